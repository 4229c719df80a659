"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP product path never does.  It wraps the plain C
implementation in mpt_oracle.c through ctypes and takes the same numpy
inputs the workload generators produce.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmpt_oracle.so")

CONVERGED, MAXITER, STALLED, DIVERGED, DEGENERATE, BAD_INPUT, LOCALMIN = range(7)

TAU_RES = 1e-9     # acceptance threshold on |R|_inf (the paper's "threshold")
MIN_SEG = 1e-6     # shortest admissible segment, metres


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP); returns the library path."""
    src = os.path.join(HERE, "mpt_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", src, "-o", LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Scene(C.Structure):
    _fields_ = [("tx", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("n_pl", C.c_int32), ("n_ln", C.c_int32), ("n_q", C.c_int32), ("n_c", C.c_int32),
                ("pl", C.c_void_p), ("ln", C.c_void_p), ("q", C.c_void_p), ("c", C.c_void_p),
                ("wd", C.c_void_p), ("sd", C.c_void_p), ("rf", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol_step", C.c_double), ("tol_res", C.c_double),
                ("tau_root", C.c_double), ("lambda0", C.c_double),
                ("plateau_win", C.c_int32), ("plateau_frac", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or (os.path.getmtime(LIB) < os.path.getmtime(os.path.join(HERE, "mpt_oracle.c"))):
            build()
        L = C.CDLL(LIB)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.orc_residual.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp]
        L.orc_residual.restype = C.c_int
        L.orc_init_line.argtypes = [vp, vp, C.c_int, vp, vp]
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_init_random.argtypes = [vp, C.c_uint64, i64, C.c_int, vp, vp]
        L.orc_init_random_batch.argtypes = [vp, C.c_uint64, i64, vp, vp, vp]
        L.orc_solve_one.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_solve_one.restype = C.c_int
        L.orc_accept_one.argtypes = [vp, vp, C.c_int, vp, vp, C.c_int, d, d]
        L.orc_accept_one.restype = C.c_int
        L.orc_solve_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
        L.orc_solve_batch_param.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
        L.orc_solve_one_param.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_solve_one_param.restype = C.c_int
        L.orc_param_residual.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp]
        L.orc_param_residual.restype = C.c_int
        L.orc_accept_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, d, d, vp, C.c_int]
        L.orc_visible_one.argtypes = [vp, vp, C.c_int, vp, vp, d]
        L.orc_visible_one.restype = C.c_int
        L.orc_visible_batch.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, d, vp, C.c_int]
        L.orc_samples.argtypes = [vp, C.c_int, C.c_int, vp]
        L.orc_samples.restype = C.c_int
        L.orc_visibility.argtypes = [vp, C.c_int, d, vp, vp, C.c_int]
        L.orc_visibility_rx.argtypes = [vp, vp, C.c_int, C.c_int, d, vp, vp, C.c_int]
        L.orc_candidates.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, i64, vp, vp, vp]
        L.orc_candidates.restype = i64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


class OracleScene:
    """Keeps the numpy arrays alive for the C struct that points at them."""

    def __init__(self, scene):
        self.keep = [np.ascontiguousarray(getattr(scene, k), dtype=np.float64)
                     for k in ("planes", "lines", "quadrics", "circles")]
        wd = getattr(scene, "wedges", None)
        self.wd = np.ascontiguousarray(wd, dtype=np.float64) if wd is not None and len(wd) else None
        sd = getattr(scene, "sides", None)
        self.sd = np.ascontiguousarray(sd, dtype=np.float64) if sd is not None and len(sd) else None
        rf = getattr(scene, "refraction", None)
        self.rf = np.ascontiguousarray(rf, dtype=np.float64) if rf is not None and len(rf) else None
        s = _Scene()
        s.tx[:] = list(scene.tx)
        s.lo[:] = list(scene.aabb_lo)
        s.hi[:] = list(scene.aabb_hi)
        s.n_pl, s.n_ln, s.n_q, s.n_c = (len(a) for a in self.keep)
        s.pl, s.ln, s.q, s.c = (_p(a) for a in self.keep)
        s.wd = _p(self.wd)
        s.sd = _p(self.sd)
        s.rf = _p(self.rf)
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def default_opts(max_iter=200, plateau_win=10, plateau_frac=0.999):
    """The parity configuration: 200 iterations, plateau window 10 at 0.999."""
    return _Opts(max_iter=max_iter, tol_step=1e-12, tol_res=1e-13, tau_root=TAU_RES, lambda0=1e-3,
                 plateau_win=plateau_win, plateau_frac=plateau_frac)


def residual(scene, rx, ids, X, jac=True):
    """Residual rows R and dense Jacobian J (rows x 3n) at points X (3n)."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    n = len(ids)
    X = np.ascontiguousarray(X, dtype=np.float64)
    R = np.zeros(4 * 5)
    J = np.zeros(4 * 5 * 3 * n) if jac else None
    m = lib().orc_residual(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), n, _p(ids),
                           _p(X), _p(R), _p(J) if jac else None)
    if m < 0:
        return None, None
    return R[:m].copy(), (J[: m * 3 * n].reshape(m, 3 * n).copy() if jac else None)


def init_line(scene, rx, ids):
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    X = np.zeros(3 * len(ids))
    lib().orc_init_line(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), len(ids), _p(ids), _p(X))
    return X


def splitmix64(seed, c):
    """Output number c+1 of SplitMix64 started from state `seed`."""
    return int(lib().orc_splitmix64(seed & (2**64 - 1), c))


def init_random(scene, seed, sid, ids):
    """Random start of solve `sid`: projections of box-uniform points."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    X = np.zeros(3 * len(ids))
    lib().orc_init_random(os_.ref, seed, sid, len(ids), _p(ids), _p(X))
    return X


def init_random_batch(scene, batch, seed):
    """[15, n] random starts of every solve of a workloads.Batch."""
    os_ = OracleScene(scene)
    x = np.zeros((15, batch.n))
    lib().orc_init_random_batch(os_.ref, seed, batch.n, _p(batch.order), _p(batch.prim), _p(x))
    return x


def param_residual(scene, rx, ids, U, jac=True):
    """Parametric form: law rows R at X(U), J = dR/dU, and X(U)."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    n = len(ids)
    U = np.ascontiguousarray(U, dtype=np.float64)
    R = np.zeros(20)
    J = np.zeros(20 * len(U)) if jac else None
    X = np.zeros(3 * n)
    m = lib().orc_param_residual(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), n, _p(ids), _p(U),
                                 _p(R), _p(J) if jac else None, _p(X))
    if m < 0:
        return None, None, None
    return R[:m].copy(), (J[: m * len(U)].reshape(m, len(U)).copy() if jac else None), X


def solve_one(scene, rx, ids, x0=None, opts=None, form="implicit"):
    """Returns (X, cost, iters, status) for one candidate path; form
    "implicit" (Eq. 12) or "param" (Eq. 15)."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    n = len(ids)
    X = np.zeros(15)
    c = C.c_double()
    it = C.c_int32()
    o = opts or default_opts()
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    f = lib().orc_solve_one_param if form == "param" else lib().orc_solve_one
    st = f(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), n, _p(ids),
           _p(x0a), C.byref(o), _p(X), C.byref(c), C.byref(it))
    return X[: 3 * n].copy(), c.value, it.value, st


def accept_one(scene, rx, ids, X, status, tau_res=TAU_RES, min_seg=MIN_SEG):
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    return bool(lib().orc_accept_one(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), len(ids),
                                     _p(ids), _p(X), int(status), tau_res, min_seg))


def solve_batch(scene, batch, x0=None, opts=None, nthreads=0, form="implicit"):
    """Solve every candidate of a workloads.Batch; returns dict of arrays
    x [15, n], cost, iters, status.  form "implicit" or "param"."""
    os_ = OracleScene(scene)
    nb = batch.n
    x = np.zeros((15, nb))
    cost = np.zeros(nb)
    iters = np.zeros(nb, np.int32)
    status = np.zeros(nb, np.uint8)
    o = opts or default_opts()
    x0 = batch.x0 if x0 is None else x0
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    f = lib().orc_solve_batch_param if form == "param" else lib().orc_solve_batch
    f(os_.ref, nb, _p(batch.rx), _p(batch.rx_index), _p(batch.order),
      _p(batch.prim), _p(x0a), C.byref(o), _p(x), _p(cost), _p(iters),
      _p(status), int(nthreads))
    return {"x": x, "cost": cost, "iters": iters, "status": status}


def accept_batch(scene, batch, x, status, tau_res=TAU_RES, min_seg=MIN_SEG, nthreads=0):
    os_ = OracleScene(scene)
    acc = np.zeros(batch.n, np.uint8)
    x = np.ascontiguousarray(x, dtype=np.float64)
    status = np.ascontiguousarray(status, dtype=np.uint8)
    lib().orc_accept_batch(os_.ref, batch.n, _p(batch.rx), _p(batch.rx_index), _p(batch.order),
                           _p(batch.prim), _p(x), _p(status), tau_res, min_seg, _p(acc), int(nthreads))
    return acc


def visible_one(scene, rx, ids, X, min_seg=MIN_SEG):
    """Physical validation of one path: no segment crosses another facet or
    paraboloid patch."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    X = np.ascontiguousarray(X, dtype=np.float64)
    return bool(lib().orc_visible_one(os_.ref, _p(np.ascontiguousarray(rx, dtype=np.float64)), len(ids), _p(ids),
                                      _p(X), min_seg))


def visible_batch(scene, batch, x, accept, min_seg=MIN_SEG, nthreads=0):
    """Visibility flags of the accepted paths of a batch (0 for the others)."""
    os_ = OracleScene(scene)
    vis = np.zeros(batch.n, np.uint8)
    x = np.ascontiguousarray(x, dtype=np.float64)
    accept = np.ascontiguousarray(accept, dtype=np.uint8)
    lib().orc_visible_batch(os_.ref, batch.n, _p(batch.rx), _p(batch.rx_index), _p(batch.order),
                            _p(batch.prim), _p(x), _p(accept), min_seg, _p(vis), int(nthreads))
    return vis


# ------------------------------------------------------------ candidate generation
def samples(scene, g, k):
    """Sample points [m, 3] of object g with k per side."""
    os_ = scene if isinstance(scene, OracleScene) else OracleScene(scene)
    pts = np.zeros((k * k + 2 * k, 3))
    m = lib().orc_samples(os_.ref, int(g), int(k), _p(pts))
    return pts[:m]


def visibility(scene, k=4, min_seg=MIN_SEG, nthreads=0):
    """Visibility matrix V [n, n] (bool, symmetric) and BS row B [n] of Alg. 1."""
    os_ = OracleScene(scene)
    n = scene.n_prims
    V = np.zeros((n, n), np.uint8)
    B = np.zeros(n, np.uint8)
    lib().orc_visibility(os_.ref, int(k), float(min_seg), _p(V), _p(B), int(nthreads))
    return V.astype(bool), B.astype(bool)


def visibility_rx(scene, rx, k=4, min_seg=MIN_SEG, nthreads=0):
    """UE columns U [n_rx, n] (object j sees receiver r) and line of sight [n_rx]."""
    os_ = OracleScene(scene)
    rx = np.ascontiguousarray(rx, dtype=np.float64).reshape(-1, 3)
    n = scene.n_prims
    U = np.zeros((len(rx), n), np.uint8)
    los = np.zeros(len(rx), np.uint8)
    lib().orc_visibility_rx(os_.ref, _p(rx), len(rx), int(k), float(min_seg), _p(U), _p(los), int(nthreads))
    return U.astype(bool), los.astype(bool)


def candidates(scene, rx, V, B, U, max_order, edge_last=False):
    """Interaction lists of Alg. 1: every simple path BS -> objects -> UE with
    1..max_order objects, receiver by receiver, order by order, in increasing
    object ids: dict of rx_index [m], order [m], prim [5, m]."""
    os_ = OracleScene(scene)
    V8 = np.ascontiguousarray(V, dtype=np.uint8)
    B8 = np.ascontiguousarray(B, dtype=np.uint8)
    U8 = np.ascontiguousarray(U, dtype=np.uint8)
    rx = np.ascontiguousarray(rx, dtype=np.float64).reshape(-1, 3)
    L = lib()
    total = L.orc_candidates(os_.ref, _p(V8), _p(B8), _p(U8), len(rx), int(max_order), int(edge_last), 0,
                             None, None, None)
    if total < 0:
        raise ValueError("bad candidate arguments")
    ri = np.zeros(max(total, 1), np.int32)
    order = np.zeros(max(total, 1), np.int32)
    prim = np.full((5, max(total, 1)), -1, np.int32)
    L.orc_candidates(os_.ref, _p(V8), _p(B8), _p(U8), len(rx), int(max_order), int(edge_last), int(total),
                     _p(ri), _p(order), _p(prim))
    return {"rx_index": ri[:total], "order": order[:total], "prim": np.ascontiguousarray(prim[:, :total])}
