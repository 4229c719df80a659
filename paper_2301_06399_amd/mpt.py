"""Thin ctypes binding of libmpt.so (include/mpt.h).

Argument marshalling only: numpy inputs become torch device tensors, torch
tensors are handed to the library as raw device pointers, and every step of
the solve runs in the library's HIP kernels.  There is no CPU fallback: if
the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmpt.so")

MPT_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVALID_ARG", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NO_SCENE",
                5: "E_UNSUPPORTED", 6: "E_NO_MODEL", 7: "E_CAPACITY"}
CONVERGED, MAXITER, STALLED, DIVERGED, DEGENERATE, BAD_INPUT, LOCALMIN, OUTSIDE = range(8)
FALLBACK = 0x80
ROW = 16  # doubles per solve in a point array (MPT_ROW)
FP64_PLAIN, FP32_POLISH64 = 0, 1
INIT_LINE, INIT_USER, INIT_LEARNED, INIT_LEARNED_ALL, INIT_RANDOM = 0, 1, 2, 3, 4
FORM_IMPLICIT, FORM_PARAMETRIC, FORM_AUTO = 0, 1, 2
SCHED_PER_ORDER, SCHED_PERSISTENT, SCHED_AUTO, SCHED_SPLIT = 0, 1, 2, 3


class MptError(RuntimeError):
    pass


class SceneDesc(C.Structure):
    _fields_ = [("tx", C.c_double * 3), ("aabb_lo", C.c_double * 3), ("aabb_hi", C.c_double * 3),
                ("n_planes", C.c_int32), ("n_lines", C.c_int32), ("n_quadrics", C.c_int32),
                ("n_circles", C.c_int32), ("planes", C.c_void_p), ("lines", C.c_void_p),
                ("quadrics", C.c_void_p), ("circles", C.c_void_p), ("wedges", C.c_void_p),
                ("sides", C.c_void_p), ("refraction", C.c_void_p)]


class BatchDesc(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_rx", C.c_int32), ("rx", C.c_void_p), ("rx_index", C.c_void_p),
                ("order", C.c_void_p), ("prim", C.c_void_p), ("x0", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("init", C.c_int32), ("max_iter", C.c_int32),
                ("max_iter32", C.c_int32), ("polish_steps", C.c_int32), ("fallback", C.c_int32),
                ("plateau_win", C.c_int32), ("sched", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("max_iter_fb", C.c_int32), ("graph", C.c_int32),
                ("plateau_frac", C.c_double), ("tol_step", C.c_double), ("tol_res", C.c_double),
                ("tau_root", C.c_double), ("lambda0", C.c_double), ("tol_step32", C.c_double),
                ("tol_res32", C.c_double), ("tau_root32", C.c_double), ("polish_gate", C.c_double),
                ("seed", C.c_uint64), ("spill", C.c_int32), ("form", C.c_int32),
                ("stat_tol", C.c_double), ("stat_win", C.c_int32), ("refill", C.c_int32),
                ("max_iter32_planar", C.c_int32), ("extent_skip", C.c_double),
                ("learned_gain", C.c_double)]


class SolveOut(C.Structure):
    _fields_ = [("x", C.c_void_p), ("cost", C.c_void_p), ("iters", C.c_void_p), ("status", C.c_void_p),
                ("stage_iters", C.c_void_p)]


EXPORTS = ["mpt_create", "mpt_destroy", "mpt_last_error", "mpt_set_stream", "mpt_synchronize",
           "mpt_scene_upload", "mpt_default_opts", "mpt_solve_batch", "mpt_accept", "mpt_mlp_init",
           "mpt_mlp_train_step", "mpt_mlp_predict", "mpt_mlp_save", "mpt_mlp_load", "mpt_last_timings",
           "mpt_flops_per_iter", "mpt_flops_assembly", "mpt_autotune", "mpt_mlp_grad", "mpt_mlp_features", "mpt_mlp_param_count",
           "mpt_gemm_bf16_check", "mpt_last_lm_timings", "mpt_mlp_predict_unfused", "mpt_visible",
           "mpt_visibility", "mpt_visibility_rx", "mpt_candidates", "mpt_last_launch", "mpt_set_timing",
           "mpt_solve_batch_noalloc", "mpt_mlp_grad_fp32"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmpt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MptError(f"{path} is missing: build it with paper_2301_06399_amd.build.build()")
    # the library and torch must share one HIP runtime: torch's, loaded first
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, st = C.c_void_p, C.c_int
    L.mpt_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.mpt_destroy.argtypes = [vp]
    L.mpt_last_error.argtypes = [vp]
    L.mpt_last_error.restype = C.c_char_p
    L.mpt_set_stream.argtypes = [vp, vp]
    L.mpt_synchronize.argtypes = [vp]
    L.mpt_scene_upload.argtypes = [vp, C.POINTER(SceneDesc)]
    L.mpt_default_opts.argtypes = [C.POINTER(SolveOpts)]
    L.mpt_default_opts.restype = None
    L.mpt_solve_batch.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(SolveOpts), C.POINTER(SolveOut)]
    L.mpt_solve_batch_noalloc.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(SolveOpts), C.POINTER(SolveOut)]
    L.mpt_accept.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(SolveOut), C.c_double, C.c_double, vp, vp, vp,
                             C.POINTER(C.c_int64)]
    L.mpt_visible.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(SolveOut), vp, C.c_double, vp, vp,
                              C.POINTER(C.c_int64)]
    L.mpt_visibility.argtypes = [vp, C.c_int32, C.c_double, vp, vp]
    L.mpt_visibility_rx.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_double, vp, vp]
    L.mpt_candidates.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int64, vp, vp, vp,
                                 C.POINTER(C.c_int64)]
    L.mpt_mlp_init.argtypes = [vp, C.c_uint64]
    L.mpt_mlp_train_step.argtypes = [vp, C.POINTER(BatchDesc), vp, vp, vp, C.c_int32, C.c_float, vp]
    L.mpt_mlp_grad.argtypes = [vp, C.POINTER(BatchDesc), vp, vp, vp, C.c_int32, vp, vp]
    L.mpt_mlp_grad_fp32.argtypes = [vp, C.POINTER(BatchDesc), vp, vp, vp, C.c_int32, vp, vp]
    L.mpt_mlp_features.argtypes = [vp, C.POINTER(BatchDesc), vp]
    L.mpt_mlp_param_count.argtypes = [C.POINTER(C.c_size_t)]
    L.mpt_gemm_bf16_check.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int32, vp, C.c_int32, vp,
                                      C.c_int32]
    L.mpt_mlp_predict.argtypes = [vp, C.POINTER(BatchDesc), vp]
    L.mpt_mlp_predict_unfused.argtypes = [vp, C.POINTER(BatchDesc), vp]
    L.mpt_mlp_save.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.mpt_mlp_load.argtypes = [vp, vp, C.c_size_t]
    L.mpt_last_timings.argtypes = [vp, C.POINTER(C.c_float)]
    L.mpt_flops_per_iter.argtypes = [C.c_int, vp, C.c_int32, vp]
    L.mpt_flops_assembly.argtypes = [C.c_int, vp, C.c_int32, vp]
    L.mpt_last_lm_timings.argtypes = [vp, C.POINTER(C.c_float)]
    L.mpt_last_launch.argtypes = [vp, C.POINTER(C.c_int32)]
    L.mpt_set_timing.argtypes = [vp, C.c_int32]
    L.mpt_autotune.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(SolveOpts), C.POINTER(SolveOut),
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_float),
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    for f in EXPORTS:
        getattr(L, f).restype = st if f not in ("mpt_last_error", "mpt_default_opts") else getattr(L, f).restype
    _lib = L
    return L


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().mpt_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def to_rows(x):
    """[15][n] points (the host batches' layout) -> the library's [n][ROW]
    rows, zero beyond the 15 coordinates."""
    x = np.asarray(x, np.float64)
    r = np.zeros((x.shape[1], ROW), np.float64)
    r[:, :x.shape[0]] = x.T
    return r


class DeviceBatch:
    """A batch's arrays resident in device memory (torch tensors)."""

    def __init__(self, batch, device="cuda"):
        import torch
        self.n = int(batch.n)
        self.n_rx = int(len(batch.rx))
        self.rx = torch.from_numpy(np.ascontiguousarray(batch.rx, np.float64)).to(device)
        self.rx_index = torch.from_numpy(np.ascontiguousarray(batch.rx_index, np.int32)).to(device)
        self.order = torch.from_numpy(np.ascontiguousarray(batch.order, np.int32)).to(device)
        self.prim = torch.from_numpy(np.ascontiguousarray(batch.prim, np.int32)).to(device)
        self.x0 = None if batch.x0 is None else torch.from_numpy(to_rows(batch.x0)).to(device)

    def desc(self) -> BatchDesc:
        return BatchDesc(self.n, self.n_rx, _ptr(self.rx), _ptr(self.rx_index), _ptr(self.order), _ptr(self.prim),
                         _ptr(self.x0))


def unpack_bits(words, n: int) -> np.ndarray:
    """Bit words (a tensor or array [..., W]) -> bool array [..., n]."""
    w = words.cpu().numpy() if hasattr(words, "cpu") else np.asarray(words)
    w = np.ascontiguousarray(w).view(np.uint32)
    bits = (w[..., :, None] >> np.arange(32, dtype=np.uint32)) & 1
    return bits.reshape(*w.shape[:-1], -1)[..., :n].astype(bool)


def device_batch(rx, rx_index, order, prim):
    """A DeviceBatch over device tensors already in place (e.g. candidates)."""
    db = DeviceBatch.__new__(DeviceBatch)
    db.n, db.n_rx = int(rx_index.shape[0]), int(rx.shape[0])
    db.rx, db.rx_index, db.order, db.prim, db.x0 = rx, rx_index, order, prim, None
    return db


class DeviceOut:
    def __init__(self, n, device="cuda", stages=False):
        import torch
        # one row of ROW doubles per solve (the library's point layout)
        self.x = torch.empty((max(n, 0), ROW), dtype=torch.float64, device=device)
        self.cost = torch.empty(max(n, 0), dtype=torch.float64, device=device)
        self.iters = torch.empty(max(n, 0), dtype=torch.int32, device=device)
        self.status = torch.empty(max(n, 0), dtype=torch.uint8, device=device)
        self.stage = torch.empty((4, max(n, 0)), dtype=torch.int32, device=device) if stages else None

    def desc(self) -> SolveOut:
        return SolveOut(_ptr(self.x), _ptr(self.cost), _ptr(self.iters), _ptr(self.status), _ptr(self.stage))

    def points(self):
        """The points as a [15][n] view of the row-major array."""
        return self.x[:, :15].t()

    def numpy(self):
        r = {"x": np.ascontiguousarray(self.points().cpu().numpy()), "cost": self.cost.cpu().numpy(),
             "iters": self.iters.cpu().numpy(),
             "status": self.status.cpu().numpy()}
        if self.stage is not None:
            r["stage"] = self.stage.cpu().numpy()
        return r


def flops_per_iter(types, form=FORM_IMPLICIT) -> dict:
    """Algorithmic FLOPs of one LM iteration / polish step / residual
    evaluation for a path with the given primitive types (host only)."""
    L = load_library()
    t = np.ascontiguousarray(types, np.int32)
    out = np.zeros(4, np.int64)
    rc = L.mpt_flops_per_iter(len(t), t.ctypes.data, int(form), out.ctypes.data)
    if rc != MPT_OK:
        raise MptError(f"mpt_flops_per_iter: {STATUS_NAMES.get(rc, rc)}")
    a = np.zeros(1, np.int64)
    rc = L.mpt_flops_assembly(len(t), t.ctypes.data, int(form), a.ctypes.data)
    if rc != MPT_OK:
        raise MptError(f"mpt_flops_assembly: {STATUS_NAMES.get(rc, rc)}")
    return {"lm": int(out[0]), "polish": int(out[1]), "residual": int(out[2]), "sqrt_div": int(out[3]),
            "assembly": int(a[0])}


def flops_table(form=FORM_IMPLICIT) -> dict:
    """FLOPs per iteration for every order 1..5 and type combination, as
    dense arrays indexed by the base-4 code sum(type_k * 4**k)."""
    tab = {}
    for n in range(1, 6):
        lm = np.zeros(4 ** n, np.int64)
        po = np.zeros(4 ** n, np.int64)
        re_ = np.zeros(4 ** n, np.int64)
        asm = np.zeros(4 ** n, np.int64)
        for code in range(4 ** n):
            types = [(code // 4 ** k) % 4 for k in range(n)]
            f = flops_per_iter(types, form)
            lm[code], po[code], re_[code], asm[code] = f["lm"], f["polish"], f["residual"], f["assembly"]
        tab[n] = {"lm": lm, "polish": po, "residual": re_, "assembly": asm}
    return tab


class Context:
    """One library context on one GPU.

    The library enqueues on a stream of its own (a torch stream of default
    priority).  Every call first makes that stream wait for the caller's
    current stream (inputs written by torch) and afterwards makes the
    caller's current stream wait for it (outputs read by torch), so torch
    code sees the results in order without host synchronisation."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.L = load_library()
        if not torch.cuda.is_available():
            raise MptError("no HIP device available")
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        if self.stream.cuda_stream == 0:
            raise MptError("the library needs a stream other than the null stream")
        h = C.c_void_p()
        rc = self.L.mpt_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != MPT_OK:
            raise MptError(f"mpt_create failed: {STATUS_NAMES.get(rc, rc)}")
        self.h = h

    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _leave(self):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _check(self, rc, what):
        if rc != MPT_OK:
            msg = self.L.mpt_last_error(self.h).decode()
            raise MptError(f"{what}: {STATUS_NAMES.get(rc, rc)}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.L.mpt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_scene(self, scene):
        self._enter()
        keep = [np.ascontiguousarray(getattr(scene, k), np.float64) for k in ("planes", "lines", "quadrics", "circles")]
        d = SceneDesc()
        d.tx[:] = list(map(float, scene.tx))
        d.aabb_lo[:] = list(map(float, scene.aabb_lo))
        d.aabb_hi[:] = list(map(float, scene.aabb_hi))
        d.n_planes, d.n_lines, d.n_quadrics, d.n_circles = (len(a) for a in keep)
        d.planes, d.lines, d.quadrics, d.circles = (a.ctypes.data if a.size else None for a in keep)
        wd = getattr(scene, "wedges", None)
        if wd is not None and len(wd):
            wd = np.ascontiguousarray(wd, np.float64)
            if wd.shape != (len(keep[1]), 7):
                raise ValueError("wedges: one record of 7 values per straight edge")
            d.wedges = wd.ctypes.data
        sd = getattr(scene, "sides", None)
        if sd is not None and len(sd):
            sd = np.ascontiguousarray(sd, np.float64)
            if sd.shape != (len(keep[0]),):
                raise ValueError("sides: one value per plane facet")
            d.sides = sd.ctypes.data
        rf = getattr(scene, "refraction", None)
        if rf is not None and len(rf):
            rf = np.ascontiguousarray(rf, np.float64)
            if rf.shape != (len(keep[0]), 2):
                raise ValueError("refraction: two indices per plane facet")
            d.refraction = rf.ctypes.data
        self._check(self.L.mpt_scene_upload(self.h, C.byref(d)), "mpt_scene_upload")
        self.n_all = int(sum(len(a) for a in keep))

    def solve(self, dbatch: DeviceBatch, opts: SolveOpts | None = None, out: DeviceOut | None = None) -> DeviceOut:
        out = out or DeviceOut(dbatch.n)
        o = opts or default_opts()
        bd, od = dbatch.desc(), out.desc()
        self._enter()
        rc = self.L.mpt_solve_batch(self.h, C.byref(bd), C.byref(o), C.byref(od))
        self._leave()
        self._check(rc, "mpt_solve_batch")
        return out

    def solve_noalloc(self, dbatch: DeviceBatch, opts: SolveOpts, out: DeviceOut) -> DeviceOut:
        """mpt_solve_batch_noalloc: the caller's outputs, the library's static
        scratch, no allocation."""
        bd, od = dbatch.desc(), out.desc()
        self._enter()
        rc = self.L.mpt_solve_batch_noalloc(self.h, C.byref(bd), C.byref(opts), C.byref(od))
        self._leave()
        self._check(rc, "mpt_solve_batch_noalloc")
        return out

    def accept(self, dbatch: DeviceBatch, out: DeviceOut, tau_res=1e-9, min_seg=1e-6, sync=True):
        torch = self.torch
        n = dbatch.n
        acc = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
        idx = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        cnt = torch.empty(1, dtype=torch.int32, device="cuda")
        hc = C.c_int64(0)
        bd, od = dbatch.desc(), out.desc()
        self._enter()
        rc = self.L.mpt_accept(self.h, C.byref(bd), C.byref(od), tau_res, min_seg, _ptr(acc), _ptr(idx),
                               _ptr(cnt), C.byref(hc) if sync else None)
        self._leave()
        self._check(rc, "mpt_accept")
        k = int(hc.value) if sync else None
        return acc[:n], (idx[:k] if sync else idx), (k if sync else cnt)

    def visible(self, dbatch: DeviceBatch, out: DeviceOut, accept, min_seg=1e-6, sync=True):
        """Physical validation of the accepted paths: returns (visible flags
        [n] uint8 device tensor, count or None)."""
        torch = self.torch
        vis = torch.empty(max(dbatch.n, 1), dtype=torch.uint8, device="cuda")
        cnt = torch.empty(1, dtype=torch.int32, device="cuda")
        hc = C.c_int64(0)
        bd, od = dbatch.desc(), out.desc()
        self._enter()
        rc = self.L.mpt_visible(self.h, C.byref(bd), C.byref(od), _ptr(accept), min_seg, _ptr(vis), _ptr(cnt),
                                C.byref(hc) if sync else None)
        self._leave()
        self._check(rc, "mpt_visible")
        return vis[:dbatch.n], (hc.value if sync else None)

    def visibility(self, k=4, min_seg=1e-6):
        """Visibility matrix of the uploaded scene's objects and the BS row, as
        int32 tensors of bit words [n_all, W] and [W] (W = (n_all + 31) // 32)."""
        torch = self.torch
        W = (self.n_all + 31) // 32
        V = torch.empty((max(self.n_all, 1), W), dtype=torch.int32, device="cuda")
        B = torch.empty(W, dtype=torch.int32, device="cuda")
        self._enter()
        rc = self.L.mpt_visibility(self.h, int(k), float(min_seg), _ptr(V), _ptr(B))
        self._leave()
        self._check(rc, "mpt_visibility")
        return V[:self.n_all], B

    def visibility_rx(self, rx, k=4, min_seg=1e-6):
        """The objects each receiver sees (bit words [n_rx, W]) and the line
        of sight [n_rx] uint8; rx is a [n_rx, 3] float64 device tensor."""
        torch = self.torch
        W = (self.n_all + 31) // 32
        n_rx = int(rx.shape[0])
        U = torch.empty((max(n_rx, 1), W), dtype=torch.int32, device="cuda")
        los = torch.empty(max(n_rx, 1), dtype=torch.uint8, device="cuda")
        self._enter()
        rc = self.L.mpt_visibility_rx(self.h, _ptr(rx), n_rx, int(k), float(min_seg), _ptr(U), _ptr(los))
        self._leave()
        self._check(rc, "mpt_visibility_rx")
        return U[:n_rx], los[:n_rx]

    def candidates(self, V, B, U, max_order, edge_last=False):
        """Every simple path BS -> objects -> UE (Alg. 1) per receiver row of
        U: device tensors rx_index [m], order [m], prim [5, m] int32."""
        torch = self.torch
        n_rx = int(U.shape[0])
        tot = C.c_int64(0)
        self._enter()
        rc = self.L.mpt_candidates(self.h, _ptr(V), _ptr(B), _ptr(U), n_rx, int(max_order), int(edge_last), 0,
                                   None, None, None, C.byref(tot))
        self._check(rc, "mpt_candidates")
        m = tot.value
        ri = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        order = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        prim = torch.empty((5, max(m, 1)), dtype=torch.int32, device="cuda")
        if m > 0:
            rc = self.L.mpt_candidates(self.h, _ptr(V), _ptr(B), _ptr(U), n_rx, int(max_order), int(edge_last), m,
                                       _ptr(ri), _ptr(order), _ptr(prim), C.byref(tot))
        self._leave()
        self._check(rc, "mpt_candidates")
        return ri[:m], order[:m], prim[:, :m]

    def autotune(self, dbatch: DeviceBatch, opts: SolveOpts | None = None, out: DeviceOut | None = None):
        out = out or DeviceOut(dbatch.n)
        o = opts or default_opts()
        sch, blk, ms, gd, sp, fm = C.c_int32(), C.c_int32(), C.c_float(), C.c_int32(), C.c_int32(), C.c_int32()
        bd, od = dbatch.desc(), out.desc()
        self._enter()
        rc = self.L.mpt_autotune(self.h, C.byref(bd), C.byref(o), C.byref(od), C.byref(sch), C.byref(blk),
                                 C.byref(ms), C.byref(gd), C.byref(sp), C.byref(fm))
        self._leave()
        self._check(rc, "mpt_autotune")
        return {"sched": sch.value, "block": blk.value, "gdiv": gd.value, "spill": sp.value, "form": fm.value,
                "ms": ms.value}

    def synchronize(self):
        self._check(self.L.mpt_synchronize(self.h), "mpt_synchronize")

    def timings(self):
        ms = (C.c_float * 6)()
        self._check(self.L.mpt_last_timings(self.h, ms), "mpt_last_timings")
        return {"bin": ms[0], "learned": ms[1], "lm": ms[2], "resume": ms[3], "polish": ms[4], "fallback": ms[5]}

    def set_timing(self, on: bool):
        """Stage events in every solve (on by default; off saves their cost
        on the stream, and timings() then fails)."""
        self._check(self.L.mpt_set_timing(self.h, 1 if on else 0), "mpt_set_timing")

    def last_launch(self):
        """Schedule, block, grid divisor, straggler threshold and resolved
        form of the last solve's first LM pass."""
        v = (C.c_int32 * 5)()
        self._check(self.L.mpt_last_launch(self.h, v), "mpt_last_launch")
        return {"sched": v[0], "block": v[1], "gdiv": v[2], "spill": v[3], "form": v[4]}

    def lm_timings(self):
        """Per-order kernel durations (ms) of the last per-order LM pass."""
        ms = (C.c_float * 5)()
        self._check(self.L.mpt_last_lm_timings(self.h, ms), "mpt_last_lm_timings")
        return [ms[i] for i in range(5)]

    # ---------------------------------------------------------------- network
    def mlp_init(self, seed: int = 0):
        self._enter()
        rc = self.L.mpt_mlp_init(self.h, C.c_uint64(seed))
        self._leave()
        self._check(rc, "mpt_mlp_init")

    def mlp_train_step(self, dbatch: DeviceBatch, target_x, use=None, lr=1e-3, loss=None, rows=None):
        bd = dbatch.desc()
        nr = int(rows.numel()) if rows is not None else dbatch.n
        self._enter()
        rc = self.L.mpt_mlp_train_step(self.h, C.byref(bd), _ptr(target_x), _ptr(use), _ptr(rows), nr,
                                       C.c_float(lr), _ptr(loss))
        self._leave()
        self._check(rc, "mpt_mlp_train_step")

    def mlp_grad(self, dbatch: DeviceBatch, target_x, use=None, rows=None, fp32=False):
        """Loss and gradient without an update; fp32: the FP32 check mode."""
        torch = self.torch
        n = C.c_size_t(0)
        self.L.mpt_mlp_param_count(C.byref(n))
        g = torch.empty(n.value, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        bd = dbatch.desc()
        nr = int(rows.numel()) if rows is not None else dbatch.n
        self._enter()
        fn = self.L.mpt_mlp_grad_fp32 if fp32 else self.L.mpt_mlp_grad
        rc = fn(self.h, C.byref(bd), _ptr(target_x), _ptr(use), _ptr(rows), nr, _ptr(loss), _ptr(g))
        self._leave()
        self._check(rc, "mpt_mlp_grad_fp32" if fp32 else "mpt_mlp_grad")
        return float(loss.item()), g

    def mlp_features(self, dbatch: DeviceBatch):
        f = self.torch.empty((dbatch.n, 96), dtype=self.torch.float32, device="cuda")
        bd = dbatch.desc()
        self._enter()
        rc = self.L.mpt_mlp_features(self.h, C.byref(bd), _ptr(f))
        self._leave()
        self._check(rc, "mpt_mlp_features")
        return f

    def gemm_bf16_check(self, A, B, a_trans=False, b_trans=False, splits=1):
        """C = A B on the matrix cores (inputs rounded to BF16, FP32 sums).
        A, B: float32 CUDA tensors laid out as the flags say."""
        torch = self.torch
        if a_trans:
            K, M = A.shape
        else:
            M, K = A.shape
        N = B.shape[0] if b_trans else B.shape[1]
        Cm = torch.empty((M, N), dtype=torch.float32, device="cuda")
        self._enter()
        rc = self.L.mpt_gemm_bf16_check(self.h, M, N, K, _ptr(A.contiguous()), int(a_trans), _ptr(B.contiguous()),
                                        int(b_trans), _ptr(Cm), splits)
        self._leave()
        self._check(rc, "mpt_gemm_bf16_check")
        return Cm

    def mlp_predict_unfused(self, dbatch: DeviceBatch, x_out=None):
        x_out = x_out if x_out is not None else self.torch.zeros((dbatch.n, ROW), dtype=self.torch.float64,
                                                                 device="cuda")
        bd = dbatch.desc()
        self._enter()
        rc = self.L.mpt_mlp_predict_unfused(self.h, C.byref(bd), _ptr(x_out))
        self._leave()
        self._check(rc, "mpt_mlp_predict_unfused")
        return x_out[:, :15].t()

    def mlp_predict(self, dbatch: DeviceBatch, x_out=None):
        x_out = x_out if x_out is not None else self.torch.empty((dbatch.n, ROW), dtype=self.torch.float64,
                                                                 device="cuda")
        bd = dbatch.desc()
        self._enter()
        rc = self.L.mpt_mlp_predict(self.h, C.byref(bd), _ptr(x_out))
        self._leave()
        self._check(rc, "mpt_mlp_predict")
        return x_out[:, :15].t()

    def mlp_save(self) -> bytes:
        n = C.c_size_t(0)
        self._check(self.L.mpt_mlp_save(self.h, None, C.byref(n)), "mpt_mlp_save")
        buf = (C.c_char * n.value)()
        self._check(self.L.mpt_mlp_save(self.h, buf, C.byref(n)), "mpt_mlp_save")
        return bytes(buf)

    def mlp_load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._enter()
        rc = self.L.mpt_mlp_load(self.h, buf, len(blob))
        self._leave()
        self._check(rc, "mpt_mlp_load")
