"""Closed-form answers for paths of planes and straight edges.

Test infrastructure, written independently of the oracle and of the HIP
library: no residual rows, no Levenberg-Marquardt, no shared helpers.  It
answers "does this interaction list have a path, and where are its points"
from two facts the paper and the mathematics fix:

* Image method (Sec. III-A, Eqs. (5)-(6)): on planes, mirror TX through the
  planes in order, then intersect backwards from RX.  A path exists iff
  every backward intersection lies strictly between its start and the
  image (fraction t in (0, 1)); then it is unique.
* Fermat's principle (Sec. II, Eqs. (1) and (3)): on infinite planes and
  straight lines the total length sum |X_{k+1} - X_k| is a sum of norms of
  affine maps of the objects' parameters, so it is convex.  The reflection
  law up to its sign and the Keller law are exactly its stationarity
  where no segment is empty.  A path exists iff the global minimiser has
  no empty segment and each reflection returns to the incoming side (the
  sign of Eq. (1)).  The minimiser is found by Newton's method on the
  smoothed length sum sqrt(|d|^2 + eps^2), with eps driven to zero, so the
  kink of an empty segment cannot stall it.

The acceptance rule on top of existence (finite extents, shortest segment,
no grazing reflection) is restated here from its definition.
"""
from __future__ import annotations

import os

import numpy as np

MIN_SEG = 1e-6      # shortest admissible segment (m)
GRAZE = 1e-9        # smallest admissible |cos| between incoming ray and normal


def _orthonormal_pair(n):
    """Any orthonormal pair spanning the plane with unit normal n, rows [B,3]."""
    a = np.zeros_like(n)
    i = np.argmin(np.abs(n), axis=1)
    a[np.arange(len(n)), i] = 1.0
    u = np.cross(n, a)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u, np.cross(n, u)


# ---------------------------------------------------------------- image method
def image_method(tx, rx, normals, offsets):
    """Eqs. (5)-(6) for a batch of reflection-only chains.

    tx [3]; rx [B,3]; normals [B,n,3] unit; offsets [B,n] (n.x = d).
    Returns points [B,n,3] and the backward fractions t [B,n]; a path exists
    iff every t is in (0, 1)."""
    B, n, _ = normals.shape
    I = [np.broadcast_to(np.asarray(tx, float), (B, 3))]
    for k in range(n):
        nv, d = normals[:, k], offsets[:, k]
        s = np.einsum("bi,bi->b", I[-1], nv) - d
        I.append(I[-1] - 2.0 * s[:, None] * nv)
    X = np.empty((B, n, 3))
    t = np.empty((B, n))
    nxt = np.asarray(rx, float)
    with np.errstate(divide="ignore", invalid="ignore"):
        for k in range(n - 1, -1, -1):
            nv, d = normals[:, k], offsets[:, k]
            v = I[k + 1] - nxt
            den = np.einsum("bi,bi->b", v, nv)
            tk = (d - np.einsum("bi,bi->b", nxt, nv)) / den
            X[:, k] = nxt + tk[:, None] * v
            t[:, k] = tk
            nxt = X[:, k]
    return X, t


# ---------------------------------------------------------------- Fermat
def _fermat_eval(tx, rx, O, Bm, z, eps, want_hess=True, wt=None):
    """Smoothed optical length sum_j wt_j sqrt(|d_j|^2 + eps^2) (wt: the
    refractive index of each segment's medium, 1 by default), its gradient
    and Hessian in the parameters z [B,n,2] of the points P_k = O_k + Bm_k z_k
    (O [B,n,3], Bm [B,n,3,2] with orthonormal columns; a line's second
    column is zero).

    With w = d/s the unit-ish segment directions, the Hessian of one term
    is wt (I - w w^T)/s; its blocks in z are wt B_k^T (I - w w^T) B_l / s,
    formed from the Gram matrices B_k^T B_l and the projections B_k^T w."""
    B, n = z.shape[0], z.shape[1]
    if wt is None:
        wt = np.ones((B, n + 1))
    X = O + (Bm @ z[..., None])[..., 0]
    P = np.concatenate([np.broadcast_to(tx, (B, 1, 3)), X, rx[:, None]], axis=1)
    d = P[:, 1:] - P[:, :-1]                                  # [B,n+1,3]
    s = np.sqrt((d * d).sum(-1) + eps * eps)                  # [B,n+1]
    f = (wt * s).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = d / s[..., None]
        Bt = np.swapaxes(Bm, -1, -2)
        a = (Bt @ w[:, :-1, :, None])[..., 0]                 # B_k^T w (segment into X_k)
        c = (Bt @ w[:, 1:, :, None])[..., 0]                  # B_k^T w (segment out of X_k)
        wi, wo = wt[:, :-1, None], wt[:, 1:, None]
        g = wi * a - wo * c                                   # [B,n,2]
        if not want_hess:
            return f, g, None, X
        si, so = s[:, :-1, None, None], s[:, 1:, None, None]
        G = Bt @ Bm                                           # [B,n,2,2]
        Dg = (wi[..., None] * (G - a[..., :, None] * a[..., None, :]) / si
              + wo[..., None] * (G - c[..., :, None] * c[..., None, :]) / so)
        Ck = Bt[:, :-1] @ Bm[:, 1:]                           # [B,n-1,2,2]
        Of = -wt[:, 1:-1, None, None] * (Ck - c[:, :-1, :, None] * a[:, 1:, None, :]) / s[:, 1:-1, None, None]
    H = np.zeros((B, n, 2, n, 2))
    k = np.arange(n)
    H[:, k, :, k, :] = np.moveaxis(Dg, 1, 0)
    if n > 1:
        H[:, k[:-1], :, k[1:], :] = np.moveaxis(Of, 1, 0)
        H[:, k[1:], :, k[:-1], :] = np.moveaxis(np.swapaxes(Of, -1, -2), 1, 0)
    return f, g, H.reshape(B, 2 * n, 2 * n), X


def fermat_minimiser(tx, rx, O, Bm, free, z0, wt=None):
    """Global minimiser of the total length over infinite planes and lines.

    O [B,n,3] is a point of each object and Bm [B,n,3,2] an orthonormal
    basis of its directions (a line's second column is zero and its second
    parameter is not free: free [B,n,2]).  Damped Newton with backtracking
    on the smoothed length, eps = 1, 1e-2, ..., 1e-12, then exact Newton
    steps where no segment is nearly empty.  wt [B,n+1]: the refractive index
    of each segment's medium (the optical length), 1 by default.  Returns the
    points [B,n,3], the largest exact gradient component and the shortest
    segment."""
    tx = np.asarray(tx, float)
    z = z0 * free
    B, n = z.shape[0], z.shape[1]
    wt = np.ones((B, n + 1)) if wt is None else np.asarray(wt, float)
    fixed = (~free).reshape(B, 2 * n).astype(float)
    ladder = 0.5 ** np.arange(12)

    def newton_dir(H, g, idx):
        Hr = H + (1e-14 * np.abs(np.einsum("bii->b", H))[:, None] + fixed[idx])[:, :, None] * np.eye(2 * n)
        gr = g.reshape(len(idx), 2 * n) * (1 - fixed[idx])
        return -np.linalg.solve(Hr, gr[..., None])[..., 0].reshape(len(idx), n, 2)

    for eps in (1.0, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12):
        act = np.arange(B)
        for _ in range(80):
            if not len(act):
                break
            Oi, Bi, rxi, zi = O[act], Bm[act], rx[act], z[act]
            f, g, H, _ = _fermat_eval(tx, rxi, Oi, Bi, zi, eps, wt=wt[act])
            dz = newton_dir(H, g, act)
            slope = (g * dz).sum((1, 2))
            # backtracking: the full step first, then ladders of shorter ones,
            # each ladder tried at once
            m = len(act)
            f1, _, _, _ = _fermat_eval(tx, rxi, Oi, Bi, zi + dz, eps, want_hess=False, wt=wt[act])
            step = np.where(f1 <= f + 1e-4 * slope, 1.0, 0.0)
            for lad in range(6):
                pend = np.where(step == 0.0)[0]
                if not len(pend):
                    break
                lv = ladder * 0.5 ** (1 + 12 * lad)
                L = len(lv)
                q = len(pend)
                zt = zi[pend][:, None] + lv[None, :, None, None] * dz[pend][:, None]
                ft, _, _, _ = _fermat_eval(tx, np.repeat(rxi[pend], L, 0), np.repeat(Oi[pend], L, 0),
                                           np.repeat(Bi[pend], L, 0), zt.reshape(q * L, n, 2), eps,
                                           want_hess=False, wt=np.repeat(wt[act][pend], L, 0))
                ok = ft.reshape(q, L) <= f[pend, None] + 1e-4 * lv[None, :] * slope[pend, None]
                hit = ok.any(1)
                step[pend[hit]] = lv[ok[hit].argmax(1)]
            z[act] = zi + step[:, None, None] * dz
            moved = np.abs(step[:, None, None] * dz).max((1, 2))
            # a smoothed stage only warm-starts the next one; the last is
            # taken to rounding level
            tol = max(1e-13, 1e-4 * eps)
            done = (moved <= tol * (1 + np.abs(zi).max((1, 2)))) | (np.abs(g).max((1, 2)) <= 1e-15)
            act = act[~done]
    f, g, _, X = _fermat_eval(tx, rx, O, Bm, z, 0.0, want_hess=False, wt=wt)
    P = np.concatenate([np.broadcast_to(tx, (B, 1, 3)), X, rx[:, None]], axis=1)
    smin = np.linalg.norm(np.diff(P, axis=1), axis=2).min(1)
    smooth = np.where(smin > 1e-9)[0]
    for _ in range(3):
        if not len(smooth):
            break
        Oi, Bi, rxi = O[smooth], Bm[smooth], rx[smooth]
        f0, g0, H0, _ = _fermat_eval(tx, rxi, Oi, Bi, z[smooth], 0.0, wt=wt[smooth])
        dz = newton_dir(H0, g0, smooth)
        _, g1, _, _ = _fermat_eval(tx, rxi, Oi, Bi, z[smooth] + dz, 0.0, want_hess=False, wt=wt[smooth])
        better = np.abs(g1 * free[smooth]).max((1, 2)) < np.abs(g0 * free[smooth]).max((1, 2))
        z[smooth[better]] += dz[better]
    f, g, _, X = _fermat_eval(tx, rx, O, Bm, z, 0.0, want_hess=False, wt=wt)
    P = np.concatenate([np.broadcast_to(tx, (B, 1, 3)), X, rx[:, None]], axis=1)
    smin = np.linalg.norm(np.diff(P, axis=1), axis=2).min(1)
    gn = np.nan_to_num(np.abs(g * free).max((1, 2)), nan=np.inf)
    return X, gn, smin


# ---------------------------------------------------------------- acceptance
def _rect_coords(rec, X):
    o, eu, ev = rec[:, 4:7], rec[:, 7:10], rec[:, 10:13]
    w = X - o
    return (np.einsum("bi,bi->b", w, eu), np.einsum("bi,bi->b", eu, eu),
            np.einsum("bi,bi->b", w, ev), np.einsum("bi,bi->b", ev, ev), np.linalg.norm(eu, axis=1),
            np.linalg.norm(ev, axis=1))


def planar_paths_closed_form(scene, batch, idx=None, margin=1e-7):
    """Closed-form accept flags of paths whose objects are all planes and
    straight edges (the planes reflect, or refract where the scene gives
    them refractive indices).

    Returns (idx, accept, ambiguous, X): the solve ids considered (the
    planar ones among `idx`), the flags the acceptance rule gives at the
    closed-form root, a mask of solves whose decision lies within `margin`
    of one of its thresholds (a point on the border of its extent, a
    segment of about 1e-6 m, a nearly grazing reflection, a nearly empty
    segment at the minimiser), and the closed-form points [n, 15]."""
    npl, nln = len(scene.planes), len(scene.lines)
    if idx is None:
        idx = np.arange(batch.n)
    idx = np.asarray(idx)
    order = batch.order[idx]
    prim = batch.prim[:, idx]
    typ = np.where(prim < 0, -1, np.where(prim < npl, 0, np.where(prim < npl + nln, 1, 2)))
    act = np.arange(5)[:, None] < order[None, :]
    planar = np.all(~act | (typ <= 1), axis=0) & (order >= 1)
    idx, order, prim, typ = idx[planar], order[planar], prim[:, planar], typ[:, planar]
    acc = np.zeros(len(idx), bool)
    amb = np.zeros(len(idx), bool)
    Xall = np.zeros((len(idx), 15))
    tx = np.asarray(scene.tx, float)
    # a dummy record where a scene has no planes or no lines, so that the
    # per-slot gathers below always have a row to read
    planes = scene.planes if npl else np.array([[0, 0, 1.0] + [0.0] * 10])
    lines = scene.lines if nln else np.zeros((1, 8))
    rxall = batch.rx[batch.rx_index[idx]]
    # refractive indices (front, back) of each facet slot; (0, 0): a mirror
    rfi = (scene.refraction if len(getattr(scene, "refraction", [])) else np.zeros((max(npl, 1), 2)))
    refr = (typ == 0) & (rfi[np.where(typ == 0, prim, 0), 0] > 0)
    # reflection-only chains take the image method, the others Fermat (the
    # optical length where a facet refracts); both are grouped by order
    refl_only = (np.all(~act[:, planar] | (typ == 0), axis=0) & ~np.any(refr, axis=0)) if len(idx) \
        else np.zeros(0, bool)
    code = order * 2 + refl_only
    for c in np.unique(code):
        sel = np.where(code == c)[0]
        n = int(order[sel[0]])
        kinds = typ[:n, sel]                                  # [n, B]
        rx = rxall[sel]
        pl = [planes[np.where(kinds[k] == 0, prim[k, sel], 0)] for k in range(n)]
        ln = [lines[np.where(kinds[k] == 1, prim[k, sel] - npl, 0)] for k in range(n)]
        if refl_only[sel[0]]:
            X, t = image_method(tx, rx, np.stack([r[:, 0:3] for r in pl], 1), np.stack([r[:, 3] for r in pl], 1))
            exists = np.all((t > 0) & (t < 1), axis=1)
            unsure = np.any((np.abs(t) < 1e-9) | (np.abs(t - 1) < 1e-9), axis=1)
            X = np.where(np.isfinite(X), X, 0.0)
        else:
            Bn = len(sel)
            O = np.empty((Bn, n, 3))
            Bm = np.zeros((Bn, n, 3, 2))
            free = np.ones((Bn, n, 2), bool)
            z0 = np.empty((Bn, n, 2))
            for k in range(n):
                isp = kinds[k] == 0
                u, v = _orthonormal_pair(pl[k][:, 0:3])
                O[:, k] = np.where(isp[:, None], pl[k][:, 0:3] * pl[k][:, 3:4], ln[k][:, 0:3])
                Bm[:, k, :, 0] = np.where(isp[:, None], u, ln[k][:, 3:6])
                Bm[:, k, :, 1] = np.where(isp[:, None], v, 0.0)
                free[:, k, 1] = isp
                Pk = tx + (k + 1) / (n + 1) * (rx - tx)
                z0[:, k] = (np.swapaxes(Bm[:, k], 1, 2) @ (Pk - O[:, k])[..., None])[..., 0]
            rf = refr[:n, sel]                                # [n, B]
            nfk = [np.where(rf[k], rfi[np.where(kinds[k] == 0, prim[k, sel], 0), 0], 0.0) for k in range(n)]
            nbk = [np.where(rf[k], rfi[np.where(kinds[k] == 0, prim[k, sel], 0), 1], 0.0) for k in range(n)]
            first = np.argmax(rf, axis=0)                     # first refracting slot (if any)
            has_rf = rf.any(axis=0)
            starts = ([np.ones(Bn)] if not has_rf.any() else
                      [np.where(has_rf, np.choose(first, nfk), 1.0), np.where(has_rf, np.choose(first, nbk), 1.0)])
            exists = np.zeros(Bn, bool)
            unsure = np.zeros(Bn, bool)
            Xbest = None
            for m0 in starts:
                # the medium of each segment: a refracting facet takes the ray
                # to its other side's index, a reflection keeps it
                wt = np.empty((Bn, n + 1))
                m = m0.copy()
                for k in range(n):
                    wt[:, k] = m
                    m = np.where(rf[k], np.where(m == nfk[k], nbk[k], nfk[k]), m)
                wt[:, n] = m
                X, gn, smin = fermat_minimiser(tx, rx, O, Bm, free, z0, wt=wt)
                P = np.concatenate([np.broadcast_to(tx, (Bn, 1, 3)), X, rx[:, None]], axis=1)
                # a minimiser with a segment far below the shortest admissible
                # one is never accepted, whether it is a kink or not
                smooth = smin > 1e-7
                signed = np.ones(Bn, bool)
                for k in range(n):
                    nv = pl[k][:, 0:3]
                    a = np.einsum("bi,bi->b", P[:, k + 1] - P[:, k], nv)
                    b = np.einsum("bi,bi->b", P[:, k + 2] - P[:, k + 1], nv)
                    # reflections return to the incoming side; refractions
                    # cross, arriving from the side whose index is the
                    # segment's medium
                    arrive = np.where(a < 0, nfk[k], nbk[k])
                    ok_r = (a * b > 0) & (arrive == wt[:, k])
                    signed &= np.where(kinds[k] != 0, True, np.where(rf[k], ok_r, a * b < 0))
                ex = smooth & signed
                take = ex & ~exists
                Xbest = X if Xbest is None else np.where(take[:, None, None], X, Xbest)
                unsure |= ex & (gn > 1e-9)
                exists |= ex
            X = Xbest
        # acceptance at the closed-form root
        P = np.concatenate([np.broadcast_to(tx, (len(sel), 1, 3)), X, rx[:, None]], axis=1)
        seg = np.linalg.norm(np.diff(P, axis=1), axis=2)
        ok = exists & np.all(seg >= MIN_SEG, axis=1)
        near = np.any(np.abs(seg - MIN_SEG) <= margin, axis=1)
        for k in range(n):
            Xk = X[:, k]
            isp = kinds[k] == 0
            a, aa, b, bb, lu, lv = _rect_coords(pl[k], Xk)
            in_rect = (a >= 0) & (a <= aa) & (b >= 0) & (b <= bb)
            near_rect = ((np.abs(a) <= margin * lu) | (np.abs(a - aa) <= margin * lu)
                         | (np.abs(b) <= margin * lv) | (np.abs(b - bb) <= margin * lv))
            dd = P[:, k + 1] - P[:, k]
            with np.errstate(divide="ignore", invalid="ignore"):
                cs = np.abs(np.einsum("bi,bi->b", dd, pl[k][:, 0:3])) / np.linalg.norm(dd, axis=1)
            s_ = np.einsum("bi,bi->b", Xk - ln[k][:, 0:3], ln[k][:, 3:6])
            in_seg = (s_ >= ln[k][:, 6]) & (s_ <= ln[k][:, 7])
            near_seg = (np.abs(s_ - ln[k][:, 6]) <= margin) | (np.abs(s_ - ln[k][:, 7]) <= margin)
            ok &= np.where(isp, in_rect & (cs >= GRAZE), in_seg)
            near |= np.where(isp, near_rect | (np.abs(cs - GRAZE) <= 1e-10), near_seg)
        acc[sel] = ok
        amb[sel] = unsure | (near & exists)
        Xall[sel, :3 * n] = X.reshape(len(sel), 3 * n)
    return idx, acc, amb, Xall


_JOB = None


def _chunk(bounds):
    scene, batch, idx = _JOB
    return planar_paths_closed_form(scene, batch, idx[bounds[0]:bounds[1]])


def planar_paths_closed_form_parallel(scene, batch, idx=None, workers=None, chunk=32768):
    """planar_paths_closed_form over forked worker processes (the arithmetic is
    per solve, so the chunks are independent)."""
    import multiprocessing as mp
    global _JOB
    idx = np.arange(batch.n) if idx is None else np.asarray(idx)
    workers = workers or min(8, os.cpu_count() or 1)
    bounds = [(a, min(a + chunk, len(idx))) for a in range(0, len(idx), chunk)]
    _JOB = (scene, batch, idx)
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_chunk, bounds)
    finally:
        _JOB = None
    if not parts:
        return (np.zeros(0, np.int64), np.zeros(0, bool), np.zeros(0, bool), np.zeros((0, 15)))
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(4))
