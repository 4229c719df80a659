"""Pins of the oracle's refraction (Sec. VI: Snell's law as one more law
equation, on facets that refract instead of reflecting).

* A ray through parallel interfaces (a single interface, a slab) keeps its
  ray parameter p = n sin(theta) (Snell); its points follow from the one
  scalar equation "lateral offset = sum of h_j p / sqrt(n_j^2 - p^2)",
  solved here by bisection, independently of the oracle.
* A refracted path is a stationary point of the optical length
  sum n_j |X_{j+1} - X_j| (Fermat), convex over infinite planes and lines:
  on the glazed street canyon every accepted solve is that minimiser and
  every root it defines is found (closed_forms.py).
* A transmitted ray crosses the facet: TX and RX on the same side of a
  lone refracting facet have no path.
"""
import numpy as np
import pytest

import oracle as O
from paper_2301_06399_amd import workloads as W
import closed_forms as CF


def big_plane(nv, d, size=1e4):
    nv = np.asarray(nv, float) / np.linalg.norm(nv)
    a = np.eye(3)[np.argmin(np.abs(nv))]
    u = np.cross(nv, a)
    u /= np.linalg.norm(u)
    v = np.cross(nv, u)
    c = nv * d
    return W.plane_rect(nv, d, c - size * (u + v), 2 * size * u, 2 * size * v)


def layered_points(tx, rx, nrm, offsets, idx):
    """Points where a ray from tx to rx crosses the parallel planes
    nrm . x = offsets[j] (in order along nrm), the media having indices
    idx[0] (at tx) .. idx[-1] (at rx): bisection on the ray parameter."""
    tx, rx, nrm = (np.asarray(v, float) for v in (tx, rx, nrm))
    levels = [tx @ nrm] + list(offsets) + [rx @ nrm]
    h = np.abs(np.diff(levels))
    lat = (rx - tx) - ((rx - tx) @ nrm) * nrm
    D = np.linalg.norm(lat)
    u = lat / D
    lo, hi = 0.0, min(idx) * (1 - 1e-16)
    for _ in range(300):
        p = 0.5 * (lo + hi)
        if sum(hj * p / np.sqrt(nj * nj - p * p) for hj, nj in zip(h, idx)) < D:
            lo = p
        else:
            hi = p
    p = 0.5 * (lo + hi)
    pts, x = [], tx.copy()
    for j, dj in enumerate(offsets):
        x = x + h[j] * p / np.sqrt(idx[j] ** 2 - p * p) * u
        x = x + (dj - x @ nrm) * nrm
        pts.append(x.copy())
    return np.array(pts)


@pytest.mark.parametrize("form", ["implicit", "param"])
def test_single_interface_follows_snell(form):
    rng = np.random.default_rng(31)
    n_ok = 0
    misses = []
    for trial in range(200):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        d0 = rng.uniform(-1, 1)
        n1, n2 = rng.uniform(1.0, 2.0, 2)
        # the facet's normal points into medium 1, where TX is
        sc = W.Scene(tx=rng.uniform(-5, 5, 3), planes=np.array([big_plane(nrm, d0)]),
                     refraction=np.array([[n1, n2]]), aabb_lo=-10 * np.ones(3), aabb_hi=10 * np.ones(3))
        sc.tx = sc.tx + (d0 + rng.uniform(0.5, 5) - sc.tx @ nrm) * nrm
        rx = rng.uniform(-5, 5, 3)
        rx = rx + (d0 - rng.uniform(0.5, 5) - rx @ nrm) * nrm
        Xcf = layered_points(sc.tx, rx, -nrm, [-d0], [n1, n2])
        X, c, it, st = O.solve_one(sc, rx, [0], form=form)
        if st != O.CONVERGED:
            # the implicit form can stall next to grazing incidence: a non-root
            # end, and a start next to the closed form converges to it
            assert form == "implicit" and c > 1e-6, (trial, st, c)
            X, c, it, st = O.solve_one(sc, rx, [0], x0=Xcf[0] + 1e-3 * rng.normal(size=3), form=form)
            misses.append(trial)
        assert st == O.CONVERGED, (trial, st, c)
        np.testing.assert_allclose(X, Xcf[0], atol=1e-9 * (1 + np.abs(Xcf).max()))
        assert O.accept_one(sc, rx, [0], X, st)
        # Snell's law itself: n1 sin(theta1) = n2 sin(theta2)
        i, r = X - sc.tx, rx - X
        s1 = np.linalg.norm(np.cross(i / np.linalg.norm(i), nrm))
        s2 = np.linalg.norm(np.cross(r / np.linalg.norm(r), nrm))
        assert abs(n1 * s1 - n2 * s2) < 1e-10
        # swapping the indices (the normal pointing into the other medium)
        # must give the same path once the facet is turned around
        sc2 = W.Scene(tx=sc.tx, planes=np.array([big_plane(-nrm, -d0)]), refraction=np.array([[n2, n1]]),
                      aabb_lo=sc.aabb_lo, aabb_hi=sc.aabb_hi)
        X2, c2, it2, st2 = O.solve_one(sc2, rx, [0], x0=X, form=form)
        assert st2 == O.CONVERGED
        np.testing.assert_allclose(X2, Xcf[0], atol=1e-9 * (1 + np.abs(Xcf).max()))
        n_ok += 1
    assert n_ok == 200 and len(misses) <= 4, misses


@pytest.mark.parametrize("form", ["implicit", "param"])
def test_slab_closed_form(form):
    """Through a slab of index ng between two parallel facets (normals
    outward, air outside): both points as the bisection gives them."""
    rng = np.random.default_rng(32)
    found = 0
    for trial in range(200):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        d0, t, ng = rng.uniform(-1, 1), rng.uniform(0.1, 2), rng.uniform(1.2, 2.0)
        tx = rng.uniform(-5, 5, 3)
        tx = tx + (d0 - rng.uniform(0.5, 5) - tx @ nrm) * nrm
        rx = rng.uniform(-5, 5, 3)
        rx = rx + (d0 + t + rng.uniform(0.5, 5) - rx @ nrm) * nrm
        sc = W.Scene(tx=tx, planes=np.array([big_plane(-nrm, -d0), big_plane(nrm, d0 + t)]),
                     refraction=np.array([[1.0, ng], [1.0, ng]]), aabb_lo=-10 * np.ones(3), aabb_hi=10 * np.ones(3))
        Xcf = layered_points(tx, rx, nrm, [d0, d0 + t], [1.0, ng, 1.0])
        X, c, it, st = O.solve_one(sc, rx, [0, 1], form=form)
        atol = 1e-9 * (1 + np.abs(Xcf).max())
        if st == O.CONVERGED:
            np.testing.assert_allclose(X.reshape(2, 3), Xcf, atol=atol)
            assert O.accept_one(sc, rx, [0, 1], X, st)
            found += 1
        else:
            # a non-root end; a restart from the closed-form neighbourhood
            # reaches the root
            X2, c2, it2, st2 = O.solve_one(sc, rx, [0, 1], x0=Xcf.ravel() + 1e-3 * rng.normal(size=6), form=form)
            assert st2 == O.CONVERGED
            np.testing.assert_allclose(X2.reshape(2, 3), Xcf, atol=atol)
    assert found >= 195


def test_same_side_has_no_transmitted_path():
    """A refracting facet passes the ray to its other side: with TX and RX
    on the same side no solve is accepted (a root of the tangential law
    that turns back is rejected)."""
    rng = np.random.default_rng(33)
    for trial in range(100):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        tx = rng.uniform(-5, 5, 3)
        tx = tx + (rng.uniform(0.5, 5) - tx @ nrm) * nrm
        rx = rng.uniform(-5, 5, 3)
        rx = rx + (rng.uniform(0.5, 5) - rx @ nrm) * nrm
        sc = W.Scene(tx=tx, planes=np.array([big_plane(nrm, 0.0)]), refraction=np.array([[1.0, 1.5]]),
                     aabb_lo=-10 * np.ones(3), aabb_hi=10 * np.ones(3))
        for form in ("implicit", "param"):
            X, c, it, st = O.solve_one(sc, rx, [0], form=form)
            assert not O.accept_one(sc, rx, [0], X, st)


def test_refraction_jacobian_matches_central_differences():
    rng = np.random.default_rng(34)
    for trial in range(20):
        planes = [big_plane(rng.normal(size=3), rng.uniform(-2, 2)) for _ in range(3)]
        sc = W.Scene(tx=rng.uniform(-3, 3, 3), planes=np.array(planes),
                     refraction=np.array([[1.0, 1.5], [0.0, 0.0], [1.3, 1.1]]),
                     lines=np.array([W.line_seg(rng.uniform(-2, 2, 3), np.array([0, 0, 1.0]), -1e4, 1e4)]),
                     aabb_lo=-10 * np.ones(3), aabb_hi=10 * np.ones(3))
        ids = [0, 3, 2, 1]
        X = rng.uniform(-3, 3, 3 * len(ids))
        rx = rng.uniform(-3, 3, 3)
        R, J = O.residual(sc, rx, ids, X)
        Jfd = np.zeros_like(J)
        for j in range(len(X)):
            h = 1e-6 * max(1.0, abs(X[j]))
            e = np.zeros(len(X))
            e[j] = h
            Rp, _ = O.residual(sc, rx, ids, X + e, jac=False)
            Rm, _ = O.residual(sc, rx, ids, X - e, jac=False)
            Jfd[:, j] = (Rp - Rm) / (2 * h)
        np.testing.assert_allclose(J, Jfd, atol=2e-6 * (1 + np.abs(J).max()), rtol=1e-5)


@pytest.mark.parametrize("form", ["implicit", "param"])
def test_glazed_street_matches_optical_fermat(form):
    """The glazed street canyon (lists through a glass pane, 256 receivers x
    64): accept flags equal to the optical-length closed form, accepted
    points within 1e-9 m, no false root.  The parametric form misses at
    most a few roots (each a non-root end that an Alg. 1 restart recovers);
    the implicit form, whose object rows are penalties, ends about 10% of
    them in valleys next to the thin slabs (a reading: the library runs the
    parametric form on these scenes)."""
    sc, b = W.config6(n_rx=256)
    idx, exp, amb, Xcf = CF.planar_paths_closed_form(sc, b)
    assert len(idx) == b.n and amb.sum() <= 3
    r = O.solve_batch(sc, b, form=form)
    acc = O.accept_batch(sc, b, r["x"], r["status"]).astype(bool)
    assert exp.sum() > 1500
    false_root = acc & ~exp & ~amb
    assert not false_root.any(), np.where(false_root)[0][:10]
    both = acc & exp
    for n in range(1, 6):
        m = both & (b.order == n)
        if m.any():
            assert np.abs(r["x"][:3 * n, m].T - Xcf[m, :3 * n]).max() <= 1e-9
    missed = np.where(exp & ~acc & ~amb)[0]
    if form == "param":
        assert len(missed) <= 3, missed
        for i in missed:
            n = int(b.order[i])
            ids, rx = b.prim[:n, i], b.rx[b.rx_index[i]]
            assert r["status"][i] != O.CONVERGED
            hit = any(O.solve_one(sc, rx, ids, x0=O.init_random(sc, s, int(i), ids), form=form)[3] == O.CONVERGED
                      for s in range(8))
            assert hit, i
    else:
        assert len(missed) <= 0.15 * exp.sum()
        assert (r["status"][missed] != O.CONVERGED).all()
