"""Pins of the oracle's candidate generation (Alg. 1: visibility matrix,
adjacency matrix, all simple paths from BS to UE).

- The paper's own example: the adjacency matrix printed in Fig. 4 for the
  two-triangle scenario of Fig. 3, and its pruned form when a diffraction
  may only come last.
- The path enumeration against brute force over permutations and against
  closed-form path counts from matrix products.
- The visibility of the street-canyon objects against an independent
  slab-method segment/box test, and the room's closed form.
- The sample points lie on their objects, inside their extents.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2301_06399_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAMES = ["s%d" % i for i in range(1, 7)] + ["e%d" % i for i in range(1, 7)]


def fig4():
    g = json.load(open(os.path.join(GOLD, "fig4_adjacency.json")))
    idx = {nm: i for i, nm in enumerate(NAMES)}
    V = np.zeros((12, 12), bool)
    B = np.zeros(12, bool)
    U = np.zeros(12, bool)
    for nm in g["rows"]["BS"]:
        if nm != "UE":
            B[idx[nm]] = True
    for r in NAMES:
        for nm in g["rows"][r]:
            if nm == "UE":
                U[idx[r]] = True
            else:
                V[idx[r], idx[nm]] = True
    return V, B, U, "UE" in g["rows"]["BS"]


@pytest.mark.parametrize("k", [2, 4, 8])
def test_fig4_adjacency_matrix(k):
    """Sec. II-C, Fig. 4: the visibility matrix, the BS row and the UE
    column of the Fig. 3 scenario, as printed."""
    V0, B0, U0, los0 = fig4()
    sc, ue = W.fig3_scene()
    V, B = O.visibility(sc, k=k)
    U, los = O.visibility_rx(sc, ue, k=k)
    assert np.array_equal(V, V0), np.argwhere(V != V0)
    assert np.array_equal(B, B0)
    assert np.array_equal(U[0], U0)
    assert los[0] == los0


def cand(sc, rx, V, B, U, max_order, edge_last=False):
    c = O.candidates(sc, rx, V, B, U, max_order, edge_last)
    return W.Batch(np.asarray(rx).reshape(-1, 3), c["rx_index"], c["order"], c["prim"])


def brute_paths(V, B, U, edge, max_order, edge_last):
    out = []
    n = len(B)
    for o in range(1, max_order + 1):
        for p in itertools.permutations(range(n), o):
            ok = B[p[0]] and U[p[-1]]
            for a, b in zip(p, p[1:]):
                ok = ok and V[a, b] and not (edge_last and edge[a])
            if ok:
                out.append((o,) + p)
    return out


@pytest.mark.parametrize("edge_last", [False, True])
def test_fig4_simple_paths_brute_force(edge_last):
    """Alg. 1's all_simple_paths on the Fig. 4 graph, orders 1-4: the same
    lists in the same order as brute force over permutations; with the
    pruning of Fig. 4 (red entries), edges only come last and fewer
    candidates remain."""
    V, B, U, _ = fig4()
    sc, ue = W.fig3_scene()
    edge = np.arange(12) >= 6
    b = cand(sc, ue, V, B, U[None, :], 4, edge_last)
    got = [(int(o),) + tuple(int(v) for v in b.prim[:o, i]) for i, o in enumerate(b.order)]
    assert got == brute_paths(V, B, U, edge, 4, edge_last)
    assert (b.rx_index == 0).all()
    if edge_last:
        full = cand(sc, ue, V, B, U[None, :], 4, False)
        assert b.n < full.n
        for i, o in enumerate(b.order):
            assert not edge[b.prim[:o - 1, i]].any()


def test_candidate_counts_closed_form():
    """Street canyon with 12 buildings: per receiver, the number of simple
    paths of orders 1-3 equals B.U, B^T V U and B^T V^2 U minus the paths
    that come back to their first object."""
    sc = W.street_canyon_scene(2, n_boxes=12)
    rng = np.random.default_rng(3)
    rx = np.column_stack([sc._free_xy(rng, 5), np.full(5, 1.5)])
    V, B = O.visibility(sc, k=2)
    U, _ = O.visibility_rx(sc, rx, k=2)
    b = cand(sc, rx, V, B, U, 3)
    Vi, Bi = V.astype(np.int64), B.astype(np.int64)
    V2 = Vi @ Vi
    for r in range(len(rx)):
        Ui = U[r].astype(np.int64)
        want = [Bi @ Ui, Bi @ Vi @ Ui, Bi @ V2 @ Ui - (Bi * Ui * np.diag(V2)).sum()]
        for o in (1, 2, 3):
            assert ((b.rx_index == r) & (b.order == o)).sum() == want[o - 1]
    # canonical order: receiver, order, then increasing object ids
    key = [(int(b.rx_index[i]), int(b.order[i])) + tuple(int(v) for v in b.prim[:b.order[i], i]) for i in range(b.n)]
    assert key == sorted(key)


def segment_enters_any_box(P, Q, boxes, margin):
    lo = np.column_stack([boxes[:, 0] - boxes[:, 2] / 2, boxes[:, 1] - boxes[:, 3] / 2, np.zeros(len(boxes))])
    hi = np.column_stack([boxes[:, 0] + boxes[:, 2] / 2, boxes[:, 1] + boxes[:, 3] / 2, boxes[:, 4]])
    d = Q - P
    L = np.linalg.norm(d)
    t0 = np.full(len(boxes), margin / L)
    t1 = np.full(len(boxes), 1.0 - margin / L)
    inside = np.ones(len(boxes), bool)
    for i in range(3):
        if d[i] == 0.0:
            inside &= (lo[:, i] < P[i]) & (P[i] < hi[:, i])
            continue
        a, b = (lo[:, i] - P[i]) / d[i], (hi[:, i] - P[i]) / d[i]
        t0, t1 = np.maximum(t0, np.minimum(a, b)), np.minimum(t1, np.maximum(a, b))
    return bool((inside & (t0 < t1)).any())


def box_of(sc, g):
    """Building of an object of the street canyon (-1 for the ground)."""
    npl = len(sc.planes)
    return (g - 1) // 5 if g < npl else (g - npl) // 8


def test_street_visibility_matches_slab_test():
    """Two objects of different buildings (or the ground) see each other iff
    some pair of their sample points is joined by a segment that enters no
    building (slab test); two objects of one convex building never do; the
    BS row and UE columns likewise."""
    sc = W.street_canyon_scene(2, n_boxes=6)
    k = 2
    n = sc.n_prims
    V, B = O.visibility(sc, k=k)
    S = [O.samples(sc, g, k) for g in range(n)]
    boxes = sc._boxes
    for i in range(n):
        for j in range(i + 1, n):
            if box_of(sc, i) == box_of(sc, j) and box_of(sc, i) >= 0:
                assert not V[i, j]
                continue
            want = any(not segment_enters_any_box(p, q, boxes, O.MIN_SEG) for p in S[i] for q in S[j])
            assert V[i, j] == want, (i, j)
    assert V.sum() > 0.1 * n * n
    for j in range(n):
        assert B[j] == any(not segment_enters_any_box(sc.tx, q, boxes, O.MIN_SEG) for q in S[j]), j
    rng = np.random.default_rng(9)
    rx = np.column_stack([sc._free_xy(rng, 3), np.full(3, 1.5)])
    U, los = O.visibility_rx(sc, rx, k=k)
    for r in range(3):
        assert los[r] == (not segment_enters_any_box(sc.tx, rx[r], boxes, O.MIN_SEG))
        for j in range(n):
            assert U[r, j] == any(not segment_enters_any_box(q, rx[r], boxes, O.MIN_SEG) for q in S[j]), (r, j)


def test_room_visibility_closed_form():
    """Inside the convex room every wall sees every other wall, TX and RX;
    a junction edge sees every object except the two walls that meet there
    (their segments would graze the wall)."""
    sc, b = W.config1(n_rx=4)
    V, B = O.visibility(sc, k=3)
    U, los = O.visibility_rx(sc, b.rx, k=3)
    want = ~np.eye(8, dtype=bool)
    for e, walls in ((6, (0, 2)), (7, (3, 5))):
        for w in walls:
            want[e, w] = want[w, e] = False
    assert np.array_equal(V, want)
    assert B.all() and U.all() and los.all()


def test_samples_on_objects_and_in_extents():
    """Sample counts (k^2 per rectangle, k per edge, 2k per circle, the
    aperture's grid points per paraboloid) and every sample on its object
    and inside its finite extent."""
    rng = np.random.default_rng(4)
    sc3 = W.curved_scene(3, n_quad=6, n_circ=6, rng=rng)
    sc2 = W.street_canyon_scene(2, n_boxes=3)
    for k in (1, 2, 3, 5):
        for sc in (sc2, sc3):
            npl, nln, nq = len(sc.planes), len(sc.lines), len(sc.quadrics)
            for g in range(sc.n_prims):
                S = O.samples(sc, g, k)
                if g < npl:
                    r = sc.planes[g]
                    assert len(S) == k * k
                    w = S - r[4:7]
                    a, bb = w @ r[7:10] / (r[7:10] @ r[7:10]), w @ r[10:13] / (r[10:13] @ r[10:13])
                    assert (a > 0).all() and (a < 1).all() and (bb > 0).all() and (bb < 1).all()
                    assert np.abs(S @ r[:3] - r[3]).max() < 1e-9
                elif g < npl + nln:
                    r = sc.lines[g - npl]
                    assert len(S) == k
                    s = (S - r[:3]) @ r[3:6]
                    assert (s > r[6]).all() and (s < r[7]).all()
                    assert np.abs(S - r[:3] - s[:, None] * r[3:6]).max() < 1e-9
                elif g < npl + nln + nq:
                    r = sc.quadrics[g - npl - nln]
                    want = sum((2 * a + 1 - k) ** 2 + (2 * c + 1 - k) ** 2 < k * k for a in range(k) for c in range(k))
                    assert len(S) == want
                    A = np.array([[r[3], r[4], r[5]], [r[4], r[6], r[7]], [r[5], r[7], r[8]]])
                    w = S - r[:3]
                    f = np.einsum("ij,jk,ik->i", w, A, w) + w @ r[9:12] + r[12]
                    assert np.abs(f).max() < 1e-9
                    perp = w - (w @ r[13:16])[:, None] * r[13:16]
                    assert (np.linalg.norm(perp, axis=1) < r[16]).all()
                else:
                    r = sc.circles[g - npl - nln - nq]
                    assert len(S) == 2 * k
                    w = S - r[:3]
                    assert np.abs(w @ r[3:6]).max() < 1e-9
                    assert np.abs(np.linalg.norm(w, axis=1) - r[6]).max() < 1e-9
