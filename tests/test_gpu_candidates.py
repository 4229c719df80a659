"""Candidate generation on the GPU (mpt_visibility, mpt_visibility_rx,
mpt_candidates) against the oracle on the same scenes.  Every output is
integer: visibility bits from the same IEEE FP64 tests in the same order
without contraction, and path lists in the same canonical order, so they
must agree exactly."""
import numpy as np
import pytest

import oracle as O
from paper_2301_06399_amd import workloads as W

from test_oracle_candidates import fig4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_06399_amd import mpt
    c = mpt.Context(0)
    yield c
    c.close()


def gpu_vis(ctx, sc, rx, k):
    import torch
    from paper_2301_06399_amd import mpt
    ctx.upload_scene(sc)
    V, B = ctx.visibility(k)
    R = torch.from_numpy(np.ascontiguousarray(rx, np.float64).reshape(-1, 3)).cuda()
    U, los = ctx.visibility_rx(R, k)
    n = sc.n_prims
    return (V, B, U, R), (mpt.unpack_bits(V, n), mpt.unpack_bits(B, n), mpt.unpack_bits(U, n),
                          los.cpu().numpy().astype(bool))


def test_fig4_on_the_gpu(ctx):
    """Sec. II-C, Fig. 4: the GPU's bits are the printed matrix."""
    V0, B0, U0, los0 = fig4()
    sc, ue = W.fig3_scene()
    for k in (2, 4, 8):
        _, (V, B, U, los) = gpu_vis(ctx, sc, ue, k)
        assert np.array_equal(V, V0) and np.array_equal(B, B0)
        assert np.array_equal(U[0], U0) and los[0] == los0


@pytest.mark.parametrize("which", ["street", "room", "curved", "stress"])
def test_visibility_matches_oracle(ctx, which):
    """Street canyon (651 objects), room, curved objects (paraboloid patches
    block, circles do not) and the stress scene: the same bits as the
    oracle."""
    rng = np.random.default_rng(21)
    if which == "street":
        sc, k = W.street_canyon_scene(2), 2
        rx = np.column_stack([sc._free_xy(rng, 24), np.full(24, 1.5)])
    elif which == "room":
        sc, b = W.config1(n_rx=8)
        rx, k = b.rx, 3
    elif which == "curved":
        sc, k = W.curved_scene(3, n_quad=60, n_circ=30), 3
        rx = rng.uniform(sc.aabb_lo, sc.aabb_hi, (16, 3))
    else:
        sc, k = W.stress_scene(), 2
        rx = np.column_stack([sc._free_xy(rng, 8), np.full(8, 1.5)])
    _, (V, B, U, los) = gpu_vis(ctx, sc, rx, k)
    oV, oB = O.visibility(sc, k=k)
    oU, olos = O.visibility_rx(sc, rx, k=k)
    assert np.array_equal(V, oV), np.argwhere(V != oV)[:5]
    assert np.array_equal(B, oB)
    assert np.array_equal(U, oU), np.argwhere(U != oU)[:5]
    assert np.array_equal(los, olos)
    assert 0 < V.sum() < V.size


@pytest.mark.parametrize("edge_last", [False, True])
def test_candidates_match_oracle(ctx, edge_last):
    """Interaction lists of 12 street-canyon receivers (12 buildings, orders
    1-3) and of the Fig. 3 scenario (orders 1-5): the same lists in the same
    order as the oracle's enumeration."""
    rng = np.random.default_rng(5)
    cases = []
    sc = W.street_canyon_scene(2, n_boxes=12)
    cases.append((sc, np.column_stack([sc._free_xy(rng, 12), np.full(12, 1.5)]), 3))
    sc3, ue = W.fig3_scene()
    cases.append((sc3, ue.reshape(1, 3), 5))
    for sc, rx, mo in cases:
        (V, B, U, R), (Vb, Bb, Ub, _) = gpu_vis(ctx, sc, rx, 2)
        ri, order, prim = ctx.candidates(V, B, U, mo, edge_last)
        want = O.candidates(sc, rx, Vb, Bb, Ub, mo, edge_last)
        assert ri.shape[0] == len(want["order"]) > 0
        assert np.array_equal(ri.cpu().numpy(), want["rx_index"])
        assert np.array_equal(order.cpu().numpy(), want["order"])
        assert np.array_equal(prim.cpu().numpy(), want["prim"])


def test_alg1_pipeline_end_to_end(ctx):
    """Alg. 1 on the GPU: visibility -> candidates -> solve -> accept ->
    validate, for 8 street-canyon receivers up to 2 interactions; the kept
    paths equal the oracle's chain on the same candidate lists."""
    from paper_2301_06399_amd import mpt
    rng = np.random.default_rng(8)
    sc = W.street_canyon_scene(2, n_boxes=12)
    rx = np.column_stack([sc._free_xy(rng, 8), np.full(8, 1.5)])
    (V, B, U, R), (Vb, Bb, Ub, _) = gpu_vis(ctx, sc, rx, 2)
    ri, order, prim = ctx.candidates(V, B, U, 2)
    db = mpt.device_batch(R, ri, order, prim)
    out = ctx.solve(db, mpt.default_opts())
    acc, idx, k = ctx.accept(db, out)
    vis, nv = ctx.visible(db, out, acc)
    b = W.Batch(rx, ri.cpu().numpy(), order.cpu().numpy(), prim.cpu().numpy())
    orc = O.solve_batch(sc, b)
    oacc = O.accept_batch(sc, b, orc["x"], orc["status"])
    ovis = O.visible_batch(sc, b, orc["x"], oacc)
    assert np.array_equal(acc.cpu().numpy(), oacc)
    assert np.array_equal(vis.cpu().numpy(), ovis)
    assert nv > 0


def test_candidate_edge_cases(ctx):
    """No receivers; capacity too small; samples per side outside 1..16."""
    import torch
    from paper_2301_06399_amd import mpt
    sc, ue = W.fig3_scene()
    (V, B, U, R), _ = gpu_vis(ctx, sc, ue, 2)
    ri, order, prim = ctx.candidates(V, B, U[:0], 3)
    assert ri.shape[0] == 0
    tot = __import__("ctypes").c_int64(0)
    buf = torch.empty((5, 1), dtype=torch.int32, device="cuda")
    rc = ctx.L.mpt_candidates(ctx.h, mpt._ptr(V), mpt._ptr(B), mpt._ptr(U), 1, 3, 0, 1, mpt._ptr(buf[0]),
                              mpt._ptr(buf[1]), mpt._ptr(buf), __import__("ctypes").byref(tot))
    assert rc == 7 and tot.value > 1
    with pytest.raises(mpt.MptError):
        ctx.visibility(17)
    with pytest.raises(mpt.MptError):
        ctx.visibility(0)
