"""Physical validation on the GPU (mpt_visible) against the oracle's test on
the same inputs: the decisions are integer flags, so they must agree bit for
bit (the kernel computes the oracle's IEEE FP64 operations in the same order
without contraction)."""
import numpy as np
import pytest

import oracle as O
from paper_2301_06399_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_06399_amd import mpt
    c = mpt.Context(0)
    yield c
    c.close()


def run(ctx, sc, b, **opts):
    from paper_2301_06399_amd import mpt
    ctx.upload_scene(sc)
    db = mpt.DeviceBatch(b)
    out = ctx.solve(db, mpt.default_opts(**opts))
    acc, idx, k = ctx.accept(db, out)
    vis, nv = ctx.visible(db, out, acc)
    g = out.numpy()
    return g, acc.cpu().numpy(), vis.cpu().numpy(), nv


@pytest.mark.parametrize("cfg", [2, 3])
def test_visibility_matches_oracle_on_the_same_points(ctx, cfg):
    """Street canyon (all 262,144 solves) and curved subset: the oracle's
    validation of the GPU's own accepted points gives the same flags."""
    sc, b = W.config2() if cfg == 2 else W.config3(n_rx=256, per_rx=64)
    g, acc, vis, nv = run(ctx, sc, b, form=2)
    ovis = O.visible_batch(sc, b, g["x"], acc)
    assert np.array_equal(vis, ovis), np.where(vis != ovis)[0][:10]
    assert nv == int(vis.sum())
    assert ((vis == 1) <= (acc == 1)).all()
    assert 0 < nv < acc.sum()


def test_visibility_full_pipeline_against_oracle(ctx):
    """The whole chain - solve, accept, validate - on the GPU and in the
    oracle gives the same kept paths of the room and a street-canyon subset
    (planes and straight edges: unique roots)."""
    for sc, b in (W.config1(), W.config2(n_rx=256, per_rx=64)):
        g, acc, vis, nv = run(ctx, sc, b)
        orc = O.solve_batch(sc, b)
        oacc = O.accept_batch(sc, b, orc["x"], orc["status"])
        ovis = O.visible_batch(sc, b, orc["x"], oacc)
        assert np.array_equal(vis, ovis)


def test_visibility_wedges_match_oracle(ctx):
    """Double diffractions through the buildings (the wedges decide), and
    the room's inner corners: the same flags as the oracle on the GPU's
    points, and none of the through-building paths kept."""
    from test_oracle_visibility import diagonal_edge_batch
    sc = W.street_canyon_scene(2)
    b = diagonal_edge_batch(sc)
    g, acc, vis, nv = run(ctx, sc, b)
    assert acc.sum() > 200
    assert np.array_equal(vis, O.visible_batch(sc, b, g["x"], acc))
    sc, b = W.config1()
    g, acc, vis, nv = run(ctx, sc, b)
    assert np.array_equal(vis, O.visible_batch(sc, b, g["x"], acc))


def test_visibility_edge_cases(ctx):
    """An empty batch; a margin longer than every segment leaves only the
    wedges to decide (nothing can be crossed strictly inside): without wedges
    every accepted path is kept, with them the oracle's flags."""
    from paper_2301_06399_amd import mpt
    sc, b = W.config2(n_rx=16, per_rx=64)
    e = b.subset(np.arange(0))
    ctx.upload_scene(sc)
    db = mpt.DeviceBatch(e)
    out = ctx.solve(db, mpt.default_opts())
    acc, idx, k = ctx.accept(db, out)
    vis, nv = ctx.visible(db, out, acc)
    assert nv == 0
    db = mpt.DeviceBatch(b)
    out = ctx.solve(db, mpt.default_opts())
    acc, idx, k = ctx.accept(db, out)
    vis, nv = ctx.visible(db, out, acc, min_seg=1e4)
    g, a = out.numpy(), acc.cpu().numpy()
    assert np.array_equal(vis.cpu().numpy(), O.visible_batch(sc, b, g["x"], a, min_seg=1e4))
    assert 0 < nv < k
    bare = W.Scene(tx=sc.tx, planes=sc.planes, lines=sc.lines, aabb_lo=sc.aabb_lo, aabb_hi=sc.aabb_hi)
    ctx.upload_scene(bare)
    vis, nv = ctx.visible(db, out, acc, min_seg=1e4)
    assert nv == k and np.array_equal(vis.cpu().numpy(), a)
