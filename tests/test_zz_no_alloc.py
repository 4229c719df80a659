"""The allocation-free solve against mpt_solve_batch (run on an MI355X).

mpt_solve_batch_noalloc runs the same kernels on a static device scratch;
with the same launch choices (no straggler launch) its outputs must equal
mpt_solve_batch's bit for bit.  Two calls in a row share the scratch, the
second with a smaller batch, so the counters must be cleared between them.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2301_06399_amd import workloads as W

pytestmark = pytest.mark.gpu


def _arrays(out):
    return {k: v.cpu().numpy().copy() for k, v in (("x", out.x), ("cost", out.cost), ("iters", out.iters),
                                                    ("status", out.status))}


@pytest.mark.parametrize("prec,form", [(1, 2), (0, 0), (1, 0)])
def test_noalloc_matches_solve_batch(prec, form):
    from paper_2301_06399_amd import mpt
    ctx = mpt.Context(0)
    try:
        sc, b = W.config5(n_rx=96, per_rx=256)          # facets, edges and paraboloids, orders 3-5
        sc2, b2 = W.config2(n_rx=40, per_rx=64)          # the second call: a smaller batch
        b2 = b2.subset(np.arange(b2.n - 13))
        assert b2.n < b.n
        for scene, batch in ((sc, b), (sc2, b2)):
            ctx.upload_scene(scene)
            db = mpt.DeviceBatch(batch)
            opts = mpt.default_opts(precision=mpt.FP32_POLISH64 if prec else mpt.FP64_PLAIN, form=form, spill=0)
            ref = ctx.solve(db, opts)
            torch.cuda.synchronize()
            r = _arrays(ref)
            launch_ref = ctx.last_launch()
            out = mpt.DeviceOut(batch.n)
            out.x.fill_(np.nan)
            out.status.fill_(255)
            ctx.solve_noalloc(db, opts, out)
            torch.cuda.synchronize()
            g = _arrays(out)
            assert ctx.last_launch() == launch_ref
            for k in ("x", "cost", "iters", "status"):
                assert np.array_equal(r[k], g[k], equal_nan=True), k
            acc_r, _, n_r = ctx.accept(db, ref)
            acc_g, _, n_g = ctx.accept(db, out)
            assert n_r == n_g and torch.equal(acc_r, acc_g)
            assert n_g > 0
    finally:
        ctx.close()


def test_noalloc_rejects_what_needs_allocation():
    from paper_2301_06399_amd import mpt
    ctx = mpt.Context(0)
    try:
        sc, b = W.config2(n_rx=4, per_rx=16)
        ctx.upload_scene(sc)
        db = mpt.DeviceBatch(b)
        out = mpt.DeviceOut(b.n)
        ctx.mlp_init(1)
        for bad in (dict(init=mpt.INIT_LEARNED), dict(graph=1)):
            with pytest.raises(mpt.MptError):
                ctx.solve_noalloc(db, mpt.default_opts(**bad), out)
    finally:
        ctx.close()
