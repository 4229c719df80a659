"""Training of the learned warm start (network kernels in libmpt.so).

The network is trained on the GPU by the library's own forward, backward and
Adam kernels on solver outputs: problems drawn from the workload's generator
on the "train" seed stream (the same scene, other receivers and lists) are
solved by the plain FP64 solver, and the converged points are the targets.
Only index shuffling of minibatches is done with torch.
"""
from __future__ import annotations

import math
import sys
import time

import numpy as np

from . import mpt
from . import workloads as W


def targets(ctx, db, form=mpt.FORM_IMPLICIT, ends=False):
    """Training targets: the plain FP64 solver's end points from the straight
    line, in `form`.  Only the roots (CONVERGED), or with `ends` every end
    point of a finished descent (roots and non-root stationary points), so
    that the network learns where the descent from the line ends."""
    import torch
    out = ctx.solve(db, mpt.default_opts(precision=mpt.FP64_PLAIN, form=form))
    st = out.status.to(torch.int32) & 0x7F
    if ends:
        ok = (st == mpt.CONVERGED) | (st == mpt.LOCALMIN) | (st == mpt.MAXITER) | (st == mpt.STALLED)
        ok &= torch.isfinite(out.x).all(dim=1)
    else:
        ok = st == mpt.CONVERGED
    return out, ok.to(torch.uint8)


def train(ctx, scene, train_batch, steps=3000, batch_rows=4096, lr=1e-3, seed=1, log=None,
          form=mpt.FORM_IMPLICIT, ends=False):
    """Solve `train_batch` with the plain FP64 solver, then train for `steps`
    Adam steps with cosine-decayed learning rate.  Returns the loss history."""
    import torch
    ctx.upload_scene(scene)
    db = mpt.DeviceBatch(train_batch)
    out, use = targets(ctx, db, form, ends)
    ctx.mlp_init(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = train_batch.n
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    perm = torch.randperm(n, device="cuda", generator=gen).to(torch.int32)
    pos = 0
    for it in range(steps):
        if pos + batch_rows > n:
            perm = torch.randperm(n, device="cuda", generator=gen).to(torch.int32)
            pos = 0
        rows = perm[pos:pos + batch_rows]
        pos += batch_rows
        a = lr * 0.5 * (1.0 + math.cos(math.pi * it / max(1, steps)))
        ctx.mlp_train_step(db, out.x, use=use, lr=a, loss=loss, rows=rows)
        if it % 1000 == 0 or it == steps - 1:
            hist.append((it, float(loss.item())))
            if log:
                print(f"# train step {it}: loss {hist[-1][1]:.5f}", file=log, flush=True)
    return hist


def train_joint(ctx, parts, steps=4000, batch_rows=4096, lr=1e-3, seed=1, log=None):
    """One network for several scenes: `parts` is a list of (scene, batch);
    each part's problems are solved by the plain FP64 solver (targets), then
    the Adam steps cycle through the parts, uploading each part's scene
    before its minibatch.  Returns the loss history (step, part, loss)."""
    import torch
    data = []
    for sc, tb in parts:
        ctx.upload_scene(sc)
        db = mpt.DeviceBatch(tb)
        out = ctx.solve(db, mpt.default_opts(precision=mpt.FP64_PLAIN))
        use = (out.status == mpt.CONVERGED).to(torch.uint8)
        data.append((sc, db, out, use))
    ctx.mlp_init(seed)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for it in range(steps):
        j = it % len(data)
        sc, db, out, use = data[j]
        if len(data) > 1 or it == 0:
            ctx.upload_scene(sc)
        rows = torch.randint(0, db.n, (batch_rows,), device="cuda", generator=gen, dtype=torch.int32)
        a = lr * 0.5 * (1.0 + math.cos(math.pi * it / max(1, steps)))
        ctx.mlp_train_step(db, out.x, use=use, lr=a, loss=loss, rows=rows)
        if it % 250 < len(data) or it == steps - 1:
            hist.append((it, j, float(loss.item())))
            if log:
                print(f"# train step {it} (scene {j}): loss {hist[-1][2]:.5f}", file=log, flush=True)
    return hist


def prepare(ctx, scene, batch, steps=None, n_rx=16384, log=sys.stderr):
    """Train the network for the workload of `scene` (the curved and the
    stress scenes) on held-apart problems (about a million, targets from the
    parametric form the solver runs); returns True when the learned start is
    ready."""
    if len(scene.lines) and len(scene.quadrics):
        cfg, n_rx, per_rx = 5, max(1, n_rx // 16), 1024   # the stress scene
    elif len(scene.quadrics) or len(scene.circles):
        cfg, per_rx = 3, 64
    else:
        # planes and straight edges only: the learned start serves no path
        # (their roots are reached from the straight line), so the network
        # is initialised but not trained
        ctx.mlp_init(1)
        if log:
            print("# no curved objects: the learned start serves no path (network not trained)", file=log,
                  flush=True)
        return True
    t = time.time()
    sc, tb = W.training_batch(cfg, n_rx=n_rx, per_rx=per_rx)
    same = all(np.shape(getattr(sc, k)) == np.shape(getattr(scene, k)) and
               np.allclose(getattr(sc, k), getattr(scene, k)) for k in ("planes", "lines", "quadrics", "circles"))
    if not same:
        return False  # no training generator for this scene
    hist = train(ctx, sc, tb, steps=steps or 20000, log=log, form=mpt.FORM_PARAMETRIC)
    ctx.upload_scene(scene)
    if log:
        print(f"# learned start trained in {time.time() - t:.1f}s, final loss {hist[-1][1]:.5f}", file=log, flush=True)
    return True
