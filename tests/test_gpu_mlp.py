"""The learned start's kernels on the GPU: the matrix-core GEMM, the
features, the gradients (against the FP64 reference), training, save/load,
and the learned start inside the solver."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp_ref as R
from paper_2301_06399_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2301_06399_amd import mpt
    c = mpt.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("at,bt", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K,splits", [(100, 70, 77, 1), (64, 64, 32, 1), (33, 257, 300, 3), (256, 16, 4096, 16)])
def test_mfma_gemm_matches_cpu(ctx, at, bt, M, N, K, splits):
    """C = A B on the matrix cores with BF16 inputs: equal to the FP64 product
    of the BF16-rounded inputs up to FP32 accumulation error (this also pins
    the MFMA operand and result lane layout)."""
    import torch
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.normal(size=(K, M) if at else (M, K)).astype(np.float32)
    B = rng.normal(size=(N, K) if bt else (K, N)).astype(np.float32)
    Cg = ctx.gemm_bf16_check(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), bool(at), bool(bt), splits)
    Ar, Br = R.bf16(A), R.bf16(B)
    Cr = (Ar.T if at else Ar) @ (Br.T if bt else Br)
    err = np.abs(Cg.cpu().numpy() - Cr).max()
    assert err <= 1e-5 * np.sqrt(K) * max(1.0, np.abs(Cr).max()), err


def test_features_match_reference(ctx):
    from paper_2301_06399_amd import mpt
    for cfg in (2, 3):
        sc, b = W.training_batch(cfg, n_rx=8, per_rx=64)
        ctx.upload_scene(sc)
        f = ctx.mlp_features(mpt.DeviceBatch(b)).cpu().numpy()
        np.testing.assert_allclose(f, R.features(sc, b), atol=2e-6, rtol=1e-6)


def solved_training_set(ctx, cfg, n_rx):
    from paper_2301_06399_amd import mpt
    sc, b = W.training_batch(cfg, n_rx=n_rx, per_rx=64)
    ctx.upload_scene(sc)
    db = mpt.DeviceBatch(b)
    out = ctx.solve(db, mpt.default_opts(precision=mpt.FP64_PLAIN))
    return sc, b, db, out


def test_gradients_match_fp64_reference(ctx):
    """Loss and gradient of the BF16 kernels against the FP64 reference: to
    FP32-accumulation precision when the reference rounds where the kernels
    store BF16, and to BF16 precision against the exact FP64 network."""
    import torch
    from paper_2301_06399_amd import mpt
    sc, b, db, out = solved_training_set(ctx, 2, 32)
    use = (out.status == 0).to(torch.uint8)
    ctx.mlp_init(7)
    rows = torch.arange(0, 2000, dtype=torch.int32, device="cuda")
    loss_g, g = ctx.mlp_grad(db, out.x, use=use, rows=rows)
    hdr, w, _, _ = R.parse_blob(ctx.mlp_save())
    P = R.unpack(w)
    sb = b.subset(np.arange(2000))
    X = R.features(sc, sb)
    T = R.targets(sc, sb, out.numpy()["x"][:, :2000])
    mask = np.zeros((2000, 16))
    u = use.cpu().numpy()[:2000]
    for i in range(2000):
        mask[i, :3 * sb.order[i]] = u[i]
    G_gpu = R.unpack(g.cpu().numpy())
    for rounding, tol, ltol in ((True, 5e-3, 1e-4), (False, 2e-2, 1e-2)):
        loss_r, G, _ = R.loss_and_grad(P, X, T, mask, rounding=rounding)
        assert abs(loss_g - loss_r) <= ltol * loss_r, (rounding, loss_g, loss_r)
        for k in G:
            rel = np.linalg.norm(G_gpu[k] - G[k]) / max(np.linalg.norm(G[k]), 1e-30)
            assert rel <= tol, (rounding, k, rel)


def test_fp32_gradients_match_fp64_reference(ctx):
    """The backward pass run in FP32 throughout (no BF16 rounding anywhere)
    against the exact FP64 network and its gradient: relative error at the
    level of FP32 accumulation."""
    import torch
    sc, b, db, out = solved_training_set(ctx, 3, 16)
    use = (out.status == 0).to(torch.uint8)
    ctx.mlp_init(11)
    rows = torch.arange(0, 512, dtype=torch.int32, device="cuda")
    loss_g, g = ctx.mlp_grad(db, out.x, use=use, rows=rows, fp32=True)
    hdr, w, _, _ = R.parse_blob(ctx.mlp_save())
    P = R.unpack(w)
    sb = b.subset(np.arange(512))
    X = R.features(sc, sb)
    T = R.targets(sc, sb, out.numpy()["x"][:, :512])
    mask = np.zeros((512, 16))
    u = use.cpu().numpy()[:512]
    for i in range(512):
        mask[i, :3 * sb.order[i]] = u[i]
    assert mask.sum() > 100
    loss_r, G, _ = R.loss_and_grad(P, X, T, mask, rounding=False)
    assert abs(loss_g - loss_r) <= 1e-6 * loss_r, (loss_g, loss_r)
    G_gpu = R.unpack(g.cpu().numpy())
    for k in G:
        rel = np.linalg.norm(G_gpu[k] - G[k]) / max(np.linalg.norm(G[k]), 1e-30)
        assert rel <= 1e-6, (k, rel)


def test_training_lowers_loss_and_blob_roundtrip(ctx):
    import torch
    from paper_2301_06399_amd import learned, mpt
    sc, b = W.training_batch(2, n_rx=256, per_rx=64)
    hist = learned.train(ctx, sc, b, steps=300, batch_rows=2048)
    assert hist[-1][1] < 0.5 * hist[0][1], hist
    db = mpt.DeviceBatch(b)
    p1 = ctx.mlp_predict(db).cpu().numpy()
    blob = ctx.mlp_save()
    hdr, w, m, v = R.parse_blob(blob)
    assert hdr["step"] == 300 and hdr["layers"] == [96, 256, 256, 256, 15]
    ctx.mlp_init(99)
    assert not np.array_equal(ctx.mlp_predict(db).cpu().numpy(), p1)
    ctx.mlp_load(blob)
    assert np.array_equal(ctx.mlp_predict(db).cpu().numpy(), p1)
    # predictions are finite world points, zero beyond each order
    for i in range(0, b.n, 97):
        assert np.isfinite(p1[:3 * b.order[i], i]).all() and (p1[3 * b.order[i]:, i] == 0).all()


def test_learned_start_keeps_parity(ctx):
    """Started from the network's points (for every path), the solver still
    reaches the oracle's accept flags on planes and edges (unique roots)."""
    from paper_2301_06399_amd import learned, mpt
    sc, tb = W.training_batch(2, n_rx=512, per_rx=64)
    learned.train(ctx, sc, tb, steps=400, batch_rows=4096)
    hsc, hb = W.training_batch(2, n_rx=128, per_rx=64, stream="heldout")
    ctx.upload_scene(hsc)
    db = mpt.DeviceBatch(hb)
    out = ctx.solve(db, mpt.default_opts(init=mpt.INIT_LEARNED_ALL))
    acc, idx, k = ctx.accept(db, out)
    g = out.numpy()
    gacc = acc.cpu().numpy()
    orc = O.solve_batch(hsc, hb)
    oacc = O.accept_batch(hsc, hb, orc["x"], orc["status"])
    missed = np.where((gacc == 0) & (oacc == 1))[0]
    extra = np.where((gacc == 1) & (oacc == 0))[0]
    assert len(missed) <= 0.002 * max(1, oacc.sum()), missed[:10]
    for i in extra:  # a root the oracle's straight-line run did not reach
        n = hb.order[i]
        X, c, it, st = O.solve_one(hsc, hb.rx[hb.rx_index[i]], hb.prim[:n, i], x0=g["x"][:3 * n, i])
        assert st == O.CONVERGED and np.abs(X - g["x"][:3 * n, i]).max() <= 1e-6
    both = (gacc == 1) & (oacc == 1)
    for i in np.where(both)[0]:
        n = hb.order[i]
        assert np.abs(g["x"][:3 * n, i] - orc["x"][:3 * n, i]).max() <= 1e-6


def test_fused_inference_matches_layerwise_and_reference(ctx):
    """The fused inference kernel (activations in LDS) against the layer-by-
    layer GEMM path and the FP64 reference with BF16 rounding."""
    from paper_2301_06399_amd import learned, mpt
    sc, b = W.training_batch(3, n_rx=64, per_rx=64)
    learned.train(ctx, sc, b, steps=100, batch_rows=1024)
    ctx.upload_scene(sc)
    sb = b.subset(np.arange(b.n - 29))  # ragged last block
    db = mpt.DeviceBatch(sb)
    xf = ctx.mlp_predict(db).cpu().numpy()
    xu = ctx.mlp_predict_unfused(db).cpu().numpy()
    hdr, w, _, _ = R.parse_blob(ctx.mlp_save())
    P = R.unpack(w)
    X = R.features(sc, sb)
    _, _, Y = R.loss_and_grad(P, X, np.zeros((sb.n, 16)), np.ones((sb.n, 16)), rounding=True)
    L = np.linalg.norm(sb.rx[sb.rx_index] - sc.tx, axis=1)
    for i in range(0, sb.n, 7):
        n = sb.order[i]
        yf = (xf[:3 * n, i] - np.tile(sc.tx, n)) / L[i]
        yu = (xu[:3 * n, i] - np.tile(sc.tx, n)) / L[i]
        assert np.abs(yf - yu).max() <= 2e-2 * (1 + np.abs(yu).max())
        assert np.abs(yf - Y[i, :3 * n]).max() <= 2e-2 * (1 + np.abs(Y[i, :3 * n]).max())
        assert (xf[3 * n:, i] == 0).all()


def test_learned_start_on_curved_paths(ctx):
    """On paraboloids and circles the learned start serves every path: each
    GPU-accepted root is a root the oracle confirms from the GPU point, and
    the roots the oracle's straight-line run finds are mostly found too."""
    from paper_2301_06399_amd import learned, mpt
    sc, tb = W.training_batch(3, n_rx=512, per_rx=64)
    hsc, hb = W.training_batch(3, n_rx=48, per_rx=64, stream="heldout")
    for form, train_form, ofm, bar in ((mpt.FORM_IMPLICIT, mpt.FORM_IMPLICIT, "implicit", 0.03),
                                       (mpt.FORM_AUTO, mpt.FORM_PARAMETRIC, "param", 0.01)):
        learned.train(ctx, sc, tb, steps=1000, batch_rows=4096, form=train_form)
        ctx.upload_scene(hsc)
        db = mpt.DeviceBatch(hb)
        out = ctx.solve(db, mpt.default_opts(init=mpt.INIT_LEARNED, form=form))
        acc, idx, k = ctx.accept(db, out)
        g = out.numpy()
        gacc = acc.cpu().numpy()
        orc = O.solve_batch(hsc, hb, form=ofm)
        oacc = O.accept_batch(hsc, hb, orc["x"], orc["status"])
        for i in np.where(gacc == 1)[0]:
            n = hb.order[i]
            X, c, it, st = O.solve_one(hsc, hb.rx[hb.rx_index[i]], hb.prim[:n, i], x0=g["x"][:3 * n, i], form=ofm)
            assert st == O.CONVERGED and np.abs(X - g["x"][:3 * n, i]).max() <= 1e-6
            assert O.accept_one(hsc, hb.rx[hb.rx_index[i]], hb.prim[:n, i], X, st)
        missed = int(((gacc == 0) & (oacc == 1)).sum())
        print(ofm, "oracle roots", int(oacc.sum()), "GPU roots", int(gacc.sum()), "missed", missed)
        assert missed <= bar * max(1, oacc.sum())


def test_learned_start_gain_over_straight_line(ctx):
    """What the trained network buys on held-out curved problems.  In the
    implicit form: fewer FP32 iterations than the straight-line start and no
    fewer accepted paths.  In the automatic form the library runs on these
    scenes (parametric), with a network trained on that form's descent ends:
    at least as many accepted paths, at an iteration count that stays within
    a quarter of the straight line's (the parametric descent from the line
    is already short, and the network's points are not closer to its ends)."""
    from paper_2301_06399_amd import learned, mpt
    sc, tb = W.training_batch(3, n_rx=2048, per_rx=64)
    hsc, hb = W.training_batch(3, n_rx=256, per_rx=64, stream="heldout")
    for form, train_form, ends in ((mpt.FORM_IMPLICIT, mpt.FORM_IMPLICIT, False),
                                   (mpt.FORM_AUTO, mpt.FORM_PARAMETRIC, False)):
        learned.train(ctx, sc, tb, steps=1500, batch_rows=4096, form=train_form, ends=ends)
        ctx.upload_scene(hsc)
        db = mpt.DeviceBatch(hb)
        res = {}
        for name, init in (("line", mpt.INIT_LINE), ("learned", mpt.INIT_LEARNED)):
            out = mpt.DeviceOut(hb.n, stages=True)
            ctx.solve(db, mpt.default_opts(init=init, form=form), out)
            acc, idx, k = ctx.accept(db, out)
            r = out.numpy()
            res[name] = (float(r["stage"][0].mean()), k)
        print("form", form, "FP32 iterations and accepted paths, straight line vs learned:", res)
        if form == mpt.FORM_IMPLICIT:
            assert res["learned"][0] <= 0.95 * res["line"][0]
            assert res["learned"][1] >= 0.99 * res["line"][1]
        else:
            assert res["learned"][1] >= res["line"][1]
            assert res["learned"][0] <= 1.25 * res["line"][0]
