#!/usr/bin/env python3
"""Benchmark of the batched Min-Path-Tracing solve on one MI355X.

One step = one pass of the whole hot path over the street-canyon workload
(50 boxes, 651 primitives, 4096 receivers x 64 interaction lists of order
1-3 = 262,144 solves): order binning, [learned start], FP32
Levenberg-Marquardt, FP64 Gauss-Newton polish, FP64 fallback, FP64
acceptance test with ordered compaction.  Inputs are resident on the GPU
before timing starts.  `value` = accepted paths per second.

Also reported: the plain FP64 solver (P) and FP32+polish without the learned
start (S) on the same workload, the roofline of the dominant kernel (the
first LM pass) with its time measured by HIP events on the library's stream,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WKEY = {1: "room", 2: "street_canyon", 3: "curved", 5: "stress"}
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12, "bf16": 2.5e15}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("mpt_device.hpp", "mpt_solve.hip", "mpt_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2301_06399_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def type_codes(scene, batch):
    """Base-4 code of each solve's primitive-type sequence."""
    t = scene.type_of(np.maximum(batch.prim, 0))
    code = np.zeros(batch.n, np.int64)
    for k in range(5):
        code += np.where(batch.order > k, t[k], 0).astype(np.int64) * (4 ** k)
    return code


def algorithmic_flops(table, order, code, iters, kind):
    tot = 0
    for n in range(1, 6):
        m = order == n
        if m.any():
            tot += int((table[n][kind][code[m]] * iters[m].astype(np.int64)).sum())
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--n-rx", type=int, default=0, help="receivers (0: the configuration's own)")
    ap.add_argument("--variant", default="auto", choices=["auto", "L", "S", "P"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0: about 20 s of work)")
    ap.add_argument("--train-steps", type=int, default=0, help="network training steps before timing (L)")
    ap.add_argument("--only-main", action="store_true", help="time only the headline variant")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tuner: launch choices from MPT_AUTOTUNE_CACHE, else the defaults")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2301_06399_amd import mpt
    from paper_2301_06399_amd import workloads as W

    t0 = time.time()
    if args.config == 5:
        scene, batch = W.config5(n_rx=args.n_rx or 1024)
    elif args.n_rx:
        scene, batch = W.CONFIGS[args.config](n_rx=args.n_rx)
    else:
        scene, batch = W.CONFIGS[args.config]()
    names = {1: "room 10x10x3 m, 6 walls + 2 edges, 256 RX x 64 lists (order 1-2)",
             2: "street canyon 50 boxes (251 facets + 400 edges), 4096 RX x 64 lists (order 1-3)",
             3: "curved: 200 paraboloids + 100 circles, 16384 RX x 64 lists (order 1-5)",
             5: "stress: street canyon + 30 paraboloids, lists of order 3-5 with >= 2 diffractions"}
    print(f"# workload generated in {time.time() - t0:.1f}s: {batch.n} solves", file=sys.stderr, flush=True)

    ctx = mpt.Context(0)
    ctx.upload_scene(scene)
    db = mpt.DeviceBatch(batch)
    out = mpt.DeviceOut(batch.n, stages=True)
    n = batch.n
    acc = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    idx = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    import ctypes as C

    learned_ok = False
    variant = args.variant
    if variant in ("auto", "L"):
        try:
            from paper_2301_06399_amd import learned
            learned_ok = learned.prepare(ctx, scene, batch, steps=args.train_steps or None)
        except (ImportError, mpt.MptError) as e:
            print(f"# learned start unavailable: {e}", file=sys.stderr)
            learned_ok = False
        if variant == "L" and not learned_ok:
            print(json.dumps({"error": "learned start requested but unavailable"}))
            sys.exit(3)
        variant = "L" if learned_ok else "S"

    def opts_for(v):
        if v == "P":
            return mpt.default_opts(precision=mpt.FP64_PLAIN)
        if v == "S":
            return mpt.default_opts(precision=mpt.FP32_POLISH64)
        return mpt.default_opts(precision=mpt.FP32_POLISH64, init=mpt.INIT_LEARNED)

    def step(o):
        ctx.solve(db, o, out)
        bd, od = db.desc(), out.desc()
        rc = ctx.L.mpt_accept(ctx.h, C.byref(bd), C.byref(od), 1e-9, 1e-6, mpt._ptr(acc), mpt._ptr(idx),
                              mpt._ptr(cnt), None)
        ctx._check(rc, "mpt_accept")

    def timed(v, steps, warmup):
        o = opts_for(v)
        for _ in range(warmup):
            step(o)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step(o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        k = int(cnt.item())
        # per-stage durations (events on the library's stream), averaged
        st = {"bin": 0.0, "learned": 0.0, "lm": 0.0, "polish": 0.0, "fallback": 0.0}
        per_order = [0.0] * 5
        reps = min(steps, 10)
        for _ in range(reps):
            ctx.solve(db, o, out)
            tm = ctx.timings()
            for key in st:
                st[key] += tm[key] / reps
            try:
                po = ctx.lm_timings()
                per_order = [a + b / reps for a, b in zip(per_order, po)]
            except mpt.MptError:
                per_order = None
        st["lm_per_order"] = per_order
        return dt, k, st

    if args.copy_mib:
        # a plain copy of known size: what the HBM byte counters read for it
        # calibrates them for the solver kernels
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)  # one elementwise kernel: reads and writes copy_mib MiB
        torch.cuda.synchronize()
        del src, dst

    variants = [variant] if args.only_main else [variant] + [x for x in ("S", "P") if x != variant]
    # launch choices picked by the autotuner (untimed)
    tuned = {}
    for v in variants:
        tuned[v] = None if args.no_autotune else ctx.autotune(db, opts_for(v), out)
        print(f"# autotune {v}: {tuned[v]}", file=sys.stderr, flush=True)

    results = {}
    for v in variants:
        steps = args.steps if v == variant else max(5, args.steps // 4)
        warm = args.warmup if v == variant else 1
        dt, k, st = timed(v, steps, warm)
        r = out.numpy()
        results[v] = {"ms_per_step": dt * 1e3, "accepted": k, "paths_per_s": k / dt, "stage_ms": st,
                      "fallback": int((r["status"] & 0x80).astype(bool).sum()),
                      "iters_mean": float(r["iters"].mean()), "lm_iters_mean": float(r["stage"][0].mean()),
                      "launch": tuned[v],
                      "_r": r}
        print(f"# {v}: {dt * 1e3:.3f} ms/step, {k} accepted, {k / dt:.4g} paths/s, stages {st}", file=sys.stderr,
              flush=True)

    main_r = results[variant]
    r = main_r.pop("_r") if "_r" in main_r else None
    # the last out is from the last variant run: recompute the main one's stages
    step(opts_for(variant))
    ctx.synchronize()
    r = out.numpy()
    for v in results:
        results[v].pop("_r", None)

    # ---------------- roofline of the dominant kernel (first LM pass)
    table = mpt.flops_table()
    code = type_codes(scene, batch)
    prec = "fp64" if variant == "P" else "fp32"
    per_order_flops = []
    for nn in range(1, 6):
        m = batch.order == nn
        per_order_flops.append(algorithmic_flops(table, batch.order[m], code[m], r["stage"][0][m], "lm"))
    flops_pass = sum(per_order_flops)
    st = main_r["stage_ms"]
    mode = 1 if prec == "fp32" else 0
    if st.get("lm_per_order"):
        # concurrent per-order launches: the dominant one is the order with
        # the most algorithmic work, timed by its own events
        dom = int(np.argmax(per_order_flops))
        kname, kfile = f"k_lm_one<{mode}, {dom + 1}, ...>", f"k_lm_one_order{dom + 1}_{prec}"
        flops_dom, ms_dom = per_order_flops[dom], st["lm_per_order"][dom]
    else:
        kname, kfile = f"k_lm<{mode}, ...> (all orders)", f"k_lm_{prec}"
        flops_dom, ms_dom = flops_pass, st["lm"]
    achieved = flops_dom / (ms_dom * 1e-3)
    # HBM bytes per launch from the committed counter summary of this kernel
    # and workload, valid while the solver sources are unchanged
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"hbm_{kfile}_{WKEY[args.config]}.txt")
    if os.path.exists(tfile):
        kv = dict(l.split(":", 1) for l in open(tfile).read().splitlines() if ":" in l and not l.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("source_hash") == kernel_source_hash():
            traffic = float(kv["hbm_bytes_per_launch"])
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[prec], "traffic": traffic, "kernel": kname,
                "flops_per_launch": flops_dom, "launch_ms": ms_dom,
                "lm_pass": {"flops": flops_pass, "ms": st["lm"], "tflops": flops_pass / (st["lm"] * 1e-3) / 1e12,
                            "flops_per_order": per_order_flops, "ms_per_order": st.get("lm_per_order")}}

    # ---------------- parity on a sample and the CPU baseline (oracle)
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.lib()
        ncores = os.cpu_count() or 1
        try:
            ncores = len(os.sched_getaffinity(0))
        except AttributeError:
            pass
        ncores = min(ncores, 16)
        # the whole workload when it is small enough (else a seeded uniform
        # sample), solved and accepted again until about 10 s of CPU work
        m = min(n, args.cpu_sample or 2_000_000)
        samp = np.arange(n) if m == n else np.sort(np.random.default_rng(11).choice(n, size=m, replace=False))
        sb = batch.subset(samp) if m < n else batch
        reps, t_cpu, acc_cpu = 0, 0.0, 0
        while reps < 1 or (t_cpu < 10.0 and reps < 64):
            t = time.perf_counter()
            o_ = O.solve_batch(scene, sb, nthreads=ncores)
            a_ = O.accept_batch(scene, sb, o_["x"], o_["status"], nthreads=ncores)
            t_cpu += time.perf_counter() - t
            acc_cpu += int(a_.sum())
            if reps == 0:
                orc, oacc = o_, a_
            reps += 1
        what = "the whole workload" if m == n else f"a seeded uniform sample of {m} of the {n} solves"
        cpu = {"value": acc_cpu / t_cpu, "unit": "accepted paths/s", "cores": ncores, "kind": "oracle",
               "sample": f"{what} ({m} solves), solve + accept, {reps} passes, {t_cpu:.1f} s",
               "solves_per_s": reps * m / t_cpu}
        gacc = acc[:n].cpu().numpy()[samp]
        curved = np.zeros(len(samp), bool)
        for k in range(5):
            curved |= (sb.order > k) & np.isin(scene.type_of(np.maximum(sb.prim[k], 0)), (2, 3))
        both = (gacc == 1) & (oacc == 1)
        errs, other_root, unverified = [], 0, 0
        for i in np.where(both | ((gacc == 1) & curved))[0]:
            o_ = sb.order[i]
            xg = r["x"][:3 * o_, samp[i]]
            e = np.inf
            if oacc[i]:
                e = float(np.linalg.norm((xg - orc["x"][:3 * o_, i]).reshape(o_, 3), axis=1).max())
            if e <= 1e-6 or not curved[i]:
                errs.append(e)
                continue
            # a curved path may have several roots: the GPU's is verified by an
            # oracle polish from the GPU point (same root, accepted)
            X, c_, it_, st_ = O.solve_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], x0=xg)
            ok = st_ == O.CONVERGED and O.accept_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], X, st_) and \
                np.linalg.norm((X - xg).reshape(o_, 3), axis=1).max() <= 1e-6
            other_root += int(ok)
            unverified += int(not ok)
        errs = np.array(errs) if errs else np.zeros(1)
        flat = ~curved
        parity = {"sample": int(len(samp)),
                  "flag_mismatches_planar": int((gacc[flat] != oacc[flat]).sum()),
                  "gpu_only": int(((gacc == 1) & (oacc == 0)).sum()),
                  "oracle_only": int(((gacc == 0) & (oacc == 1)).sum()),
                  "curved_other_root_verified": other_root, "curved_unverified": unverified,
                  "point_err_m": {"max": float(errs.max()), "p50": float(np.percentile(errs, 50)),
                                  "p99": float(np.percentile(errs, 99))}}

    value = main_r["paths_per_s"]
    line = {
        "metric": "accepted paths/sec at 1e-6 m point error vs FP64 oracle (learned+FP32 vs plain)",
        "value": value,
        "unit": "accepted paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if variant != "P" else "f64",
        "data": "synthetic (seeded generators)",
        "config": {"workload": names[args.config], "solves": int(n),
                   "variant": {"L": "learned start + FP32 LM + FP64 polish + fallback",
                               "S": "straight-line start + FP32 LM + FP64 polish + fallback",
                               "P": "plain FP64 LM"}[variant]},
        "variants": {v: {k: (round(x, 6) if isinstance(x, float) else x) for k, x in d.items()}
                     for v, d in results.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
