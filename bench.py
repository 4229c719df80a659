#!/usr/bin/env python3
"""Benchmark of the batched Min-Path-Tracing solve on one MI355X.

One step = one pass of the whole hot path over one batch: order binning,
[learned start], FP32 Levenberg-Marquardt, FP64 Gauss-Newton polish, FP64
fallback, FP64 acceptance test with ordered compaction.  Inputs are resident
on the GPU before timing starts.  `value` = accepted paths per second.

Default workload: the multi-diffraction stress workload (the street canyon
plus 30 paraboloids; 16,384 receivers x 1024 lists of order 3-5 with at
least two diffractions = 16,777,216 solves), the largest configuration, with
the learned start trained on held-apart problems of the same scene and the
timed steps replayed from a captured HIP graph.  --config 1 / 2 / 3 / 6
select the room, the street canyon, the curved scene and the glazed street
canyon (refraction through glass panes); --config 4 is the
learned-start evaluation (one network trained on 2 M solver outputs of the
street-canyon and curved generators, timed on 1 M held-out problems).

Also reported: the plain FP64 solver (P, Pp) and FP32+polish without the
learned start (S, Si) on the same workload, the roofline of the dominant
kernel with its time measured by HIP events on the stream it runs on, and
the FP64 CPU oracle timed on the same workload (or a bounded sample of it)
on the host's cores and on one thread.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WKEY = {1: "room", 2: "street_canyon", 3: "curved", 4: "learned_heldout", 5: "stress", 6: "glazed"}
NAMES = {1: "room 10x10x3 m, 6 walls + 2 edges, 256 RX x 64 lists (order 1-2)",
         2: "street canyon 50 boxes (251 facets + 400 edges), 4096 RX x 64 lists (order 1-3)",
         3: "curved: 200 paraboloids + 100 circles, 16384 RX x 64 lists (order 1-5)",
         4: "learned start, held-out: street canyon 8192 RX x 64 (order 1-3) + curved 8192 RX x 64 (order 1-5)",
         5: "stress: street canyon + 30 paraboloids, 16384 RX x 1024 lists of order 3-5 with >= 2 diffractions",
         6: "glazed street canyon: 50 boxes + 40 glass panes (refracting facets), 4096 RX x 64 lists of order 2-4 "
            "through a pane"}
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "hbm": 8.0e12, "bf16": 2.5e15}
MLP_FLOPS_PER_ROW = 2 * (96 * 256 + 256 * 256 + 256 * 256 + 256 * 15)
# variant: (precision, start, form); form 0 = implicit (Eq. 12), 1 = parametric
# (Eq. 15), 2 = the library's choice (parametric with curved objects, else
# the tuner's)
VARIANTS = {"L": (1, "learned", 2), "A": (1, "learned_all", 2), "S": (1, "line", 2), "Si": (1, "line", 0),
            "Sp": (1, "line", 1), "P": (0, "line", 0), "Pp": (0, "line", 1)}
VARIANT_TEXT = {"L": "learned start (paths with curved objects) + FP32 LM + FP64 polish + fallback, form auto",
                "A": "learned start (every path) + FP32 LM + FP64 polish + fallback, form auto",
                "S": "straight-line start + FP32 LM + FP64 polish + fallback, form auto",
                "Si": "straight-line start + FP32 LM + FP64 polish + fallback, implicit form",
                "Sp": "straight-line start + FP32 LM + FP64 polish + fallback, parametric form",
                "P": "plain FP64 LM from the straight-line start, implicit form (Eq. 12)",
                "Pp": "plain FP64 LM from the straight-line start, parametric form (Eq. 15)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def algorithmic_flops(table, order, code, iters, kind, kept=False):
    """FLOPs of `iters` iterations of each path at its order and types.
    kept: the FP32 solver of orders 1-3 keeps the normal equations after a
    rejected step and skips their assembly in the next iteration; the
    number of such iterations is not recorded, so they are bounded from
    below: every iteration after a path's first is charged without its
    assembly (a lower bound of the work done)."""
    tot = 0
    for n in range(1, 6):
        m = order == n
        if m.any():
            it = iters[m].astype(np.int64)
            f = table[n][kind][code[m]] * it
            if kept and n <= 3 and kind == "lm":
                f = f - table[n]["assembly"][code[m]] * np.maximum(it - 1, 0)
            tot += int(f.sum())
    return tot


def opts_for(mpt, v, graph=0):
    prec, start, form = VARIANTS[v]
    init = {"line": mpt.INIT_LINE, "learned": mpt.INIT_LEARNED, "learned_all": mpt.INIT_LEARNED_ALL}[start]
    return mpt.default_opts(precision=mpt.FP32_POLISH64 if prec else mpt.FP64_PLAIN, init=init, form=form,
                            graph=graph)


class Runner:
    """A resident workload on the GPU: batch, outputs and accept buffers."""

    def __init__(self, torch, mpt, ctx, scene, batch):
        self.torch, self.mpt, self.ctx, self.scene, self.batch = torch, mpt, ctx, scene, batch
        self.db = mpt.DeviceBatch(batch)
        self.out = mpt.DeviceOut(batch.n, stages=True)
        n = max(batch.n, 1)
        self.acc = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.idx = torch.empty(n, dtype=torch.int32, device="cuda")
        self.cnt = torch.empty(1, dtype=torch.int32, device="cuda")

    def step(self, o):
        ctx, mpt = self.ctx, self.mpt
        ctx.solve(self.db, o, self.out)
        bd, od = self.db.desc(), self.out.desc()
        rc = ctx.L.mpt_accept(ctx.h, C.byref(bd), C.byref(od), 1e-9, 1e-6, mpt._ptr(self.acc),
                              mpt._ptr(self.idx), mpt._ptr(self.cnt), None)
        ctx._check(rc, "mpt_accept")

    def run(self, v, steps, warmup, tune, graph=True):
        """Autotune (optional, untimed), then time `steps` steps after
        `warmup` (replayed from a captured HIP graph with `graph`); stage and
        per-order durations from the library's events of separate solves."""
        torch, ctx, mpt = self.torch, self.ctx, self.mpt
        o = opts_for(mpt, v)
        launch = ctx.autotune(self.db, o, self.out) if tune else None
        o_step = opts_for(mpt, v, graph=1 if graph else 0)
        # the timed steps record no stage events; the stage times come from
        # separate timed solves below
        ctx.set_timing(False)
        # untimed warm-up: the requested steps, and at least 0.3 s of them
        t = time.perf_counter()
        w = 0
        while w < warmup or (time.perf_counter() - t < 0.3 and w < 1000):
            self.step(o_step)
            torch.cuda.synchronize()
            w += 1
        t = time.perf_counter()
        for _ in range(steps):
            self.step(o_step)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        k = int(self.cnt.item())
        st = {"bin": 0.0, "learned": 0.0, "lm": 0.0, "resume": 0.0, "polish": 0.0, "fallback": 0.0}
        per_order = [0.0] * 5
        reps = min(max(steps, 1), 10)
        ctx.set_timing(True)
        for _ in range(reps):
            ctx.solve(self.db, o, self.out)
            tm = ctx.timings()
            for key in st:
                st[key] += tm[key] / reps
            try:
                per_order = [a + b / reps for a, b in zip(per_order, ctx.lm_timings())]
            except mpt.MptError:
                per_order = None
        st["lm_per_order"] = per_order
        self.step(o)  # leave this variant's outputs and flags in place
        torch.cuda.synchronize()
        launch = dict(launch or {}, **ctx.last_launch())
        r = self.out.numpy()
        res = {"ms_per_step": dt * 1e3, "graph": bool(graph), "accepted": k, "paths_per_s": k / dt, "stage_ms": st,
               "fallback": int((r["status"] & 0x80).astype(bool).sum()),
               "iters_mean": float(r["iters"].mean()), "lm_iters_mean": float(r["stage"][0].mean()),
               "polished": int((r["stage"][1] > 0).sum()), "launch": launch}
        log(f"# {v}: {dt * 1e3:.3f} ms/step, {k} accepted, {k / dt:.4g} paths/s, LM iters "
            f"{res['lm_iters_mean']:.2f}, stages { {a: round(b, 4) for a, b in st.items() if a != 'lm_per_order'} }")
        return res, r

    def flags(self):
        return self.acc[:self.batch.n].cpu().numpy()

    def ctx_form_auto_is_param(self):
        """Whether every quadric of the scene is a paraboloid of revolution
        (then the automatic form is the parametric one)."""
        q = self.scene.quadrics
        for r in q:
            A = np.array([[r[3], r[4], r[5]], [r[4], r[6], r[7]], [r[5], r[7], r[8]]])
            ax = r[13:16]
            kap = 0.5 * np.trace(A)
            if not (kap > 0 and np.abs(A - kap * (np.eye(3) - np.outer(ax, ax))).max() <= 1e-9 * (1 + kap)
                    and np.abs(r[9:12] + ax).max() <= 1e-9 * (1 + kap) and abs(r[12]) <= 1e-9 * (1 + kap)):
                return False
        return True


def lm_roofline(scene, batch, r, st, prec, cfg, mpt, form=0, sched=None):
    """Roofline of the dominant solver kernel: algorithmic FLOPs of the first
    LM pass (iterations actually run in it x FLOPs per iteration of each
    path's order and types, in the variant's form) over its measured
    duration."""
    table = mpt.flops_table(form)
    code = type_codes(scene, batch)
    it1 = r["stage"][0] - r["stage"][3]   # iterations before a straggler was parked
    kept = prec == "fp32"
    per_order_flops, per_order_upper = [], []
    for nn in range(1, 6):
        m = batch.order == nn
        per_order_flops.append(algorithmic_flops(table, batch.order[m], code[m], it1[m], "lm", kept))
        per_order_upper.append(algorithmic_flops(table, batch.order[m], code[m], it1[m], "lm"))
    flops_pass = sum(per_order_flops)
    flops_resume = algorithmic_flops(table, batch.order, code, r["stage"][3], "lm", kept)
    mode = 1 if prec == "fp32" else 0
    if st.get("lm_per_order"):
        # concurrent per-order launches: they share the GPU for the whole
        # pass (which order's kernel ends first depends on how the hardware
        # queues interleave them), so the unit is the pass, timed from the
        # fork to the join on the solve's stream
        kname = f"LM pass: k_lm_one<{mode}, 1..5, ..., {form}> (per-order launches, concurrent)"
        kfile = f"lm_pass_{prec}" + ("_param" if form else "")
        flops_dom, ms_dom = flops_pass, st["lm"]
    elif sched == mpt.SCHED_SPLIT and sum(per_order_flops[3:]) == 0:
        # orders 1-3 in one launch; the launches of orders 4 and 5 found
        # nothing to do
        kname, kfile = f"k_lm_low<{mode}, ..., {form}> (orders 1-3)", f"k_lm_low_{prec}" + ("_param" if form else "")
        flops_dom, ms_dom = flops_pass, st["lm"]
    else:
        kname, kfile = f"k_lm<{mode}, ..., {form}> (all orders)", f"k_lm_{prec}" + ("_param" if form else "")
        if sched == mpt.SCHED_SPLIT:
            kname = f"split launches k_lm_low + k_lm_one<{mode}, 4 / 5, ..., {form}> (all orders, concurrent)"
            kfile = None
        flops_dom, ms_dom = flops_pass, st["lm"]
    achieved = flops_dom / (ms_dom * 1e-3)
    # HBM bytes per launch from the committed counter summary of this kernel
    # and workload, valid while the solver sources are unchanged
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"hbm_{kfile}_{WKEY[cfg]}.txt") if kfile else ""
    if kfile and os.path.exists(tfile):
        kv = dict(l.split(":", 1) for l in open(tfile).read().splitlines() if ":" in l and not l.startswith("#"))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv.get("source_hash") == kernel_source_hash():
            traffic = float(kv["hbm_bytes_per_launch"])
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK[prec] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK[prec],
            # every iteration charged with its assembly: the upper bound of the work
            "frac_upper": sum(per_order_upper) / (ms_dom * 1e-3) / PEAK[prec],
            "traffic": traffic, "kernel": kname,
            "flops_per_launch": flops_dom, "launch_ms": ms_dom,
            "lm_pass": {"flops": flops_pass, "ms": st["lm"], "tflops": flops_pass / (st["lm"] * 1e-3) / 1e12,
                        "flops_upper": sum(per_order_upper),
                        "flops_per_order": per_order_flops, "ms_per_order": st.get("lm_per_order"),
                        "straggler_flops": flops_resume, "straggler_ms": st["resume"]}}


def used_form(form, launch, scene):
    """The form a solve ran in: the one the library reports for the variant's
    last solve."""
    if form != 2:
        return form
    return launch["form"]


def ncores():
    """The host cores this process may use: its CPU affinity, or the thread
    count the host allots it (OMP_NUM_THREADS) when that is smaller."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        c = min(c, int(env))
    return c


def oracle_run(O, scene, batch, cores, budget_s, max_n, form="implicit"):
    """The oracle (solve + accept) on the whole workload or a seeded uniform
    sample of at most max_n solves, repeated until about budget_s seconds."""
    n = batch.n
    m = min(n, max_n)
    samp = np.arange(n) if m == n else np.sort(np.random.default_rng(11).choice(n, size=m, replace=False))
    sb = batch.subset(samp) if m < n else batch
    reps, t_cpu, acc_cpu = 0, 0.0, 0
    while reps < 1 or (t_cpu < budget_s and reps < 64):
        t = time.perf_counter()
        o_ = O.solve_batch(scene, sb, nthreads=cores, form=form)
        a_ = O.accept_batch(scene, sb, o_["x"], o_["status"], nthreads=cores)
        t_cpu += time.perf_counter() - t
        acc_cpu += int(a_.sum())
        if reps == 0:
            orc, oacc = o_, a_
        reps += 1
    return {"samp": samp, "sb": sb, "orc": orc, "oacc": oacc, "reps": reps, "t": t_cpu, "acc": acc_cpu, "m": m}


def oracle_single_thread(O, scene, sb, budget_s, form):
    """The oracle on one thread over the leading part of the sample, grown
    until a pass takes about budget_s seconds."""
    m = min(sb.n, 4096)
    while True:
        part = sb.subset(np.arange(m))
        t = time.perf_counter()
        o_ = O.solve_batch(scene, part, nthreads=1, form=form)
        a_ = O.accept_batch(scene, part, o_["x"], o_["status"], nthreads=1)
        dt = time.perf_counter() - t
        if dt >= 0.5 * budget_s or m >= sb.n:
            return {"value": int(a_.sum()) / dt, "solves_per_s": m / dt, "solves": m, "s": dt}
        m = min(sb.n, int(m * max(2.0, budget_s / max(dt, 1e-3))))


def parity(O, scene, run, r, gacc):
    """GPU flags and points against the oracle's on the same solves.  Planes
    and straight edges: flags must match and points agree; curved paths may
    have several roots, so a GPU root that differs from the oracle's is
    verified by an oracle solve started at the GPU point."""
    samp, sb, orc, oacc = run["samp"], run["sb"], run["orc"], run["oacc"]
    gacc = gacc[samp]
    curved = np.zeros(len(samp), bool)
    for k in range(5):
        curved |= (sb.order > k) & np.isin(scene.type_of(np.maximum(sb.prim[k], 0)), (2, 3))
    both = (gacc == 1) & (oacc == 1)
    errs, other_root, unverified, n_ok = [], 0, 0, 0
    for i in np.where(both | ((gacc == 1) & curved))[0]:
        o_ = sb.order[i]
        xg = r["x"][:3 * o_, samp[i]]
        e = np.inf
        if oacc[i]:
            e = float(np.linalg.norm((xg - orc["x"][:3 * o_, i]).reshape(o_, 3), axis=1).max())
        if e <= 1e-6 or not curved[i]:
            errs.append(e)
            n_ok += int(e <= 1e-6)
            continue
        X, c_, it_, st_ = O.solve_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], x0=xg)
        ok = st_ == O.CONVERGED and O.accept_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], X, st_) and \
            np.linalg.norm((X - xg).reshape(o_, 3), axis=1).max() <= 1e-6
        other_root += int(ok)
        unverified += int(not ok)
        n_ok += int(ok)
    # planes and straight edges: a GPU root the oracle's straight-line run
    # did not reach is checked by an oracle solve from the GPU point (the
    # root is unique, so a confirmed point is that root)
    flat = ~curved
    planar_gpu_only = np.where(flat & (gacc == 1) & (oacc == 0))[0]
    planar_confirmed = 0
    for i in planar_gpu_only:
        o_ = sb.order[i]
        xg = r["x"][:3 * o_, samp[i]]
        X, c_, it_, st_ = O.solve_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], x0=xg)
        planar_confirmed += int(st_ == O.CONVERGED and
                                O.accept_one(scene, sb.rx[sb.rx_index[i]], sb.prim[:o_, i], X, st_) and
                                np.linalg.norm((X - xg).reshape(o_, 3), axis=1).max() <= 1e-6)
    # n_ok: GPU-accepted paths that meet the bar (the oracle's root within
    # 1e-6 m, a verified other root of a curved path, or a confirmed root of
    # a planar path the oracle's straight-line run did not reach)
    n_ok += planar_confirmed
    n_gpu = int((gacc == 1).sum())
    over = int((np.array(errs) > 1e-6).sum()) if errs else 0
    errs = np.array(errs) if errs else np.zeros(1)
    mism = np.where(flat & (gacc != oacc))[0]
    oracle_only = int(((gacc == 0) & (oacc == 1)).sum())
    # misses: roots the oracle's straight-line run found and the GPU did not
    # accept, GPU roots the oracle could not confirm (curved or planar), and
    # points beyond the bar
    misses = oracle_only + unverified + (len(planar_gpu_only) - planar_confirmed) + over
    return {"sample": int(len(samp)), "gpu_accepted": n_gpu, "accepted_within_bar": n_ok,
            "misses": int(misses), "recall": n_ok / max(1, n_ok + oracle_only),
            "over_1e-6_m": over,
            "flag_mismatches_planar": int(len(mism)),
            "planar_mismatch_solves": [int(samp[i]) for i in mism[:8]],
            "planar_gpu_only_confirmed_by_oracle": planar_confirmed,
            "gpu_only": int(((gacc == 1) & (oacc == 0)).sum()),
            "oracle_only": oracle_only,
            "curved_other_root_verified": other_root, "curved_unverified": unverified,
            "point_err_m": {"max": float(errs.max()), "p50": float(np.percentile(errs, 50)),
                            "p99": float(np.percentile(errs, 99))}}


def emit(args, value, ms, variant, dtype, workload, n, variants, roofline, cpu, par, extra=None):
    line = {
        "metric": "accepted paths/sec at 1e-6 m point error vs FP64 oracle (learned+FP32 vs plain)",
        "value": value,
        "unit": "accepted paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded generators)",
        "config": {"workload": workload, "solves": int(n), "variant": VARIANT_TEXT[variant]},
        "variants": {v: {k: (round(x, 6) if isinstance(x, float) else x) for k, x in d.items()}
                     for v, d in variants.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": par,
    }
    if extra:
        line.update(extra)
    print(json.dumps(line))


def main_single(args, torch, mpt, W):
    t0 = time.time()
    if args.config == 5:
        scene, batch = W.config5(n_rx=args.n_rx or 16384)
    elif args.n_rx:
        scene, batch = W.CONFIGS[args.config](n_rx=args.n_rx)
    else:
        scene, batch = W.CONFIGS[args.config]()
    n = batch.n
    log(f"# workload generated in {time.time() - t0:.1f}s: {n} solves")
    ctx = mpt.Context(0)
    ctx.upload_scene(scene)

    variant = args.variant
    if variant in ("auto", "L", "A"):
        ok = False
        try:
            from paper_2301_06399_amd import learned
            ok = learned.prepare(ctx, scene, batch, steps=args.train_steps or None)
        except (ImportError, mpt.MptError) as e:
            log(f"# learned start unavailable: {e}")
        if variant in ("L", "A") and not ok:
            print(json.dumps({"error": "learned start requested but unavailable"}))
            sys.exit(3)
        variant = variant if variant != "auto" else ("L" if ok else "S")

    if args.copy_mib:
        # a plain copy of known size: what the HBM byte counters read for it
        # calibrates them for the solver kernels
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)  # one elementwise kernel: reads and writes copy_mib MiB
        torch.cuda.synchronize()
        del src, dst

    run = Runner(torch, mpt, ctx, scene, batch)
    # S runs in the parametric form whenever the scene allows it, so Sp is
    # the same run; it is listed only for scenes that need the implicit form
    others = ("S", "Si", "P", "Pp") if run.ctx_form_auto_is_param() else ("S", "Sp", "P", "Pp")
    variants = [variant] if args.only_main else [variant] + [x for x in others if x != variant]
    results, outs, flags = {}, {}, {}
    for v in variants:
        steps = args.steps if v == variant else max(5, args.steps // 4)
        warm = args.warmup if v == variant else 1
        results[v], outs[v] = run.run(v, steps, warm, tune=not args.no_autotune, graph=not args.no_graph)
        flags[v] = run.flags()
    main_r, r = results[variant], outs[variant]
    # physical validation of the headline variant's accepted paths (after
    # the step; reported beside it, not part of the metric)
    acc_t = torch.from_numpy(flags[variant]).to("cuda")
    out_v = mpt.DeviceOut(n)
    out_v.x.zero_()
    out_v.points().copy_(torch.from_numpy(r["x"]).to("cuda"))
    vis, nvis = ctx.visible(run.db, out_v, acc_t)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(10):
        ctx.visible(run.db, out_v, acc_t, sync=False)
    torch.cuda.synchronize()
    validation = {"visible": nvis, "ms": (time.perf_counter() - t) * 100.0}
    prec = "fp32" if VARIANTS[variant][0] else "fp64"
    form = used_form(VARIANTS[variant][2], main_r["launch"], scene)
    main_r["form_used"] = form
    roof = lm_roofline(scene, batch, r, main_r["stage_ms"], prec, args.config, mpt, form,
                       (main_r.get("launch") or {}).get("sched"))

    cpu = par = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.lib()
        cores = ncores()
        fname = "param" if form else "implicit"
        orun = oracle_run(O, scene, batch, cores, 10.0, args.cpu_sample or 2_000_000, fname)
        what = "the whole workload" if orun["m"] == n else f"a seeded uniform sample of the {n} solves"
        one = oracle_single_thread(O, scene, orun["sb"], 6.0, fname)
        cpu = {"value": orun["acc"] / orun["t"], "unit": "accepted paths/s", "cores": cores, "kind": "oracle",
               "sample": f"{what} ({orun['m']} solves), {fname} form, solve + accept, {orun['reps']} passes, "
                         f"{orun['t']:.1f} s on {cores} threads; one thread: the first {one['solves']} solves "
                         f"of it, {one['s']:.1f} s",
               "solves_per_s": orun["reps"] * orun["m"] / orun["t"],
               "single_thread": {"value": one["value"], "solves_per_s": one["solves_per_s"]}}
        par = parity(O, scene, orun, r, flags[variant])
        ovis = O.visible_batch(scene, batch, r["x"], flags[variant], nthreads=cores)
        validation["oracle_flag_mismatches"] = int((ovis != vis.cpu().numpy()).sum())
    # the metric counts the accepted paths that meet the 1e-6 m bar against
    # the oracle: exact when the whole workload was checked, else the
    # checked sample's share
    value = main_r["paths_per_s"]
    if par and par["gpu_accepted"]:
        value *= par["accepted_within_bar"] / par["gpu_accepted"]
    emit(args, value, main_r["ms_per_step"], variant, "f32+f64" if VARIANTS[variant][0] else "f64",
         NAMES[args.config], n, results, roof, cpu, par, extra={"validation": validation})


def main_learned(args, torch, mpt, W):
    """Learned-start evaluation: one network trained on the outputs of the
    plain FP64 solver for 2 M problems (half street canyon, half curved, the
    "train" seed stream), then L / A / S / P timed on 1 M held-out problems
    (the "heldout" stream), each half with its scene resident."""
    from paper_2301_06399_amd import learned
    n_rx = args.n_rx or 16384
    t0 = time.time()
    train = [W.training_batch(2, n_rx=n_rx), W.training_batch(3, n_rx=n_rx)]
    held = [W.training_batch(2, n_rx=n_rx // 2, stream="heldout"),
            W.training_batch(3, n_rx=n_rx // 2, stream="heldout")]
    log(f"# workloads generated in {time.time() - t0:.1f}s: train {sum(b.n for _, b in train)}, "
        f"held-out {sum(b.n for _, b in held)}")
    ctx = mpt.Context(0)
    t0 = time.time()
    hist = learned.train_joint(ctx, train, steps=args.train_steps or 6000, log=sys.stderr)
    log(f"# joint training {time.time() - t0:.1f}s, final losses {hist[-2:]}")
    del train
    variants = ["L", "A", "S", "Si", "P", "Pp"]
    per = {v: [] for v in variants}
    outs, flags = {}, {}
    for h, (sc, b) in enumerate(held):
        ctx.upload_scene(sc)
        run = Runner(torch, mpt, ctx, sc, b)
        for v in variants:
            res, r = run.run(v, args.steps, args.warmup, tune=not args.no_autotune)
            per[v].append(res)
            outs[(h, v)], flags[(h, v)] = r, run.flags()
    results = {}
    for v in variants:
        ms = sum(x["ms_per_step"] for x in per[v])
        k = sum(x["accepted"] for x in per[v])
        results[v] = {"ms_per_step": ms, "accepted": k, "paths_per_s": k / (ms * 1e-3),
                      "halves": [{kk: x[kk] for kk in ("ms_per_step", "accepted", "lm_iters_mean", "iters_mean",
                                                        "polished", "fallback", "stage_ms")} for x in per[v]]}
    # the network kernel on the curved half (every path served): MFMA roofline
    rows = held[1][1].n
    ms_net = per["L"][1]["stage_ms"]["learned"]
    ach = MLP_FLOPS_PER_ROW * rows / (ms_net * 1e-3)
    roof = {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK["bf16"] / 1e12, "unit": "TFLOP/s",
            "frac": ach / PEAK["bf16"], "traffic": None, "kernel": "k_mlp_fused (curved half, every row)",
            "flops_per_launch": MLP_FLOPS_PER_ROW * rows, "launch_ms": ms_net}
    cpu = par = None
    if not args.no_cpu_baseline:
        import oracle as O
        O.lib()
        cores = ncores()
        tot_t = tot_acc = tot_m = 0
        par = []
        for h, (sc, b) in enumerate(held):
            fm = used_form(VARIANTS["L"][2], per["L"][h].get("launch"), sc)
            orun = oracle_run(O, sc, b, cores, 5.0, args.cpu_sample or 2_000_000, "param" if fm else "implicit")
            tot_t += orun["t"]
            tot_acc += orun["acc"]
            tot_m += orun["m"] * orun["reps"]
            par.append(parity(O, sc, orun, outs[(h, "L")], flags[(h, "L")]))
        cpu = {"value": tot_acc / tot_t, "unit": "accepted paths/s", "cores": cores, "kind": "oracle",
               "sample": f"the whole held-out set (both halves), solve + accept, {tot_t:.1f} s",
               "solves_per_s": tot_m / tot_t}
    n = sum(b.n for _, b in held)
    value = results["L"]["paths_per_s"]
    if par and sum(p["gpu_accepted"] for p in par):
        value *= sum(p["accepted_within_bar"] for p in par) / sum(p["gpu_accepted"] for p in par)
    emit(args, value, results["L"]["ms_per_step"], "L", "bf16+f32+f64", NAMES[4], n,
         results, roof, cpu, par, extra={"training": {"problems": 2 * n_rx * 64, "loss_history": hist[-4:]}})


def main_alg1(args, torch, mpt, W):
    """Alg. 1 end to end on the street canyon for a block of receivers:
    visibility matrix, UE columns, every simple path up to max_order objects
    as candidates, then the solve (FP32 + polish + fallback), acceptance and
    physical validation.  One step = the whole chain for every receiver."""
    import oracle as O
    scene, full = W.config2()
    n_rx = args.n_rx or 64
    rx = np.ascontiguousarray(full.rx[:n_rx])
    k, mo = args.samples, args.max_order
    ctx = mpt.Context(0)
    ctx.upload_scene(scene)
    R = torch.from_numpy(rx).cuda()
    opts = mpt.default_opts(form=2)

    def step(sync_each=False, t=None):
        def mark(name):
            if sync_each:
                torch.cuda.synchronize()
                t[name] = time.perf_counter()
        mark("start")
        V, B = ctx.visibility(k)
        mark("visibility")
        U, los = ctx.visibility_rx(R, k)
        mark("ue_columns")
        ri, order, prim = ctx.candidates(V, B, U, mo, args.edge_last)
        mark("candidates")
        db = mpt.device_batch(R, ri, order, prim)
        out = ctx.solve(db, opts)
        mark("solve")
        acc, idx, na = ctx.accept(db, out)
        mark("accept")
        vis, nv = ctx.visible(db, out, acc)
        mark("validate")
        return V, B, U, db, out, acc, vis, na, nv

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        V, B, U, db, out, acc, vis, na, nv = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    marks = {}
    step(True, marks)
    names = ["visibility", "ue_columns", "candidates", "solve", "accept", "validate"]
    prev, stages = marks["start"], {}
    for nm in names:
        stages[nm] = round((marks[nm] - prev) * 1e3, 4)
        prev = marks[nm]
    m = db.n
    # the candidate fill writes rx_index, order and prim (28 B per path)
    cand_ms = stages["candidates"]
    fill_bytes = 28.0 * m
    roof = {"bound": "hbm", "achieved": fill_bytes / (cand_ms * 1e-3) / 1e9, "peak": PEAK["hbm"] / 1e9,
            "unit": "GB/s", "frac": fill_bytes / (cand_ms * 1e-3) / PEAK["hbm"], "traffic": None,
            "kernel": "mpt_candidates (count + scan + fill), sync to sync", "bytes_per_launch": fill_bytes}
    # parity: the oracle's visibility and lists for the first receivers, and
    # its chain on their candidates
    nr = min(n_rx, 2)
    Vb, Bb, Ub = mpt.unpack_bits(V, scene.n_prims), mpt.unpack_bits(B, scene.n_prims), mpt.unpack_bits(U, scene.n_prims)
    t = time.perf_counter()
    oV, oB = O.visibility(scene, k=k, nthreads=ncores())
    oU, _ = O.visibility_rx(scene, rx[:nr], k=k, nthreads=ncores())
    oc = O.candidates(scene, rx[:nr], oV, oB, oU, mo, args.edge_last)
    sel = np.where(db.rx_index.cpu().numpy() < nr)[0]
    ob = W.Batch(rx[:nr], oc["rx_index"], oc["order"], oc["prim"])
    # the oracle in the form the library ran (the forms can accept different
    # paths on hard planar chains)
    fm = "param" if ctx.last_launch().get("form", 0) == 1 else "implicit"
    orc = O.solve_batch(scene, ob, nthreads=ncores(), form=fm)
    oacc = O.accept_batch(scene, ob, orc["x"], orc["status"], nthreads=ncores())
    ovis = O.visible_batch(scene, ob, orc["x"], oacc, nthreads=ncores())
    t_cpu = time.perf_counter() - t
    same_lists = (np.array_equal(db.prim.cpu().numpy()[:, sel], oc["prim"]) and
                  np.array_equal(db.order.cpu().numpy()[sel], oc["order"]))
    par = {"receivers": nr, "visibility_equal": bool(np.array_equal(Vb, oV) and np.array_equal(Bb, oB)),
           "ue_equal": bool(np.array_equal(Ub[:nr], oU)), "candidate_lists_equal": bool(same_lists),
           "form": fm, "accept_equal": bool(np.array_equal(acc.cpu().numpy()[sel], oacc)),
           "accept_mismatches": int((acc.cpu().numpy()[sel] != oacc).sum()),
           "kept_equal": bool(np.array_equal(vis.cpu().numpy()[sel], ovis)),
           "kept_mismatches": int((vis.cpu().numpy()[sel] != ovis).sum())}
    # the validation itself on the same points: the oracle's test of the GPU's
    # accepted points (a path that grazes a facet can flip with the last bits
    # of its points, the GPU's and the oracle's solves differing there)
    gx = out.numpy()["x"][:, sel]
    ovis_g = O.visible_batch(scene, ob, gx, acc.cpu().numpy()[sel], nthreads=ncores())
    par["kept_equal_same_points"] = bool(np.array_equal(vis.cpu().numpy()[sel], ovis_g))
    cpu = {"value": int(ovis.sum()) / t_cpu, "unit": "kept paths/s", "cores": ncores(), "kind": "oracle",
           "sample": f"Alg. 1 for the first {nr} receivers (visibility matrix, their UE columns, "
                     f"{len(oc['order'])} candidates solved, accepted and validated)"}
    line = {
        "metric": "Alg. 1 kept paths/sec (visibility + candidates + solve + accept + validation)",
        "value": nv / (ms * 1e-3), "unit": "kept paths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic (seeded generators)",
        "config": {"workload": f"street canyon 50 boxes (651 objects), {n_rx} receivers, simple paths of "
                               f"1-{mo} objects, {k} samples per side" +
                               (", edges only last" if args.edge_last else ""), "receivers": n_rx, "max_order": mo,
                   "samples_per_side": k, "edge_last": bool(args.edge_last)},
        "candidates": m, "candidates_per_s": m / (ms * 1e-3), "accepted": na, "kept": nv, "stages_ms": stages,
        "roofline": roof, "cpu_baseline": cpu, "parity_sample": par}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=5, choices=[1, 2, 3, 4, 5, 6])
    ap.add_argument("--n-rx", type=int, default=0, help="receivers (0: the configuration's own)")
    ap.add_argument("--variant", default="auto", choices=["auto", "L", "A", "S", "Si", "Sp", "P", "Pp"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="largest oracle sample (0: 2,000,000 solves)")
    ap.add_argument("--train-steps", type=int, default=0, help="network training steps before timing")
    ap.add_argument("--only-main", action="store_true", help="time only the headline variant")
    ap.add_argument("--no-graph", action="store_true", help="launch the timed steps directly (no HIP graph)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the tuner: launch choices from MPT_AUTOTUNE_CACHE, else the defaults")
    ap.add_argument("--alg1", action="store_true",
                    help="Alg. 1 end to end: visibility, candidates, solve, accept, validation")
    ap.add_argument("--max-order", type=int, default=3, help="Alg. 1: most objects per candidate path")
    ap.add_argument("--samples", type=int, default=4, help="Alg. 1: sample points per side of an object")
    ap.add_argument("--edge-last", action="store_true", help="Alg. 1: a diffraction only as the last interaction")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2301_06399_amd import mpt
    from paper_2301_06399_amd import workloads as W
    if args.alg1:
        main_alg1(args, torch, mpt, W)
    elif args.config == 4:
        main_learned(args, torch, mpt, W)
    else:
        main_single(args, torch, mpt, W)


if __name__ == "__main__":
    main()
