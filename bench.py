#!/usr/bin/env python
"""Throughput benchmark of tree field integration on one MI355X.

Default workload: random recursive tree, N = 100,000 (vertex i attaches to a
uniform parent in [0, i)), integer weights uniform in {1..8}, field
F[N x 16] FP32 ~ N(0, 1), two kernels f(d) = exp(-0.05 d) and
f(d) = 1 / (1 + d)^2. One step integrates the field with both kernels
(2 N d vertex-channels). Inputs are resident on the GPU before timing.

Prints one JSON line: throughput (vertex-channels per second), parity
against the CPU FP64 oracle on 512 sampled rows, the roofline of the
dominant kernel stage (HIP events recorded by the library on the launch
stream during the timed steps), and the oracle's own throughput on the
host cores for a bounded sample of rows.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("vertex·channels integrated/s, fwd+bwd batched vs plain fwd, "
          "at rel err ≤1e-4")


# published dense peaks of one MI355X (FP32 vector includes packed issue)
PEAK_TFLOPS = {"mfma": {"f32": 157.3, "f64": 78.6}, "alu": {"f32": 157.3, "f64": 78.6}}
# the vector roof without packed FP32 issue, which the library's build turns
# off: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
ALU_UNPACKED_TFLOPS = {"f32": 78.6, "f64": 78.6}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


LIB_SOURCES = ["kernels.hpp", "kernels_expsum.hpp", "kernels_conv1d.hpp", "kernels_cells.hpp",
               "kernels_hankel.hpp",
               "tfi.hip", "plan.cpp", "plan.hpp"]


def measured_traffic(workload, stage, plan="-"):
    """HBM bytes per launch of a stage from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the summary has
    no line for it, the plan differs (leaf-tile size and direct/FFT rule,
    where the workload tunes them) or the library sources changed since it
    was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_pmc.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for name in LIB_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_34025_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    pat = re.compile(r"<!-- traffic workload=(\S+) stage=(\S+) (?:plan=(\S+) )?"
                     r"bytes_per_launch=(\d+) sources_sha256=([0-9a-f]+) -->")
    with open(path) as fh:
        for line in fh:
            m = pat.search(line)
            if (m and m.group(1) == workload and m.group(2) == stage
                    and (m.group(3) or "-") == plan and m.group(5) == sha):
                return int(m.group(4))
    return None


def stage_roofline(name, sd, dtype, workload=None, plan="-"):
    """Roofline entry of one profiled stage ({launches, ms, bytes, flops})."""
    sec = sd["ms"] * 1e-3
    gbs = sd["bytes"] / sec / 1e9
    unit = "mfma" if name.endswith("_mfma") else "alu"
    peak_tf = PEAK_TFLOPS[unit][dtype]
    flops = sd.get("flops", 0.0)
    if flops and flops / (peak_tf * 1e12) > sd["bytes"] / (HBM_PEAK_GBS * 1e9):
        tfs = flops / sec / 1e12
        r = {"bound": unit, "achieved": round(tfs, 3), "peak": peak_tf, "unit": "TFLOP/s",
             "frac": round(tfs / peak_tf, 4), "hbm_gbs": round(gbs, 2)}
        if unit == "alu":
            up = ALU_UNPACKED_TFLOPS[dtype]
            r.update({"peak_unpacked": up, "frac_unpacked": round(tfs / up, 4)})
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4)}
        if flops:
            r["tflops"] = round(flops / sec / 1e12, 3)
    r.update({"kernel": name,
              "traffic": measured_traffic(workload, name, plan) if workload else None,
              "launch_us": round(1e3 * sd["ms"] / sd["launches"], 3),
              "bytes_per_launch": sd["bytes"] / sd["launches"],
              "flops_per_launch": flops / sd["launches"]})
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default direct/FFT rule instead of tuning it")
    ap.add_argument("--fft-cost", type=float, default=None,
                    help="use this direct/FFT cost constant instead of tuning it")
    ap.add_argument("--batched-fft-cost", type=float, default=None,
                    help="direct/FFT cost constant of the batched table path instead of "
                         "tuning it (default: --fft-cost when given)")
    ap.add_argument("--leaf-max", type=int, default=None,
                    help="dense leaf-tile size of the plain-forward plan instead of tuning it")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched forest forward+backward measurement")
    ap.add_argument("--no-wide", action="store_true",
                    help="skip the wide-channel (C = 4160) patch-grid measurement")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched forest forward+backward measurement")
    ap.add_argument("--wide-only", action="store_true",
                    help="run only the wide-channel measurement")
    ap.add_argument("--wide-cases", default=None,
                    help="comma-separated tree:side cases of the wide-channel measurement "
                         "(default: serpentine 32..512, random/comb/fishbone 256)")
    ap.add_argument("--families", action="store_true",
                    help="also run the policy sweep over the paper's fifteen families "
                         "(off by default: one run of it ended in a host segmentation "
                         "fault with no cause shown yet)")
    ap.add_argument("--no-families", action="store_true",
                    help="(default) leave the family sweep out")
    ap.add_argument("--families-only", action="store_true",
                    help="run only the backbone-policy family sweep")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the FP64 2000-vertex, Sinkhorn and 2M-vertex configurations")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 2M-vertex forward + dF measurement")
    ap.add_argument("--large-trees", default="cater2m,binary2m",
                    help="comma-separated trees of that measurement")
    ap.add_argument("--configs-only", action="store_true",
                    help="run only those three configurations")
    ap.add_argument("--ablation", action="store_true",
                    help="also run the decomposition/evaluator ablation on six families, in "
                         "a child process (off by default: its one run ended in a host "
                         "heap-corruption abort, no cause shown yet)")
    ap.add_argument("--ablation-only", action="store_true",
                    help="run only that ablation")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    if args.copy_probe:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.batched_only:
        print(json.dumps({"batched_fwd_bwd": batched_fwd_bwd(args, None)}), flush=True)
        return
    if args.wide_only:
        print(json.dumps({"wide_channel": wide_channel(args)}), flush=True)
        return
    if args.families_only:
        print(json.dumps({"family_sweep": family_sweep(args)}), flush=True)
        return
    if args.ablation_only:
        print(json.dumps({"policy_ablation": policy_ablation(args)}), flush=True)
        return
    if args.large_only:
        print(json.dumps({"large": large_trees(args)}), flush=True)
        return
    if args.configs_only:
        print(json.dumps({"small_fp64": small_fp64(args), "sinkhorn": sinkhorn_sphere(args),
                          "large": large_trees(args)}), flush=True)
        return
    W = S.workload("rrt100k")
    p, w, F = W["parent"], W["weight"], W["F"]
    N, d = F.shape
    def tables(K):
        return [torch.tensor(fn(K), dtype=torch.float32, device=dev) for _, fn in W["kernels"]]

    t0 = time.perf_counter()
    leaf_tuning = None
    if args.leaf_max is not None or args.fft_cost is not None or args.no_autotune:
        tfi = TreeIntegrator(p, w, device=0, leaf_max=args.leaf_max or 0)
        build_s = time.perf_counter() - t0
        fs = tables(tfi.kernel_length)
        t0 = time.perf_counter()
        if args.fft_cost is not None:
            tfi.set_fft_cost(args.fft_cost)
            cost = args.fft_cost
        else:
            cost = tfi.autotune(fs[0], d) if not args.no_autotune else tfi.stats()["fft_cost"]
    else:
        # plan per leaf-tile size, each with its table rule autotuned; the
        # fastest is kept (setup, outside the timed steps)
        tfi = TreeIntegrator.tuned(p, w, tables, d, device=0)
        build_s = time.perf_counter() - t0
        fs = tables(tfi.kernel_length)
        cost = tfi.stats()["fft_cost"]
        leaf_tuning = tfi.tuning
    tune_s = time.perf_counter() - t0
    K = tfi.kernel_length
    tabs = [fn(K) for _, fn in W["kernels"]]
    Ft = torch.tensor(F, device=dev)
    log(f"bench: N={N} d={d} build {build_s:.2f}s kernel_length={K} "
        f"autotuned fft_cost={cost} in {tune_s:.2f}s")

    outs = [torch.empty_like(Ft) for _ in fs]
    def step():
        # both kernels in one call: the cell sums of F are formed once; the
        # results go to the same tensors every step
        tfi.integrate_many(fs, Ft, out=outs)

    def step_separate():
        for i, f in enumerate(fs):
            tfi.integrate(f, Ft, out=outs[i])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel durations: the same steps again with HIP events around every
    # stage on its launch stream (direct launches instead of graph replay;
    # the kernels are the same)
    tfi.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tfi.profile(False)
    stages = tfi.profile_report()
    ms_per_step = 1e3 * elapsed / args.steps
    value = 2 * N * d / (elapsed / args.steps)
    # the same step as two separate integrations, for reference
    for _ in range(args.warmup):
        step_separate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_separate()
    torch.cuda.synchronize()
    separate_ms = 1e3 * (time.perf_counter() - t0) / args.steps
    step()
    log(f"bench: {ms_per_step:.4f} ms/step, {value:.4e} vertex*channels/s")

    # the exponential kernel through each evaluator (per integration)
    lam_t = torch.tensor([float(np.exp(-0.05))], dtype=torch.float32, device=dev)
    one_t = torch.ones(1, dtype=torch.float32, device=dev)
    exp_ms = {}
    for name, call in (("table", lambda: tfi.integrate(fs[0], Ft)),
                       ("sweep", lambda: tfi.integrate_expsum(one_t, lam_t, Ft))):
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            y_exp = call()
        torch.cuda.synchronize()
        exp_ms[name] = 1e3 * (time.perf_counter() - t0) / args.steps
    rows_e = np.random.default_rng(98).choice(N, 256, replace=False)
    ref_e = oracle.integrate(p, w, tabs[0], F.astype(np.float64), rows=rows_e)
    exp_sweep_err = float(np.linalg.norm(y_exp.cpu().numpy()[rows_e] - ref_e) / np.linalg.norm(ref_e))
    log(f"bench: exp kernel per integration: table {exp_ms['table']:.4f} ms, "
        f"sweep {exp_ms['sweep']:.4f} ms (sweep parity {exp_sweep_err:.2e})")

    # parity on 512 sampled rows of the last step's outputs
    rows = np.random.default_rng(99).choice(N, 512, replace=False)
    errs = {}
    for (name, _), tab, out in zip(W["kernels"], tabs, outs):
        ref = oracle.integrate(p, w, tab, F.astype(np.float64), rows=rows)
        y = out.cpu().numpy()[rows].astype(np.float64)
        errs[name] = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    ok = all(e <= 1e-4 for e in errs.values())
    log(f"bench: parity {errs} ok={ok}")

    # dominant stage and its roofline: algorithmic bytes and, for the
    # contraction stages, flops per launch over the event-timed launch
    # duration; the bound is whichever peak the stage's work would take
    # longer to reach
    dom = max(stages, key=lambda k: stages[k]["ms"])
    leaf_used = int(getattr(tfi, "leaf_max", None) or args.leaf_max or 32)
    # plan key of the counter lines: leaf-tile size and how many tables the
    # direct/FFT rule sends to the FFT (the tuned constant itself may differ
    # between runs that assign the same methods)
    plan_key = f"leaf{leaf_used}_fft{tfi.stats()['fft_jobs']}"
    roofline = stage_roofline(dom, stages[dom], "f32", "rrt100k", plan=plan_key)

    cpu = None
    if not args.no_cpu_baseline:
        Fd = F.astype(np.float64)
        cores = oracle.num_threads()
        # marginal cost per row from two probe sizes (each call also pays a
        # fixed setup: adjacency build and thread start)
        probe_t = []
        for m in (64, 512):
            probe = np.random.default_rng(m).choice(N, m, replace=False)
            t0 = time.perf_counter()
            for tab in tabs:
                oracle.integrate(p, w, tab, Fd, rows=probe)
            probe_t.append(time.perf_counter() - t0)
        per_row = max((probe_t[1] - probe_t[0]) / 448, probe_t[1] / 512 * 0.25, 1e-9)
        nrows = int(min(N, max(512, args.cpu_seconds / per_row)))
        sample = np.random.default_rng(7).choice(N, nrows, replace=False)
        t0 = time.perf_counter()
        for tab in tabs:
            oracle.integrate(p, w, tab, Fd, rows=sample)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": 2 * nrows * d / cpu_s, "unit": "vertex*channels/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{nrows} uniformly sampled rows of the same workload, both kernels, "
                         f"{cpu_s:.1f} s, FP64"}
        log(f"bench: oracle {cpu['value']:.3e} vertex*channels/s on {cores} threads")

    batched = None if args.no_batched else batched_fwd_bwd(args, value)
    wide = None if args.no_wide else wide_channel(args)
    small = sink = large = None
    if not args.no_configs:
        small, sink, large = small_fp64(args), sinkhorn_sphere(args), large_trees(args)
    families = family_sweep(args) if (args.families and not args.no_families) else None
    ablation = child_section("--ablation-only", "policy_ablation") if args.ablation else None

    rec = {
        "metric": METRIC, "value": value, "unit": "vertex*channels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain forward, one tree: random recursive tree N=100000, "
                               "weights U{1..8}, F[N x 16] fp32 ~ N(0,1), kernels "
                               "exp(-0.05 d) and 1/(1+d)^2 (one step = both kernels, one "
                               "tfi_integrate_multi call: the cell sums of F are formed once)",
                   "N": int(N), "d": int(d), "kernels": 2,
                   "kernel_length": int(K), "build_s": round(build_s, 3),
                   "fft_cost": cost,
                   "leaf_max": leaf_used, "plan_key": plan_key,
                   "leaf_tuning_ms": ({str(k): round(v, 4) for k, v in leaf_tuning.items()}
                                      if leaf_tuning else None)},
        "parity": {"rows": 512, "rel_err": errs, "ok": ok},
        "ms_per_step_two_calls": round(separate_ms, 5),
        "exp_kernel_ms_per_integration": {k: round(v, 5) for k, v in exp_ms.items()},
        "exp_kernel_sweep_rel_err": exp_sweep_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_fwd_bwd": batched,
        "wide_channel": wide,
        "k3_roofline": (wide or {}).get("k3_roofline"),
        "small_fp64": small,
        "sinkhorn": sink,
        "large": large,
        "family_sweep": families,
        "policy_ablation": ablation,
        "stages": stages,
    }
    print(json.dumps(rec), flush=True)


def batched_fwd_bwd(args, plain_value):
    """Training step on a forest: 512 minimum spanning trees of sqrt(n) x
    sqrt(n) grids (side uniform in {14..64}, weights U{1..16}), F[n x 64]
    FP32, learnable kernel f(d) = sum_{k<8} a_k exp(-b_k d); loss
    sum(W * out). One step = forward + backward (dF, da, db) through an
    autograd function, timed for two evaluators of the same kernel: the
    backbone sweeps for exponential sums (ExpSumIntegrate, the reported
    value) and the general kernel-table path (TreeIntegrate with the table
    built from a, b; its direct/FFT rule autotuned on forward+adjoint
    passes). Parity of each: out and dF on 512 sampled rows against the
    oracle; da exactly against the oracle's exp-kernel recursion
    (da_k = <W, K_k F> with K_k the single exponential e^{-b_k d}); db by a
    central difference of that recursion in b_k."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import (ExpSumIntegrate, TreeIntegrator, TreeIntegrate,
                                      expsum_table)
    from paper_2609_34025_amd import synth as S

    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    W = S.workload("grid512")
    gen_s = time.perf_counter() - t0
    p, w, F = W["parent"], W["weight"], W["F"]
    n, d = F.shape
    t0 = time.perf_counter()
    tfi = TreeIntegrator(p, w, device=0)
    build_s = time.perf_counter() - t0
    K = tfi.kernel_length
    rng = np.random.default_rng(33)
    pinned = args.batched_fft_cost if args.batched_fft_cost is not None else args.fft_cost
    if pinned is not None:
        tfi.set_fft_cost(pinned)
        cost = pinned
    elif not args.no_autotune:
        ftune = torch.tensor(W["kernels"][0][1](K), dtype=torch.float32, device=dev)
        cost = tfi.autotune(ftune, d, backward=True)
    else:
        cost = tfi.stats()["fft_cost"]
    log(f"batched: {len(W['offsets']) - 1} trees, n={n} d={d} gen {gen_s:.1f}s "
        f"build {build_s:.2f}s kernel_length={K} table-path fft_cost={cost}")
    Wt = torch.tensor(rng.standard_normal((n, d)), dtype=torch.float32, device=dev)
    a = torch.tensor(W["a"], dtype=torch.float32, device=dev, requires_grad=True)
    b = torch.tensor(W["b"], dtype=torch.float32, device=dev, requires_grad=True)
    Ft = torch.tensor(F, device=dev, requires_grad=True)

    # oracle references, shared by both evaluators
    rows = np.random.default_rng(99).choice(n, 512, replace=False)
    A = a.detach().double().cpu().numpy()
    B = b.detach().double().cpu().numpy()
    ftab = (A[None, :] * np.exp(-np.arange(K)[:, None] * B[None, :])).sum(1)
    Fd = F.astype(np.float64)
    Wd = Wt.double().cpu().numpy()
    ref_out = oracle.integrate(p, w, ftab, Fd, rows=rows)
    ref_dF = oracle.integrate(p, w, ftab, Wd, rows=rows)
    da_ref = np.array([np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k])], Fd))
                       for k in range(8)])
    hb = 1e-5
    db_ref = np.array([A[k] * (np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k] - hb)], Fd))
                               - np.sum(Wd * oracle.expdp(p, w, [1.0], [np.exp(-B[k] + hb)], Fd)))
                       / (2 * hb) for k in range(8)])

    def rel(x, r):
        return float(np.linalg.norm(x - r) / np.linalg.norm(r))

    paths = {
        "sweep": lambda: ExpSumIntegrate.apply(tfi, Ft, a, b),
        "table": lambda: TreeIntegrate.apply(tfi, Ft, expsum_table(a, b, K)),
    }
    results = {}
    for name, fwd in paths.items():
        res = {}

        def step():
            a.grad = b.grad = Ft.grad = None
            out = fwd()
            (Wt * out).sum().backward()
            res["out"] = out

        steps = max(5, args.steps // 5)
        for _ in range(max(2, args.warmup)):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        value = n * d / (el / steps)
        log(f"batched[{name}]: {1e3 * el / steps:.3f} ms/step fwd+bwd, "
            f"{value:.4e} vertex*channels/s")
        tfi.profile(True)
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        tfi.profile(False)
        stages = tfi.profile_report()
        for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["ms"]):
            log(f"batched[{name}] stage {k:16s} {v['launches']:4d} launches "
                f"{1e3 * v['ms'] / v['launches']:10.2f} us/launch")
        dom = max(stages, key=lambda k: stages[k]["ms"])
        errs = {"out": rel(res["out"].detach().double().cpu().numpy()[rows], ref_out),
                "dF": rel(Ft.grad.double().cpu().numpy()[rows], ref_dF),
                "da": rel(a.grad.double().cpu().numpy(), da_ref),
                "db": rel(b.grad.double().cpu().numpy(), db_ref)}
        ok = all(e <= 1e-4 for e in errs.values())
        log(f"batched[{name}]: parity {errs} ok={ok}")
        plan = "-" if name == "sweep" else f"fft{tfi.stats()['fft_jobs']}"
        wl = "grid512_sweep" if name == "sweep" else "grid512"
        results[name] = {"value": value, "steps": steps, "ms_per_step": 1e3 * el / steps,
                         "parity": {"rows": 512, "rel_err": errs, "ok": ok},
                         "roofline": stage_roofline(dom, stages[dom], "f32", wl, plan=plan),
                         # the FFT cross-interaction stages of the step
                         "k3_roofline": {k: stage_roofline(k, sd, "f32", wl, plan=plan)
                                         for k, sd in stages.items()
                                         if (k.startswith("fft") or k.startswith("df_fft"))
                                         and sd["ms"] > 0},
                         "stages": stages}
    best = results["sweep"]
    return {"value": best["value"], "unit": "vertex*channels/s", "steps": best["steps"],
            "ms_per_step": best["ms_per_step"],
            "ratio_vs_plain_fwd": best["value"] / plain_value if plain_value else None,
            "evaluator": "backbone sweeps for exponential sums (ExpSumIntegrate)",
            "workload": "forward+backward (dF, da, db) of 512 grid-MST trees, sides U{14..64}, "
                        "weights U{1..16}, F[n x 64] fp32, f = sum of 8 exponentials; "
                        "loss sum(W * out)",
            "n": int(n), "d": int(d), "trees": int(len(W["offsets"]) - 1),
            "kernel_length": int(K), "build_s": round(build_s, 3),
            "parity": best["parity"], "roofline": best["roofline"], "stages": best["stages"],
            "table_path": {"value": results["table"]["value"],
                           "ms_per_step": results["table"]["ms_per_step"],
                           "ratio_vs_plain_fwd": (results["table"]["value"] / plain_value
                                                  if plain_value else None),
                           "fft_cost": cost, "plan_key": f"fft{tfi.stats()['fft_jobs']}",
                           "parity": results["table"]["parity"],
                           "roofline": results["table"]["roofline"],
                           "k3_roofline": results["table"]["k3_roofline"],
                           "stages": results["table"]["stages"]}}



# The paper's 32-core CPU timings of one integration at C = 4160 (seconds;
# tables "vit-runtime" and "vit-crossover"), quoted as context only.
PAPER_CPU_S = {("serpentine", 1024): 0.39, ("serpentine", 4096): 1.76,
               ("serpentine", 16384): 8.02, ("serpentine", 65536): 37.82,
               ("serpentine", 262144): 165.67, ("random", 65536): 121.4,
               ("comb", 65536): 231.1, ("fishbone", 65536): 91.4}


def wide_channel(args):
    """Masked-linear-attention payload (C = 4160 channels) on patch-grid
    spanning trees: serpentine paths from a 32x32 to a 512x512 grid, and the
    random, comb and fishbone trees at 256x256. FP32 forward, graph replay,
    parity on sampled rows x channels against the FP64 oracle."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    if args.wide_cases:
        cases = [(c.split(":")[0], int(c.split(":")[1])) for c in args.wide_cases.split(",")]
    else:
        cases = [("serpentine", s) for s in (32, 64, 128, 256, 384, 512)]
        cases += [("random", 256), ("comb", 256), ("fishbone", 256)]
    out_cases = []
    roofline = None
    k3 = {}
    for kind, side in cases:
        W = S.workload("attn", tree=kind, side=side)
        p, w = W["parent"], W["weight"]
        n, C = len(p), W["d"]
        t0 = time.perf_counter()
        tfi = TreeIntegrator(p, w, device=0)
        build_s = time.perf_counter() - t0
        K = tfi.kernel_length
        tab = W["kernels"][0][1](K)
        f = torch.tensor(tab, dtype=torch.float32, device=dev)
        phi = torch.from_numpy(W["phi"]).to(dev)
        v = torch.from_numpy(W["v"]).to(dev)
        # payload [phi v^T | phi] built on the device (input preparation)
        F = torch.cat([(phi[:, :, None] * v[:, None, :]).reshape(n, -1), phi], 1).contiguous()
        del phi, v
        cost = tfi.autotune(f, C)
        reps = 3 if n >= 100000 else 5
        for _ in range(2):
            y = tfi.integrate(f, F)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            y = tfi.integrate(f, F)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        tfi.profile(True)
        tfi.integrate(f, F)
        torch.cuda.synchronize()
        tfi.profile(False)
        stages = tfi.profile_report()
        rng = np.random.default_rng(side)
        rows = np.sort(rng.choice(n, 32, replace=False))
        chans = np.sort(rng.choice(C, 64, replace=False))
        Fs = F[:, chans].double().cpu().numpy()
        ref = oracle.integrate(p, w, tab, Fs, rows=rows)
        got = y[rows][:, chans].double().cpu().numpy()
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        rec = {"tree": kind, "side": side, "N": n, "C": C, "ms": round(ms, 4),
               "value": n * C / (ms * 1e-3), "build_s": round(build_s, 3),
               "fft_cost": cost, "rel_err": err, "ok": err <= 1e-4,
               "stages_ms": {k: round(v["ms"], 4) for k, v in stages.items()}}
        if (kind, n) in PAPER_CPU_S:
            rec["paper_cpu_s"] = PAPER_CPU_S[(kind, n)]
        out_cases.append(rec)
        log(f"wide[{kind} {side}x{side}] N={n} C={C}: {ms:.3f} ms/integration "
            f"({rec['value']:.3e} vertex*channels/s), parity {err:.2e}")
        if kind == "serpentine" and side == 512:
            dom = max(stages, key=lambda k: stages[k]["ms"])
            roofline = stage_roofline(dom, stages[dom], "f32", "serpentine512")
        # the FFT cross-interaction stages of this case (1-D convolution,
        # 2-D LDS and global passes): algorithmic bytes over event time
        for k, sd in stages.items():
            if k.startswith("fft") and sd["ms"] > 0:
                k3[f"{kind}{side}/{k}"] = stage_roofline(k, sd, "f32", f"{kind}{side}")
        del tfi, F, y
        torch.cuda.empty_cache()
    return {"unit": "vertex*channels/s (forward, one integration)", "dtype": "f32",
            "payload": "x_j = [vec(phi_j v_j^T) | phi_j], r = dh = 64, C = 4160; "
                       "mask f = exp(u d^2 + v d + w), u=-1e-5, v=-0.01, w=0.5",
            "parity": "32 sampled rows x 64 sampled channels vs FP64 oracle",
            "paper_cpu_s": "32-core CPU, context only",
            "cases": out_cases, "roofline": roofline, "k3_roofline": k3}



def _timed(call, reps, warm=2):
    import torch
    for _ in range(warm):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def _stages(tfi, call):
    import torch
    tfi.profile(True)
    call()
    torch.cuda.synchronize()
    tfi.profile(False)
    return tfi.profile_report()


def small_fp64(args):
    """Plain forward of the small configuration: random recursive tree
    N = 2000 (parent of i uniform in [0, i)), weights U{1..4}, F[N x 4] FP64
    ~ N(0, 1), f(d) = exp(-0.1 d). Timed as graph replays into one output;
    parity on every row against the FP64 oracle (bar 1e-10)."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    W = S.workload("small")
    p, w, F = W["parent"], W["weight"], W["F"]
    n, d = F.shape
    tfi = TreeIntegrator(p, w, device=0)
    K = tfi.kernel_length
    tab = W["kernels"][0][1](K)
    f = torch.tensor(tab, dtype=torch.float64, device=dev)
    Ft = torch.tensor(F, device=dev)
    cost = tfi.autotune(f, d)
    out = torch.empty_like(Ft)
    ms = _timed(lambda: tfi.integrate(f, Ft, out=out), max(20, args.steps))
    stages = _stages(tfi, lambda: tfi.integrate(f, Ft, out=out))
    tfi.integrate(f, Ft, out=out)
    ref = oracle.integrate(p, w, tab, F)
    err = float(np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref))
    dom = max(stages, key=lambda k: stages[k]["ms"])
    log(f"small fp64: N={n} d={d} {ms:.4f} ms/integration, parity {err:.2e}")
    return {"workload": "plain forward, random recursive tree N=2000, weights U{1..4}, "
                        "F[N x 4] fp64 ~ N(0,1), f = exp(-0.1 d)",
            "dtype": "f64", "N": n, "d": d, "ms": round(ms, 5),
            "value": n * d / (ms * 1e-3), "unit": "vertex*channels/s", "fft_cost": cost,
            "parity": {"rows": "all", "rel_err": err, "ok": err <= 1e-10},
            "roofline": stage_roofline(dom, stages[dom], "f64")}


def sinkhorn_sphere(args):
    """Iterated solve: Sinkhorn scaling on the minimum spanning tree of the
    symmetrised 8-NN graph of 50,000 points uniform on the sphere, lengths
    quantised to 1/64, f(k) = exp(-k / 3.2) (exp(-d / 0.05)), marginals
    ~ Dirichlet(1). The products run through the kernel table (per-table
    rule autotuned) and, since f is one exponential, through the backbone
    sweeps; for each, 200 iterations of two FP32 products are timed (no
    residual checks inside the timed loop), then every product of a second
    200-iteration run is checked against the FP64 exp-kernel tree recursion
    applied to the same rounded input vector. The faster evaluator is the
    record's value."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S
    from paper_2609_34025_amd.sinkhorn import sinkhorn

    dev = torch.device("cuda", 0)
    W = S.workload("sphere50k")
    p, w = W["parent"], W["weight"]
    n = len(p)
    tfi = TreeIntegrator(p, w, device=0)
    K = tfi.kernel_length
    lam = float(np.exp(-1.0 / 3.2))
    table = torch.tensor(lam ** np.arange(K), dtype=torch.float32, device=dev)
    sweep = (torch.ones(1, dtype=torch.float32, device=dev),
             torch.full((1,), lam, dtype=torch.float32, device=dev))
    a = torch.tensor(W["a"], device=dev)
    b = torch.tensor(W["b"], device=dev)
    cost = tfi.autotune(table, 1)
    iters = 200
    x = torch.rand(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    runs = {}
    for name, f, prod in (("table", table, lambda: tfi.integrate(table, x, out=y)),
                          ("sweep", sweep, lambda: tfi.integrate_expsum(sweep[0], sweep[1], x))):
        sinkhorn(tfi, f, a, b, iters=5, check_every=10 ** 9)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sinkhorn(tfi, f, a, b, iters=iters, check_every=10 ** 9)
        torch.cuda.synchronize()
        ms_iter = 1e3 * (time.perf_counter() - t0) / iters
        ms_prod = _timed(prod, 200)
        stages = _stages(tfi, prod)
        errs = []

        def check(xin, yv):
            ref = oracle.expdp(p, w, [1.0], [lam], xin.double().cpu().numpy())
            errs.append(float(np.linalg.norm(yv.double().cpu().numpy() - ref) /
                              np.linalg.norm(ref)))

        _, _, res = sinkhorn(tfi, f, a, b, iters=iters, on_product=check)
        dom = max(stages, key=lambda k: stages[k]["ms"])
        log(f"sinkhorn[{name}]: N={n} {ms_iter:.4f} ms/iteration ({ms_prod:.4f} ms/product), "
            f"{len(errs)} products checked, max rel err {max(errs):.2e}")
        runs[name] = {"ms_per_iteration": round(ms_iter, 5), "ms_per_product": round(ms_prod, 5),
                      "parity": {"products": len(errs), "max_rel_err": max(errs),
                                 "ok": max(errs) <= 1e-4},
                      "residual_first_last": [res[0][1], res[-1][1]],
                      "roofline": stage_roofline(dom, stages[dom], "f32")}
    best = min(runs, key=lambda k: runs[k]["ms_per_iteration"])
    r = runs[best]
    return {"workload": "200 Sinkhorn iterations (2 fp32 products each) on the MST of the 8-NN "
                        "graph of 50000 points on the sphere, lengths in units of 1/64, "
                        "f(k) = exp(-k/3.2), marginals Dirichlet(1)",
            "N": n, "d": 1, "iterations": iters, "evaluator": best,
            "ms_per_iteration": r["ms_per_iteration"], "ms_per_product": r["ms_per_product"],
            "value": n / (r["ms_per_product"] * 1e-3),
            "unit": "vertex*channels/s (one product)", "fft_cost": cost,
            "parity": dict(r["parity"], oracle="fp64 exp-kernel tree recursion on the same "
                                               "fp32 input"),
            "residual_first_last": r["residual_first_last"], "roofline": r["roofline"],
            "evaluators": runs}


def large_trees(args):
    """Large forward + adjoint: N = 2,000,000 as a caterpillar (spine of
    N/4, three leaves per spine vertex) and as a binary random recursive
    tree, weights U{1..8}, F[N x 32] FP32 ~ N(0, 1), f(d) = exp(-0.01 d),
    gout ~ N(0, 1), under a 64 GB device-memory budget (kernel spectra are
    formed again in the adjoint, nothing is kept between the passes).
    Forward and dF are timed; parity on 512 sampled rows against the BFS
    oracle and on all rows against the exp-kernel tree recursion."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    budget = 64 << 30
    out_cases = []
    for name in args.large_trees.split(","):
        t0 = time.perf_counter()
        W = S.workload(name)
        p, w, F = W["parent"], W["weight"], W["F"]
        n, d = F.shape
        tfi = TreeIntegrator(p, w, device=0, memory_budget=budget)
        build_s = time.perf_counter() - t0
        K = tfi.kernel_length
        lam = float(np.exp(-0.01))
        tab = lam ** np.arange(K)
        f = torch.tensor(tab, dtype=torch.float32, device=dev)
        Ft = torch.tensor(F, device=dev)
        G = torch.tensor(np.random.default_rng(55).standard_normal(F.shape), dtype=torch.float32,
                         device=dev)
        out = torch.empty_like(Ft)
        ms_f = _timed(lambda: tfi.integrate(f, Ft, out=out), 3, warm=1)
        dF = {}

        def bwd():
            dF["x"], _ = tfi.backward(f, Ft, G, need_df=False)

        ms_b = _timed(bwd, 3, warm=1)
        stages = _stages(tfi, lambda: tfi.integrate(f, Ft, out=out))
        tfi.integrate(f, Ft, out=out)
        bwd()
        torch.cuda.synchronize()
        y, yd = out.cpu().numpy(), dF["x"].cpu().numpy()
        Fd, Gd = F.astype(np.float64), G.cpu().numpy().astype(np.float64)
        rows = np.random.default_rng(5).choice(n, 512, replace=False)
        errs = {"fwd_rows": oracle.integrate(p, w, tab, Fd, rows=rows),
                "dF_rows": oracle.integrate(p, w, tab, Gd, rows=rows)}
        errs = {"fwd_rows": float(np.linalg.norm(y[rows] - errs["fwd_rows"]) /
                                  np.linalg.norm(errs["fwd_rows"])),
                "dF_rows": float(np.linalg.norm(yd[rows] - errs["dF_rows"]) /
                                 np.linalg.norm(errs["dF_rows"]))}
        r = oracle.expdp(p, w, [1.0], [lam], Fd)
        errs["fwd_all"] = float(np.linalg.norm(y - r) / np.linalg.norm(r))
        r = oracle.expdp(p, w, [1.0], [lam], Gd)
        errs["dF_all"] = float(np.linalg.norm(yd - r) / np.linalg.norm(r))
        st = tfi.stats()
        dom = max(stages, key=lambda k: stages[k]["ms"])
        rec = {"tree": name, "N": n, "d": d, "build_s": round(build_s, 2),
               "ms_fwd": round(ms_f, 3), "ms_bwd_dF": round(ms_b, 3),
               "value": 2 * n * d / ((ms_f + ms_b) * 1e-3),
               "device_GiB": round(st["device_bytes"] / 2 ** 30, 2),
               "parity": {"rel_err": errs, "ok": max(errs.values()) <= 1e-4},
               "roofline": stage_roofline(dom, stages[dom], "f32", name),
               "stages": stages}
        # the FFT cross-interaction stages of this tree (K3)
        rec["k3_roofline"] = {k: stage_roofline(k, sd, "f32", name)
                              for k, sd in stages.items() if k.startswith("fft") and sd["ms"] > 0}
        out_cases.append(rec)
        log(f"large[{name}] N={n} d={d}: fwd {ms_f:.2f} ms, bwd dF {ms_b:.2f} ms, "
            f"{rec['device_GiB']} GiB, parity {errs}")
        del tfi, Ft, G, out, dF
        torch.cuda.empty_cache()
    return {"unit": "vertex*channels/s (forward + adjoint dF)", "dtype": "f32",
            "budget_bytes": budget, "cases": out_cases}


# The paper's CPU timings (ms) of the scalar forward with f(d) = 1/(1+d) at
# the largest size of each family (table "synthetic-largest"), quoted as
# context only: FTFI (centroid baseline), D2 (diameter + 2-D FFT), A2
# (adaptive + 2-D FFT).
PAPER_FAMILY_MS = {
    "path": (59.31, 1.15, 2.09), "balanced_binary": (64.10, 23.80, 56.63),
    "complete_3ary": (56.36, 29.72, 61.63), "caterpillar": (84.25, 35.43, 38.02),
    "caterpillar_hanging_paths": (64.77, 6.68, 16.67), "comb": (67.53, 24.11, 25.74),
    "broom": (54.76, 10.57, 11.80), "double_broom": (26.70, 5.32, 5.83),
    "uniform_spider": (44.51, 4.57, 5.86), "short_arm_spider": (41.22, 25.65, 30.51),
    "long_arm_spider": (259.52, 382.98, 20.33), "star": (25.25, 23.52, 25.02),
    "random_recursive": (43.73, 18.29, 38.83), "random_mst_topology": (46.37, 17.09, 41.79),
    "preferential_attachment": (38.42, 21.14, 33.22)}


def child_section(flag, key, timeout=900):
    """Run one section of this script in a child process (its own HIP
    context) and return its record; a child that fails leaves an error
    record instead of ending the whole run."""
    import subprocess
    t0 = time.perf_counter()
    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), flag],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                       timeout=timeout)
    for line in r.stderr.splitlines():
        if line.startswith("bench") or line.startswith("ablation"):
            log(line)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"child exited with status {r.returncode}",
                "stderr_tail": r.stderr[-2000:], "s": round(time.perf_counter() - t0, 1)}
    return json.loads(lines[-1])[key]


# Diameter-1D times of table "synthetic-largest" (CPU, Python; context only)
PAPER_D1_MS = {"balanced_binary": 49.46, "complete_3ary": 63.56,
               "caterpillar_hanging_paths": 62.78, "uniform_spider": 32.04,
               "long_arm_spider": 70288.89, "random_recursive": 37.48}

ABLATION_VARIANTS = [  # (label, policy, table method)
    ("centroid_fft", "centroid", "fft"),   # centroid-only decomposition (FTFI-style)
    ("D1", "diameter", "fft1d"),           # Diameter + per-depth-pair 1-D FFTs
    ("D2", "diameter", "fft"),             # Diameter + 2-D FFT
    ("A2", "adaptive", "fft"),             # Adaptive + 2-D FFT
    ("diameter_hankel", "diameter", "hankel"),  # Diameter + Hankel product
    ("adaptive_auto", "adaptive", "auto"),  # the library's default rule
]


def policy_ablation(args):
    """Decomposition and evaluator variants of the paper's ablation (table
    "synthetic-largest": FTFI, D1, D2, A2) plus the Hankel product and the
    library's default, on six of the fifteen families at their largest
    sizes: ms per integration (graph replay) of a scalar FP64 field with
    f(d) = 1/(1+d), the paper's setting, and of an FP32 field of 64
    channels; parity against the FP64 oracle on every row (scalar) or 16
    sampled rows (64 channels). One handle per (family, variant)."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    fams = {name: (p, w) for name, p, w in S.paper_families()}
    out = []
    worst = 0.0
    for name in PAPER_D1_MS:
        p, w = fams[name]
        n = len(p)
        rng = np.random.default_rng(321)
        F1 = rng.standard_normal(n)
        F64 = rng.standard_normal((n, 64)).astype(np.float32)
        rows = np.sort(rng.choice(n, 16, replace=False))
        rec = {"family": name, "N": n, "ms_scalar_fp64": {}, "ms_d64_fp32": {},
               "root": {}, "methods": {},
               "paper_cpu_ms": {"FTFI": PAPER_FAMILY_MS[name][0], "D1": PAPER_D1_MS[name],
                                "D2": PAPER_FAMILY_MS[name][1], "A2": PAPER_FAMILY_MS[name][2]}}
        for label, pol, meth in ABLATION_VARIANTS:
            tfi = TreeIntegrator(p, w, device=0, policy=pol, table_method=meth)
            K = tfi.kernel_length
            tab = 1.0 / (1.0 + np.arange(K, dtype=np.float64))
            st = tfi.stats()
            rec["root"][label] = [st["root"]["m"], st["root"]["H"]]
            m = tfi.export("job_method")
            rec["methods"][label] = {k: int((m == v).sum()) for k, v in
                                     (("direct", 0), ("fft", 1), ("fft1d", 2), ("hankel", 3))}
            for key, dt, Fh, bar in (("ms_scalar_fp64", torch.float64, F1, 1e-10),
                                     ("ms_d64_fp32", torch.float32, F64, 1e-4)):
                f = torch.tensor(tab, dtype=dt, device=dev)
                Fd = torch.tensor(Fh, device=dev)
                for _ in range(3):
                    y = tfi.integrate(f, Fd)
                torch.cuda.synchronize()
                reps = 20
                t0 = time.perf_counter()
                for _ in range(reps):
                    y = tfi.integrate(f, Fd)
                torch.cuda.synchronize()
                rec[key][label] = round(1e3 * (time.perf_counter() - t0) / reps, 4)
                if Fh.ndim == 1:
                    ref = oracle.integrate(p, w, tab, Fh)
                    got = y.cpu().numpy()
                else:
                    ref = oracle.integrate(p, w, tab, Fh.astype(np.float64), rows=rows)
                    got = y[rows].double().cpu().numpy()
                err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
                worst = max(worst, err / bar)
            tfi.close()
        out.append(rec)
        log(f"ablation[{name} N={n}] scalar fp64 ms {rec['ms_scalar_fp64']}")
    return {"unit": "ms per integration (graph replay)", "kernel": "f(d) = 1/(1+d)",
            "variants": {l: f"policy {p}, table method {m}" for l, p, m in ABLATION_VARIANTS},
            "parity_ok": worst <= 1.0, "worst_err_over_bar": worst,
            "paper_cpu_ms": "table synthetic-largest, CPU Python, context only",
            "families": out}


def family_sweep(args):
    """Backbone policies (adaptive = the paper's score, diameter, centroid)
    on the fifteen synthetic families at their largest sizes: forward time
    per integration of a scalar FP64 field with f(d) = 1/(1+d) (the paper's
    setting) and of an FP32 field of C = 4160 channels, each policy with
    its own tuned direct/FFT rule; parity against the FP64 oracle on every
    row (scalar) or on sampled rows x channels (wide)."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_34025_amd import TreeIntegrator, synth as S

    dev = torch.device("cuda", 0)
    policies = ("adaptive", "diameter", "centroid")
    fams = []
    worst = 0.0
    for name, p, w in S.paper_families():
        n = len(p)
        rng = np.random.default_rng(123)
        F1 = rng.standard_normal(n)
        phi, v = S.attention_features(n, 64, 64, rng)
        Fw = torch.from_numpy(S.attention_payload(phi, v)).to(dev)
        C = Fw.shape[1]
        rec = {"family": name, "N": n, "ms_scalar_fp64": {}, "ms_wide_fp32": {}, "plan": {}}
        if name in PAPER_FAMILY_MS:
            ftfi, d2, a2 = PAPER_FAMILY_MS[name]
            rec["paper_cpu_ms"] = {"FTFI": ftfi, "D2": d2, "A2": a2}
        widths = (("ms_scalar_fp64", torch.float64, torch.tensor(F1, device=dev), 1),
                  ("ms_wide_fp32", torch.float32, Fw, C))
        for pol in policies:
            for key, dt, Fd, d in widths:
                tfi = TreeIntegrator(p, w, device=0, policy=pol)
                K = tfi.kernel_length
                tab = 1.0 / (1.0 + np.arange(K, dtype=np.float64))
                st = tfi.stats()
                rec["plan"].setdefault(pol, {})[key] = {
                    "calls": st["calls"], "root": [st["root"]["m"], st["root"]["H"]],
                    "sum_M": st["sum_M"], "levels": st["levels"]}
                f = torch.tensor(tab, dtype=dt, device=dev)
                tfi.autotune(f, d)
                for _ in range(3):
                    y = tfi.integrate(f, Fd)
                torch.cuda.synchronize()
                reps = 20
                t0 = time.perf_counter()
                for _ in range(reps):
                    y = tfi.integrate(f, Fd)
                torch.cuda.synchronize()
                rec[key][pol] = round(1e3 * (time.perf_counter() - t0) / reps, 4)
                if d == 1:
                    ref = oracle.integrate(p, w, tab, F1)
                    err = float(np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref))
                    bar = 1e-10
                else:
                    rows = np.sort(rng.choice(n, 16, replace=False))
                    ch = np.sort(rng.choice(C, 32, replace=False))
                    ref = oracle.integrate(p, w, tab, Fw[:, ch].double().cpu().numpy(), rows=rows)
                    got = y[rows][:, ch].double().cpu().numpy()
                    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
                    bar = 1e-4
                worst = max(worst, err / bar)
                del tfi
        fams.append(rec)
        log(f"families[{name} N={n}] scalar fp64 ms {rec['ms_scalar_fp64']} | "
            f"C={C} fp32 ms {rec['ms_wide_fp32']}")
    return {"unit": "ms per integration (graph replay)", "kernel": "f(d) = 1/(1+d)",
            "scalar": "F[N] FP64 ~ N(0,1) (default_rng(123))",
            "wide": "attention payload C = 4160 FP32",
            "parity_ok": worst <= 1.0, "worst_err_over_bar": worst,
            "paper_cpu_ms": "table synthetic-largest, CPU, context only",
            "families": fams}


if __name__ == "__main__":
    main()
