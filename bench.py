"""Benchmark of the MI355X dual-tree fast Gauss transform on one GPU.

Workload (the 2-D clustered configuration): 50,000 points, D = 2, 32
anisotropic Gaussian clusters + 10% uniform background, Q = R; seven
bandwidths h* x 10^{-3..3} (h* = the LSCV optimum, tests/golden/hstar.json);
relative error eps = 1e-2 on every query.

One step = the whole hot path over that input, resident in HBM:
  kd-tree build + raw moments (dfgt_build_tree)  ->  DFGT for all seven
  bandwidths in one traversal (dfgt_gauss_sum).
value = N_Q * N_R * 7 / (seconds per step)  [query x reference pairs / s].
The kd-tree leaf size is picked before anything is timed by
dfgt_tune_leaf_size on this workload (--leaf N fixes it instead); the choice
and every candidate's time are in config.leaf_tuning.
The plain tiled brute-force GPU sum (dfgt_naive_sum) over the same seven
bandwidths is timed alongside.

batched: the 3-D batch, 8 clustered problems of 10k..200k points, each swept
over 64 log-spaced bandwidths h_S x 10^{-3..3} at h and sqrt(2) h (the LSCV
pair): 1024 sums in one traversal, eager and as a captured graph replay,
beside the brute force over the same 1024 sums; its leaf size is tuned on the
largest problem.

grad_ms (the metric's second part): the backward pass on the 16-D workload,
200,000 points (8 latent clusters embedded + N(0, 0.01 I) noise), eps 1e-4,
bandwidths {h_S, h*} (h* of its seeded 5,000-point subsample,
tests/golden/hstar.json): dfgt_lscv_score with dCV/dh (sums at h and sqrt(2) h
with their h-derivatives) plus dfgt_gauss_sum_backward for dG/dq, tree built
once outside the timed region.

Prints ONE JSON line.  --gpus must be 1 (this build targets one GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "query×ref pairs/s at rel-err 1e-2 (dual-tree vs brute-force GPU) + grad ms"
SCALES = [1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0, 1000.0]
EPS = 1e-2

# Exhaustive-tile roofline (bound "alu"): the algorithmic work per point pair is
# 2D+1 FP32 VALU operations (D differences, D-1 fused multiply-adds + 1 multiply,
# 1 add) and one v_exp_f32.  Peak pair rate = 256 CUs x 64 lanes x 2.4 GHz /
# (2D+1 + EXP_SLOTS) VALU issue slots, EXP_SLOTS = issue cost of v_exp_f32 in
# full-rate slots (transcendentals run at a quarter of the VALU rate).  Rates
# are also quoted in TFLOP/s at FLOPS_PER_PAIR = 3D+1 (D subtractions, D
# squares, D-1 additions, the exponential, the accumulation).
CUS, LANES, CLOCK = 256, 64, 2.4e9
EXP_SLOTS = 4

# HBM bytes per launch of the mixed-precision exhaustive-tile kernel
# (k_etile<2, false, false>) in one step of this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the counters of a 256 MiB
# device copy: profiles/dfgt_c2_sweep_hbm_traffic.md.  Valid for the kernel
# as profiled; None when it has changed since.
K_ETILE_TRAFFIC_BYTES = {64: 9.90e6 + 2.99e6, 128: 8.41e6 + 2.90e6}  # by leaf size; others: not measured (null)


def flops_per_pair(d):
    return 3 * d + 1


def base_peak_pairs(d):
    return CUS * LANES * CLOCK / (2 * d + 1 + EXP_SLOTS)


def per_bandwidth(torch, dfgt, x, hs, leaf, reps=3):
    """Median ms per single-bandwidth call: DFGT, DFD ablation, brute force."""
    R = dfgt.build_tree(x, leaf_size=leaf)

    def med(f):
        f()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[reps // 2] * 1e3

    rows = []
    for s, h in zip(SCALES, hs):
        rows.append({
            "h_over_hstar": s,
            "dfgt_ms": med(lambda: dfgt.gauss_sum(R, R, [h], EPS)),
            "dfd_ms": med(lambda: dfgt.gauss_sum(R, R, [h], EPS, force_method=dfgt.FORCE_CENTROID)),
            "bruteforce_ms": med(lambda: dfgt.naive_sum(x, x, [h])),
        })
    return {"what": "single-bandwidth calls, tree built once, eps 1e-2: DFGT, the DFD ablation (only the "
                    "centroid finite-difference prune), brute force", "rows": rows}


def batched_bench(torch, dfgt, synth, leaf):
    """The 3-D batch: eager call, graph replays, brute force; returns details.

    leaf 0: the leaf size comes from dfgt_tune_leaf_size on the largest problem
    at 16 of its bandwidths (outside the timed region)."""
    xs = [synth.c4_problem(k) for k in range(8)]
    xd = [torch.as_tensor(x, device="cuda") for x in xs]
    torch.cuda.synchronize()
    tuning = None
    if leaf == 0:
        big = int(np.argmax([len(x) for x in xs]))
        hb = synth.silverman_h(xs[big]) * np.geomspace(1e-3, 1e3, 16)
        leaf, tms = dfgt.tune_leaf_size(xd[big], hb, EPS, reps=2)
        tuning = {"on": f"the largest problem (N = {len(xs[big])}), 16 log-spaced bandwidths, 2 repetitions",
                  "candidates_ms": {str(k): v for k, v in tms.items()}}
    t0 = time.perf_counter()
    trees = [dfgt.build_tree(x, leaf_size=leaf) for x in xd]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    probs = []
    for x, t in zip(xs, trees):
        base = synth.silverman_h(x) * np.geomspace(1e-3, 1e3, 64)
        probs.append((t, t, np.concatenate([base, np.sqrt(2.0) * base])))
    dfgt.gauss_sum_batched(probs, EPS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dfgt.gauss_sum_batched(probs, EPS)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    b = dfgt.Batch(probs, EPS, stats=True)
    b.run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    b.check()
    t0 = time.perf_counter()
    worst = 0.0
    for x, (t, _, h), G in zip(xd, probs, b.G):
        Gb = dfgt.naive_sum(x, x, h)
        worst = max(worst, float(((G - Gb).abs() / Gb).max()))
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t0
    pairs = float(sum(x.shape[0] ** 2 for x in xs)) * 128
    return {
        "workload": "3-D, 8 clustered problems N = 10k..200k (sum 690k), 64 log-spaced h x {1, sqrt2}, eps 1e-2",
        "sums": 8 * 128, "leaf_size": leaf, "leaf_tuning": tuning,
        "build_ms": t_build * 1e3, "eager_ms": t_eager * 1e3, "graph_replay_ms": t_graph * 1e3,
        "pairs_per_s_graph": pairs / t_graph, "bruteforce_ms": t_bf * 1e3, "bruteforce_pairs_per_s": pairs / t_bf,
        "speedup_vs_bruteforce": t_bf / t_graph, "max_rel_err_vs_bruteforce": worst,
        "node_pairs": b.stats["node_pairs"], "base_point_pairs": b.stats["base_point_pairs"],
    }


def grad_bench(args, torch, dfgt, synth):
    """Backward on the 16-D workload; returns (ms, details)."""
    hj = json.load(open(os.path.join(ROOT, "tests", "golden", "hstar.json")))
    x5 = synth.c5()
    n5, d5 = x5.shape
    hs5 = [synth.silverman_h(x5), hj["c5_sub5k"]["h_star"]]
    eps5 = 1e-4
    xd = torch.as_tensor(x5, device="cuda")
    R = dfgt.build_tree(xd, leaf_size=args.grad_leaf)
    dG = torch.full((len(hs5), n5), 1.0 / n5, dtype=torch.float64, device="cuda")

    def one():
        cv, dcv = dfgt.lscv_score(R, hs5, eps5, variant=1, grad=True)
        dh, dq = dfgt.gauss_sum_backward(R, R, hs5, eps5, dG)
        return cv, dcv, dq

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.grad_steps):
        cv, dcv, dq = one()
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / args.grad_steps
    # where the time goes: one profiled gradient-mode call over the four LSCV sums
    hh = hs5 + [np.sqrt(2.0) * h for h in hs5]
    _, _, _, st = dfgt.gauss_sum_grad(R, R, hh, eps5, dq=False, stats=True, profile=True)
    em_ms = st["kernel_ms"]["etile"]
    pairs = st["base_point_pairs"]
    # matrix-core roofline of the exhaustive tiles in gradient mode: per pair
    # 2 D flops for q.r plus 2 D for the kernel-weighted reference sums
    flops = pairs * 4.0 * d5
    peak = 78.6e12
    det = {
        "workload": f"16-D clustered, {n5} points (Q = R), bandwidths h_S, h* (+ sqrt2 h for LSCV), eps {eps5}",
        "h": hs5, "leaf_size": args.grad_leaf, "steps": args.grad_steps,
        "cv": [float(v) for v in cv], "dcv_dh": [float(v) for v in dcv],
        "lscv_grad_call": {"kernel_ms": st["kernel_ms"], "base_point_pairs": pairs, "node_pairs": st["node_pairs"]},
        "roofline_emfma": {"bound": "mfma", "achieved": flops / (em_ms * 1e-3) / 1e12 if em_ms > 0 else None,
                           "peak": peak / 1e12, "unit": "TFLOP/s",
                           "frac": flops / (em_ms * 1e-3) / peak if em_ms > 0 else None,
                           "flops_per_pair": 4 * d5, "dtype": "f64"},
    }
    return t_grad * 1e3, det


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the 16-D backward timing")
    ap.add_argument("--no-batched", action="store_true", help="skip the 3-D batched sweep")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a kernel of known traffic that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    ap.add_argument("--grad-steps", type=int, default=3)
    ap.add_argument("--grad-leaf", type=int, default=128)
    ap.add_argument("--leaf", type=int, default=0,
                    help="leaf size of the 2-D and batched workloads; 0 = dfgt_tune_leaf_size picks it (untimed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1102_2878_amd import dfgt, synth

    hstar = json.load(open(os.path.join(ROOT, "tests", "golden", "hstar.json")))["c2"]["h_star"]
    hs = [hstar * s for s in SCALES]
    x_host = synth.c2()
    n, d = x_host.shape
    x = torch.as_tensor(x_host, device="cuda")
    torch.cuda.synchronize()
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the leaf size: tuned on this workload before anything is timed
    leaf = args.leaf
    leaf_tuning = None
    if leaf == 0:
        leaf, tms = dfgt.tune_leaf_size(x, hs, EPS, reps=3)
        leaf_tuning = {"on": "this workload (build + the 7-bandwidth sums), 3 repetitions",
                       "candidates_ms": {str(k): v for k, v in tms.items()}}

    def step(profile):
        t = dfgt.build_tree(x, leaf_size=leaf)
        if not profile:
            return dfgt.gauss_sum(t, t, hs, EPS), None
        return dfgt.gauss_sum(t, t, hs, EPS, stats=True, profile=True)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    # timed region: K steps exactly as a caller runs them (no events, no stats)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G, _ = step(False)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps

    # the same steps with HIP events around every launch, for the per-kernel breakdown
    agg_ms = {}
    agg_launch = {}
    base_pairs = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = step(True)
        for k, v in st["kernel_ms"].items():
            agg_ms[k] = agg_ms.get(k, 0.0) + v
            agg_launch[k] = agg_launch.get(k, 0) + st["kernel_launches"][k]
        base_pairs += st["base_point_pairs"]
    torch.cuda.synchronize()
    t_step_prof = (time.perf_counter() - t0) / args.steps
    stats = st

    # base-case tiles: one call with every leaf pair exhaustive at h*, at the
    # tuned leaf size and at leaf 32 (one block per query leaf: 1,563 leaves
    # give every CU work, where the 391 leaves of leaf 128 leave it partly idle)
    base_cases = {}
    for bl in sorted({leaf, 32}):
        tree_x = dfgt.build_tree(x, leaf_size=bl)
        for _ in range(2):
            _, st_x = dfgt.gauss_sum(tree_x, tree_x, [hstar], EPS, force_method=dfgt.FORCE_EXACT, stats=True,
                                     profile=True)
        base_cases[bl] = {"pairs": st_x["base_point_pairs"], "k_etile_ms": st_x["kernel_ms"]["etile"]}
        del tree_x

    # per-bandwidth comparison (the layout of the paper's Table 1 on the
    # synthetic stand-in): DFGT, the DFD ablation (centroid finite-difference
    # prune only, p_max = 1 rule of the same code) and the brute force, one
    # bandwidth per call, tree built once
    per_h = per_bandwidth(torch, dfgt, x, hs, leaf)

    # build alone
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dfgt.build_tree(x, leaf_size=leaf)
    torch.cuda.synchronize()
    t_build = (time.perf_counter() - t0) / args.steps

    # brute-force comparator, same inputs and bandwidths
    for _ in range(max(1, args.warmup)):
        dfgt.naive_sum(x, x, hs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Gb = dfgt.naive_sum(x, x, hs)
    torch.cuda.synchronize()
    t_bf = (time.perf_counter() - t0) / args.steps

    pairs = float(n) * n * len(hs)
    value = pairs / t_step

    # roofline of the exhaustive tiles (DFGTBase) in the timed step, from the
    # HIP events around their launches on the stream they run on
    et_ms = agg_ms.get("etile", 0.0)
    et_launches = max(agg_launch.get("etile", 0), 1)
    dominant = max(agg_ms, key=agg_ms.get) if agg_ms else None
    pair_rate = (base_pairs / (et_ms * 1e-3)) if et_ms > 0 else 0.0
    peak = base_peak_pairs(d)
    fpp = flops_per_pair(d)
    roofline = {
        "kernel": "k_etile (DFGTBase exhaustive leaf-leaf tiles, mixed precision; on a side stream beside the "
                  "local-moment kernels, timed as it runs there)",
        "bound": "alu",
        "achieved": pair_rate * fpp / 1e12,
        "peak": peak * fpp / 1e12,
        "unit": "TFLOP/s",
        "frac": pair_rate / peak,
        "traffic": K_ETILE_TRAFFIC_BYTES.get(leaf),
        "traffic_unit": "HBM bytes per launch (read + written)",
        "flops_per_pair": fpp,
        "pairs_per_s": pair_rate,
        "peak_pairs_per_s": peak,
        "avg_launch_ms": et_ms / et_launches,
        "pairs_per_launch": base_pairs / et_launches,
        "dominant_kernel_in_step": dominant,
        "dominant_kernel_note": "k_traverse is latency-bound (one wave per segment, one launch per tree level): "
                                "it has no throughput roofline; see traversal.node_pairs_per_s",
    }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-exp/f64-sum",
        "data": "synthetic",
        "config": {
            "workload": "2-D clustered mixture, 50,000 points (Q = R), 7 bandwidths h* x 10^-3..10^3, eps 1e-2",
            "n": n, "d": d, "n_bandwidths": len(hs), "eps": EPS, "h_star": hstar, "leaf_size": leaf,
            "leaf_tuning": leaf_tuning,
            "p_max": 6,
        },
        "bruteforce_gpu": {"value": pairs / t_bf, "unit": "pairs/s", "ms_per_sweep": t_bf * 1e3},
        "speedup_vs_bruteforce": t_bf / t_step,
        "phases_ms": {"build_tree": t_build * 1e3, "step_with_events_and_stats": t_step_prof * 1e3,
                      **{f"kernel_{k}": v / args.steps for k, v in agg_ms.items() if not k.startswith("unused")}},
        "traversal": {**{k: stats[k] for k in ("node_pairs", "prune_f", "prune_d", "prune_t", "prune_centroid",
                                               "base_leaf_pairs", "base_point_pairs", "levels", "max_order",
                                               "segments", "max_segment", "local_nodes", "max_local_ops")},
                      "node_pairs_per_s": stats["node_pairs"] / (agg_ms.get("traverse", 0.0) / args.steps * 1e-3)
                      if agg_ms.get("traverse", 0.0) > 0 else None,
                      "us_per_level": agg_ms.get("traverse", 0.0) / args.steps / max(stats["levels"], 1) * 1e3},
        "roofline": roofline,
        "base_case_tiles": {
            "what": "one call with every leaf pair exhaustive (forced), bandwidth h*: the exhaustive-tile kernel "
                    "(one block per query leaf), at the tuned leaf size and at leaf 32",
            **{f"leaf_{bl}": {
                "pairs": bc["pairs"], "k_etile_ms": bc["k_etile_ms"],
                "pairs_per_s": bc["pairs"] / (bc["k_etile_ms"] * 1e-3),
                "tflops": bc["pairs"] / (bc["k_etile_ms"] * 1e-3) * fpp / 1e12,
                "frac_of_alu_peak": bc["pairs"] / (bc["k_etile_ms"] * 1e-3) / base_peak_pairs(d),
            } for bl, bc in base_cases.items()},
        },
        "per_bandwidth": per_h,
        "grad_ms": None,
    }

    if not args.no_batched:
        out["batched"] = batched_bench(torch, dfgt, synth, args.leaf)
    if not args.no_grad:
        out["grad_ms"], out["grad"] = grad_bench(args, torch, dfgt, synth)

    if not args.no_cpu_baseline:
        import oracle

        # rate estimate: one untimed call starts the oracle's threads, then a small sample over
        # every bandwidth (the cost per pair depends on h)
        oracle.naive_kde_rows(x_host, synth.subsample(x_host, 64, 98), x_host, hs[3])
        rng_rows = synth.subsample(x_host, 256, 99)
        t0 = time.perf_counter()
        for h in hs:
            oracle.naive_kde_rows(x_host, rng_rows, x_host, h)
        rate = len(rng_rows) * n * len(hs) / max(time.perf_counter() - t0, 1e-6)
        m = int(min(n, max(64, args.cpu_seconds * rate / (n * len(hs)))))
        rows = synth.subsample(x_host, m, 100)
        t0 = time.perf_counter()
        ref = np.stack([oracle.naive_kde_rows(x_host, rows, x_host, h) for h in hs])
        t_cpu = time.perf_counter() - t0
        Gs = G.cpu().numpy()[:, rows]
        Gbs = Gb.cpu().numpy()[:, rows]
        out["cpu_baseline"] = {
            "value": m * n * len(hs) / t_cpu, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{m} query rows x {n} references x {len(hs)} bandwidths (seeded subsample), {t_cpu:.1f} s",
        }
        out["max_rel_err_sampled"] = {"dfgt": float(np.max(np.abs(Gs - ref) / ref)),
                                      "bruteforce_gpu": float(np.max(np.abs(Gbs - ref) / ref)),
                                      "rows": m}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
