"""Benchmark of the MI355X dual-tree fast Gauss transform on one GPU.

Headline workload (the batched configuration): eight 3-D clustered problems
of 10k, 20k, 40k, 60k, 80k, 120k, 160k and 200k points (Q = R each), every
problem swept over 64 log-spaced bandwidths h_S x 10^{-3..3} at h and sqrt(2) h
(the pair the least-squares cross-validation score needs): 1,024 Gaussian
sums with relative error eps = 1e-2 on every query, in one traversal, captured
once as a HIP graph (dfgt_batch_create) and replayed.

One step = one replay of that graph over inputs resident in HBM (the trees,
built once beforehand, are timed separately as build_ms).
value = sum_k N_k^2 x 128 / (seconds per step)  [query x reference pairs / s].
The leaf size is picked before anything is timed, by timing the eager
batched call at each candidate leaf size (--leaf N fixes it instead).  The same 1,024 sums as one
eager dfgt_gauss_sum_batched call, and the plain tiled brute-force GPU sum
(dfgt_naive_sum) over them, are timed alongside.

Secondary workloads in the same line:
  c2    2-D, 50,000 points, 7 bandwidths h* x 10^{-3..3}: tree build + sums
        per step, the brute force, single-bandwidth calls (DFGT, the DFD
        ablation, brute force) and every leaf pair forced exhaustive;
  c3    5-D, 100,000 points, the same 7 scales of its h*, expansion orders 6
        and 2 per dimension at eps 1e-2 and 1e-4 (leaf size tuned per order),
        beside the brute force;
  grad  16-D, 200,000 points, eps 1e-4: dfgt_lscv_score with dCV/dh plus the
        dG/dq backward (grad_ms).
Every workload's error is checked against the oracle's exact sums on seeded
query rows; the CPU baseline is the oracle itself timed on the host's cores.

Prints ONE JSON line.  --gpus must be 1: the benchmark runs on one GPU.
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

# Roofline of the exhaustive leaf-leaf tiles (DFGTBase), the dominant kernel:
# the algorithmic work per point pair is 3D + 2 flops (D differences, D
# squares, D - 1 additions, the exponential, the weighted accumulation as a
# multiply-add), priced against MI355X's published FP32 vector peak.
FP32_PEAK = 157.3e12
CUS, CLOCK = 256, 2.4e9
# Issue-slot model of the same work, from a throughput probe on the MI355X
# (lane-operations per CU-clock: FP32 FMA 98.6, v_exp_f32 27.9, measured
# serially, not co-issued): on the vector ALUs a pair takes 2D + 1 FP32 VALU
# slots and one exp; in the matrix-core tiles (squared distances from MFMA)
# one FMA and one exp.
FMA_RATE, EXP_RATE = 98.6, 27.9
LEAF_CANDIDATES = (64, 128, 256)


def flops_per_pair(d):
    return 3 * d + 2


def slot_peak_pairs(d):
    return CUS * CLOCK / ((2 * d + 1) / FMA_RATE + 1.0 / EXP_RATE)


def slot_peak_pairs_mx():
    # matrix-core tiles: the vector ALU issues one exp2 and one FMA per pair
    return CUS * CLOCK / (1.0 / FMA_RATE + 1.0 / EXP_RATE)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_etile_mx32_3d_batch_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1102_2878_amd", "csrc", "dfgt.hip")


def recorded_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, when the kernel source is still the one
    the counters were taken on (else None)."""
    import hashlib
    try:
        txt = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None, "no rocprofv3 traffic summary"
    rec = {ln.split(":", 1)[0].strip(): ln.split(":", 1)[1].strip() for ln in txt.splitlines() if ":" in ln}
    if rec.get("dfgt.hip sha256 at measurement") != src:
        return None, "the kernel source changed since the FETCH_SIZE / WRITE_SIZE counters were taken"
    return float(rec["traffic_bytes_per_launch"]), ("rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by a "
                                                    "256 MiB copy: profiles/k_etile_mx32_3d_batch_hbm_traffic.md")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def median_ms(torch, f, reps=3):
    f()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        f()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[reps // 2] * 1e3


def rel_err(G, ref):
    return float(np.max(np.abs(G - ref) / ref))


# ------------------------------------------------------------------ 3-D batch (headline)
def batched_setup(torch, dfgt, synth, leaf):
    xs = [synth.c4_problem(k) for k in range(8)]
    xd = [torch.as_tensor(x, device="cuda") for x in xs]
    torch.cuda.synchronize()
    tuning = None

    def problems(lf):
        trees = [dfgt.build_tree(x, leaf_size=lf) for x in xd]
        out = []
        for x, t in zip(xs, trees):
            base = synth.silverman_h(x) * np.geomspace(1e-3, 1e3, 64)
            out.append((t, t, np.concatenate([base, np.sqrt(2.0) * base])))
        return out

    if leaf == 0:
        # the workload itself decides: the eager batched call per candidate
        # (median of 3 after a warm-up call), the smallest leaf within 2% of
        # the fastest
        tms = {}
        for lf in LEAF_CANDIDATES:
            pr = problems(lf)
            tms[lf] = median_ms(torch, lambda: dfgt.gauss_sum_batched(pr, EPS), reps=3)
            del pr
        best = min(tms.values())
        leaf = min(lf for lf, v in tms.items() if v <= 1.02 * best)
        tuning = {"on": "this workload (the eager batched call, median of 3 after a warm-up)",
                  "candidates_ms": {str(k): v for k, v in tms.items()}}
    dfgt.build_tree(xd[0], leaf_size=leaf)  # warm the build path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trees = [dfgt.build_tree(x, leaf_size=leaf) for x in xd]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    probs = []
    for x, t in zip(xs, trees):
        base = synth.silverman_h(x) * np.geomspace(1e-3, 1e3, 64)
        probs.append((t, t, np.concatenate([base, np.sqrt(2.0) * base])))
    return xs, xd, trees, probs, leaf, tuning, t_build


def batched_extras(torch, dfgt, xd, probs, b):
    """Eager call, per-kernel event times of one eager call, brute force."""
    t_eager = median_ms(torch, lambda: dfgt.gauss_sum_batched(probs, EPS))
    _, st = dfgt.gauss_sum_batched(probs, EPS, stats=True, profile=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for x, (t, _, h), G in zip(xd, probs, b.G):
        Gb = dfgt.naive_sum(x, x, h)
        worst = max(worst, float(((G - Gb).abs() / Gb).max()))
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t0
    return t_eager, st, t_bf, worst


# ------------------------------------------------------------------ 2-D sweep
def c2_bench(torch, dfgt, synth, args):
    hstar = json.load(open(os.path.join(ROOT, "tests", "golden", "hstar.json")))["c2"]["h_star"]
    hs = [hstar * s for s in SCALES]
    xh = synth.c2()
    n = xh.shape[0]
    x = torch.as_tensor(xh, device="cuda")
    leaf, tuning = args.leaf, None
    if leaf == 0:
        leaf, tms = dfgt.tune_leaf_size(x, hs, EPS, reps=3)
        tuning = {"on": "this workload (build + the 7-bandwidth sums), 3 repetitions",
                  "candidates_ms": {str(k): v for k, v in tms.items()}}

    def step():
        t = dfgt.build_tree(x, leaf_size=leaf)
        return dfgt.gauss_sum(t, t, hs, EPS)

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G = step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    R = dfgt.build_tree(x, leaf_size=leaf)
    _, st = dfgt.gauss_sum(R, R, hs, EPS, stats=True, profile=True)
    _, st = dfgt.gauss_sum(R, R, hs, EPS, stats=True, profile=True)
    t_build = median_ms(torch, lambda: dfgt.build_tree(x, leaf_size=leaf), reps=5)
    t_bf = median_ms(torch, lambda: dfgt.naive_sum(x, x, hs), reps=3)
    forced = {}
    for bl in sorted({leaf, 32}):
        tx = dfgt.build_tree(x, leaf_size=bl)
        for scale in (1.0, 10.0):
            for _ in range(2):
                _, sx = dfgt.gauss_sum(tx, tx, [hstar * scale], EPS, force_method=dfgt.FORCE_EXACT, profile=True)
            rate = sx["base_point_pairs"] / (sx["kernel_ms"]["etile"] * 1e-3)
            forced[f"leaf_{bl}_h{scale:g}hstar"] = {
                "pairs": sx["base_point_pairs"], "k_etile_ms": sx["kernel_ms"]["etile"], "pairs_per_s": rate,
                "frac_fp32_peak": rate * flops_per_pair(2) / FP32_PEAK, "frac_issue_slots": rate / slot_peak_pairs(2)}
    rows = []
    for s, h in zip(SCALES, hs):
        rows.append({"h_over_hstar": s,
                     "dfgt_ms": median_ms(torch, lambda: dfgt.gauss_sum(R, R, [h], EPS)),
                     "dfd_ms": median_ms(torch, lambda: dfgt.gauss_sum(R, R, [h], EPS,
                                                                      force_method=dfgt.FORCE_CENTROID)),
                     "bruteforce_ms": median_ms(torch, lambda: dfgt.naive_sum(x, x, [h]))})
    pairs = float(n) * n * len(hs)
    out = {
        "workload": "2-D clustered mixture, 50,000 points (Q = R), 7 bandwidths h* x 10^-3..10^3, eps 1e-2; "
                    "step = tree build + sums",
        "h_star": hstar, "leaf_size": leaf, "leaf_tuning": tuning, "p_max": 6,
        "ms_per_step": t_step * 1e3, "pairs_per_s": pairs / t_step,
        "bruteforce_ms": t_bf, "bruteforce_pairs_per_s": pairs / (t_bf * 1e-3),
        "speedup_vs_bruteforce": t_bf / (t_step * 1e3),
        "build_ms": t_build, "kernel_ms": st["kernel_ms"], "kernel_launches": st["kernel_launches"],
        "traversal": {k: st[k] for k in ("node_pairs", "prune_f", "prune_d", "prune_t", "prune_centroid",
                                         "base_leaf_pairs", "base_point_pairs", "levels", "segments")},
        "exhaustive_tile_rate": {
            "pairs_per_s": st["base_point_pairs"] / (st["kernel_ms"]["etile"] * 1e-3),
            "frac_fp32_peak": st["base_point_pairs"] / (st["kernel_ms"]["etile"] * 1e-3) * flops_per_pair(2)
            / FP32_PEAK},
        "forced_exhaustive": forced,
        "per_bandwidth": {"what": "single-bandwidth calls, tree built once: DFGT, the DFD ablation (only the "
                                  "centroid finite-difference prune), brute force", "rows": rows},
    }
    return xh, hs, G, out


# ------------------------------------------------------------------ 5-D workload
def c3_bench(torch, dfgt, synth, oracle):
    hstar = json.load(open(os.path.join(ROOT, "tests", "golden", "hstar.json")))["c3"]["h_star"]
    hs = [hstar * s for s in SCALES]
    xh = synth.c3()
    x = torch.as_tensor(xh, device="cuda")
    rows = synth.subsample(xh, 300, 45)
    ref = np.stack([oracle.naive_kde_rows(xh, rows, xh, h) for h in hs])
    t_bf = median_ms(torch, lambda: dfgt.naive_sum(x, x, hs), reps=3)
    out = {"workload": "5-D correlated mixture + 5% Student-t outliers, 100,000 points (Q = R), 7 bandwidths "
                       "h* x 10^-3..10^3", "h_star": hstar, "bruteforce_ms": t_bf, "rows": []}
    for pmax in (6, 2):
        for eps in (1e-2, 1e-4):
            leaf, _ = dfgt.tune_leaf_size(x, hs, eps, reps=1, p_max=pmax)
            R = dfgt.build_tree(x, p_max=pmax, leaf_size=leaf)
            ms = median_ms(torch, lambda: dfgt.gauss_sum(R, R, hs, eps))
            G, st = dfgt.gauss_sum(R, R, hs, eps, stats=True)
            err = rel_err(G.cpu().numpy()[:, rows], ref)
            out["rows"].append({"p_max": pmax, "eps": eps, "leaf_size": leaf, "ms": ms,
                                "speedup_vs_bruteforce": t_bf / ms,
                                "max_rel_err_oracle": err, "oracle_rows": len(rows),
                                "base_point_pairs": st["base_point_pairs"], "max_order": st["max_order"]})
    return out


# ------------------------------------------------------------------ 16-D gradients
def grad_bench(args, torch, dfgt, synth, oracle):
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
    hh = hs5 + [np.sqrt(2.0) * h for h in hs5]
    _, _, _, st = dfgt.gauss_sum_grad(R, R, hh, eps5, dq=False, stats=True, profile=True)
    em_ms = st["kernel_ms"]["etile"]
    pairs = st["base_point_pairs"]
    flops = pairs * 4.0 * d5  # q.r and the kernel-weighted reference sums, 2 D each
    # oracle check of G, dG/dh and dG/dq on seeded query rows against all 200,000 references
    G, Gh, Gq = dfgt.gauss_sum_grad(R, R, hs5, eps5)
    rows = synth.subsample(x5, 200, 56)
    idx = torch.as_tensor(rows, device="cuda")
    G, Gh, Gq = G[:, idx].cpu().numpy(), Gh[:, idx].cpu().numpy(), Gq[:, idx].cpu().numpy()
    errs = {"G": 0.0, "dGdh": 0.0, "dGdq": 0.0}
    for k, h in enumerate(hs5):
        g, gh, gq = oracle.naive_kde_grad(x5[rows], x5, h)
        qs = oracle.naive_kde_qscale(x5[rows], x5, h)
        errs["G"] = max(errs["G"], rel_err(G[k], g))
        errs["dGdh"] = max(errs["dGdh"], float(np.max(np.abs(Gh[k] - gh) / gh)))
        errs["dGdq"] = max(errs["dGdq"], float(np.max(np.linalg.norm(Gq[k] - gq, axis=1) / qs)))
    det = {
        "workload": f"16-D clustered, {n5} points (Q = R), bandwidths h_S, h* (+ sqrt2 h for LSCV), eps {eps5}",
        "h": hs5, "leaf_size": args.grad_leaf, "steps": args.grad_steps,
        "cv": [float(v) for v in cv], "dcv_dh": [float(v) for v in dcv],
        "lscv_grad_call": {"kernel_ms": st["kernel_ms"], "base_point_pairs": pairs, "node_pairs": st["node_pairs"]},
        "max_rel_err_oracle": {**errs, "rows": len(rows), "units": "G and dG/dh relative to themselves, dG/dq "
                               "relative to h^-2 sum_j K_j |q - r_j|"},
        "roofline_emfma": {"bound": "mfma", "achieved": flops / (em_ms * 1e-3) / 1e12 if em_ms > 0 else None,
                           "peak": 78.6, "unit": "TFLOP/s",
                           "frac": flops / (em_ms * 1e-3) / 78.6e12 if em_ms > 0 else None,
                           "flops_per_pair": 4 * d5, "dtype": "f64"},
    }
    return t_grad * 1e3, det


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=200, help="oracle query rows per problem for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="only the headline (3-D batch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a kernel of known traffic that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    ap.add_argument("--grad-steps", type=int, default=3)
    ap.add_argument("--grad-leaf", type=int, default=128)
    ap.add_argument("--leaf", type=int, default=0,
                    help="leaf size of the 3-D and 2-D workloads; 0 = dfgt_tune_leaf_size picks it (untimed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1102_2878_amd import dfgt, synth

    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline: the captured 3-D batch
    xs, xd, trees, probs, leaf, tuning, t_build = batched_setup(torch, dfgt, synth, args.leaf)
    b = dfgt.Batch(probs, EPS, stats=True)
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    b.check()
    pairs = float(sum(x.shape[0] ** 2 for x in xs)) * 128
    value = pairs / t_step
    t_eager, st, t_bf, worst_bf = batched_extras(torch, dfgt, xd, probs, b)

    # roofline of the dominant kernel, the matrix-core exhaustive tiles with
    # FP32 products (k_etile_mx32_1): the HIP events around its launch on the
    # stream it runs on (a side stream, beside the local-moment and per-leaf
    # kernels) in one eager call of the same jobs, over the pairs it computed
    km, kl = st["kernel_ms"], st["kernel_launches"]
    et_ms, et_n = km["etile_mx32"], max(kl["etile_mx32"], 1)
    traffic, traffic_note = recorded_traffic()
    ep = st["e_pairs"]["fp32"]
    rate = ep / (et_ms * 1e-3)
    roofline = {
        "kernel": "k_etile_mx32_1 (DFGTBase exhaustive leaf-leaf tiles, D = 3: squared distances from "
                  "v_mfma_f32_16x16x4f32, exp2 and the weighted sums on the vector ALUs)",
        "bound": "alu",
        "achieved": rate * flops_per_pair(3) / 1e12,
        "peak": FP32_PEAK / 1e12,
        "unit": "TFLOP/s",
        "frac": rate * flops_per_pair(3) / FP32_PEAK,
        "traffic": traffic,
        "traffic_note": traffic_note,
        "flops_per_pair": flops_per_pair(3),
        "pairs_per_launch": ep / et_n,
        "avg_launch_ms": et_ms / et_n,
        "pairs_per_s": rate,
        "issue_slot_frac": rate / slot_peak_pairs_mx(),
        "issue_slot_peak_pairs_per_s": slot_peak_pairs_mx(),
        "issue_slot_model": "per pair one v_exp_f32 and one FMA on the vector ALU, the matrix cores overlapped",
        "pairs_fp64_products": st["e_pairs"]["fp64"],
        "kernel_ms_of_one_eager_call": km,
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
            "workload": "3-D batch: 8 clustered problems N = 10k..200k (sum 690k, Q = R), 64 log-spaced "
                        "bandwidths h_S x 10^-3..10^3 at h and sqrt2 h (1,024 sums), eps 1e-2, one captured "
                        "graph replayed per step",
            "problems": [int(x.shape[0]) for x in xs], "d": 3, "sums": 1024, "eps": EPS, "leaf_size": leaf,
            "leaf_tuning": tuning, "p_max": 4, "parts": b.stats["parts"],
        },
        "build_ms": t_build * 1e3,
        "eager_ms": t_eager,
        "bruteforce_gpu": {"value": pairs / t_bf, "unit": "pairs/s", "ms": t_bf * 1e3},
        "speedup_vs_bruteforce": t_bf / t_step,
        "max_rel_err_vs_bruteforce": worst_bf,
        "traversal": {k: st[k] for k in ("node_pairs", "prune_f", "prune_d", "prune_t", "prune_centroid",
                                         "base_leaf_pairs", "base_point_pairs", "levels", "segments")},
        "roofline": roofline,
        "grad_ms": None,
    }

    import oracle

    if not args.no_cpu_baseline:
        # the oracle on the host cores over seeded query rows of every problem, each row against all its
        # references at all 128 bandwidths; the same rows check the replay's sums
        oracle.naive_kde_rows(xs[0], synth.subsample(xs[0], 16, 97), xs[0], 0.01)
        t0 = time.perf_counter()
        worst, npairs = 0.0, 0.0
        for k, (x, (t, _, h), G) in enumerate(zip(xs, probs, b.G)):
            rows = synth.subsample(x, args.cpu_rows, 90 + k)
            ref = np.stack([oracle.naive_kde_rows(x, rows, x, hk) for hk in h])
            Gs = G[:, torch.as_tensor(rows, device=G.device)].cpu().numpy()
            worst = max(worst, rel_err(Gs, ref))
            npairs += len(rows) * x.shape[0] * len(h)
        t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": npairs / t_cpu, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{args.cpu_rows} seeded query rows per problem x all its references x all 128 bandwidths "
                      f"(8 problems), {t_cpu:.1f} s",
        }
        out["max_rel_err_oracle"] = {"value": worst, "rows_per_problem": args.cpu_rows, "bandwidths": 128}

    if not args.no_secondary:
        xh2, hs2, G2, c2 = c2_bench(torch, dfgt, synth, args)
        rows2 = synth.subsample(xh2, 400, 28)
        ref2 = np.stack([oracle.naive_kde_rows(xh2, rows2, xh2, h) for h in hs2])
        c2["max_rel_err_oracle"] = {"value": rel_err(G2.cpu().numpy()[:, rows2], ref2), "rows": len(rows2)}
        out["c2"] = c2
        out["c3"] = c3_bench(torch, dfgt, synth, oracle)
        out["grad_ms"], out["grad"] = grad_bench(args, torch, dfgt, synth, oracle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
