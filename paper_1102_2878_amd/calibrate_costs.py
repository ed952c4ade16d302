"""Measures the GPU's per-unit costs of the summarisation methods relative to
one exhaustive point pair, the weights of the library's ChooseBestMethod
(Section 3.8) cost model.

For each workload shape (dimension, expansion order, leaf size) it times one
call per method forced alone (dfgt_options.force_method) with HIP events and
divides each method's kernel time by its algorithmic work from dfgt_stats:
  E  exhaustive pairs                  (k_etile)
  F  sum N_Q p^D over far-field pairs  (k_leaf, less its time with no series)
  D  sum N_R p^D over direct pairs     (local-op kernels + the k_leaf increase)
  T  sum D p^2D over translation pairs (the same)
and prints w_X = (time per unit of X) / (time per exhaustive pair).
Needs the GPU; the inputs are the seeded synthetic workloads.
Usage: python -m paper_1102_2878_amd.calibrate_costs
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def measure(dfgt, torch, x, hs, leaf, pmax, eps):
    xd = torch.as_tensor(x, device="cuda")
    R = dfgt.build_tree(xd, leaf_size=leaf, p_max=pmax)

    def run(force):
        dfgt.gauss_sum(R, R, hs, eps, force_method=force, profile=True)
        _, st = dfgt.gauss_sum(R, R, hs, eps, force_method=force, profile=True)
        return st

    ex = run(dfgt.FORCE_EXACT)
    t_e = ex["kernel_ms"]["etile"] / max(ex["base_point_pairs"], 1)
    leaf_base = ex["kernel_ms"]["leaf"]
    out = {"t_E_ps": t_e * 1e9}
    for name, force, key in (("F", dfgt.FORCE_F, "work_f"), ("D", dfgt.FORCE_D, "work_d"),
                             ("T", dfgt.FORCE_T, "work_t")):
        st = run(force)
        work = st[key]
        if work <= 0:
            out["w_" + name] = None
            continue
        ms = st["kernel_ms"]["leaf"] - leaf_base
        if name != "F":
            ms += st["kernel_ms"]["local"]
        out["w_" + name] = max(ms, 0.0) / work / t_e
        out["work_" + name] = work
    return out


def main():
    import torch

    from paper_1102_2878_amd import dfgt, synth

    hj = json.load(open(os.path.join(ROOT, "tests", "golden", "hstar.json")))
    res = {}
    x2 = synth.c2()
    hs2 = [hj["c2"]["h_star"] * s for s in (1.0, 10.0, 100.0)]
    res["d2_p6_leaf128"] = measure(dfgt, torch, x2, hs2, 128, 0, 1e-2)
    x3 = synth.c4_problem(7)
    hs3 = synth.silverman_h(x3) * np.array([0.1, 0.3, 1.0])
    res["d3_p4_leaf128"] = measure(dfgt, torch, x3, hs3, 128, 0, 1e-2)
    x5 = synth.c3()
    hs5 = [hj["c3"]["h_star"] * s for s in (10.0, 100.0)]
    res["d5_p2_leaf64"] = measure(dfgt, torch, x5, hs5, 64, 2, 1e-2)
    res["d5_p6_leaf64"] = measure(dfgt, torch, x5, hs5, 64, 6, 1e-2)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
