"""Writes tests/golden/hstar.json: the least-squares cross-validation optimum h*
of each synthetic workload, computed with the oracle's exact sums only.

The paper sweeps seven bandwidths 10^-3 .. 10^3 times the LSCV optimum
(Section 4), "according to the standard least-squares cross-validation score"
of Silverman's book.  For the synthetic stand-ins h* is found here as the
minimiser of that standard score, whose integral of the squared estimate keeps
its diagonal (the oracle's LSCV variant 1; the fully leave-one-out reading of
Section 1, eq. 4 has no small-h penalty and dips spuriously once a few close
pairs dominate): a log-spaced grid over
h_S * [1e-2, 10] (h_S = Silverman's rule), then golden-section search on log h
to 1e-3 relative.

    python tests/golden/make_hstar.py c2 [c3 c5_sub5k ...]

c5_sub5k is the 16-D workload's seeded 5,000-point subsample: its h* stands
for the full set's (the LSCV sums over 200,000 points are out of the
oracle's reach).
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1102_2878_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hstar.json")


def c5_sub5k():
    """The 16-D workload's seeded 5,000-point subsample (its h* is estimated there)."""
    x = synth.c5()
    return x[synth.subsample(x, 5000, 5)]


GENERATORS = {"c1": synth.c1, "c2": synth.c2, "c3": synth.c3, "c5_sub5k": c5_sub5k}
GEN_NAMES = {"c5_sub5k": "tests/golden/make_hstar.py:c5_sub5k() = synth.c5()[synth.subsample(x, 5000, 5)]"}


def cv(x, h):
    return float(oracle.lscv(x, [h], 1)[0][0])


def hstar(x, grid=24):
    hs = synth.silverman_h(x)
    lg = np.linspace(math.log(hs * 1e-2), math.log(hs * 10.0), grid)
    vals = [cv(x, math.exp(v)) for v in lg]
    i = int(np.argmin(vals))
    a, b = lg[max(i - 1, 0)], lg[min(i + 1, grid - 1)]
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = cv(x, math.exp(c)), cv(x, math.exp(d))
    while b - a > 1e-3:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = cv(x, math.exp(c))
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = cv(x, math.exp(d))
    h = math.exp((a + b) / 2)
    return h, hs, cv(x, h)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        x = GENERATORS[nm]()
        t = time.time()
        h, hs, v = hstar(x)
        data[nm] = {"h_star": h, "h_silverman": hs, "cv_ls": v, "lscv_variant": 1, "n": int(x.shape[0]), "d": int(x.shape[1]),
                    "generator": GEN_NAMES.get(nm, f"paper_1102_2878_amd.synth.{nm}()"),
                    "seconds": round(time.time() - t, 1)}
        print(nm, data[nm], flush=True)
        json.dump(data, open(OUT, "w"), indent=2, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
