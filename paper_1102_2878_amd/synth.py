"""Seeded synthetic point sets shaped like the paper's workloads.

This module holds input generators only: it contains none of the kernel-sum
arithmetic and is imported by both the oracle-side tests and the GPU path.

The paper evaluates on clustered astronomy and pharmaceutical data (Section 4,
dataset list) that is not available here; these mixtures stand in for it:

* ``c1``: 2,000 points, D=2, four isotropic Gaussians (sigma 0.05).
* ``c2``: 50,000 points, D=2, 32 anisotropic Gaussians plus 10% uniform
  background (shaped like the 2-D astronomy sets sj2-50000-2 / colors50k).
* ``c3``: 100,000 points, D=5, 16 correlated Gaussians plus 5% Student-t(3)
  outliers (shaped like the 5-D bio5 set).
* ``c4``: eight 3-D clustered problems of uneven size (10k..200k points).
* ``c5``: 200,000 points, D=16: eight latent 3-D clusters linearly embedded
  plus isotropic noise.

All generators use ``numpy.random.Generator(PCG64(seed))``, return float64
row-major ``(N, D)`` arrays, and shuffle the rows so that user order carries no
cluster structure.
"""
from __future__ import annotations

import numpy as np

C4_SIZES = (10_000, 20_000, 40_000, 60_000, 80_000, 120_000, 160_000, 200_000)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def _counts(rng, n, k):
    return rng.multinomial(n, np.full(k, 1.0 / k))


def _haar_orthogonal(rng, d):
    a = rng.standard_normal((d, d))
    qm, rm = np.linalg.qr(a)
    return qm * np.sign(np.diag(rm))[None, :]


def c1(n: int = 2000, seed: int = 1) -> np.ndarray:
    """Four isotropic Gaussians (sigma=0.05), means uniform in the unit square."""
    rng = _rng(seed)
    means = rng.uniform(0.0, 1.0, size=(4, 2))
    parts = [m + 0.05 * rng.standard_normal((c, 2)) for m, c in zip(means, _counts(rng, n, 4))]
    x = np.concatenate(parts)
    return x[rng.permutation(n)]


def c2(n: int = 50_000, seed: int = 2) -> np.ndarray:
    """32 anisotropic Gaussians (eigenvalues log-uniform in [1e-4, 1e-2]) + 10% uniform."""
    rng = _rng(seed)
    n_bg = n // 10
    n_cl = n - n_bg
    k = 32
    means = rng.uniform(0.0, 1.0, size=(k, 2))
    theta = rng.uniform(0.0, np.pi, size=k)
    lam = _loguniform(rng, 1e-4, 1e-2, (k, 2))
    parts = []
    for j, c in enumerate(_counts(rng, n_cl, k)):
        ct, st = np.cos(theta[j]), np.sin(theta[j])
        rot = np.array([[ct, -st], [st, ct]])
        z = rng.standard_normal((c, 2)) * np.sqrt(lam[j])[None, :]
        parts.append(means[j] + z @ rot.T)
    parts.append(rng.uniform(0.0, 1.0, size=(n_bg, 2)))
    x = np.concatenate(parts)
    return x[rng.permutation(n)]


def c3(n: int = 100_000, seed: int = 3) -> np.ndarray:
    """16 correlated 5-D Gaussians + 5% heavy-tailed Student-t(3) outliers."""
    rng = _rng(seed)
    d = 5
    n_out = n // 20
    n_cl = n - n_out
    k = 16
    means = rng.uniform(0.0, 1.0, size=(k, d))
    parts = []
    for j, c in enumerate(_counts(rng, n_cl, k)):
        o = _haar_orthogonal(rng, d)
        lam = _loguniform(rng, 1e-4, 1e-2, d)
        z = rng.standard_normal((c, d)) * np.sqrt(lam)[None, :]
        parts.append(means[j] + z @ o.T)
    z = rng.standard_normal((n_out, d))
    w = rng.chisquare(3, size=n_out)
    parts.append(0.5 + 0.1 * z / np.sqrt(w / 3.0)[:, None])
    x = np.concatenate(parts)
    return x[rng.permutation(n)]


def c4_problem(k: int) -> np.ndarray:
    """k-th batched problem (k in 0..7): 3-D, 8 isotropic clusters, sigma log-uniform [0.01, 0.05]."""
    n = C4_SIZES[k]
    rng = _rng(40 + k)
    means = rng.uniform(0.0, 1.0, size=(8, 3))
    sig = _loguniform(rng, 0.01, 0.05, 8)
    parts = [means[j] + sig[j] * rng.standard_normal((c, 3)) for j, c in enumerate(_counts(rng, n, 8))]
    x = np.concatenate(parts)
    return x[rng.permutation(n)]


def c5(n: int = 200_000, seed: int = 5) -> np.ndarray:
    """8 latent 3-D clusters (sigma 0.05) embedded in 16-D by orthonormal columns, + N(0, 0.01 I)."""
    rng = _rng(seed)
    means = rng.uniform(0.0, 1.0, size=(8, 3))
    lat = np.concatenate([m + 0.05 * rng.standard_normal((c, 3)) for m, c in zip(means, _counts(rng, n, 8))])
    a, _ = np.linalg.qr(rng.standard_normal((16, 3)))
    x = lat @ a.T + np.sqrt(0.01) * rng.standard_normal((n, 16))
    return x[rng.permutation(n)]


def bichromatic_queries(x: np.ndarray, seed: int) -> np.ndarray:
    """A second draw from the same bounding region, for bichromatic tests (Q != R)."""
    rng = _rng(seed + 100)
    lo, hi = x.min(axis=0), x.max(axis=0)
    n = x.shape[0]
    take = x[rng.integers(0, n, size=n)]
    jitter = 0.02 * (hi - lo) * rng.standard_normal(x.shape)
    return take + jitter


def silverman_h(x: np.ndarray) -> float:
    """Silverman's normal-reference bandwidth with the mean per-dimension variance."""
    n, d = x.shape
    sig = np.sqrt(np.mean(np.var(x, axis=0, ddof=1)))
    return float(sig * (4.0 / ((d + 2) * n)) ** (1.0 / (d + 4)))


def subsample(x: np.ndarray, m: int, seed: int) -> np.ndarray:
    """Seeded index sample (without replacement) of m rows."""
    rng = _rng(seed + 7)
    return np.sort(rng.choice(x.shape[0], size=min(m, x.shape[0]), replace=False))


def weights(n: int, seed: int, kind: str = "exp") -> np.ndarray:
    """Seeded non-negative point weights for weighted sums.

    ``exp``: exponential(1); ``wide``: log-uniform over [1e-6, 1e3];
    ``sparse``: exponential(1) with about 30% zeros; ``int``: integers 0..3
    (at least one non-zero)."""
    rng = _rng(seed + 31)
    if kind == "exp":
        return rng.exponential(size=n)
    if kind == "wide":
        return _loguniform(rng, 1e-6, 1e3, n)
    if kind == "sparse":
        w = rng.exponential(size=n)
        w[rng.random(n) < 0.3] = 0.0
        w[0] = max(w[0], 1.0)
        return w
    if kind == "int":
        w = rng.integers(0, 4, size=n).astype(np.float64)
        w[0] = max(w[0], 1.0)
        return w
    raise ValueError(kind)
