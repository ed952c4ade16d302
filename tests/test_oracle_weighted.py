"""Pins for the oracle's weighted sums G_w(q) = sum_j w_j K(q, r_j) (the sums of
Section 1 with a weight per reference point) and their derivatives: a closed
form, duplicated points, dropped points, linearity and central differences."""
import math

import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth


def test_single_point_closed_form():
    # |q - r| = 5 and 2 h^2 = 25: K = e^-1, so G_w = 2 / e; dG/dh = w K |q-r|^2 / h^3,
    # dG/dq = -w K (q - r) / h^2 at h^2 = 12.5
    q = np.array([[0.0, 0.0]])
    r = np.array([[3.0, 4.0]])
    h = math.sqrt(12.5)
    G, gh, gq = oracle.naive_kde_weighted(q, r, [2.0], h)
    assert G[0] == pytest.approx(2.0 / math.e, rel=1e-15)
    assert gh[0] == pytest.approx(2.0 / math.e * 25.0 / h**3, rel=1e-14)
    assert gq[0] == pytest.approx([2.0 / math.e * 3.0 / 12.5, 2.0 / math.e * 4.0 / 12.5], rel=1e-14)


def test_integer_weights_are_duplicated_points():
    x = synth.c1(n=200, seed=3)
    q = synth.c1(n=50, seed=4)
    rng = np.random.default_rng(5)
    k = rng.integers(0, 4, size=x.shape[0])
    k[0] = 1
    dup = np.repeat(x, k, axis=0)
    for h in (0.02, 0.1, 0.5):
        G, gh, gq = oracle.naive_kde_weighted(q, x, k.astype(float), h)
        G0, gh0, gq0 = oracle.naive_kde_grad(q, dup, h)
        np.testing.assert_allclose(G, oracle.naive_kde(q, dup, h), rtol=1e-13)
        np.testing.assert_allclose(gh, gh0, rtol=1e-12)
        np.testing.assert_allclose(gq, gq0, rtol=1e-10, atol=1e-12 * np.abs(gq0).max())


def test_unit_weights_are_the_plain_sum_and_zero_weights_drop_points():
    x = synth.c1(n=300, seed=6)
    q = x[:40]
    for h in (0.01, 0.2):
        G, _, _ = oracle.naive_kde_weighted(q, x, np.ones(len(x)), h)
        np.testing.assert_allclose(G, oracle.naive_kde(q, x, h), rtol=1e-14)
        w = np.ones(len(x))
        w[::3] = 0.0
        Gz, _, _ = oracle.naive_kde_weighted(q, x, w, h)
        np.testing.assert_allclose(Gz, oracle.naive_kde(q, x[w > 0], h), rtol=1e-13)


def test_linear_in_the_weights():
    x = synth.c1(n=250, seed=7)
    q = synth.c1(n=30, seed=8)
    rng = np.random.default_rng(9)
    w1, w2 = rng.random(len(x)), rng.exponential(size=len(x))
    a, b = 0.7, 3.25
    for h in (0.03, 0.3):
        G1, h1, q1 = oracle.naive_kde_weighted(q, x, w1, h)
        G2, h2, q2 = oracle.naive_kde_weighted(q, x, w2, h)
        G, gh, gq = oracle.naive_kde_weighted(q, x, a * w1 + b * w2, h)
        np.testing.assert_allclose(G, a * G1 + b * G2, rtol=1e-13)
        np.testing.assert_allclose(gh, a * h1 + b * h2, rtol=1e-12)
        np.testing.assert_allclose(gq, a * q1 + b * q2, rtol=1e-9, atol=1e-12 * np.abs(gq).max())


def test_derivatives_vs_central_differences():
    rng = np.random.default_rng(10)
    x = rng.normal(size=(120, 3))
    w = rng.exponential(size=120)
    q = rng.normal(size=(5, 3))
    h = 0.6
    _, gh, gq = oracle.naive_kde_weighted(q, x, w, h)
    dh = 1e-6
    fd = (oracle.naive_kde_weighted(q, x, w, h + dh)[0] - oracle.naive_kde_weighted(q, x, w, h - dh)[0]) / (2 * dh)
    np.testing.assert_allclose(gh, fd, rtol=1e-7)
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1e-6
        fq = (oracle.naive_kde_weighted(q + e, x, w, h)[0] - oracle.naive_kde_weighted(q - e, x, w, h)[0]) / 2e-6
        np.testing.assert_allclose(gq[:, c], fq, rtol=1e-6, atol=1e-9)
