"""Pins for the oracle's exact kernel sums (Section 1.1, eq. gaussian_kernel_sums;
Alg. NaiveKDE) and their derivatives.  Every check compares against something
computed independently of the oracle: arbitrary-precision mpmath sums, numpy /
scipy library routines, closed forms or finite differences."""
import mpmath as mp
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from paper_1102_2878_amd import synth


def _mp_sum(q, r, h):
    mp.mp.dps = 40
    out = []
    for qi in q:
        s = mp.mpf(0)
        for rj in r:
            d2 = sum((mp.mpf(float(a)) - mp.mpf(float(b))) ** 2 for a, b in zip(qi, rj))
            s += mp.e ** (-d2 / (2 * mp.mpf(float(h)) ** 2))
        out.append(float(s))
    return np.array(out)


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_tiny_brute_force_vs_mpmath(d):
    rng = np.random.default_rng(10 + d)
    q = rng.uniform(size=(7, d))
    r = rng.uniform(size=(13, d))
    for h in (0.03, 0.3, 3.0):
        got = oracle.naive_kde(q, r, h)
        ref = _mp_sum(q, r, h)
        # exp(-x) carries a relative error ~ x * u from rounding its argument
        xmax = ((q[:, None] - r[None]) ** 2).sum(-1).max() / (2 * h * h)
        np.testing.assert_allclose(got, ref, rtol=1e-14 * (2 + xmax), atol=1e-300)


def test_matches_library_distance_route():
    x = synth.c1(n=500, seed=4)
    for h in (0.01, 0.1, 1.0):
        ref = np.exp(-cdist(x, x, "sqeuclidean") / (2 * h * h)).sum(axis=1)
        np.testing.assert_allclose(oracle.naive_kde(x, x, h), ref, rtol=1e-12)


def test_coincident_points_give_count():
    x = np.tile(np.array([[0.25, -1.5, 3.0]]), (37, 1))
    np.testing.assert_array_equal(oracle.naive_kde(x, x, 1e-3), np.full(37, 37.0))


def test_huge_bandwidth_tends_to_count():
    x = synth.c1(n=300, seed=6)
    ext = np.ptp(x, axis=0).max()
    g = oracle.naive_kde(x, x, 1e6 * ext)
    assert np.all(np.abs(g / 300 - 1) < 1e-10)


def test_single_reference_point_closed_form():
    q = np.array([[0.1, 0.2], [0.4, -0.3]])
    r = np.array([[0.0, 0.5]])
    h = 0.37
    d2 = ((q - r) ** 2).sum(1)
    np.testing.assert_allclose(oracle.naive_kde(q, r, h), np.exp(-d2 / (2 * h * h)), rtol=1e-15)


def test_separated_clusters_at_tiny_bandwidth_count_duplicates():
    rng = np.random.default_rng(3)
    base = rng.uniform(size=(20, 2))
    mult = rng.integers(1, 5, size=20)
    x = np.repeat(base, mult, axis=0)
    g = oracle.naive_kde(x, x, 1e-9)
    np.testing.assert_array_equal(g, np.repeat(mult, mult).astype(float))


def test_rows_variant_equals_full():
    x = synth.c1(n=400, seed=8)
    rows = np.array([0, 5, 399, 17])
    np.testing.assert_array_equal(oracle.naive_kde_rows(x, rows, x, 0.05), oracle.naive_kde(x, x, 0.05)[rows])


def test_gradients_vs_mpmath_derivative():
    q = np.array([[0.3, 0.1]])
    r = np.array([[0.0, 0.0], [0.2, 0.5], [0.9, -0.2]])
    h = 0.4
    G, gh, gq = oracle.naive_kde_grad(q, r, h)
    mp.mp.dps = 30

    def f(hh, x0, x1):
        return sum(mp.e ** (-((x0 - a) ** 2 + (x1 - b) ** 2) / (2 * hh * hh)) for a, b in r)

    x0, x1 = mp.mpf(0.3), mp.mpf(0.1)
    assert abs(gh[0] - float(mp.diff(lambda t: f(t, x0, x1), mp.mpf(h)))) < 1e-13
    assert abs(gq[0, 0] - float(mp.diff(lambda t: f(mp.mpf(h), t, x1), x0))) < 1e-13
    assert abs(gq[0, 1] - float(mp.diff(lambda t: f(mp.mpf(h), x0, t), x1))) < 1e-13
    np.testing.assert_allclose(G, oracle.naive_kde(q, r, h), rtol=1e-15)


def test_gradients_vs_central_differences():
    x = synth.c1(n=200, seed=9)
    q = x[:20]
    h = 0.05
    _, gh, gq = oracle.naive_kde_grad(q, x, h)
    dh = 1e-5 * h
    fd = (oracle.naive_kde(q, x, h + dh) - oracle.naive_kde(q, x, h - dh)) / (2 * dh)
    np.testing.assert_allclose(gh, fd, rtol=1e-7)
    for k in range(2):
        e = np.zeros(2)
        e[k] = 1e-6
        fdq = np.array([(oracle.naive_kde(qi[None] + e, x, h) - oracle.naive_kde(qi[None] - e, x, h))[0] / 2e-6
                        for qi in q])
        np.testing.assert_allclose(gq[:, k], fdq, rtol=1e-6, atol=1e-6)


def test_coincident_points_zero_gradient():
    x = np.tile(np.array([[1.0, 2.0]]), (9, 1))
    _, gh, gq = oracle.naive_kde_grad(x, x, 0.3)
    assert np.all(gh == 0) and np.all(gq == 0)


def test_qscale_single_reference_closed_form():
    """One reference at distance rho: h^-2 e^{-rho^2/2h^2} rho."""
    q = np.array([[0.1, -0.2, 0.3]])
    r = np.array([[0.4, 0.2, 0.3]])
    h = 0.7
    rho = 0.5
    np.testing.assert_allclose(oracle.naive_kde_qscale(q, r, h), [np.exp(-rho ** 2 / (2 * h * h)) * rho / h ** 2],
                               rtol=1e-14)


def test_qscale_equals_gradient_norm_on_one_side():
    """In one dimension with every reference on one side of the query, every
    term of dG/dq has the same sign, so the sum of their norms is |dG/dq|
    (the oracle's analytic gradient, pinned by mpmath and differences)."""
    rng = np.random.default_rng(61)
    r = rng.uniform(0.0, 1.0, size=(300, 1))
    q = np.array([[-0.05], [-0.3], [1.2]])
    for h in (0.05, 0.4, 3.0):
        _, _, gq = oracle.naive_kde_grad(q, r, h)
        np.testing.assert_allclose(oracle.naive_kde_qscale(q, r, h), np.abs(gq[:, 0]), rtol=1e-13)


def test_qscale_sphere_and_inequalities():
    """References on a sphere of radius rho around q: N K(rho) rho / h^2
    exactly.  In general |dG/dq| <= qscale <= sqrt(G h^3 dG/dh) / h^2
    (triangle and Cauchy-Schwarz inequalities against the pinned gradient)."""
    rng = np.random.default_rng(62)
    q = np.array([[0.3, 0.6]])
    ang = rng.uniform(0.0, 2 * np.pi, 200)
    rho, h = 0.25, 0.2
    r = q + rho * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    np.testing.assert_allclose(oracle.naive_kde_qscale(q, r, h), [200 * np.exp(-rho ** 2 / (2 * h * h)) * rho / h ** 2],
                               rtol=1e-12)
    x = synth.c1(n=800, seed=63)
    qs = x[:50]
    for h in (0.01, 0.1, 1.0):
        G, gh, gq = oracle.naive_kde_grad(qs, x, h)
        s = oracle.naive_kde_qscale(qs, x, h)
        assert np.all(np.linalg.norm(gq, axis=1) <= s * (1 + 1e-12))
        assert np.all(s <= np.sqrt(G * gh * h ** 3) / h ** 2 * (1 + 1e-12))
