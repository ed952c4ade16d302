"""Pins for the oracle's recursive DFGT (Section 3.9) against the paper's three
theorems (Section 3.10) and exact brute-force sums, plus the LSCV score
(Section 1, eq. 4) against closed forms and quadrature."""
import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_1102_2878_amd import synth


def _check_theorems(x, q, h, eps, **kw):
    G = oracle.naive_kde(q, x, h)
    Gt, info = oracle.dfgt(q, x, h, eps, G_exact=G, **kw)
    rel = np.abs(Gt - G) / G
    assert rel.max() <= eps * (1 + 1e-9) + 1e-13, rel.max()          # global relative error theorem
    assert np.all(info["coverage"] == x.shape[0])                      # partition theorem
    assert info["bound_violations"] == 0                               # bounds theorem (checked inside)
    assert np.all(info["G_lower"] <= G * (1 + 1e-12) + 1e-12)
    assert np.all(info["G_upper"] >= G * (1 - 1e-12) - 1e-12)
    return rel, info


@pytest.mark.parametrize("scale", [0.1, 1.0, 10.0])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_c1_guarantee(scale, eps):
    x = synth.c1()
    h = synth.silverman_h(x) * scale
    _check_theorems(x, x, h, eps)


@pytest.mark.parametrize("scale", [1e-3, 1e-1, 1.0, 10.0, 1e3])
def test_clustered_2d_sweep(scale):
    x = synth.c2(n=3000, seed=12)
    _check_theorems(x, x, synth.silverman_h(x) * scale, 1e-2)


@pytest.mark.parametrize("d", [3, 5])
def test_higher_dimensions(d):
    x = synth.c3(n=1500, seed=13)[:, :d] if d <= 5 else None
    for scale in (0.3, 3.0):
        _check_theorems(x, x, synth.silverman_h(x) * scale, 1e-2)
    _check_theorems(x, x, synth.silverman_h(x), 1e-2, pmax=6 if d == 3 else 3)


def test_bichromatic():
    x = synth.c1(n=1500, seed=14)
    q = synth.bichromatic_queries(x, 14)[:700]
    for scale in (0.2, 2.0):
        _check_theorems(x, q, synth.silverman_h(x) * scale, 1e-2)


def test_eps_zero_is_brute_force_to_rounding():
    x = synth.c1(n=800, seed=15)
    h = synth.silverman_h(x)
    G = oracle.naive_kde(x, x, h)
    Gt, info = oracle.dfgt(x, x, h, 0.0)
    np.testing.assert_allclose(Gt, G, rtol=1e-12)


def test_coincident_points_prune_at_root_with_order_one():
    x = np.tile(np.array([[0.3, 0.7]]), (200, 1))
    Gt, info = oracle.dfgt(x, x, 0.01, 0.0)
    np.testing.assert_array_equal(Gt, np.full(200, 200.0))
    assert info["pairs"] == 1 and info["base_cases"] == 0 and info["max_order"] == 1


@pytest.mark.parametrize("force", [1, 2, 3, 4])
def test_each_summarize_method_alone_keeps_the_guarantee(force):
    # force: 1 = only far-field evaluation, 2 = only direct local, 3 = only
    # far-to-local, 4 = only the centroid form; everything else goes exhaustive
    x = synth.c1(n=1200, seed=16)
    h = synth.silverman_h(x) * 3.0
    rel, info = _check_theorems(x, x, h, 1e-2, force=force)
    key = {1: "prune_F", 2: "prune_D", 3: "prune_T", 4: "prune_centroid"}[force]
    assert info[key] > 0


def test_centroid_prune_dominates_at_tiny_bandwidth():
    x = synth.c2(n=4000, seed=17)
    h = synth.silverman_h(x) * 1e-3
    rel, info = _check_theorems(x, x, h, 1e-2)
    assert info["prune_centroid"] > 0 and info["base_pairs"] < 0.05 * 4000 ** 2


# ---- LSCV (Section 1, eq. 4) --------------------------------------------------------------------
def test_lscv_two_points_closed_form():
    mp.mp.dps = 30
    for d in (1, 2, 3):
        x = np.zeros((2, d))
        x[1, 0] = 0.7
        for h in (0.2, 1.3):
            cv, _ = oracle.lscv(x, h, variant=0)
            hh, dd = mp.mpf(h), mp.mpf(0.7)
            ref = (4 * mp.pi * hh ** 2) ** (-mp.mpf(d) / 2) * mp.e ** (-dd ** 2 / (4 * hh ** 2)) \
                - 2 * (2 * mp.pi * hh ** 2) ** (-mp.mpf(d) / 2) * mp.e ** (-dd ** 2 / (2 * hh ** 2))
            assert cv[0] == pytest.approx(float(ref), rel=1e-13)


def test_convolution_kernel_is_root_two_bandwidth():
    # int K_h(x - a) K_h(x - b) dx = K_{sqrt2 h}(a - b) for normalised Gaussians (reading A7)
    h, a, b = 0.3, 0.1, 0.55
    k = lambda x, c, hh: np.exp(-(x - c) ** 2 / (2 * hh * hh)) / np.sqrt(2 * np.pi * hh * hh)
    val, _ = integrate.quad(lambda x: k(x, a, h) * k(x, b, h), -10, 10, epsabs=1e-14, epsrel=1e-13)
    assert val == pytest.approx(k(a, b, np.sqrt(2) * h), rel=1e-11)
    # two dimensions
    a2, b2 = np.array([0.1, -0.2]), np.array([0.4, 0.3])
    k2 = lambda x, y, c, hh: np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2 * hh * hh)) / (2 * np.pi * hh * hh)
    val2, _ = integrate.dblquad(lambda y, x: k2(x, y, a2, h) * k2(x, y, b2, h), -5, 5, -5, 5,
                                epsabs=1e-13, epsrel=1e-11)
    ref2 = np.exp(-((a2 - b2) ** 2).sum() / (4 * h * h)) / (4 * np.pi * h * h)
    assert val2 == pytest.approx(ref2, rel=1e-9)


def test_lscv_gradient_vs_central_differences():
    x = synth.c1(n=400, seed=18)
    for variant in (0, 1):
        for h in (0.01, 0.05, 0.2):
            cv, dcv = oracle.lscv(x, h, variant)
            dh = 1e-5 * h
            fd = (oracle.lscv(x, h + dh, variant)[0] - oracle.lscv(x, h - dh, variant)[0]) / (2 * dh)
            assert dcv[0] == pytest.approx(fd[0], rel=1e-6)


def test_lscv_variants_differ_by_the_diagonal():
    x = synth.c1(n=300, seed=19)
    h = 0.04
    n, d = x.shape
    cv0, _ = oracle.lscv(x, h, 0)
    cv1, _ = oracle.lscv(x, h, 1)
    S2 = (oracle.naive_kde(x, x, np.sqrt(2) * h) - 1).sum()
    a = (4 * np.pi * h * h) ** (-d / 2)
    assert cv1[0] - cv0[0] == pytest.approx(a * (n + S2) / n ** 2 - a * S2 / (n * (n - 1)), rel=1e-10)


# ---- LCV and the density estimate (Section 1) ---------------------------------------------------
def test_lcv_two_points_closed_form():
    # each point's leave-one-out estimate is the other point's kernel:
    # CV_LK = -d^2/(2h^2) - (D/2) log(2 pi h^2), dCV/dh = d^2/h^3 - D/h
    for d in (1, 2, 5):
        x = np.zeros((2, d))
        x[1, -1] = 0.45
        for h in (0.1, 0.8):
            cv, dcv = oracle.lcv(x, h)
            assert cv[0] == pytest.approx(-0.45 ** 2 / (2 * h * h) - 0.5 * d * np.log(2 * np.pi * h * h), rel=1e-13)
            assert dcv[0] == pytest.approx(0.45 ** 2 / h ** 3 - d / h, rel=1e-12)


def test_lcv_leave_one_out_and_duplicates():
    # three points, two of them coincident: the duplicate pair contributes
    # K = 1 to each other's estimate, the third point sees both at distance 1
    x = np.array([[0.0, 0.0], [0.0, 0.0], [0.6, 0.8]])
    h = 0.5
    k = np.exp(-1.0 / (2 * h * h))
    V = 2 * np.pi * h * h
    ref = np.mean(np.log(np.array([1 + k, 1 + k, 2 * k]) / (2 * V)))
    assert oracle.lcv(x, h)[0][0] == pytest.approx(ref, rel=1e-13)


def test_lcv_gradient_vs_central_differences_and_underflow():
    x = synth.c1(n=300, seed=21)
    for h in (0.01, 0.05, 0.3):
        cv, dcv = oracle.lcv(x, h)
        dh = 1e-6 * h
        fd = (oracle.lcv(x, h + dh)[0] - oracle.lcv(x, h - dh)[0]) / (2 * dh)
        assert dcv[0] == pytest.approx(fd[0], rel=1e-6)
    # an isolated point whose leave-one-out sum underflows: the score is -inf
    y = np.array([[0.0], [0.001], [50.0]])
    assert oracle.lcv(y, 0.01)[0][0] == -np.inf


def test_density_integrates_to_one():
    # the normalising constant V_Dh = (2 pi h^2)^{D/2}: trapezoid quadrature of
    # the estimate over a box holding all the mass
    r1 = np.array([[0.1], [0.35], [-0.4], [0.2]])
    g = np.linspace(-4.0, 4.0, 8001)
    p = oracle.kde_density(g[:, None], r1, 0.3)
    assert np.trapezoid(p, g) == pytest.approx(1.0, rel=1e-10)
    r2 = np.array([[0.1, -0.2], [0.4, 0.3], [-0.3, 0.0]])
    g2 = np.linspace(-3.0, 3.0, 601)
    X, Y = np.meshgrid(g2, g2, indexing="ij")
    p2 = oracle.kde_density(np.stack([X.ravel(), Y.ravel()], 1), r2, 0.25).reshape(X.shape)
    assert np.trapezoid(np.trapezoid(p2, g2, axis=1), g2) == pytest.approx(1.0, rel=1e-8)


def test_final_point_bounds_are_tight_when_everything_is_pruned():
    # At a huge bandwidth every pair prunes with K(d^l) ~ K(d^u) ~ 1, so the
    # postponed bound changes pushed to the points pin G^l and G^u close to G.
    x = synth.c1(n=600, seed=20)
    h = 1e3 * np.ptp(x)
    G = oracle.naive_kde(x, x, h)
    Gt, info = oracle.dfgt(x, x, h, 1e-2, G_exact=G)
    assert np.all(info["G_lower"] >= G * (1 - 1e-5))
    assert np.all(info["G_upper"] <= G * (1 + 1e-5))
    assert info["base_cases"] == 0
