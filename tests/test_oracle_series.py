"""Pins for the oracle's series-expansion machinery: Hermite functions and the
multi-index layout (Section 3.1, Appendix), far-field / local expansions and
their operators (Sections 3.3, 3.4, 3.7), truncation bounds and order choice
(Sections 3.5, 3.6, 3.8), node-pair distance bounds (Section 2.2).

The reference values come from numpy's Hermite series, mpmath, direct
exponentials and exact algebraic identities, never from the oracle itself."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import hermite as nph

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _kernel(q, r, h):
    return np.exp(-((q[:, None, :] - r[None, :, :]) ** 2).sum(-1) / (2 * h * h)).sum(1)


# ---- Hermite functions ---------------------------------------------------------------------
def test_printed_hermite_polynomials():
    t = np.linspace(-3, 3, 41)
    H = oracle.hermite_table(t, 3) * np.exp(t * t)[:, None]  # h_n e^{t^2} = H_n
    for n, key in enumerate(("H0", "H1", "H2")):
        coef = GOLDEN["hermite_polynomials"][key]
        np.testing.assert_allclose(H[:, n], np.polyval(coef[::-1], t), rtol=1e-13, atol=1e-12)


def test_hermite_functions_vs_numpy_series():
    t = np.linspace(-6, 6, 101)
    H = oracle.hermite_table(t, 20)
    for n in range(20):
        c = np.zeros(n + 1)
        c[n] = 1
        ref = nph.hermval(t, c) * np.exp(-t * t)
        np.testing.assert_allclose(H[:, n], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_generating_function():
    # e^{-(t - s)^2} = sum_n s^n / n! h_n(t)   (Section 3.1)
    t = np.linspace(-2, 2, 9)
    H = oracle.hermite_table(t, 41)
    for s in (-0.7, 0.2, 0.9):
        series = sum(s ** n / math.factorial(n) * H[:, n] for n in range(41))
        np.testing.assert_allclose(series, np.exp(-(t - s) ** 2), rtol=1e-13, atol=1e-14)


def test_szasz_inequality_used_by_the_lemmas():
    # (1/n!) |h_n(x)| <= 2^{n/2} / sqrt(n!) e^{-x^2/2}  (proof of the far-field lemma)
    x = np.linspace(-15, 15, 30001)
    H = oracle.hermite_table(x, 41)
    for n in range(41):
        lhs = np.abs(H[:, n]) / math.factorial(n)
        rhs = 2 ** (n / 2) / math.sqrt(math.factorial(n)) * np.exp(-x * x / 2)
        assert np.all(lhs <= rhs * (1 + 1e-12) + 1e-300)


# ---- Multi-index layout ----------------------------------------------------------------------
def test_position_multiindex_roundtrip_and_last_dim_fastest():
    assert oracle.pos_to_mi(1, 2, 3) == (0, 1)
    assert oracle.pos_to_mi(3, 2, 3) == (1, 0)
    for d, p in ((1, 5), (2, 4), (3, 3), (5, 2)):
        for i in range(p ** d):
            a = oracle.pos_to_mi(i, d, p)
            assert oracle.mi_to_pos(a, p) == i
            assert a == tuple(int(v) for v in np.unravel_index(i, (p,) * d))


def test_multiindex_expansion_vs_numpy_powers():
    x = np.array([0.3, -1.2])
    out = oracle.mi_expansion(x, 4)
    assert out.size == GOLDEN["multi_index_expansion_figure"]["terms"]
    for i, a in enumerate(itertools.product(range(4), repeat=2)):
        assert out[i] == pytest.approx(np.prod(x ** np.array(a)), rel=1e-15)
    # sub-box of radix p inside radix-pmax storage (A15)
    y = np.array([0.5, 2.0, -1.0])
    out = oracle.mi_expansion(y, 2, pmax=3)
    for a in itertools.product(range(2), repeat=3):
        assert out[oracle.mi_to_pos(a, 3)] == pytest.approx(np.prod(y ** np.array(a)))


# ---- Expansions: high-order exactness (eq. primal, eq. dual) --------------------------------
@pytest.mark.parametrize("d", [1, 2])
def test_far_field_expansion_converges_to_kernel(d):
    rng = np.random.default_rng(d)
    h = 0.5
    r = rng.uniform(-0.3, 0.3, size=(6, d))
    c = np.zeros(d)
    q = rng.uniform(-1.5, 1.5, size=(10, d))
    p = 30 if d == 1 else 24
    M = oracle.p2m(r, c, h, p)
    got = oracle.far_eval(M, c, h, p, p, q)
    np.testing.assert_allclose(got, _kernel(q, r, h), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2])
def test_direct_local_expansion_converges_to_kernel(d):
    rng = np.random.default_rng(20 + d)
    h = 0.5
    r = rng.uniform(-2, 2, size=(6, d))
    cq = np.full(d, 0.1)
    q = cq + rng.uniform(-0.3, 0.3, size=(10, d))
    p = 30 if d == 1 else 24
    L = oracle.direct_local(r, cq, h, p, p)
    got = oracle.local_eval(L, cq, h, p, p, q)
    np.testing.assert_allclose(got, _kernel(q, r, h), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2])
def test_far_to_local_converges_to_kernel(d):
    rng = np.random.default_rng(30 + d)
    h = 1.0
    cr = np.zeros(d)
    cq = np.full(d, 0.8)
    r = cr + rng.uniform(-0.15, 0.15, size=(5, d))
    q = cq + rng.uniform(-0.15, 0.15, size=(7, d))
    p = 18
    M = oracle.p2m(r, cr, h, p)
    L = oracle.f2l(M, cr, cq, h, p, p)
    got = oracle.local_eval(L, cq, h, p, p, q)
    np.testing.assert_allclose(got, _kernel(q, r, h), rtol=1e-11, atol=1e-12)


def test_points_at_centre_are_exact_at_order_one():
    # every reference point at R.c: M = (|R|, 0, ...), F-eval = G exactly for p >= 1
    c = np.array([0.2, -0.4, 1.0])
    r = np.tile(c, (11, 1))
    M = oracle.p2m(r, c, 0.3, 3)
    assert M[0] == 11.0 and np.all(M[1:] == 0.0)
    q = np.random.default_rng(1).uniform(-1, 1, size=(5, 3))
    for p in (1, 2, 3):
        np.testing.assert_allclose(oracle.far_eval(M, c, 0.3, p, 3, q), _kernel(q, r, 0.3), rtol=1e-14)


def test_direct_local_at_centre_gives_exact_zeroth_moment():
    # a local expansion evaluated at Q.c reduces to L_0 = G(Q.c, R)
    rng = np.random.default_rng(5)
    r = rng.uniform(size=(9, 2))
    cq = np.array([0.4, 0.6])
    L = oracle.direct_local(r, cq, 0.2, 4, 4)
    assert L[0] == pytest.approx(_kernel(cq[None], r, 0.2)[0], rel=1e-14)
    assert oracle.local_eval(L, cq, 0.2, 4, 4, cq[None])[0] == pytest.approx(L[0], rel=1e-15)


def test_f2l_zeroth_term_is_far_field_at_query_centre():
    rng = np.random.default_rng(6)
    r = rng.uniform(-0.2, 0.2, size=(8, 2))
    cr = np.zeros(2)
    cq = np.array([0.5, -0.3])
    M = oracle.p2m(r, cr, 0.4, 5)
    L = oracle.f2l(M, cr, cq, 0.4, 5, 5)
    assert L[0] == pytest.approx(oracle.far_eval(M, cr, 0.4, 5, 5, cq[None])[0], rel=1e-13)


# ---- Hierarchical operators: exact re-centring (Section 3.7) ------------------------------------
@pytest.mark.parametrize("d,pmax", [(1, 8), (2, 6), (3, 4), (5, 2)])
def test_f2f_equals_direct_moments_at_parent(d, pmax):
    rng = np.random.default_rng(40 + d)
    h = 0.3
    a = rng.uniform(0, 0.2, size=(7, d))
    b = rng.uniform(0.1, 0.3, size=(5, d))
    ca, cb, cp = a.mean(0), b.mean(0), np.concatenate([a, b]).mean(0) + 0.01
    Mp = oracle.f2f(oracle.p2m(a, ca, h, pmax), ca, cp, h, pmax)
    Mp = oracle.f2f(oracle.p2m(b, cb, h, pmax), cb, cp, h, pmax, Mp)
    direct = oracle.p2m(np.concatenate([a, b]), cp, h, pmax)
    np.testing.assert_allclose(Mp, direct, rtol=1e-12, atol=1e-13 * np.abs(direct).max())


@pytest.mark.parametrize("d,p", [(1, 7), (2, 5), (3, 3)])
def test_l2l_preserves_the_local_polynomial(d, p):
    rng = np.random.default_rng(50 + d)
    h = 0.4
    Lp = rng.standard_normal(p ** d)
    cp = rng.uniform(size=d)
    cc = cp + rng.uniform(-0.1, 0.1, size=d)
    q = cc + rng.uniform(-0.05, 0.05, size=(9, d))
    Lc = oracle.l2l(Lp, cp, cc, h, p, p)
    np.testing.assert_allclose(oracle.local_eval(Lc, cc, h, p, p, q), oracle.local_eval(Lp, cp, h, p, p, q),
                               rtol=1e-12, atol=1e-12)


# ---- Truncation bounds (Section 3.5) ------------------------------------------------------------
def _box_points(rng, c, half, n, d):
    return c + rng.uniform(-1, 1, size=(n, d)) * half


@pytest.mark.parametrize("d", [1, 2, 3])
def test_far_field_error_within_lemma_bound(d):
    rng = np.random.default_rng(60 + d)
    for _ in range(60):
        h = rng.uniform(0.2, 2.0)
        r_ = rng.uniform(0.05, 0.95)
        half = r_ * h
        c = rng.uniform(-1, 1, size=d)
        pts = _box_points(rng, c, half, 12, d)
        q = c + rng.uniform(-4, 4, size=(20, d)) * h
        p = int(rng.integers(1, 7))
        M = oracle.p2m(pts, c, h, p)
        err = np.abs(oracle.far_eval(M, c, h, p, p, q) - _kernel(q, pts, h)).max()
        assert err <= oracle.bound_far(r_, p, d, 12) * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("d", [1, 2, 3])
def test_local_error_within_lemma_bound(d):
    rng = np.random.default_rng(70 + d)
    for _ in range(60):
        h = rng.uniform(0.2, 2.0)
        r_ = rng.uniform(0.05, 0.95)
        cq = rng.uniform(-1, 1, size=d)
        q = _box_points(rng, cq, r_ * h, 15, d)
        pts = cq + rng.uniform(-4, 4, size=(9, d)) * h
        p = int(rng.integers(1, 7))
        L = oracle.direct_local(pts, cq, h, p, p)
        err = np.abs(oracle.local_eval(L, cq, h, p, p, q) - _kernel(q, pts, h)).max()
        assert err <= oracle.bound_local(r_, p, d, 9) * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("d", [1, 2, 3])
def test_far_to_local_error_within_lemma_bound(d):
    rng = np.random.default_rng(80 + d)
    for _ in range(60):
        h = rng.uniform(0.2, 2.0)
        r_ = rng.uniform(0.02, 0.48)
        cq, cr = rng.uniform(-1, 1, size=d), rng.uniform(-1, 1, size=d)
        q = _box_points(rng, cq, r_ * h, 10, d)
        pts = _box_points(rng, cr, r_ * h, 10, d)
        p = int(rng.integers(1, 7))
        L = oracle.f2l(oracle.p2m(pts, cr, h, p), cr, cq, h, p, p)
        err = np.abs(oracle.local_eval(L, cq, h, p, p, q) - _kernel(q, pts, h)).max()
        assert err <= oracle.bound_f2l(r_, p, d, 10) * (1 + 1e-9) + 1e-14


def test_bounds_shrink_with_order_and_vanish_at_zero_width():
    for d in (1, 2, 5):
        b = [oracle.bound_far(0.4, p, d, 100) for p in range(1, 10)]
        assert all(x > y for x, y in zip(b, b[1:]))
        assert oracle.bound_far(0.0, 1, d, 100) == 0.0
        assert oracle.bound_f2l(0.0, 1, d, 100) == 0.0


# ---- Distance bounds (Section 2.2) and the centroid bound (Section 3.10) ----------------------
def test_distance_bounds_enclose_all_pair_distances():
    rng = np.random.default_rng(90)
    for _ in range(200):
        d = int(rng.integers(1, 6))
        qlo = rng.uniform(-1, 1, d)
        qhi = qlo + rng.uniform(0, 1, d)
        rlo = rng.uniform(-1, 1, d)
        rhi = rlo + rng.uniform(0, 1, d)
        dl, du = oracle.dist_bounds(qlo, qhi, rlo, rhi)
        q = rng.uniform(qlo, qhi, size=(30, d))
        r = rng.uniform(rlo, rhi, size=(30, d))
        dist = np.sqrt(((q[:, None] - r[None]) ** 2).sum(-1))
        assert dist.min() >= dl - 1e-12 and dist.max() <= du + 1e-12
        # the corners attain the bounds
        corners_q = np.array(list(itertools.product(*zip(qlo, qhi))))
        corners_r = np.array(list(itertools.product(*zip(rlo, rhi))))
        dmax = np.sqrt(((corners_q[:, None] - corners_r[None]) ** 2).sum(-1)).max()
        assert du == pytest.approx(dmax, rel=1e-12)


def test_centroid_bound_covers_centroid_error():
    rng = np.random.default_rng(91)
    for _ in range(100):
        d = 2
        h = rng.uniform(0.05, 1.0)
        qlo = rng.uniform(-1, 1, d)
        qhi = qlo + rng.uniform(0, 0.5, d)
        rlo = rng.uniform(-1, 1, d)
        rhi = rlo + rng.uniform(0, 0.5, d)
        q = rng.uniform(qlo, qhi, size=(20, d))
        r = rng.uniform(rlo, rhi, size=(15, d))
        dl, du = oracle.dist_bounds(qlo, qhi, rlo, rhi)
        dc = np.linalg.norm((qlo + qhi) / 2 - (rlo + rhi) / 2)
        approx = 15 * np.exp(-dc * dc / (2 * h * h))
        err = np.abs(_kernel(q, r, h) - approx).max()
        assert err <= oracle.centroid_bound(dl, du, dc, h, 15) + 1e-13


# ---- Order selection (Section 3.6) and ChooseBestMethod (Section 3.8) --------------------------
def test_orders_are_least_admissible():
    for d in (1, 2, 3):
        for tau in (1e-1, 1e-3, 1e-6):
            w, h, n = 0.5, 1.0, 50
            p = oracle.far_field_order(w, h, d, n, tau, 8)
            r = w / (2 * h)
            if p:
                assert oracle.bound_far(r, p, d, n) <= tau
                assert p == 1 or oracle.bound_far(r, p - 1, d, n) > tau
            else:
                assert all(oracle.bound_far(r, q, d, n) > tau for q in range(1, 9))
            pt = oracle.f2l_order(0.3, 0.4, h, d, n, tau, 8)
            if pt:
                assert oracle.bound_f2l(0.4 / 2, pt, d, n) <= tau
    assert oracle.far_field_order(2.0, 1.0, 2, 10, 1.0, 6) == 0  # width 2h: r = 1, inadmissible
    assert oracle.f2l_order(1.0, 0.1, 1.0, 2, 10, 1.0, 6) == 0   # side length h: r = 1/2


def test_choose_method_prefers_cheapest():
    # tiny far-away reference box: the centroid form of T costs D and wins
    m, p = oracle.choose_method([0, 0], [1, 1], [50, 50], [50.1, 50.1], 1000, 10, 1.0, 1e-3, 6)
    assert (m, p) == (oracle.METHOD_T, 1)
    # unprunable (overlapping, wide) pair -> E
    m, p = oracle.choose_method([0, 0], [10, 10], [0, 0], [10, 10], 1000, 1000, 1.0, 1e-6, 6)
    assert m == oracle.METHOD_E and p == 0
    # one query, many references, small reference box, query far outside the T range -> F
    m, p = oracle.choose_method([0, 0], [3, 3], [1, 1], [1.2, 1.2], 1, 5000, 1.0, 1.0, 6)
    assert m == oracle.METHOD_F and p >= 1
    # many queries in a small box, few references -> D
    m, p = oracle.choose_method([1, 1], [1.2, 1.2], [0, 0], [3, 3], 5000, 2, 1.0, 1e-3, 6)
    assert m == oracle.METHOD_D and p >= 1


def test_bounds_equal_the_proof_product_form():
    # The lemma's right-hand side is |R| (prod_d (U + V) - prod_d U) with the per-dimension
    # geometric-series bounds U, V from the proof; evaluate that product form in mpmath.
    import mpmath as mp
    mp.mp.dps = 40
    for d in (1, 2, 3, 5):
        for r in (0.05, 0.3, 0.45):
            for p in (1, 2, 4, 6):
                R = mp.mpf(r)
                U = (1 - R ** p) / (1 - R)
                V = R ** p / ((1 - R) * mp.sqrt(mp.factorial(p)))
                far = 37 * ((U + V) ** d - U ** d)
                assert oracle.bound_far(r, p, d, 37) == pytest.approx(float(far), rel=1e-12)
                assert oracle.bound_local(r, p, d, 37) == pytest.approx(float(far), rel=1e-12)
                T = 2 * R
                U2 = ((1 - T ** p) / (1 - T)) ** 2
                V2 = (1 - T ** p) / (1 - T) * T ** p / ((1 - T) * mp.sqrt(mp.factorial(p)))
                W2 = T ** p / ((1 - T) ** 2 * mp.sqrt(mp.factorial(p)))
                f2l = 37 * ((U2 + V2 + W2) ** d - U2 ** d)
                assert oracle.bound_f2l(r, p, d, 37) == pytest.approx(float(f2l), rel=1e-12)


def test_choose_method_cost_model_and_ties():
    # D = 2, both boxes tiny relative to h: F, D and T are all admissible at order 1.
    # One query: c_F = 2*1*1 = 2 = c_T = 2*1 -> tie, F first.
    m, p = oracle.choose_method([0, 0], [1e-3, 1e-3], [5, 5], [5.001, 5.001], 1, 1000, 1.0, 10.0, 6)
    assert (m, p) == (oracle.METHOD_F, 1)
    # at tau = 1 the order-1 far-field bound (~1.0005) fails, p_F = 2 costs 8 > c_T = 2
    m, p = oracle.choose_method([0, 0], [1e-3, 1e-3], [5, 5], [5.001, 5.001], 1, 1000, 1.0, 1.0, 6)
    assert (m, p) == (oracle.METHOD_T, 1)
    # Many queries, one reference: c_D = 2*1*1 = 2 ties c_T = 2 -> D before T.
    m, p = oracle.choose_method([0, 0], [1e-3, 1e-3], [5, 5], [5.001, 5.001], 1000, 1, 1.0, 10.0, 6)
    assert (m, p) == (oracle.METHOD_D, 1)
    # Overlapping boxes (no centroid prune), all three lemma orders admissible at tau:
    # check the choice is the argmin of the A12 costs.
    qlo, qhi, rlo, rhi = [0, 0], [0.3, 0.3], [0.2, 0.2], [0.5, 0.5]
    for nQ, nR, tau in ((1, 500, 1e-4), (3, 500, 1e-6), (500, 2, 1e-6), (4000, 4000, 1e-3)):
        pF = oracle.far_field_order(0.3, 1.0, 2, nR, tau, 6)
        pD = oracle.local_order(0.3, 1.0, 2, nR, tau, 6)
        pT = oracle.f2l_order(0.3, 0.3, 1.0, 2, nR, tau, 6)
        costs = [(2 * nQ * pF ** 2) if pF else np.inf, (2 * nR * pD ** 2) if pD else np.inf,
                 (2 * pT ** 4) if pT else np.inf, 2 * nQ * nR]
        want = int(np.argmin(costs))
        m, p = oracle.choose_method(qlo, qhi, rlo, rhi, nQ, nR, 1.0, tau, 6)
        assert m == [oracle.METHOD_F, oracle.METHOD_D, oracle.METHOD_T, oracle.METHOD_E][want]
        assert p == [pF, pD, pT, 0][want]
