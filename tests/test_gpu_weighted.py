"""GPU parity of the weighted sums G_w(q) = sum_j w_j K(q, r_j) (a reference
tree built with dfgt_build_tree_weighted) against the oracle's exact weighted
FP64 sums and derivatives.

The guarantee is the unweighted one with G_w in place of G: every query within
eps G_w(q) of the exact weighted sum.  Unit weights give bit-identical results
to the unweighted tree (the stored weights are exactly 1, the node weights are
exact sums of ones); integer weights give the sums over duplicated points (the
same exact values, each side within eps of them)."""
import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth
from tests.gpu_util import cuda, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfgt():
    from paper_1102_2878_amd import dfgt as m
    return m


def _wtree(dfgt, x, w, leaf=32):
    return dfgt.build_tree(cuda(x), leaf_size=leaf, weights=cuda(w))


@pytest.mark.parametrize("kind", ["exp", "wide", "sparse"])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_weighted_2d_matches_oracle(dfgt, kind, precision, eps):
    x = synth.c2(n=6000, seed=41)
    w = synth.weights(len(x), 41, kind)
    hS = synth.silverman_h(x)
    hs = [hS * s for s in (0.01, 0.3, 1.0, 30.0)]
    note(f"weighted 2-D kind={kind} precision={precision} eps={eps}")
    R = _wtree(dfgt, x, w)
    G = dfgt.gauss_sum(R, R, hs, eps, precision=precision).cpu().numpy()
    for k, h in enumerate(hs):
        ref, _, _ = oracle.naive_kde_weighted(x, x, w, h)
        pos = ref > 0
        rel = np.abs(G[k][pos] - ref[pos]) / ref[pos]
        assert rel.max() <= eps, (kind, h, rel.max())
        # queries whose exact sum underflows to 0 (every nearby weight is 0): at most
        # a subnormal remainder of the FP64 exponentials, never a spurious value
        assert np.all(np.abs(G[k][~pos]) <= 1e-300)


@pytest.mark.parametrize("d,maker", [(5, "c3"), (16, "c5")])
def test_weighted_higher_dimensions(dfgt, d, maker):
    x = getattr(synth, maker)(n=8000, seed=43)
    q = synth.bichromatic_queries(x, 43)[:3000]
    w = synth.weights(len(x), 43, "wide")
    hS = synth.silverman_h(x)
    hs = [hS * s for s in (0.5, 1.0, 4.0)]
    note(f"weighted D={d} bichromatic")
    R = _wtree(dfgt, x, w)
    Q = dfgt.build_tree(cuda(q))
    G = dfgt.gauss_sum(Q, R, hs, 1e-3).cpu().numpy()
    for k, h in enumerate(hs):
        ref, _, _ = oracle.naive_kde_weighted(q, x, w, h)
        rel = np.abs(G[k] - ref) / ref
        assert rel.max() <= 1e-3, (d, h, rel.max())


def test_unit_weights_are_bit_identical_to_unweighted(dfgt):
    for maker, n in (("c2", 5000), ("c3", 4000), ("c5", 3000)):
        x = getattr(synth, maker)(n=n, seed=44)
        hs = [synth.silverman_h(x) * s for s in (0.3, 1.0, 5.0)]
        note(f"unit weights {maker}")
        # separate query trees throughout: a call with Q = R is monochromatic and
        # uses the self-term prior, which a weighted R does not allow
        Q = dfgt.build_tree(cuda(x))
        R0 = dfgt.build_tree(cuda(x))
        R1 = _wtree(dfgt, x, np.ones(len(x)))
        G0 = dfgt.gauss_sum(Q, R0, hs, 1e-3).cpu().numpy()
        G1 = dfgt.gauss_sum(Q, R1, hs, 1e-3).cpu().numpy()
        assert np.array_equal(G0, G1), maker
        # weights on a query tree are ignored
        Qw = _wtree(dfgt, x, synth.weights(len(x), 44, "exp"))
        G2 = dfgt.gauss_sum(Qw, R0, hs, 1e-3).cpu().numpy()
        assert np.array_equal(G0, G2), maker


def test_integer_weights_are_duplicated_points(dfgt):
    x = synth.c2(n=5000, seed=45)
    w = synth.weights(len(x), 45, "int")
    dup = np.repeat(x, w.astype(np.int64), axis=0)
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    eps = 1e-3
    note("integer weights vs duplicated points")
    Rw = _wtree(dfgt, x, w)
    Rd = dfgt.build_tree(cuda(dup))
    Q = dfgt.build_tree(cuda(x))
    Gw = dfgt.gauss_sum(Q, Rw, hs, eps).cpu().numpy()
    Gd = dfgt.gauss_sum(Q, Rd, hs, eps).cpu().numpy()
    for k, h in enumerate(hs):
        ref = oracle.naive_kde(x, dup, h)
        assert (np.abs(Gw[k] - ref) / ref).max() <= eps
        assert (np.abs(Gd[k] - ref) / ref).max() <= eps
        assert (np.abs(Gw[k] - Gd[k]) / ref).max() <= 2 * eps


@pytest.mark.parametrize("maker,eps,precision", [("c2", 0.0, 1), ("c2", 1e-3, 0), ("c5", 0.0, 1), ("c5", 1e-3, 0),
                                                 ("c5", 1e-3, 1)])
def test_weighted_gradients(dfgt, maker, eps, precision):
    x = getattr(synth, maker)(n=4000, seed=46)
    w = synth.weights(len(x), 46, "exp")
    hs = [synth.silverman_h(x) * s for s in (0.5, 2.0)]
    note(f"weighted grad {maker} eps={eps} precision={precision}")
    R = _wtree(dfgt, x, w)
    G, Gh, Gq = (t.cpu().numpy() for t in dfgt.gauss_sum_grad(R, R, hs, eps, precision=precision))
    for k, h in enumerate(hs):
        g, gh, gq = oracle.naive_kde_weighted(x, x, w, h)
        assert (np.abs(G[k] - g) / g).max() <= max(eps, 1e-10)
        eh = np.abs(Gh[k] - gh)
        eq = np.linalg.norm(Gq[k] - gq, axis=1)
        if eps == 0.0:
            # FP64 exhaustive: the exact sums up to rounding (dG/dq measured against
            # its Cauchy-Schwarz size plus the floor of the scaled differences)
            sq = np.sqrt(np.maximum(g * gh * h ** 3, 0.0)) / h ** 2
            floor = 1e-13 * g * np.max(np.abs(x), axis=1) / h ** 2
            assert np.all(eh <= 1e-10 * gh + 1e-300)
            assert np.all(eq <= 1e-10 * sq + floor)
        else:
            unit = g / h
            assert np.all(eh <= 4 * eps * unit), np.max(eh / unit) / eps
            assert np.all(eq <= 4 * eps * unit), np.max(eq / unit) / eps


def test_weighted_density(dfgt):
    x = synth.c2(n=5000, seed=47)
    w = synth.weights(len(x), 47, "exp")
    q = synth.bichromatic_queries(x, 47)[:2000]
    hs = [synth.silverman_h(x) * s for s in (0.5, 2.0)]
    note("weighted density")
    R = _wtree(dfgt, x, w)
    Q = dfgt.build_tree(cuda(q))
    p = dfgt.kde_density(Q, R, hs, 1e-4).cpu().numpy()
    for k, h in enumerate(hs):
        g, _, _ = oracle.naive_kde_weighted(q, x, w, h)
        ref = g / (w.sum() * 2.0 * np.pi * h * h)
        assert (np.abs(p[k] - ref) / ref).max() <= 1e-4 * (1 + 1e-9)


def test_weighted_rejections(dfgt):
    x = synth.c1(n=500, seed=48)
    note("weighted rejections")
    for bad in (-1.0, np.nan, np.inf):
        w = np.ones(len(x))
        w[7] = bad
        with pytest.raises(dfgt.DfgtError, match="negative or not finite"):
            _wtree(dfgt, x, w)
    with pytest.raises(dfgt.DfgtError, match="all weights are zero"):
        _wtree(dfgt, x, np.zeros(len(x)))
    w = np.ones(len(x))
    w[3] = -0.0  # a negative zero is a zero weight
    R = _wtree(dfgt, x, w)
    h = synth.silverman_h(x)
    with pytest.raises(dfgt.DfgtError, match="unweighted"):
        dfgt.lscv_score(R, [h], 1e-2)
    with pytest.raises(dfgt.DfgtError, match="unweighted"):
        dfgt.lcv_score(R, [h], 1e-2)
    with pytest.raises(dfgt.DfgtError, match="unweighted"):
        dfgt.lscv_optimize(R, 0.5 * h, 2.0 * h, 1e-2)
    with pytest.raises(dfgt.DfgtError, match="weights must be"):
        dfgt.build_tree(cuda(x), weights=cuda(np.ones(len(x) - 1)))
