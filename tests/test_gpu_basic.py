"""GPU parity of the brute-force comparator, the kd-tree and the raw moments
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth
from tests.gpu_util import compare_trees, cuda, note

pytestmark = pytest.mark.gpu

# Mixed precision (FP64 differences, FP32 exp2, FP32 partial sums of <= 64
# terms, FP64 accumulation): per-term relative error <= ln2 * 126 * 2^-24 (the
# FP32 rounding of the exponent, |exponent| <= 126 before exp2 underflows)
# + 2^-22 (exp2) and <= 64 * 2^-24 for the partial sums, i.e. < 1e-5 overall.
# Terms below 2^-126 flush to zero in FP32: an absolute error <= n_r * 2^-126.
MIXED_RTOL = 1e-5


def mixed_atol(nr):
    return nr * 2.0 ** -126


@pytest.fixture(scope="module")
def dfgt():
    from paper_1102_2878_amd import dfgt as m
    return m


@pytest.mark.parametrize("prec", [1, 0])
def test_naive_c1_vs_oracle(dfgt, prec):
    x = synth.c1()
    h0 = synth.silverman_h(x)
    hs = [0.1 * h0, h0, 10 * h0]
    note(f"naive c1 prec={prec}")
    G = dfgt.naive_sum(cuda(x), cuda(x), hs, precision=prec).cpu().numpy()
    for k, h in enumerate(hs):
        ref = oracle.naive_kde(x, x, h)
        np.testing.assert_allclose(G[k], ref, rtol=1e-12 if prec == 1 else MIXED_RTOL)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 7, 16])
def test_naive_dims_and_ragged_sizes(dfgt, d):
    rng = np.random.default_rng(d)
    for nq, nr in ((1, 1), (3, 1000), (1000, 3), (777, 1531)):
        q = rng.uniform(size=(nq, d))
        r = rng.uniform(size=(nr, d))
        hs = [0.05, 0.4]
        note(f"naive d={d} nq={nq} nr={nr}")
        for prec in (0, 1):
            G = dfgt.naive_sum(cuda(q), cuda(r), hs, precision=prec).cpu().numpy()
            for k, h in enumerate(hs):
                ref = oracle.naive_kde(q, r, h)
                np.testing.assert_allclose(G[k], ref, rtol=1e-12 if prec == 1 else MIXED_RTOL,
                                           atol=1e-300 if prec == 1 else mixed_atol(nr))


def test_naive_full_size_sampled(dfgt):
    x = synth.c2()
    rows = synth.subsample(x, 300, 2)
    h = 0.004
    note("naive c2 50k sampled")
    G = dfgt.naive_sum(cuda(x), cuda(x), [h]).cpu().numpy()[0]
    ref = oracle.naive_kde_rows(x, rows, x, h)
    np.testing.assert_allclose(G[rows], ref, rtol=MIXED_RTOL)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 16, 32])
@pytest.mark.parametrize("leaf", [1, 4, 32])
def test_tree_bit_exact_random(dfgt, d, leaf):
    rng = np.random.default_rng(100 * d + leaf)
    x = rng.standard_normal((1500, d)) * rng.uniform(0.1, 2.0, size=d)
    note(f"tree d={d} leaf={leaf}")
    t = dfgt.build_tree(cuda(x), leaf_size=leaf)
    compare_trees(dfgt.tree_export(t), oracle.build_kdtree(x, leaf), t.info()["depth"])


def test_tree_rebuilds_of_one_shape(dfgt):
    # A rebuild of the same (n, d, leaf) hands the lower levels to the per-node
    # phase from the level learnt on the previous build; other data of that
    # shape may not allow it there, and the build then goes on level by level.
    for seed in (11, 12, 13):
        x = synth.c2(n=20000, seed=seed)
        ref = oracle.build_kdtree(x, 32)
        for rep in range(2):
            note(f"tree rebuild seed={seed} rep={rep}")
            t = dfgt.build_tree(cuda(x), leaf_size=32)
            compare_trees(dfgt.tree_export(t), ref, t.info()["depth"])
    # sizes around the per-node phase's node limits (512 points at D=1 with
    # leaf 1, 960 at D=2 with leaf 8, 320 at D=16 with leaf 32; a whole tree in
    # one block up to them) and far above them
    rng = np.random.default_rng(14)
    for n in (320, 321, 512, 513, 960, 961, 5000):
        for d, leaf in ((1, 1), (2, 8), (16, 32)):
            x = rng.standard_normal((n, d))
            ref = oracle.build_kdtree(x, leaf)
            for rep in range(2):
                note(f"tree sizes n={n} d={d} leaf={leaf} rep={rep}")
                t = dfgt.build_tree(cuda(x), leaf_size=leaf)
                compare_trees(dfgt.tree_export(t), ref, t.info()["depth"])


def test_tree_large_frontier(dfgt):
    # 1.5M uniform 2-D points: the first build guesses level 13 for the
    # per-node phase, where 8192 nodes share its 2048 blocks (several subtrees
    # per block); the rebuild starts at level 11, the first whose nodes hold
    # at most 1024 points (2048 nodes)
    x = np.random.default_rng(15).uniform(size=(1_500_000, 2))
    ref = oracle.build_kdtree(x, 32)
    for rep in range(2):
        note(f"tree large frontier rep={rep}")
        t = dfgt.build_tree(cuda(x), leaf_size=32)
        compare_trees(dfgt.tree_export(t), ref, t.info()["depth"])


def test_tree_deep_chain(dfgt):
    # 1.5^-k: every mid-point split cuts off the two or so largest points, so
    # the tree is a chain about n / 2 levels deep.  Its big nodes reach far
    # below any balanced-tree level, so the first build goes level by level
    # to the end; the rebuild starts the per-node phase at the level where the
    # chain's node fits (about 220), and that phase then runs some 480 levels
    # deep in one block.
    x = (1.5 ** -np.arange(1400.0))[::-1].reshape(-1, 1).copy()
    ref = oracle.build_kdtree(x, 4)
    for rep in range(2):
        note(f"tree chain rep={rep}")
        t = dfgt.build_tree(cuda(x), leaf_size=4)
        compare_trees(dfgt.tree_export(t), ref, t.info()["depth"])


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_tree_bit_exact_workloads(dfgt, name):
    gen = {"c1": lambda: synth.c1(), "c2": lambda: synth.c2(), "c3": lambda: synth.c3(n=30000),
           "c4": lambda: synth.c4_problem(0), "c5": lambda: synth.c5(n=20000)}[name]
    x = gen()
    note(f"tree workload {name} n={x.shape[0]}")
    t = dfgt.build_tree(cuda(x), leaf_size=32)
    info = t.info()
    compare_trees(dfgt.tree_export(t), oracle.build_kdtree(x, 32), info["depth"])
    assert info["n"] == x.shape[0]


def test_tree_degenerate_inputs(dfgt):
    cases = {
        "single": np.array([[0.5, 0.5]]),
        "duplicates": np.tile(np.array([[0.1, 0.2, 0.3]]), (300, 1)),
        "collinear": np.stack([np.linspace(0, 1, 999), np.full(999, 2.0)], axis=1),
        "adjacent_doubles": np.array([[1.0], [np.nextafter(1.0, 2.0)]] * 40),
        "few_points": np.random.default_rng(0).uniform(size=(5, 3)),
        "clusters_of_duplicates": np.repeat(np.random.default_rng(1).uniform(size=(50, 2)), 40, axis=0),
    }
    for name, x in cases.items():
        for leaf in (1, 8, 32):
            note(f"tree degenerate {name} leaf={leaf}")
            t = dfgt.build_tree(cuda(x), leaf_size=leaf)
            compare_trees(dfgt.tree_export(t), oracle.build_kdtree(x, leaf), t.info()["depth"])


@pytest.mark.parametrize("d,pmax", [(1, 8), (2, 6), (3, 4), (5, 2), (5, 4), (16, 1)])
def test_raw_moments_vs_oracle_p2m(dfgt, d, pmax):
    rng = np.random.default_rng(7 + d)
    x = rng.uniform(size=(3000, d)) * rng.uniform(0.2, 1.0, size=d)
    note(f"moments d={d} pmax={pmax}")
    t = dfgt.build_tree(cuda(x), leaf_size=16, p_max=pmax)
    mu = dfgt.tree_moments(t)
    tr = dfgt.tree_export(t)
    pts = x[tr["perm"]]
    # with h = 1/sqrt(2) the paper's moments M_alpha equal the raw moments
    h = 1.0 / np.sqrt(2.0)
    check = np.unique(np.concatenate([[0], rng.integers(0, tr["n_nodes"], size=60)]))
    for node in check:
        b, e = tr["begin"][node], tr["end"][node]
        c = (tr["lo"][node] + tr["hi"][node]) / 2.0
        ref = oracle.p2m(pts[b:e], c, h, pmax)
        scale = np.abs(ref).max()
        np.testing.assert_allclose(mu[node], ref, rtol=1e-11, atol=1e-12 * scale)


def test_invalid_input_rejected(dfgt):
    x = np.array([[0.0, np.nan], [1.0, 2.0]])
    with pytest.raises(dfgt.DfgtError, match="non-finite"):
        dfgt.build_tree(cuda(x))


def test_tree_perm_on_device():
    from paper_1102_2878_amd import dfgt
    x = synth.c2(n=20000, seed=91)
    note("tree perm on device")
    t = dfgt.build_tree(cuda(x), leaf_size=64)
    perm = dfgt.tree_perm(t).cpu().numpy()
    assert np.array_equal(perm, dfgt.tree_export(t)["perm"])
    assert np.array_equal(np.sort(perm), np.arange(x.shape[0]))


def test_caller_allocator():
    """With torch's caching allocator installed, the sums' workspaces come from it
    (torch's allocated bytes grow) and the results are bitwise those of the
    hipMalloc workspaces; releasing the workspace returns the memory to torch."""
    import torch

    from paper_1102_2878_amd import dfgt
    x = synth.c2(n=20000, seed=92)
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    note("caller allocator")
    t = dfgt.build_tree(cuda(x))
    ref = dfgt.gauss_sum(t, t, hs, 1e-2).cpu().numpy()
    torch.cuda.synchronize()
    dfgt.use_torch_allocator(True)
    try:
        before = torch.cuda.memory_allocated()
        G = dfgt.gauss_sum(t, t, hs, 1e-2).cpu().numpy()
        during = torch.cuda.memory_allocated()
        assert during > before + (1 << 20), (before, during)
        assert G.tobytes() == ref.tobytes()
        dfgt.lib().dfgt_release_workspace()
        assert torch.cuda.memory_allocated() < during
    finally:
        dfgt.use_torch_allocator(False)
    G2 = dfgt.gauss_sum(t, t, hs, 1e-2).cpu().numpy()
    assert G2.tobytes() == ref.tobytes()
