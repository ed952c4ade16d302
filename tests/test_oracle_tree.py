"""Pins for the oracle's kd-tree (Section 2.1, Alg. BuildKdTree; readings A1-A6),
re-derived by brute force on small inputs with numpy."""
import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth


def _check_tree(x, t, leaf):
    n, d = x.shape
    perm = t["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    m = t["n_nodes"]
    seen_leaf_ranges = []
    for i in range(m):
        b, e = t["begin"][i], t["end"][i]
        pts = x[perm[b:e]]
        # box = exact min / max of the node's points (A1)
        np.testing.assert_array_equal(t["lo"][i], pts.min(0))
        np.testing.assert_array_equal(t["hi"][i], pts.max(0))
        L, R = t["left"][i], t["right"][i]
        if L < 0:  # stable partitions keep the original relative order inside each leaf (A5)
            assert np.all(np.diff(perm[b:e]) > 0)
        w = t["hi"][i] - t["lo"][i]
        if L < 0:
            assert R < 0
            seen_leaf_ranges.append((b, e))
            if e - b > leaf:  # only a zero width or an empty side may stop a large node (A4)
                if w.max() > 0:
                    sd = int(np.argmax(w))
                    sc = (t["lo"][i][sd] + t["hi"][i][sd]) / 2.0
                    left = pts[:, sd] <= sc
                    assert left.all() or (~left).all()
            continue
        assert e - b > leaf
        sd = t["split_dim"][i]
        assert sd == int(np.argmax(w))  # widest dimension, lowest index on ties (A3)
        sc = t["split_coord"][i]
        assert sc == (t["lo"][i][sd] + t["hi"][i][sd]) / 2.0  # FP64 midpoint (A6)
        assert t["begin"][L] == b and t["end"][L] == t["begin"][R] and t["end"][R] == e
        assert np.all(x[perm[t["begin"][L]:t["end"][L]], sd] <= sc)
        assert np.all(x[perm[t["begin"][R]:t["end"][R]], sd] > sc)
        assert t["end"][L] > b and t["end"][L] < e
    # leaves tile [0, n) in tree order
    seen_leaf_ranges.sort()
    assert seen_leaf_ranges[0][0] == 0 and seen_leaf_ranges[-1][1] == n
    for (b0, e0), (b1, _) in zip(seen_leaf_ranges, seen_leaf_ranges[1:]):
        assert e0 == b1
    # pre-order numbering: left child directly follows its parent
    for i in range(m):
        if t["left"][i] >= 0:
            assert t["left"][i] == i + 1


@pytest.mark.parametrize("d", [1, 2, 3, 5, 16])
@pytest.mark.parametrize("leaf", [1, 4, 32])
def test_random_trees(d, leaf):
    rng = np.random.default_rng(100 * d + leaf)
    x = rng.standard_normal((300, d)) * rng.uniform(0.1, 2.0, size=d)
    _check_tree(x, oracle.build_kdtree(x, leaf), leaf)


def test_clustered_tree():
    x = synth.c2(n=3000, seed=11)
    _check_tree(x, oracle.build_kdtree(x, 16), 16)


def test_single_point():
    x = np.array([[0.5, 0.5]])
    t = oracle.build_kdtree(x, 8)
    assert t["n_nodes"] == 1 and t["perm"].tolist() == [0]


def test_all_duplicates_is_one_leaf():
    x = np.tile(np.array([[0.1, 0.2, 0.3]]), (100, 1))
    t = oracle.build_kdtree(x, 4)
    assert t["n_nodes"] == 1 and t["left"][0] == -1


def test_collinear_and_ties():
    x = np.stack([np.linspace(0, 1, 65), np.full(65, 2.0)], axis=1)
    t = oracle.build_kdtree(x, 4)
    _check_tree(x, t, 4)
    assert set(t["split_dim"][t["left"] >= 0].tolist()) == {0}
    # a square: equal widths split on the lowest dimension
    sq = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 1.0], [1.0, 0.0], [0.5, 0.5]])
    t2 = oracle.build_kdtree(sq, 1)
    assert t2["split_dim"][0] == 0


def test_adjacent_doubles_do_not_recurse_forever():
    a = 1.0
    b = np.nextafter(a, 2.0)
    x = np.array([[a], [b], [a], [b], [a], [b]])
    t = oracle.build_kdtree(x, 1)
    _check_tree(x, t, 1)


def test_fewer_points_than_leaf():
    x = np.random.default_rng(0).uniform(size=(5, 3))
    t = oracle.build_kdtree(x, 32)
    assert t["n_nodes"] == 1 and t["perm"].tolist() == [0, 1, 2, 3, 4]
