"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np


def cuda(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def note(msg):
    """Names the case before a GPU step, flushed, so a crash log says which case ran."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def compare_trees(gpu, ora, depth=None):
    """Walks the breadth-first GPU tree and the pre-order oracle tree together and
    asserts bit-identical structure; returns the number of nodes compared.  Also
    checks that the GPU ids are breadth-first (children left then right, level
    by level) and, given the tree's reported depth, the number of levels."""
    assert np.array_equal(gpu["perm"], ora["perm"]), "tree permutations differ"
    assert gpu["n_nodes"] == ora["n_nodes"], (gpu["n_nodes"], ora["n_nodes"])
    level, order = [0], [0]
    levels = 0
    while level:
        levels += 1
        nxt = []
        for v in level:
            if gpu["left"][v] >= 0:
                nxt += [int(gpu["left"][v]), int(gpu["right"][v])]
        order += nxt
        level = nxt
    assert order == list(range(gpu["n_nodes"])), "node ids are not breadth-first"
    if depth is not None:
        assert levels == depth, (levels, depth)
    stack = [(0, 0)]
    seen = 0
    while stack:
        g, o = stack.pop()
        seen += 1
        assert gpu["begin"][g] == ora["begin"][o] and gpu["end"][g] == ora["end"][o]
        assert np.array_equal(gpu["lo"][g], ora["lo"][o]) and np.array_equal(gpu["hi"][g], ora["hi"][o])
        gl, ol = gpu["left"][g], ora["left"][o]
        assert (gl < 0) == (ol < 0)
        if gl < 0:
            continue
        assert gpu["split_dim"][g] == ora["split_dim"][o]
        assert gpu["split_coord"][g] == ora["split_coord"][o]
        stack.append((gpu["right"][g], ora["right"][o]))
        stack.append((gl, ol))
    assert seen == gpu["n_nodes"]
    return seen
