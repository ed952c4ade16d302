"""GPU tests of the batched sweep (dfgt_gauss_sum_batched) and of its captured
graph (dfgt_batch_create / run / check): several problems of uneven size,
every bandwidth of each, in one traversal.

Every (problem, bandwidth) job only reads its own lists, so a batched result
must equal the single-problem call bitwise; the guarantee of Section 3.10 is
checked against the oracle's exact sums; graph replays are checked against
the eager result after every replay, with other GPU work in between."""
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


def _problems_2d(dfgt):
    xa = synth.c1()
    xb = synth.c2(n=6000, seed=31)
    xc = synth.c1(n=3000, seed=32)
    qc = synth.bichromatic_queries(xc, 32)[:1777]
    ta, tb, tc, tq = (dfgt.build_tree(cuda(v)) for v in (xa, xb, xc, qc))
    ha = [synth.silverman_h(xa) * s for s in (0.1, 1.0, 10.0)]
    hb = [synth.silverman_h(xb) * s for s in (0.01, 0.1, 1.0, 10.0)]
    hc = [synth.silverman_h(xc) * s for s in (0.3, 3.0)]
    probs = [(ta, ta, ha), (tb, tb, hb), (tq, tc, hc)]
    data = [(xa, xa), (xb, xb), (qc, xc)]
    return probs, data


def test_batched_equals_single_calls(dfgt):
    probs, data = _problems_2d(dfgt)
    note("batch 2-D three problems")
    outs, st = dfgt.gauss_sum_batched(probs, 1e-2, stats=True)
    for (Q, R, h), G, (q, r) in zip(probs, outs, data):
        single = dfgt.gauss_sum(Q, R, h, 1e-2)
        assert G.cpu().numpy().tobytes() == single.cpu().numpy().tobytes()
        Gn = G.cpu().numpy()
        for k, hk in enumerate(h):
            ref = oracle.naive_kde(q, r, hk)
            assert np.max(np.abs(Gn[k] - ref) / ref) <= 1e-2
    assert st["segments"] > 0


def test_batched_uneven_3d_problems(dfgt):
    """Shaped like the 3-D batch: clustered problems of uneven size, many
    log-spaced bandwidths, each at h and sqrt(2) h (the LSCV pair)."""
    sizes = (1500, 4000, 9000)
    probs, data = [], []
    for i, n in enumerate(sizes):
        x = synth.c4_problem(i)
        x = x[synth.subsample(x, n, 70 + i)]
        t = dfgt.build_tree(cuda(x))
        base = synth.silverman_h(x) * np.geomspace(1e-2, 1e2, 6)
        h = np.concatenate([base, np.sqrt(2.0) * base])
        probs.append((t, t, h))
        data.append(x)
    note("batch 3-D uneven")
    outs = dfgt.gauss_sum_batched(probs, 1e-2)
    for (t, _, h), G, x in zip(probs, outs, data):
        Gn = G.cpu().numpy()
        rows = synth.subsample(x, 400, 3)
        for k, hk in enumerate(h):
            ref = oracle.naive_kde_rows(x, rows, x, hk)
            assert np.max(np.abs(Gn[k][rows] - ref) / ref) <= 1e-2, (x.shape, hk)


def test_graph_replays_match_eager(dfgt):
    probs, data = _problems_2d(dfgt)
    note("batch graph capture")
    ref = [G.cpu().numpy() for G in dfgt.gauss_sum_batched(probs, 1e-2)]
    b = dfgt.Batch(probs, 1e-2, stats=True)
    assert b.stats["segments"] > 0
    other = dfgt.build_tree(cuda(synth.c1(n=1000, seed=5)))
    import torch
    for rep in range(3):
        note(f"batch graph replay {rep}")
        for G in b.G:
            G.fill_(-1.0)
        b.run()
        b.check()
        for G, R in zip(b.G, ref):
            assert G.cpu().numpy().tobytes() == R.tobytes(), rep
        # unrelated eager work between replays
        dfgt.gauss_sum(other, other, [0.05], 1e-2)
        torch.cuda.synchronize()


def test_batch_rejects_mixed_dimensions(dfgt):
    t2 = dfgt.build_tree(cuda(synth.c1(n=500, seed=3)))
    t3 = dfgt.build_tree(cuda(synth.c3(n=500, seed=3)[:, :3].copy()))
    with pytest.raises(dfgt.DfgtError):
        dfgt.gauss_sum_batched([(t2, t2, [0.1]), (t3, t3, [0.1])], 1e-2)
