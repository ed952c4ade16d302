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


def _problems_3d(dfgt, sizes, nbase, leaf=32):
    probs, data = [], []
    for i, n in enumerate(sizes):
        x = synth.c4_problem(i)
        if n < x.shape[0]:
            x = x[synth.subsample(x, n, 70 + i)]
        t = dfgt.build_tree(cuda(x), leaf_size=leaf)
        base = synth.silverman_h(x) * np.geomspace(1e-3, 1e3, nbase)
        probs.append((t, t, np.concatenate([base, np.sqrt(2.0) * base])))
        data.append(x)
    return probs, data


def test_split_into_parts_matches_unsplit(dfgt, monkeypatch):
    """A memory budget too small for the whole batch splits its jobs into parts
    that run in turn on the same buffers (eager) or one after another in the
    captured graph.  Jobs only read their own lists, so every part layout
    gives the unsplit result bitwise; it is also within eps of the oracle."""
    probs, data = _problems_3d(dfgt, (1500, 4000, 9000), 6)
    note("batch split: unsplit reference")
    ref, st0 = dfgt.gauss_sum_batched(probs, 1e-2, stats=True)
    ref = [G.cpu().numpy() for G in ref]
    assert st0["parts"] == 1
    monkeypatch.setenv("DFGT_MEMORY_BUDGET_MB", "48")
    note("batch split: eager, 48 MiB budget")
    outs, st = dfgt.gauss_sum_batched(probs, 1e-2, stats=True)
    assert st["parts"] >= 3, st["parts"]
    for G, R in zip(outs, ref):
        assert G.cpu().numpy().tobytes() == R.tobytes()
    note("batch split: graph capture, 48 MiB budget")
    b = dfgt.Batch(probs, 1e-2, stats=True)
    assert b.stats["parts"] >= 3, b.stats["parts"]
    import torch
    for rep in range(3):
        note(f"batch split: graph replay {rep}")
        for G in b.G:
            G.fill_(-1.0)
        b.run()
        b.check()
        for G, R in zip(b.G, ref):
            assert G.cpu().numpy().tobytes() == R.tobytes(), rep
        dfgt.gauss_sum(probs[0][0], probs[0][0], [0.05], 1e-2)
        torch.cuda.synchronize()
    monkeypatch.delenv("DFGT_MEMORY_BUDGET_MB")
    for (t, _, h), G, x in zip(probs, ref, data):
        rows = synth.subsample(x, 300, 9)
        for k in range(0, len(h), 3):
            r = oracle.naive_kde_rows(x, rows, x, h[k])
            assert np.max(np.abs(G[k][rows] - r) / r) <= 1e-2, (x.shape, h[k])


@pytest.mark.parametrize("leaf", [128, 256])
def test_full_size_3d_batch_sampled(dfgt, leaf):
    """The 3-D batch at its full size and in the bench's launch configurations:
    8 clustered problems of 10k..200k points, 64 log-spaced bandwidths
    h_S x 10^{-3..3} each at h and sqrt(2) h (1024 sums), leaf size 128 or 256
    (the candidates the bench picks between), the jobs split into as many parts
    as the default memory budget needs.  The captured graph's replay equals the
    eager call bitwise; 200 seeded rows per problem at 16 seeded bandwidths are
    within eps of the oracle; both product precisions of the matrix-core tiles
    take part."""
    import torch
    probs, data = _problems_3d(dfgt, synth.C4_SIZES, 64, leaf=leaf)
    note(f"batch 3-D full size, leaf {leaf}: eager")
    eager, st = dfgt.gauss_sum_batched(probs, 1e-2, stats=True)
    torch.cuda.synchronize()
    assert st["e_pairs"]["fp32"] > 0 and st["e_pairs"]["fp64"] > 0, st["e_pairs"]
    assert st["e_pairs"]["fp32"] + st["e_pairs"]["fp64"] <= st["base_point_pairs"]
    note(f"batch 3-D full size: graph capture ({st['parts']} parts eager)")
    b = dfgt.Batch(probs, 1e-2)
    for G in b.G:
        G.fill_(-1.0)
    note("batch 3-D full size: graph replay")
    b.run()
    b.check()
    for G, E in zip(b.G, eager):
        assert torch.equal(G, E)
    del b
    rng = np.random.default_rng(404)
    for k, ((t, _, h), G, x) in enumerate(zip(probs, eager, data)):
        rows = synth.subsample(x, 200, 80 + k)
        cols = np.sort(rng.choice(len(h), size=16, replace=False))
        Gs = G[:, torch.as_tensor(rows, device=G.device)].cpu().numpy()
        for j in cols:
            r = oracle.naive_kde_rows(x, rows, x, h[j])
            rel = np.abs(Gs[j] - r) / r
            assert rel.max() <= 1e-2, (x.shape, h[j], rel.max())


def test_batch_rejects_mixed_dimensions(dfgt):
    t2 = dfgt.build_tree(cuda(synth.c1(n=500, seed=3)))
    t3 = dfgt.build_tree(cuda(synth.c3(n=500, seed=3)[:, :3].copy()))
    with pytest.raises(dfgt.DfgtError):
        dfgt.gauss_sum_batched([(t2, t2, [0.1]), (t3, t3, [0.1])], 1e-2)
