"""GPU parity of the gradient mode (dfgt_gauss_sum_grad), the backward product
(dfgt_gauss_sum_backward, and its torch.autograd wrapper) and the LSCV score
(dfgt_lscv_score) against the oracle's exact FP64 sums and derivatives.

Scales used by the tolerances (q a query, G = G(q), h the bandwidth):
  * dG/dh and dG/dq are compared in units of G / h, the size of either
    derivative when the contributing references sit at distance ~h;
  * for eps = 0 (every leaf pair exhaustive) the derivatives are the exact
    sums up to the leaf-sum rounding: relative 1e-5 in mixed precision (FP32
    exp and partial sums over <= 64 terms), 1e-10 in FP64; dG/dq is measured
    against sqrt(G h^3 dG/dh) / h^2 >= |sum_j K_j (q - r_j)| / h^2
    (Cauchy-Schwarz), the natural size of a signed sum, plus the rounding
    floor of the FP64 scaled differences (1e-13 G |q| / h^2);
  * for eps > 0 the derivatives are held to eps relative in their own units:
    |dG~/dh - dG/dh| <= eps dG/dh, and |dG~/dq - dG/dq| <= eps h^-2 sum_j K_j
    |q - r_j| (the sum of the norms of dG/dq's terms, oracle.naive_kde_qscale);
    with the rounding floor of mixed precision (1e-5 relative) below that.
LSCV: each S(h) = sum_i (G(x_i) - 1) has |S~ - S| <= eps (S + N), which bounds
the score error; dcv/dh is compared against the oracle's analytic derivative
in units of the sum of the absolute values of its terms."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth
from tests.gpu_util import cuda, note

pytestmark = pytest.mark.gpu

EXACT_TOL = {0: 1e-5, 1: 1e-10}
HSTAR = os.path.join(os.path.dirname(__file__), "golden", "hstar.json")


@pytest.fixture(scope="module")
def dfgt():
    from paper_1102_2878_amd import dfgt as m
    return m


def _grad(dfgt, x, q, hs, eps, precision=0, force=0, leaf=32):
    R = dfgt.build_tree(cuda(x), leaf_size=leaf)
    Q = R if q is None else dfgt.build_tree(cuda(q), leaf_size=leaf)
    G, Gh, Gq, st = dfgt.gauss_sum_grad(Q, R, hs, eps, precision=precision, force_method=force, stats=True)
    return G.cpu().numpy(), Gh.cpu().numpy(), Gq.cpu().numpy(), st


def _check(x, q, hs, G, Gh, Gq, eps, precision, what):
    qq = x if q is None else q
    worst = {}
    for k, h in enumerate(hs):
        g, gh, gq = oracle.naive_kde_grad(qq, x, h)
        relG = np.abs(G[k] - g) / g
        assert relG.max() <= max(eps, EXACT_TOL[precision]), (what, h, relG.max())
        eh = np.abs(Gh[k] - gh)
        eq = np.linalg.norm(Gq[k] - gq, axis=1)
        if eps == 0.0:
            tol = EXACT_TOL[precision]
            sq = np.sqrt(np.maximum(g * gh * h ** 3, 0.0)) / h ** 2
            # floor: the scaled difference s q - s r of a (near-)coincident pair
            # is exact only to ~2^-53 |s q|, i.e. dG/dq to ~1e-16 G |q| / h^2
            floor = 1e-13 * g * np.max(np.abs(qq), axis=1) / h ** 2
            assert np.all(eh <= tol * gh + 1e-300), (what, h, np.max(eh / gh))
            assert np.all(eq <= tol * sq + floor), (what, h, np.max(eq / (sq + floor / tol)))
        else:
            tol = max(eps, EXACT_TOL[precision])
            qs = oracle.naive_kde_qscale(qq, x, h)
            worst[h] = (float(np.max(eh / gh)), float(np.max(eq / qs)))
            assert np.all(eh <= tol * gh), (what, h, np.max(eh / gh) / eps)
            assert np.all(eq <= tol * qs), (what, h, np.max(eq / qs) / eps)
    return worst


@pytest.mark.parametrize("precision", [0, 1])
def test_grad_exhaustive_is_exact(dfgt, precision):
    x = synth.c1()
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    note(f"grad c1 eps=0 precision={precision}")
    G, Gh, Gq, st = _grad(dfgt, x, None, hs, 0.0, precision)
    _check(x, None, hs, G, Gh, Gq, 0.0, precision, "eps=0")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_grad_c1(dfgt, precision, eps):
    x = synth.c1()
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    note(f"grad c1 eps={eps} precision={precision}")
    G, Gh, Gq, st = _grad(dfgt, x, None, hs, eps, precision)
    assert st["prune_centroid"] == 0  # the centroid form is not used in gradient mode
    _check(x, None, hs, G, Gh, Gq, eps, precision, "c1")


def test_grad_bichromatic_3d(dfgt):
    x = synth.c3(n=4000, seed=31)[:, :3].copy()
    q = synth.bichromatic_queries(x, 77)[:1500]
    hs = [synth.silverman_h(x) * s for s in (0.3, 1.0, 3.0)]
    note("grad bichromatic d3 eps=1e-3")
    G, Gh, Gq, st = _grad(dfgt, x, q, hs, 1e-3, 0)
    _check(x, q, hs, G, Gh, Gq, 1e-3, 0, "bichromatic")


@pytest.mark.parametrize("force", [1, 2, 3])
def test_grad_forced_methods(dfgt, force):
    """Each summarisation method alone: F, D and T derivatives."""
    x = synth.c1()
    hs = [synth.silverman_h(x) * s for s in (0.3, 1.0, 10.0)]
    note(f"grad c1 force={force}")
    G, Gh, Gq, st = _grad(dfgt, x, None, hs, 1e-3, 1, force=force)
    assert st["prune_f"] + st["prune_d"] + st["prune_t"] > 0
    _check(x, None, hs, G, Gh, Gq, 1e-3, 1, f"force={force}")


@pytest.mark.parametrize("force", [0, 1, 2, 3])
def test_grad_is_derivative_of_the_approximation(dfgt, force):
    """Central difference of the FP64 approximation itself at h (1 +- 1e-6):
    the traversal takes the same decisions at both ends (checked through its
    counters), so the difference quotient must match the analytic derivative
    of the approximation to ~1e-9 of G / h."""
    x = synth.c1()
    h = synth.silverman_h(x)
    dh = 1e-6 * h
    note(f"grad fd force={force}")
    R = dfgt.build_tree(cuda(x))
    # the gradient-mode traversal is what is differentiated: difference the
    # values it returns, through dfgt_gauss_sum_grad at h +- dh
    Gp, _, _, sp = dfgt.gauss_sum_grad(R, R, [h + dh], 1e-3, dq=False, precision=1, force_method=force, stats=True)
    Gm, _, _, sm = dfgt.gauss_sum_grad(R, R, [h - dh], 1e-3, dq=False, precision=1, force_method=force, stats=True)
    G, Gh, _ = dfgt.gauss_sum_grad(R, R, [h], 1e-3, dq=False, precision=1, force_method=force)
    keys = ("node_pairs", "prune_f", "prune_d", "prune_t", "max_order", "base_point_pairs")
    assert all(sp[k] == sm[k] for k in keys), (sp, sm)
    fd = ((Gp - Gm) / (2 * dh)).cpu().numpy()[0]
    unit = G.cpu().numpy()[0] / h
    err = np.abs(fd - Gh.cpu().numpy()[0]) / unit
    assert err.max() <= 1e-7, err.max()


def test_grad_deterministic(dfgt):
    x = synth.c2(n=5000, seed=23)
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0)]
    R = dfgt.build_tree(cuda(x))
    note("grad determinism")
    a = dfgt.gauss_sum_grad(R, R, hs, 1e-2)
    b = dfgt.gauss_sum_grad(R, R, hs, 1e-2)
    for u, v in zip(a, b):
        assert u.cpu().numpy().tobytes() == v.cpu().numpy().tobytes()


def test_backward_matches_oracle_vjp(dfgt):
    x = synth.c1()
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    eps = 1e-4
    R = dfgt.build_tree(cuda(x))
    w = np.random.default_rng(5).standard_normal((len(hs), x.shape[0]))
    note("backward c1")
    dh, dq = dfgt.gauss_sum_backward(R, R, hs, eps, cuda(w))
    dq = dq.cpu().numpy()
    dh_ref, dq_ref, bound_h, bound_q = np.zeros(len(hs)), np.zeros_like(x), np.zeros(len(hs)), np.zeros(x.shape[0])
    for k, h in enumerate(hs):
        g, gh, gq = oracle.naive_kde_grad(x, x, h)
        dh_ref[k] = np.sum(w[k] * gh)
        dq_ref += w[k][:, None] * gq
        # each query's derivatives hold to eps relative in their own units
        bound_h[k] = eps * np.sum(np.abs(w[k]) * gh)
        bound_q += eps * np.abs(w[k]) * oracle.naive_kde_qscale(x, x, h)
    assert np.all(np.abs(dh - dh_ref) <= bound_h), (dh, dh_ref, bound_h)
    assert np.all(np.linalg.norm(dq - dq_ref, axis=1) <= bound_q)


def test_autograd_function(dfgt):
    import torch

    from paper_1102_2878_amd.autograd import gauss_sum_fn

    x = synth.c1(n=1500, seed=7)
    hs = [synth.silverman_h(x) * s for s in (0.5, 2.0)]
    eps = 1e-4
    note("autograd c1")
    xq = cuda(x).requires_grad_(True)
    ht = torch.tensor(hs, dtype=torch.float64, requires_grad=True)
    G = gauss_sum_fn(xq, xq.detach(), ht, eps)
    w = np.random.default_rng(6).standard_normal(tuple(G.shape))
    (G * cuda(w)).sum().backward()
    dh_ref, dq_ref = np.zeros(len(hs)), np.zeros_like(x)
    bh, bq = np.zeros(len(hs)), np.zeros(x.shape[0])
    for k, h in enumerate(hs):
        g, gh, gq = oracle.naive_kde_grad(x, x, h)
        dh_ref[k] = np.sum(w[k] * gh)
        dq_ref += w[k][:, None] * gq
        bh[k] = eps * np.sum(np.abs(w[k]) * gh)
        bq += eps * np.abs(w[k]) * oracle.naive_kde_qscale(x, x, h)
        assert np.max(np.abs(G[k].detach().cpu().numpy() - g) / g) <= eps
    assert np.all(np.abs(ht.grad.numpy() - dh_ref) <= bh)
    assert np.all(np.linalg.norm(xq.grad.cpu().numpy() - dq_ref, axis=1) <= bq)
    with pytest.raises(NotImplementedError):
        gauss_sum_fn(xq, cuda(x).requires_grad_(True), ht, eps)


def test_autograd_backward_differentiates_its_forward(dfgt):
    """The autograd Function's backward is the exact derivative of the values
    its forward returned: central differences of gauss_sum_fn itself at
    h (1 +- 1e-6), FP64 leaf sums, match ht.grad to 1e-7 G / h (the inputs and
    tolerance of the gradient-mode difference test, whose traversal takes the
    same decisions at both ends)."""
    import torch

    from paper_1102_2878_amd.autograd import gauss_sum_fn

    x = synth.c1()
    h = synth.silverman_h(x)
    dh = 1e-6 * h
    xq = cuda(x)
    w = cuda(np.random.default_rng(8).standard_normal((1, x.shape[0])))
    note("autograd differences of its own forward")

    def fwd(hv):
        ht = torch.tensor([hv], dtype=torch.float64, requires_grad=True)
        return gauss_sum_fn(xq, xq, ht, 1e-3, precision=1), ht

    G, ht = fwd(h)
    (G * w).sum().backward()
    Gp, _ = fwd(h + dh)  # with grad enabled: the gradient-mode forward, as at h
    Gm, _ = fwd(h - dh)
    fd = float(((Gp.detach() - Gm.detach()) / (2 * dh) * w).sum())
    unit = float((G.detach().abs() * w.abs()).sum()) / h
    assert abs(fd - float(ht.grad[0])) <= 1e-7 * unit, (fd, float(ht.grad[0]), unit)


def _lscv_bounds(x, hs, eps, variant):
    """Each leave-one-out sum G(x_i) - 1 is within e of its own value (e = eps,
    or the 1e-5 leaf-sum rounding at eps = 0), so each S is within e S."""
    n, d = x.shape
    e = max(eps, 1e-5)
    out = []
    for h in hs:
        S1 = np.sum(oracle.naive_kde(x, x, h) - 1.0)
        S2 = np.sum(oracle.naive_kde(x, x, np.sqrt(2.0) * h) - 1.0)
        a = (4 * np.pi * h * h) ** (-d / 2)
        b = (2 * np.pi * h * h) ** (-d / 2)
        first = a / (n * n) if variant == 1 else a / (n * (n - 1))
        out.append(e * (first * S2 + 2 * b * S1 / (n * (n - 1))))
    return np.array(out)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-2])
def test_lscv_matches_oracle(dfgt, variant, eps):
    x = synth.c1()
    hs = np.array([synth.silverman_h(x) * s for s in (0.05, 0.2, 0.5, 1.0, 2.0)])
    R = dfgt.build_tree(cuda(x))
    note(f"lscv variant={variant} eps={eps}")
    cv, dcv = dfgt.lscv_score(R, hs, eps, variant=variant, grad=True)
    cvo, dcvo = oracle.lscv(x, hs, variant=variant)
    bound = _lscv_bounds(x, hs, eps, variant) + 1e-12 * np.abs(cvo)
    assert np.all(np.abs(cv - cvo) <= bound), (cv, cvo, bound)
    # dcv: sum of |terms| of the derivative as its scale
    n, d = x.shape
    scale = np.empty(len(hs))
    for i, h in enumerate(hs):
        _, gh1, _ = oracle.naive_kde_grad(x, x, h)
        _, gh2, _ = oracle.naive_kde_grad(x, x, np.sqrt(2.0) * h)
        S1 = np.sum(oracle.naive_kde(x, x, h) - 1.0)
        S2 = np.sum(oracle.naive_kde(x, x, np.sqrt(2.0) * h) - 1.0)
        a = (4 * np.pi * h * h) ** (-d / 2)
        b = (2 * np.pi * h * h) ** (-d / 2)
        scale[i] = (d / h * (a * (S2 + n) + 2 * b * (S1 + n)) + a * np.sqrt(2.0) * np.sum(gh2)
                    + 2 * b * np.sum(gh1)) / (n * (n - 1))
    tol = 4 * max(eps, 1e-5)
    assert np.all(np.abs(dcv - dcvo) <= tol * scale), (dcv, dcvo, np.abs(dcv - dcvo) / scale)


def test_lscv_minimum_near_hstar(dfgt):
    """The standard score (variant 1) on the 2,000-point mixture: its minimum
    over a grid bracketing h* lies next to h* from tests/golden/hstar.json."""
    import json
    import os

    x = synth.c1()
    hstar = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hstar.json")))["c1"]["h_star"]
    hs = hstar * np.geomspace(0.5, 2.0, 15)
    R = dfgt.build_tree(cuda(x))
    note("lscv grid near h*")
    cv, dcv = dfgt.lscv_score(R, hs, 1e-4, variant=1, grad=True)
    k = int(np.argmin(cv))
    assert 0 < k < len(hs) - 1
    assert hs[k - 1] <= hstar <= hs[k + 1]
    assert dcv[k - 1] <= 0.0 <= dcv[k + 1]


def _isolated_pairs(h0, seed):
    """Ten pairs of points far from everything else, partners rho h0 apart with
    rho from 6 to 30: at bandwidth h0 each leave-one-out sum is one term
    between e^-18 and e^-450 (below the FP32 range for most of them)."""
    rng = np.random.default_rng(seed)
    centres = np.stack(np.meshgrid(np.linspace(1.6, 2.4, 5), [1.7, 2.3]), axis=-1).reshape(-1, 2)
    rho = np.linspace(6.0, 30.0, 10) * h0
    ang = rng.uniform(0.0, 2.0 * np.pi, 10)
    off = 0.5 * rho[:, None] * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return np.concatenate([centres + off, centres - off])


@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-2])
def test_lcv_matches_oracle(dfgt, eps):
    """Likelihood cross-validation (dfgt_lcv_score) against the oracle's exact
    leave-one-out sums (summed over j != i).  The library's leave-one-out sums
    G - 1 are computed as such (the diagonal left out, the pruning tolerance
    scaled by a lower bound on G - 1), so each is within e of its own value
    (e = eps, or the 1e-5 leaf-sum rounding at eps = 0): each log term is
    within -log(1 - e), each derivative term G' / (G - 1) within
    2.02 e |G'| / (G - 1) (value and derivative each within e).  The data
    holds points at every degree of isolation, down to sums of e^-450 at the
    smallest bandwidth."""
    x = synth.c1()
    hS = synth.silverman_h(x)
    x = np.concatenate([x, _isolated_pairs(0.05 * hS, 12)])
    hs = np.array([hS * s for s in (0.05, 0.1, 0.5, 1.0, 3.0)])
    R = dfgt.build_tree(cuda(x))
    note(f"lcv eps={eps}")
    cv, dcv = dfgt.lcv_score(R, hs, eps, grad=True)
    cvo, dcvo = oracle.lcv(x, hs)
    e = max(eps, 1e-5)
    for k, h in enumerate(hs):
        assert np.isfinite(cvo[k]) and np.isfinite(cv[k]), (h, cv[k], cvo[k])
        bound = -np.log1p(-e)
        assert abs(cv[k] - cvo[k]) <= 1.01 * bound + 1e-12 * abs(cvo[k]), (h, cv[k], cvo[k], bound)
        # every G' >= 0, so sum_j |G'_j / (G_j - 1)| / N = dCV/dh + D / h
        dbound = 2.02 * e * (dcvo[k] + x.shape[1] / h)
        assert abs(dcv[k] - dcvo[k]) <= 1.01 * dbound + 1e-10 * abs(dcvo[k]), (h, dcv[k], dcvo[k], dbound)


def test_kde_density_matches_oracle(dfgt):
    x = synth.c1()
    q = synth.bichromatic_queries(x, 31)[:1500]
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    R = dfgt.build_tree(cuda(x))
    Q = dfgt.build_tree(cuda(q))
    note("kde density")
    p = dfgt.kde_density(Q, R, hs, 1e-2).cpu().numpy()
    for k, h in enumerate(hs):
        ref = oracle.kde_density(q, x, h)
        assert np.max(np.abs(p[k] - ref) / ref) <= 1e-2


@pytest.mark.parametrize("variant", [1, 0])
def test_lscv_optimize_finds_oracle_minimum(dfgt, variant):
    """dfgt_lscv_optimize over h_S [1e-2, 10] on the 2,000-point mixture: the
    bandwidth it returns scores, in the oracle's own exact LSCV, within 1e-4
    of the oracle's minimum (a golden-section search on the oracle's score);
    for the standard score it lies within 2% of h* of tests/golden/hstar.json.
    The reported score matches the oracle's at that bandwidth to the sums'
    error bound."""
    import json
    import os

    x = synth.c1()
    hS = synth.silverman_h(x)
    R = dfgt.build_tree(cuda(x))
    note(f"lscv optimize variant={variant}")
    lo, hi = 1e-2 * hS, 10.0 * hS
    h, cv, ne = dfgt.lscv_optimize(R, lo, hi, 1e-4, variant=variant, n_grid=16, rel_tol=1e-3)
    assert lo <= h <= hi and ne >= 16
    cvo = lambda v: float(oracle.lscv(x, [v], variant=variant)[0][0])
    # the oracle's minimiser near the returned point (golden section on log h,
    # inside the searched bracket)
    a, b = max(np.log(h) - 0.1, np.log(lo)), min(np.log(h) + 0.1, np.log(hi))
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = cvo(np.exp(c)), cvo(np.exp(d))
    while b - a > 1e-4:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = cvo(np.exp(c))
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = cvo(np.exp(d))
    best = min(fc, fd)
    assert cvo(h) - best <= 1e-4 * abs(best), (h, cvo(h), best)
    assert abs(cv - cvo(h)) <= _lscv_bounds(x, [h], 1e-4, variant)[0] + 1e-5 * abs(best)
    if variant == 1:
        hstar = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hstar.json")))["c1"]["h_star"]
        assert abs(h / hstar - 1.0) <= 0.02, (h, hstar)


@pytest.mark.parametrize("d", [8, 16, 20])
def test_grad_high_dimensions(dfgt, d):
    """Gradient mode with the matrix-core exhaustive tiles (their q-gradient
    product E^T X on the matrix cores too), against the oracle."""
    x = synth.c5(n=2500, seed=60 + d)
    if d != 16:
        rng = np.random.default_rng(d)
        x = x[:, :d] if d < 16 else np.hstack([x, 0.1 * rng.standard_normal((x.shape[0], d - 16))])
    x = np.ascontiguousarray(x)
    hs = [synth.silverman_h(x) * s for s in (1.0, 3.0)]
    note(f"grad high-d d={d}")
    G, Gh, Gq, st = _grad(dfgt, x, None, hs, 0.0, 0, leaf=48)
    _check(x, None, hs, G, Gh, Gq, 0.0, 0, f"d={d} eps=0")
    G, Gh, Gq, st = _grad(dfgt, x, None, hs, 1e-4, 0, leaf=48)
    _check(x, None, hs, G, Gh, Gq, 1e-4, 0, f"d={d} eps=1e-4")


def test_grad_16d_full_size_sampled(dfgt):
    """The differentiation workload at full size and in the bench's launch
    configuration: 200,000 points in 16-D (Q = R), eps 1e-4, leaf 128,
    bandwidths h_S and h* of the seeded 5,000-point sub-problem.  G, dG/dh and
    dG/dq of 1,000 seeded query rows, each against all 200,000 references,
    hold to 1e-4 relative in their own units (reading A31's query sample)."""
    x = synth.c5()
    hs = [synth.silverman_h(x), json.load(open(HSTAR))["c5_sub5k"]["h_star"]]
    rows = synth.subsample(x, 1000, 55)
    note("grad c5 200k d=16 eps=1e-4 leaf=128")
    R = dfgt.build_tree(cuda(x), leaf_size=128)
    G, Gh, Gq = dfgt.gauss_sum_grad(R, R, hs, 1e-4)
    import torch
    idx = torch.as_tensor(rows, device=G.device)
    G, Gh, Gq = G[:, idx].cpu().numpy(), Gh[:, idx].cpu().numpy(), Gq[:, idx].cpu().numpy()
    q = x[rows]
    for k, h in enumerate(hs):
        g, gh, gq = oracle.naive_kde_grad(q, x, h)
        qs = oracle.naive_kde_qscale(q, x, h)
        assert np.max(np.abs(G[k] - g) / g) <= 1e-4
        assert np.max(np.abs(Gh[k] - gh) / gh) <= 1e-4, np.max(np.abs(Gh[k] - gh) / gh)
        eq = np.linalg.norm(Gq[k] - gq, axis=1)
        assert np.max(eq / qs) <= 1e-4, np.max(eq / qs)
