"""GPU test of dfgt_naive_sum_noalloc, the brute-force sums (Alg. NaiveKDE,
Section 1) with every buffer in the library's fixed device region: called
through the C ABI twice in a row (the second call smaller, so it runs over
what the first left in the region) and compared with dfgt_naive_sum on the
same inputs.  With the same reference chunking both give the same bits; when
the region forces fewer chunks, the sums are the same terms added in another
grouping, and both stay within the mixed-precision rounding (1e-5 relative,
plus the flush floor N_R 2^-126) of the oracle's exact sums."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1102_2878_amd import synth
from tests.gpu_util import cuda, note

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def dfgt():
    from paper_1102_2878_amd import dfgt as m
    return m


def _noalloc(dfgt, q, r, hs, precision):
    import torch
    L = dfgt.lib()
    hv = np.ascontiguousarray(hs, dtype=np.float64)
    out = torch.full((len(hs), q.shape[0]), -1.0, dtype=torch.float64, device=q.device)
    rc = L.dfgt_naive_sum_noalloc(C.c_void_p(q.data_ptr()), q.shape[0], C.c_void_p(r.data_ptr()), r.shape[0],
                                  q.shape[1], hv.ctypes.data_as(C.POINTER(C.c_double)), len(hs), precision,
                                  C.c_void_p(out.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def _case(dfgt, x, rx, hs, precision, bitwise, rows=64):
    q, r = cuda(x), cuda(rx)
    rc, got = _noalloc(dfgt, q, r, hs, precision)
    assert rc == 0, dfgt.lib().dfgt_last_error()
    ref = dfgt.naive_sum(q, r, hs, precision=precision)
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    if bitwise:
        assert got.tobytes() == ref.tobytes()
    tol = 1e-12 if precision == 1 else MIXED_TOL
    floor = rx.shape[0] * 2.0 ** -126
    np.testing.assert_array_less(np.abs(got - ref), 2 * tol * np.abs(ref) + 2 * floor)
    idx = synth.subsample(x, rows, 7)
    for k, h in enumerate(hs):
        ex = oracle.naive_kde_rows(x, idx, rx, h)
        assert np.all(np.abs(got[k][idx] - ex) <= tol * ex + floor), (precision, h)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_2d_two_calls_second_smaller(dfgt, precision):
    x = synth.c2(n=20000, seed=81)
    hs = [synth.silverman_h(x) * s for s in (0.1, 1.0, 10.0)]
    note(f"noalloc 2-D 20000 x 20000 precision={precision}")
    _case(dfgt, x, x, hs, precision, bitwise=True)
    xs = np.ascontiguousarray(x[:3001])
    note(f"noalloc 2-D 3001 x 5003 precision={precision}")
    _case(dfgt, xs, np.ascontiguousarray(x[:5003]), hs[:2], precision, bitwise=True)


def test_noalloc_16d_matrix_cores_two_calls(dfgt):
    x = synth.c5(n=6000, seed=82)
    hs = [synth.silverman_h(x) * s for s in (0.5, 2.0)]
    note("noalloc 16-D 6000 x 6000 (matrix-core form)")
    _case(dfgt, x, x, hs, 0, bitwise=True)
    note("noalloc 16-D 1000 x 1500")
    _case(dfgt, np.ascontiguousarray(x[:1000]), np.ascontiguousarray(x[:1500]), hs[1:], 0, bitwise=True)


def test_noalloc_fewer_chunks_when_the_region_is_full(dfgt):
    """7.5M references leave room for fewer chunk partials than the allocating
    form uses: the same sums in a coarser grouping, then a small call."""
    rng = np.random.default_rng(83)
    rx = rng.uniform(0.0, 1.0, size=(7_500_000, 2))
    x = np.ascontiguousarray(rx[:10000])
    hs = [0.001, 0.01, 0.1, 1.0]
    note("noalloc 2-D 10000 x 7.5M")
    _case(dfgt, x, rx, hs, 0, bitwise=False, rows=24)
    note("noalloc 2-D 500 x 800 after it")
    _case(dfgt, np.ascontiguousarray(x[:500]), np.ascontiguousarray(rx[:800]), hs, 0, bitwise=True)


def test_noalloc_rejects_what_does_not_fit(dfgt):
    import torch
    note("noalloc rejection (no device work)")
    q = torch.zeros((4_000_000, 1), dtype=torch.float64, device="cuda")
    r = torch.zeros((5_000_000, 1), dtype=torch.float64, device="cuda")
    rc, _ = _noalloc(dfgt, q, r, [0.1], 0)
    assert rc == 1 and b"scratch region" in dfgt.lib().dfgt_last_error()
    rc, _ = _noalloc(dfgt, q[:10], r[:10], [-1.0], 0)
    assert rc == 1 and b"bandwidths" in dfgt.lib().dfgt_last_error()
