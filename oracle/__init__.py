"""Plain FP64 CPU oracle for the Dual-Tree Fast Gauss Transform (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it, and the
two share no code: the arithmetic lives in ``dfgt_oracle.c`` (host C, FP64),
compiled by :mod:`oracle.build`.

Each wrapper names the passage of the paper it follows; see the C source for
the readings applied to garbled passages.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32P = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_I64P = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")

METHOD_E, METHOD_F, METHOD_D, METHOD_T = 0, 1, 2, 3
STATS = ("pairs", "prune_F", "prune_D", "prune_T", "prune_centroid", "base_cases", "base_pairs",
         "bound_violations", "max_order")


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("DFGT_ORACLE_LIB", _build.LIB)  # a mutated copy, for pin audits
        if path == _build.LIB and (not os.path.exists(path)
                                   or os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build(force=True)
        L = C.CDLL(path)
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.oracle_naive_kde.argtypes = [_DP, i64, _DP, i64, i32, dbl, _DP]
        L.oracle_naive_kde_rows.argtypes = [_DP, _I64P, i64, _DP, i64, i32, dbl, _DP]
        L.oracle_naive_kde_grad.argtypes = [_DP, i64, _DP, i64, i32, dbl, C.c_void_p, C.c_void_p,
                                            C.c_void_p]
        L.oracle_naive_kde_qscale.argtypes = [_DP, i64, _DP, i64, i32, dbl, _DP]
        L.oracle_naive_kde_weighted.argtypes = [_DP, i64, _DP, _DP, i64, i32, dbl, C.c_void_p, C.c_void_p,
                                                C.c_void_p]
        L.oracle_build_kdtree.argtypes = [_DP, i64, i32, i32, i64, _I32P, _DP, _DP, _I64P, _I64P,
                                          _I32P, _I32P, _I32P, _DP, C.POINTER(i64)]
        L.oracle_mi_to_pos.argtypes = [C.POINTER(C.c_int), i32, i32]
        L.oracle_mi_to_pos.restype = i64
        L.oracle_pos_to_mi.argtypes = [i64, i32, i32, C.POINTER(C.c_int)]
        L.oracle_mi_expansion.argtypes = [_DP, i32, i32, i32, _DP]
        L.oracle_hermite_table.argtypes = [_DP, i32, i32, _DP]
        L.oracle_p2m.argtypes = [_DP, i64, i32, _DP, dbl, i32, i32, _DP]
        L.oracle_f2f.argtypes = [_DP, _DP, _DP, i32, dbl, i32, _DP]
        L.oracle_far_eval.argtypes = [_DP, _DP, i32, dbl, i32, i32, _DP, i64, _DP]
        L.oracle_f2l.argtypes = [_DP, _DP, _DP, i32, dbl, i32, i32, _DP]
        L.oracle_direct_local.argtypes = [_DP, i64, _DP, i32, dbl, i32, i32, _DP]
        L.oracle_l2l.argtypes = [_DP, _DP, _DP, i32, dbl, i32, i32, _DP]
        L.oracle_local_eval.argtypes = [_DP, _DP, i32, dbl, i32, i32, _DP, i64, _DP]
        for nm in ("oracle_bound_far", "oracle_bound_local", "oracle_bound_f2l"):
            getattr(L, nm).argtypes = [dbl, i32, i32, dbl]
            getattr(L, nm).restype = dbl
        L.oracle_dist_bounds.argtypes = [_DP, _DP, _DP, _DP, i32, C.POINTER(dbl), C.POINTER(dbl)]
        L.oracle_far_field_order.argtypes = [dbl, dbl, i32, dbl, dbl, i32]
        L.oracle_local_order.argtypes = [dbl, dbl, i32, dbl, dbl, i32]
        L.oracle_f2l_order.argtypes = [dbl, dbl, dbl, i32, dbl, dbl, i32, i32]
        L.oracle_centroid_bound.argtypes = [dbl, dbl, dbl, dbl, dbl]
        L.oracle_centroid_bound.restype = dbl
        L.oracle_choose_method.argtypes = [_DP, _DP, _DP, _DP, i32, dbl, dbl, dbl, dbl, i32, i32,
                                           i32, C.POINTER(C.c_int)]
        L.oracle_dfgt.argtypes = [_DP, i64, _DP, i64, i32, dbl, dbl, i32, i32, i32, i32, C.c_void_p,
                                  _DP, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_lscv.argtypes = [_DP, i64, i32, _DP, i32, i32, _DP, C.c_void_p]
        L.oracle_lcv.argtypes = [_DP, i64, i32, _DP, i32, _DP, C.c_void_p]
        L.oracle_kde_density.argtypes = [_DP, i64, _DP, i64, i32, dbl, _DP]
        L.oracle_num_threads.restype = i32
        _lib = L
    return _lib


def _pts(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    return x


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# ---- Section 1.1 / Alg. NaiveKDE ------------------------------------------------------------
def naive_kde(q, r, h):
    """Exact G(q_i, R) = sum_j exp(-|q_i - r_j|^2 / 2h^2) (eq. gaussian_kernel_sums)."""
    q, r = _pts(q), _pts(r)
    out = np.empty(q.shape[0])
    _check(lib().oracle_naive_kde(q, q.shape[0], r, r.shape[0], q.shape[1], float(h), out), "naive_kde")
    return out


def naive_kde_rows(q, rows, r, h):
    """Exact sums for the query rows ``rows`` only (sampled checks at full size)."""
    q, r = _pts(q), _pts(r)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    _check(lib().oracle_naive_kde_rows(q, rows, rows.shape[0], r, r.shape[0], q.shape[1], float(h), out),
           "naive_kde_rows")
    return out


def naive_kde_grad(q, r, h):
    """(G, dG/dh, dG/dq) of the exact sum."""
    q, r = _pts(q), _pts(r)
    n, d = q.shape
    G = np.empty(n)
    gh = np.empty(n)
    gq = np.empty((n, d))
    _check(lib().oracle_naive_kde_grad(q, n, r, r.shape[0], d, float(h), _ptr(G), _ptr(gh), _ptr(gq)),
           "naive_kde_grad")
    return G, gh, gq


def naive_kde_qscale(q, r, h):
    """h^-2 sum_j K_j |q_i - r_j|: the sum of the norms of the terms of dG/dq
    (an upper bound on |dG/dq|, the unit of its relative error)."""
    q, r = _pts(q), _pts(r)
    out = np.empty(q.shape[0])
    _check(lib().oracle_naive_kde_qscale(q, q.shape[0], r, r.shape[0], q.shape[1], float(h), out),
           "naive_kde_qscale")
    return out


def naive_kde_weighted(q, r, w, h):
    """(G_w, dG_w/dh, dG_w/dq) of the exact weighted sum G_w(q) = sum_j w_j K(q, r_j)
    (the sums of Section 1 with a weight per reference point)."""
    q, r = _pts(q), _pts(r)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (r.shape[0],):
        raise ValueError("one weight per reference point")
    n, d = q.shape
    G = np.empty(n)
    gh = np.empty(n)
    gq = np.empty((n, d))
    _check(lib().oracle_naive_kde_weighted(q, n, r, w, r.shape[0], d, float(h), _ptr(G), _ptr(gh), _ptr(gq)),
           "naive_kde_weighted")
    return G, gh, gq


# ---- Section 2.1 / Alg. BuildKdTree -----------------------------------------------------------
def build_kdtree(x, leaf_size):
    """Mid-point kd-tree; nodes in pre-order.  Returns a dict of numpy arrays."""
    x = _pts(x)
    n, d = x.shape
    cap = 2 * n + 1
    perm = np.empty(n, np.int32)
    lo = np.empty(cap * d)
    hi = np.empty(cap * d)
    b = np.empty(cap, np.int64)
    e = np.empty(cap, np.int64)
    l = np.empty(cap, np.int32)
    r = np.empty(cap, np.int32)
    sd = np.empty(cap, np.int32)
    sc = np.empty(cap)
    m = C.c_int64(0)
    _check(lib().oracle_build_kdtree(x, n, d, int(leaf_size), cap, perm, lo, hi, b, e, l, r, sd, sc,
                                     C.byref(m)), "build_kdtree")
    m = m.value
    return dict(perm=perm, lo=lo[: m * d].reshape(m, d), hi=hi[: m * d].reshape(m, d), begin=b[:m],
                end=e[:m], left=l[:m], right=r[:m], split_dim=sd[:m], split_coord=sc[:m], n_nodes=m)


# ---- Section 3.1 / Appendix: multi-index layout, Hermite functions -----------------------------
def mi_to_pos(alpha, p):
    a = (C.c_int * len(alpha))(*[int(v) for v in alpha])
    return int(lib().oracle_mi_to_pos(a, len(alpha), int(p)))


def pos_to_mi(i, d, p):
    a = (C.c_int * d)()
    lib().oracle_pos_to_mi(int(i), d, int(p), a)
    return tuple(a)


def mi_expansion(x, p, pmax=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    d = x.shape[0]
    pmax = p if pmax is None else pmax
    out = np.zeros(pmax ** d)
    lib().oracle_mi_expansion(x, d, int(p), int(pmax), out)
    return out


def hermite_table(a, n):
    """H[k, m] = h_m(a[k]) for m < n (Appendix, ComputePartialDerivatives)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    H = np.zeros(a.shape[0] * n)
    lib().oracle_hermite_table(a, a.shape[0], int(n), H)
    return H.reshape(a.shape[0], n)


# ---- Sections 3.3, 3.4, 3.7 / Appendix: moments and operators -----------------------------------
def p2m(pts, center, h, p, pmax=None):
    """Far-field moments M_alpha(R, c), alpha < p (eq. far_field_moments)."""
    pts = _pts(pts)
    d = pts.shape[1]
    pmax = p if pmax is None else pmax
    M = np.zeros(pmax ** d)
    _check(lib().oracle_p2m(pts, pts.shape[0], d, np.ascontiguousarray(center, np.float64), float(h),
                            int(p), int(pmax), M), "p2m")
    return M


def f2f(Mc, cc, cp, h, pmax, Mp=None):
    """Shift child moments (about cc) to cp and add into Mp (eq. far_to_far_translation)."""
    d = len(cc)
    Mp = np.zeros(pmax ** d) if Mp is None else Mp
    _check(lib().oracle_f2f(np.ascontiguousarray(Mc, np.float64), np.ascontiguousarray(cc, np.float64),
                            np.ascontiguousarray(cp, np.float64), d, float(h), int(pmax), Mp), "f2f")
    return Mp


def far_eval(M, center, h, p, pmax, q):
    """sum_{alpha < p} M_alpha h_alpha((q - c) s) at each query (EvalFarFieldExpansion)."""
    q = _pts(q)
    out = np.zeros(q.shape[0])
    _check(lib().oracle_far_eval(np.ascontiguousarray(M, np.float64), np.ascontiguousarray(center, np.float64),
                                 q.shape[1], float(h), int(p), int(pmax), q, q.shape[0], out), "far_eval")
    return out


def f2l(M, cr, cq, h, p, pmax, L=None):
    """Far-field (about cr) to local (about cq) (eq. farfield_to_local_formula)."""
    d = len(cr)
    L = np.zeros(pmax ** d) if L is None else L
    _check(lib().oracle_f2l(np.ascontiguousarray(M, np.float64), np.ascontiguousarray(cr, np.float64),
                            np.ascontiguousarray(cq, np.float64), d, float(h), int(p), int(pmax), L), "f2l")
    return L


def direct_local(pts, cq, h, p, pmax, L=None):
    """Direct local moments of pts about cq (eq. local_moments)."""
    pts = _pts(pts)
    d = pts.shape[1]
    L = np.zeros(pmax ** d) if L is None else L
    _check(lib().oracle_direct_local(pts, pts.shape[0], np.ascontiguousarray(cq, np.float64), d, float(h),
                                     int(p), int(pmax), L), "direct_local")
    return L


def l2l(Lp, cp, cc, h, p, pmax, Lc=None):
    """Shift a local expansion from cp to cc and add into Lc (eq. local_to_local_translation)."""
    d = len(cp)
    Lc = np.zeros(pmax ** d) if Lc is None else Lc
    _check(lib().oracle_l2l(np.ascontiguousarray(Lp, np.float64), np.ascontiguousarray(cp, np.float64),
                            np.ascontiguousarray(cc, np.float64), d, float(h), int(p), int(pmax), Lc), "l2l")
    return Lc


def local_eval(L, center, h, p, pmax, q):
    """sum_{beta < p} L_beta ((q - c) s)^beta at each query (EvalLocalExpansion)."""
    q = _pts(q)
    out = np.zeros(q.shape[0])
    _check(lib().oracle_local_eval(np.ascontiguousarray(L, np.float64), np.ascontiguousarray(center, np.float64),
                                   q.shape[1], float(h), int(p), int(pmax), q, q.shape[0], out), "local_eval")
    return out


# ---- Sections 2.2, 3.5, 3.6, 3.8: bounds, orders, method choice ---------------------------------
def bound_far(r, p, d, nR):
    return float(lib().oracle_bound_far(float(r), int(p), int(d), float(nR)))


def bound_local(r, p, d, nR):
    return float(lib().oracle_bound_local(float(r), int(p), int(d), float(nR)))


def bound_f2l(r, p, d, nR):
    return float(lib().oracle_bound_f2l(float(r), int(p), int(d), float(nR)))


def dist_bounds(qlo, qhi, rlo, rhi):
    dl, du = C.c_double(), C.c_double()
    a = [np.ascontiguousarray(v, np.float64) for v in (qlo, qhi, rlo, rhi)]
    lib().oracle_dist_bounds(*a, len(a[0]), C.byref(dl), C.byref(du))
    return dl.value, du.value


def far_field_order(wR, h, d, nR, tau, pmax):
    return int(lib().oracle_far_field_order(float(wR), float(h), int(d), float(nR), float(tau), int(pmax)))


def local_order(wQ, h, d, nR, tau, pmax):
    return int(lib().oracle_local_order(float(wQ), float(h), int(d), float(nR), float(tau), int(pmax)))


def f2l_order(wQ, wR, h, d, nR, tau, pmax, literal=False):
    return int(lib().oracle_f2l_order(float(wQ), float(wR), float(h), int(d), float(nR), float(tau),
                                      int(pmax), int(bool(literal))))


def centroid_bound(dl, du, dc, h, nR):
    return float(lib().oracle_centroid_bound(float(dl), float(du), float(dc), float(h), float(nR)))


def choose_method(qlo, qhi, rlo, rhi, nQ, nR, h, tau, pmax, force=0, literal_f2l=False):
    """(method, order) from ChooseBestMethod; method 0=E, 1=F, 2=D, 3=T."""
    a = [np.ascontiguousarray(v, np.float64) for v in (qlo, qhi, rlo, rhi)]
    order = C.c_int(0)
    m = lib().oracle_choose_method(*a, len(a[0]), float(nQ), float(nR), float(h), float(tau), int(pmax),
                                   int(force), int(bool(literal_f2l)), C.byref(order))
    return int(m), order.value


# ---- Section 3.9: DFGTMain ---------------------------------------------------------------------
def default_pmax(d):
    """p_max per dimension as fixed for the paper's experiments (Section 3.9)."""
    return {1: 6, 2: 6, 3: 4, 4: 2, 5: 2}.get(d, 1)


def dfgt(q, r, h, eps, leaf_size=32, pmax=None, force=0, literal_f2l=False, G_exact=None):
    """Recursive DFGT in the paper's order.  Returns (G~, info dict)."""
    q, r = _pts(q), _pts(r)
    nq, d = q.shape
    pmax = default_pmax(d) if pmax is None else pmax
    G = np.empty(nq)
    gl = np.empty(nq)
    gu = np.empty(nq)
    cov = np.empty(nq, np.int64)
    st = np.zeros(16, np.int64)
    gx = None if G_exact is None else np.ascontiguousarray(G_exact, np.float64)
    _check(lib().oracle_dfgt(q, nq, r, r.shape[0], d, float(h), float(eps), int(leaf_size), int(pmax),
                             int(force), int(bool(literal_f2l)), _ptr(gx), G, _ptr(gl), _ptr(gu), _ptr(cov),
                             _ptr(st)), "dfgt")
    info = dict(zip(STATS, st[: len(STATS)].tolist()))
    info.update(G_lower=gl, G_upper=gu, coverage=cov)
    return G, info


# ---- Section 1, eq. (4) -------------------------------------------------------------------------
def kde_density(q, r, h):
    """Section 1 density estimate p_h(q) = G(q, R) / (|R| (2 pi h^2)^{D/2})."""
    q, r = _pts(q), _pts(r)
    out = np.empty(q.shape[0])
    _check(lib().oracle_kde_density(q, q.shape[0], r, r.shape[0], q.shape[1], float(h), out), "kde_density")
    return out


def lcv(x, hs):
    """(CV_LK(h), dCV_LK/dh) for each h: Section 1 likelihood cross-validation."""
    x = _pts(x)
    hs = np.ascontiguousarray(np.atleast_1d(hs), np.float64)
    cv = np.empty(hs.shape[0])
    dcv = np.empty(hs.shape[0])
    _check(lib().oracle_lcv(x, x.shape[0], x.shape[1], hs, hs.shape[0], cv, _ptr(dcv)), "lcv")
    return cv, dcv


def lscv(x, hs, variant=0):
    """(CV_LS(h), dCV/dh) for each h, from exact sums at h and sqrt(2) h."""
    x = _pts(x)
    hs = np.ascontiguousarray(np.atleast_1d(hs), np.float64)
    cv = np.empty(hs.shape[0])
    dcv = np.empty(hs.shape[0])
    _check(lib().oracle_lscv(x, x.shape[0], x.shape[1], hs, hs.shape[0], int(variant), cv, _ptr(dcv)), "lscv")
    return cv, dcv
