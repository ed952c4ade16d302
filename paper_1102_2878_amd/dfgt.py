"""Thin Python binding of libdfgt.so (the C ABI in include/dfgt.h).

Argument marshalling only: every computation runs in the HIP library.  Device
buffers are torch CUDA tensors (ROCm); work is enqueued on torch's current
stream.  The library must have been built (``__graft_entry__.build()`` or
``python paper_1102_2878_amd/build.py``); a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfgt.so")

PREC_MIXED, PREC_FP64 = 0, 1
FORCE_NONE, FORCE_F, FORCE_D, FORCE_T, FORCE_CENTROID, FORCE_EXACT = range(6)


class DfgtError(RuntimeError):
    pass


class Options(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("p_max", C.c_int32), ("precision", C.c_int32),
                ("force_method", C.c_int32), ("profile", C.c_int32), ("cost_exhaustive", C.c_float),
                ("reserved", C.c_int32 * 2)]


class Stats(C.Structure):
    _fields_ = [(nm, C.c_int64) for nm in (
        "node_pairs", "prune_f", "prune_d", "prune_t", "prune_centroid", "base_leaf_pairs",
        "base_point_pairs", "levels", "max_order", "fp64_groups", "segments", "max_segment", "local_nodes",
        "max_local_ops", "mfma_tiles", "parts", "work_f", "work_d", "work_t")] + [("e_items", C.c_int64 * 6),
                                                                       ("e_pairs", C.c_int64 * 2),
                                                                       ("kernel_ms", C.c_double * 6),
                                                                       ("kernel_launches", C.c_int64 * 6)]
    KERNELS = ("traverse", "leaf", "etile", "local", "etile_fp64", "etile_mx32")

    def as_dict(self):
        d = {nm: int(getattr(self, nm)) for nm, _ in self._fields_ if nm not in ("reserved", "kernel_ms",
                                                                                 "kernel_launches", "e_items",
                                                                                 "e_pairs")}
        d["e_pairs"] = {"fp32": int(self.e_pairs[0]), "fp64": int(self.e_pairs[1])}
        d["e_items"] = dict(zip(("heavy", "short", "none", "wide", "heavy_fp64", "short_fp64"),
                                [int(v) for v in self.e_items]))
        d["kernel_ms"] = dict(zip(self.KERNELS, list(self.kernel_ms)))
        d["kernel_launches"] = dict(zip(self.KERNELS, [int(v) for v in self.kernel_launches]))
        return d


class Problem(C.Structure):
    _fields_ = [("Q", C.c_void_p), ("R", C.c_void_p), ("h_host", C.POINTER(C.c_double)), ("n_h", C.c_int32),
                ("G_dev", C.c_void_p)]


_lib = None


def lib():
    """Loads libdfgt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DfgtError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.dfgt_last_error.restype = C.c_char_p
        L.dfgt_version.restype = C.c_char_p
        L.dfgt_build_tree.argtypes = [vp, i64, i32, C.POINTER(Options), vp, C.POINTER(vp)]
        L.dfgt_build_tree_weighted.argtypes = [vp, vp, i64, i32, C.POINTER(Options), vp, C.POINTER(vp)]
        L.dfgt_tree_free.argtypes = [vp]
        L.dfgt_tree_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64), C.POINTER(i32),
                                     C.POINTER(i32)]
        L.dfgt_tree_export.argtypes = [vp] + [vp] * 9
        L.dfgt_tree_moments.argtypes = [vp, vp]
        L.dfgt_tree_perm.argtypes = [vp, vp, vp]
        L.dfgt_set_allocator.argtypes = [vp, vp, vp]
        L.dfgt_release_workspace.argtypes = []
        L.dfgt_naive_sum.argtypes = [vp, i64, vp, i64, i32, C.POINTER(dbl), i32, i32, vp, vp]
        L.dfgt_naive_sum_noalloc.argtypes = [vp, i64, vp, i64, i32, C.POINTER(dbl), i32, i32, vp, vp]
        L.dfgt_gauss_sum.argtypes = [vp, vp, C.POINTER(dbl), i32, dbl, C.POINTER(Options), vp,
                                     C.POINTER(Stats), vp]
        L.dfgt_gauss_sum_grad.argtypes = [vp, vp, C.POINTER(dbl), i32, dbl, C.POINTER(Options), vp, vp, vp,
                                          C.POINTER(Stats), vp]
        L.dfgt_gauss_sum_backward.argtypes = [vp, vp, C.POINTER(dbl), i32, dbl, C.POINTER(Options), vp,
                                              C.POINTER(dbl), vp, vp]
        L.dfgt_gauss_sum_vjp.argtypes = [i32, i64, i32, vp, vp, vp, C.POINTER(dbl), vp, vp]
        L.dfgt_lscv_score.argtypes = [vp, C.POINTER(dbl), i32, dbl, i32, C.POINTER(Options), C.POINTER(dbl),
                                      C.POINTER(dbl), C.POINTER(Stats), vp]
        L.dfgt_kde_density.argtypes = [vp, vp, C.POINTER(dbl), i32, dbl, C.POINTER(Options), vp, C.POINTER(Stats),
                                       vp]
        L.dfgt_lcv_score.argtypes = [vp, C.POINTER(dbl), i32, dbl, C.POINTER(Options), C.POINTER(dbl),
                                     C.POINTER(dbl), C.POINTER(Stats), vp]
        L.dfgt_lscv_optimize.argtypes = [vp, dbl, dbl, dbl, i32, i32, dbl, C.POINTER(Options), C.POINTER(dbl),
                                         C.POINTER(dbl), C.POINTER(i32), vp]
        L.dfgt_tune_leaf_size.argtypes = [vp, i64, i32, C.POINTER(dbl), i32, dbl, C.POINTER(Options), i32, vp,
                                          C.POINTER(i32), C.POINTER(dbl)]
        L.dfgt_gauss_sum_batched.argtypes = [C.POINTER(Problem), i32, dbl, C.POINTER(Options), C.POINTER(Stats), vp]
        L.dfgt_batch_create.argtypes = [C.POINTER(Problem), i32, dbl, C.POINTER(Options), C.POINTER(Stats), vp,
                                        C.POINTER(vp)]
        L.dfgt_batch_run.argtypes = [vp, vp]
        L.dfgt_batch_check.argtypes = [vp, vp]
        L.dfgt_batch_free.argtypes = [vp]
        for nm in ("dfgt_build_tree", "dfgt_build_tree_weighted", "dfgt_tree_free", "dfgt_tree_info", "dfgt_tree_export",
                   "dfgt_tree_moments", "dfgt_tree_perm", "dfgt_set_allocator", "dfgt_release_workspace",
                   "dfgt_naive_sum", "dfgt_naive_sum_noalloc", "dfgt_gauss_sum", "dfgt_gauss_sum_grad",
                   "dfgt_gauss_sum_backward", "dfgt_gauss_sum_vjp", "dfgt_lscv_score", "dfgt_lscv_optimize", "dfgt_gauss_sum_batched",
                   "dfgt_kde_density", "dfgt_lcv_score",
                   "dfgt_batch_create",
                   "dfgt_batch_run", "dfgt_batch_check", "dfgt_batch_free"):
            getattr(L, nm).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise DfgtError(f"libdfgt error {rc}: {lib().dfgt_last_error().decode()}")


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_points(x):
    torch = _torch()
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise DfgtError("points must be a CUDA (HIP) torch tensor")
    if x.dtype != torch.float64 or x.dim() != 2:
        raise DfgtError("points must be a 2-D float64 tensor")
    return x.contiguous()


def _hvec(h):
    h = np.ascontiguousarray(np.atleast_1d(np.asarray(h, dtype=np.float64)))
    return h, h.ctypes.data_as(C.POINTER(C.c_double))


def _opts(leaf_size=0, p_max=0, precision=PREC_MIXED, force_method=FORCE_NONE, profile=False, cost_exhaustive=0.0):
    o = Options()
    o.leaf_size, o.p_max, o.precision, o.force_method = int(leaf_size), int(p_max), int(precision), int(force_method)
    o.profile = int(bool(profile))
    o.cost_exhaustive = float(cost_exhaustive)
    return o


class Tree:
    """Owns a dfgt_tree handle."""

    def __init__(self, handle, n, d):
        self.handle = handle
        self.n, self.d = n, d

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.dfgt_tree_free(h)
            self.handle = None

    def info(self):
        return tree_info(self)


def build_tree(points, leaf_size=0, p_max=0, precision=PREC_MIXED, force_method=FORCE_NONE,
               weights=None) -> Tree:
    """dfgt_build_tree: kd-tree (+ raw moments) of an (n, d) float64 CUDA tensor.

    weights: an (n,) float64 CUDA tensor of point weights >= 0 (dfgt_build_tree_weighted):
    sums over this tree as the reference set are then sum_j w_j K(q, r_j)."""
    x = _dev_points(points)
    o = _opts(leaf_size, p_max, precision, force_method)
    h = C.c_void_p()
    if weights is None:
        _check(lib().dfgt_build_tree(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], C.byref(o), _stream(),
                                     C.byref(h)))
        return Tree(h, x.shape[0], x.shape[1])
    torch = _torch()
    if not (isinstance(weights, torch.Tensor) and weights.is_cuda and weights.dtype == torch.float64
            and weights.dim() == 1 and weights.shape[0] == x.shape[0]):
        raise DfgtError("weights must be an (n,) float64 CUDA (HIP) tensor")
    w = weights.contiguous()
    _check(lib().dfgt_build_tree_weighted(C.c_void_p(x.data_ptr()), C.c_void_p(w.data_ptr()), x.shape[0],
                                          x.shape[1], C.byref(o), _stream(), C.byref(h)))
    return Tree(h, x.shape[0], x.shape[1])


def tree_info(t: Tree):
    n, d, m, dep, pm = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()
    _check(lib().dfgt_tree_info(t.handle, C.byref(n), C.byref(d), C.byref(m), C.byref(dep), C.byref(pm)))
    return dict(n=n.value, d=d.value, n_nodes=m.value, depth=dep.value, p_max=pm.value)


def tree_export(t: Tree):
    """dfgt_tree_export: host copies of the breadth-first node arrays and the permutation."""
    info = tree_info(t)
    n, d, m = info["n"], info["d"], info["n_nodes"]
    out = dict(perm=np.empty(n, np.int32), lo=np.empty((m, d)), hi=np.empty((m, d)),
               begin=np.empty(m, np.int32), end=np.empty(m, np.int32), left=np.empty(m, np.int32),
               right=np.empty(m, np.int32), split_dim=np.empty(m, np.int32), split_coord=np.empty(m))
    order = ("perm", "lo", "hi", "begin", "end", "left", "right", "split_dim", "split_coord")
    _check(lib().dfgt_tree_export(t.handle, *[out[k].ctypes.data_as(C.c_void_p) for k in order]))
    out["n_nodes"] = m
    return out


def tree_perm(t: Tree):
    """dfgt_tree_perm: the permutation as an (n,) int32 CUDA tensor (tree position -> caller index)."""
    torch = _torch()
    out = torch.empty(t.n, dtype=torch.int32, device="cuda")
    _check(lib().dfgt_tree_perm(t.handle, C.c_void_p(out.data_ptr()), _stream()))
    return out


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
_hooks = None


def use_torch_allocator(on=True):
    """dfgt_set_allocator with torch's caching allocator (on the current stream at
    allocation time), or back to hipMalloc (on=False).  The library's workspaces
    are released first, so no buffer outlives the allocator that made it; at
    interpreter exit they are released and the hook removed."""
    global _hooks
    import atexit
    torch = _torch()
    _check(lib().dfgt_release_workspace())
    if not on:
        _check(lib().dfgt_set_allocator(None, None, None))
        _hooks = None
        return

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=torch.cuda.current_stream())
        except Exception:
            return None

    def _free(ptr, nbytes, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))  # kept alive as long as the library may call them
    _check(lib().dfgt_set_allocator(C.cast(hooks[0], C.c_void_p), C.cast(hooks[1], C.c_void_p), None))
    if _hooks is None:
        atexit.register(lambda: use_torch_allocator(False) if _hooks is not None else None)
    _hooks = hooks


def tree_moments(t: Tree):
    """dfgt_tree_moments: raw moments, (n_nodes, p_max^d) float64 host array."""
    info = tree_info(t)
    mu = np.empty((info["n_nodes"], info["p_max"] ** info["d"]))
    _check(lib().dfgt_tree_moments(t.handle, mu.ctypes.data_as(C.c_void_p)))
    return mu


def naive_sum(q, r, h, precision=PREC_MIXED, out=None):
    """dfgt_naive_sum: brute-force sums, returns an (n_h, nq) float64 CUDA tensor."""
    torch = _torch()
    q, r = _dev_points(q), _dev_points(r)
    hv, hp = _hvec(h)
    if out is None:
        out = torch.empty((hv.shape[0], q.shape[0]), dtype=torch.float64, device=q.device)
    _check(lib().dfgt_naive_sum(C.c_void_p(q.data_ptr()), q.shape[0], C.c_void_p(r.data_ptr()), r.shape[0],
                                q.shape[1], hp, hv.shape[0], int(precision), C.c_void_p(out.data_ptr()),
                                _stream()))
    return out


def naive_sum_noalloc(q, r, h, precision=PREC_MIXED, out=None):
    """dfgt_naive_sum_noalloc: the brute-force sums with no device allocation in
    the library (a fixed 64 MiB region); returns an (n_h, nq) float64 CUDA tensor
    (allocated here by torch unless `out` is given)."""
    torch = _torch()
    q, r = _dev_points(q), _dev_points(r)
    hv, hp = _hvec(h)
    if out is None:
        out = torch.empty((hv.shape[0], q.shape[0]), dtype=torch.float64, device=q.device)
    _check(lib().dfgt_naive_sum_noalloc(C.c_void_p(q.data_ptr()), q.shape[0], C.c_void_p(r.data_ptr()),
                                        r.shape[0], q.shape[1], hp, hv.shape[0], int(precision),
                                        C.c_void_p(out.data_ptr()), _stream()))
    return out


def gauss_sum(Q: Tree, R: Tree, h, eps, precision=PREC_MIXED, force_method=FORCE_NONE, stats=False, out=None,
              profile=False, cost_exhaustive=0.0):
    """dfgt_gauss_sum: DFGT sums for every bandwidth, (n_h, NQ) float64 CUDA tensor [, stats dict]."""
    torch = _torch()
    hv, hp = _hvec(h)
    if out is None:
        out = torch.empty((hv.shape[0], Q.n), dtype=torch.float64, device="cuda")
    o = _opts(precision=precision, force_method=force_method, profile=profile, cost_exhaustive=cost_exhaustive)
    stats = stats or profile
    st = Stats() if stats else None
    _check(lib().dfgt_gauss_sum(Q.handle, R.handle, hp, hv.shape[0], float(eps), C.byref(o),
                                C.c_void_p(out.data_ptr()), C.byref(st) if st is not None else None, _stream()))
    return (out, st.as_dict()) if stats else out


def _vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def gauss_sum_grad(Q: Tree, R: Tree, h, eps, dh=True, dq=True, precision=PREC_MIXED, force_method=FORCE_NONE,
                   stats=False, profile=False):
    """dfgt_gauss_sum_grad: G (n_h, NQ), dG/dh (n_h, NQ) or None, dG/dq (n_h, NQ, d) or None [, stats]."""
    torch = _torch()
    hv, hp = _hvec(h)
    nh = hv.shape[0]
    G = torch.empty((nh, Q.n), dtype=torch.float64, device="cuda")
    Gh = torch.empty((nh, Q.n), dtype=torch.float64, device="cuda") if dh else None
    Gq = torch.empty((nh, Q.n, Q.d), dtype=torch.float64, device="cuda") if dq else None
    o = _opts(precision=precision, force_method=force_method, profile=profile)
    stats = stats or profile
    st = Stats() if stats else None
    _check(lib().dfgt_gauss_sum_grad(Q.handle, R.handle, hp, nh, float(eps), C.byref(o), _vp(G), _vp(Gh), _vp(Gq),
                                     C.byref(st) if st is not None else None, _stream()))
    return (G, Gh, Gq, st.as_dict()) if stats else (G, Gh, Gq)


def gauss_sum_backward(Q: Tree, R: Tree, h, eps, dG, want_dh=True, want_dq=True, precision=PREC_MIXED,
                       force_method=FORCE_NONE):
    """dfgt_gauss_sum_backward: (dh numpy (n_h,) or None, dq CUDA tensor (NQ, d) or None)."""
    torch = _torch()
    hv, hp = _hvec(h)
    nh = hv.shape[0]
    dG = dG.to(dtype=torch.float64).contiguous()
    if tuple(dG.shape) != (nh, Q.n) or not dG.is_cuda:
        raise DfgtError(f"dG must be a float64 CUDA tensor of shape ({nh}, {Q.n})")
    dh = np.empty(nh) if want_dh else None
    dq = torch.empty((Q.n, Q.d), dtype=torch.float64, device="cuda") if want_dq else None
    o = _opts(precision=precision, force_method=force_method)
    _check(lib().dfgt_gauss_sum_backward(Q.handle, R.handle, hp, nh, float(eps), C.byref(o), _vp(dG),
                                         dh.ctypes.data_as(C.POINTER(C.c_double)) if dh is not None else None,
                                         _vp(dq), _stream()))
    return dh, dq


def gauss_sum_vjp(dG, dGdh=None, dGdq=None):
    """dfgt_gauss_sum_vjp: (dh numpy (n_h,) or None, dq CUDA tensor (NQ, d) or None) from saved
    derivatives of dfgt_gauss_sum_grad."""
    torch = _torch()
    dG = dG.to(dtype=torch.float64).contiguous()
    nh, nq = dG.shape
    d = dGdq.shape[2] if dGdq is not None else 1
    dh = np.empty(nh) if dGdh is not None else None
    dq = torch.empty((nq, d), dtype=torch.float64, device=dG.device) if dGdq is not None else None
    _check(lib().dfgt_gauss_sum_vjp(nh, nq, d, _vp(dG), _vp(dGdh), _vp(dGdq),
                                    dh.ctypes.data_as(C.POINTER(C.c_double)) if dh is not None else None,
                                    _vp(dq), _stream()))
    return dh, dq


def lscv_score(R: Tree, h, eps, variant=1, grad=False, precision=PREC_MIXED, force_method=FORCE_NONE,
               stats=False):
    """dfgt_lscv_score: cv (n_h,) numpy [, dcv/dh (n_h,)] [, stats]."""
    hv, hp = _hvec(h)
    nh = hv.shape[0]
    cv = np.empty(nh)
    dcv = np.empty(nh) if grad else None
    o = _opts(precision=precision, force_method=force_method)
    st = Stats() if stats else None
    _check(lib().dfgt_lscv_score(R.handle, hp, nh, float(eps), int(variant), C.byref(o),
                                 cv.ctypes.data_as(C.POINTER(C.c_double)),
                                 dcv.ctypes.data_as(C.POINTER(C.c_double)) if dcv is not None else None,
                                 C.byref(st) if st is not None else None, _stream()))
    out = (cv,) + ((dcv,) if grad else ()) + ((st.as_dict(),) if stats else ())
    return out[0] if len(out) == 1 else out


def kde_density(Q: Tree, R: Tree, h, eps, precision=PREC_MIXED, force_method=FORCE_NONE, stats=False):
    """dfgt_kde_density: (n_h, NQ) float64 tensor of density estimates [, stats]."""
    torch = _torch()
    hv, hp = _hvec(h)
    p = torch.empty((hv.shape[0], Q.n), dtype=torch.float64, device="cuda")
    o = _opts(precision=precision, force_method=force_method)
    st = Stats() if stats else None
    _check(lib().dfgt_kde_density(Q.handle, R.handle, hp, hv.shape[0], float(eps), C.byref(o), p.data_ptr(),
                                  C.byref(st) if st is not None else None, _stream()))
    return (p, st.as_dict()) if stats else p


def lcv_score(R: Tree, h, eps, grad=False, precision=PREC_MIXED, force_method=FORCE_NONE):
    """dfgt_lcv_score: cv (n_h,) numpy [, dcv/dh (n_h,)]."""
    hv, hp = _hvec(h)
    nh = hv.shape[0]
    cv = np.empty(nh)
    dcv = np.empty(nh) if grad else None
    o = _opts(precision=precision, force_method=force_method)
    _check(lib().dfgt_lcv_score(R.handle, hp, nh, float(eps), C.byref(o), cv.ctypes.data_as(C.POINTER(C.c_double)),
                                dcv.ctypes.data_as(C.POINTER(C.c_double)) if dcv is not None else None, None,
                                _stream()))
    return (cv, dcv) if grad else cv


TUNE_LEAVES = (16, 32, 64, 128, 256)


def tune_leaf_size(points, h, eps, reps=3, p_max=0, precision=PREC_MIXED, cost_exhaustive=0.0):
    """dfgt_tune_leaf_size: (leaf, {candidate: median ms of build + monochromatic sums})."""
    x = _dev_points(points)
    hv, hp = _hvec(h)
    o = _opts(0, p_max, precision, FORCE_NONE)
    o.cost_exhaustive = float(cost_exhaustive)
    leaf = C.c_int32()
    ms = (C.c_double * len(TUNE_LEAVES))()
    _check(lib().dfgt_tune_leaf_size(C.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], hp, hv.shape[0], float(eps),
                                     C.byref(o), int(reps), _stream(), C.byref(leaf), ms))
    return leaf.value, dict(zip(TUNE_LEAVES, list(ms)))


def lscv_optimize(R: Tree, h_lo, h_hi, eps, variant=1, n_grid=16, rel_tol=1e-3, precision=PREC_MIXED,
                  force_method=FORCE_NONE):
    """dfgt_lscv_optimize: (h_star, cv_star, n_evals)."""
    o = _opts(precision=precision, force_method=force_method)
    hs, cv, ne = C.c_double(), C.c_double(), C.c_int32()
    _check(lib().dfgt_lscv_optimize(R.handle, float(h_lo), float(h_hi), float(eps), int(variant), int(n_grid),
                                    float(rel_tol), C.byref(o), C.byref(hs), C.byref(cv), C.byref(ne), _stream()))
    return hs.value, cv.value, ne.value


def _problem_array(problems):
    """[(Q, R, h)] -> (ctypes array, outputs, kept-alive host arrays)."""
    torch = _torch()
    arr = (Problem * len(problems))()
    outs, keep = [], []
    for i, (Q, R, h) in enumerate(problems):
        hv, hp = _hvec(h)
        G = torch.empty((hv.shape[0], Q.n), dtype=torch.float64, device="cuda")
        arr[i] = Problem(Q.handle, R.handle, hp, hv.shape[0], G.data_ptr())
        outs.append(G)
        keep.append(hv)
    return arr, outs, keep


def gauss_sum_batched(problems, eps, precision=PREC_MIXED, force_method=FORCE_NONE, stats=False, profile=False,
                      cost_exhaustive=0.0):
    """dfgt_gauss_sum_batched over [(Q, R, h)]: list of (n_h, NQ) tensors [, stats]."""
    arr, outs, keep = _problem_array(problems)
    o = _opts(precision=precision, force_method=force_method, profile=profile, cost_exhaustive=cost_exhaustive)
    stats = stats or profile
    st = Stats() if stats else None
    _check(lib().dfgt_gauss_sum_batched(arr, len(problems), float(eps), C.byref(o),
                                        C.byref(st) if st is not None else None, _stream()))
    return (outs, st.as_dict()) if stats else outs


class Batch:
    """dfgt_batch_create / run / check / free: a captured sweep over [(Q, R, h)].
    ``G`` holds the output tensors, rewritten by every ``run()``."""

    def __init__(self, problems, eps, precision=PREC_MIXED, force_method=FORCE_NONE, stats=False,
                 cost_exhaustive=0.0):
        self.handle = None
        self._trees = [t for p in problems for t in p[:2]]
        arr, self.G, self._keep = _problem_array(problems)
        self._arr = arr
        o = _opts(precision=precision, force_method=force_method, cost_exhaustive=cost_exhaustive)
        st = Stats() if stats else None
        h = C.c_void_p()
        _check(lib().dfgt_batch_create(arr, len(problems), float(eps), C.byref(o),
                                       C.byref(st) if st is not None else None, _stream(), C.byref(h)))
        self.handle = h
        self.stats = st.as_dict() if st is not None else None

    def run(self):
        _check(lib().dfgt_batch_run(self.handle, _stream()))
        return self.G

    def check(self):
        _check(lib().dfgt_batch_check(self.handle, _stream()))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.dfgt_batch_free(h)
            self.handle = None
