// Internal declarations of libdfgt (HIP, gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dfgt.h"

namespace dfgt {

constexpr int kMaxD = 32;
constexpr int kMaxP = 8192;   // largest p_max^D coefficient vector
constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
void clear_error();

struct Status {
    dfgt_status code = DFGT_OK;
    bool ok() const { return code == DFGT_OK; }
};

#define DFGT_HIP(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            ::dfgt::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));            \
            return DFGT_EHIP;                                                                \
        }                                                                                    \
    } while (0)

#define DFGT_TRY(expr)                                                                       \
    do {                                                                                     \
        dfgt_status s_ = (expr);                                                             \
        if (s_ != DFGT_OK) return s_;                                                        \
    } while (0)

#define DFGT_REQUIRE(cond, msg)                                                              \
    do {                                                                                     \
        if (!(cond)) {                                                                       \
            ::dfgt::set_error(msg);                                                          \
            return DFGT_EINVAL;                                                              \
        }                                                                                    \
    } while (0)

// ---------------------------------------------------------------- device buffers
// The caller's allocator (dfgt_set_allocator), or none: hipMalloc.  `gen`
// changes with every dfgt_set_allocator call; a buffer goes back to the
// allocator that made it only while that allocator is still the current one
// (a buffer freed later, e.g. at process exit after the caller's allocator is
// gone, is left to the process).
struct AllocHook {
    dfgt_alloc_fn alloc = nullptr;
    dfgt_free_fn free = nullptr;
    void *ctx = nullptr;
    unsigned gen = 0;
};
AllocHook alloc_hook();

// A device allocation owned by host code; freed in the destructor.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    dfgt_free_fn hfree = nullptr;  // set when the caller's allocator made p
    void *hctx = nullptr;
    unsigned hgen = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (!hfree) (void)hipFree(p);
            else if (alloc_hook().gen == hgen) hfree(p, bytes, hctx);
        }
        p = nullptr;
        bytes = 0;
        hfree = nullptr;
    }
    // Ensures at least `need` bytes (contents are not preserved on growth).
    dfgt_status reserve(size_t need) {
        if (need <= bytes) return DFGT_OK;
        release();
        size_t nb = need < 256 ? 256 : need;
        const AllocHook h = alloc_hook();
        if (h.alloc) {
            p = h.alloc(nb, h.ctx);
            if (!p) {
                set_error("the caller's allocator returned NULL for " + std::to_string(nb) + " bytes");
                return DFGT_ENOMEM;
            }
            hfree = h.free;
            hctx = h.ctx;
            hgen = h.gen;
        } else if (hipMalloc(&p, nb) != hipSuccess) {
            p = nullptr;
            set_error("hipMalloc of " + std::to_string(nb) + " bytes failed");
            return DFGT_ENOMEM;
        }
        bytes = nb;
        return DFGT_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Pinned host memory for small transfers (allocated with hipHostMalloc, so
// copies run as DMA without a staging pass and do not block the host).
// Contents are not preserved on growth.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
    dfgt_status reserve(size_t need) {
        if (need <= bytes) return DFGT_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        size_t nb = need < 4096 ? 4096 : need;
        if (hipHostMalloc(&p, nb, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            set_error("hipHostMalloc of " + std::to_string(nb) + " bytes failed");
            return DFGT_ENOMEM;
        }
        bytes = nb;
        return DFGT_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// A typed view into device memory owned elsewhere (an arena).
struct DevSpan {
    void *p = nullptr;
    size_t bytes = 0;
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Device memory of freed trees, handed to later builds: otherwise every build
// pays hipMalloc (which stalls) and every free hipFree (which synchronises the
// device).  pool_put keeps an allocation with an event recorded on the stream
// whose queued work may still use it; pool_get makes the taking stream wait
// for that event.  Thread-safe; at most a bounded number of bytes are kept.
void pool_put(DevBuf &b, hipStream_t st);
dfgt_status pool_get(DevBuf &b, size_t need, hipStream_t st);

// Carves several spans out of one allocation (256-byte aligned pieces), so a
// tree costs a few allocations instead of one per array.  With a pool stream,
// a growing arena comes from the pool of freed trees.
inline dfgt_status alloc_spans(DevBuf &arena, std::initializer_list<std::pair<DevSpan *, size_t>> items,
                               hipStream_t pool_stream = nullptr, bool pooled = false) {
    size_t total = 0;
    for (auto &it : items) total += (it.second + 255) / 256 * 256;
    if (pooled && total > arena.bytes) {
        if (arena.p) pool_put(arena, pool_stream);
        DFGT_TRY(pool_get(arena, total, pool_stream));
    }
    DFGT_TRY(arena.reserve(total));
    char *base = static_cast<char *>(arena.p);
    size_t off = 0;
    for (auto &it : items) {
        it.first->p = base + off;
        it.first->bytes = it.second;
        off += (it.second + 255) / 256 * 256;
    }
    return DFGT_OK;
}

// ---------------------------------------------------------------- device views
// Read-only device view of one kd-tree (breadth-first node order).
struct DevTree {
    int32_t n, d, m, pmax, P, depth, nleaves;
    const double *lo, *hi, *ctr;          // [m][d]
    const int32_t *begin, *end;           // [m] tree-order point ranges
    const int32_t *left, *right, *parent; // [m], -1 = none
    const int32_t *leaves;                // [nleaves] node ids of the leaves
    const double *x;                      // [n][d] points in tree order (FP64)
    const int32_t *perm;                  // [n] tree position -> caller index
    const double *mu;                     // [m][P] raw far-field moments
    const double *nrm;                    // [n] squared norms |x|^2 in tree order
    const int32_t *lpath;                 // [nleaves][depth] ancestors of each leaf, the leaf first
    const int32_t *lplen;                 // [nleaves] path lengths
    const double *w;                      // [n] point weights / max weight, tree order; null: all 1
};

// Weight of reference node r (its moment mu_0, the sum of its stored point
// weights); its point count when the tree carries no weights.
__device__ __forceinline__ double node_weight(const DevTree &R, int r) {
    return R.w ? R.mu[(size_t)r * R.P] : (double)(R.end[r] - R.begin[r]);
}

}  // namespace dfgt

struct dfgt_batch_s;  // a captured batch (dfgt.hip)

// The opaque handle of the C ABI.
struct dfgt_tree_s {
    int64_t n = 0;
    int32_t d = 0, leaf = 32, pmax = 1, P = 1, depth = 0, precision = 0, force = 0;
    int64_t m = 0, nleaves = 0;
    std::vector<int32_t> level_start;  // host copy: nodes of level l are [level_start[l], level_start[l+1])
    std::vector<int32_t> level_max;    // host copy: the most points of a node of level l
    // arena0: point and node-capacity arrays; arena1: per-node and per-leaf
    // arrays sized after the build; arena2: moments, norms and the device view
    dfgt::DevBuf arena0, arena1, arena2;
    dfgt::DevSpan lo, hi, ctr, begin, end, left, right, parent, sdim, scoord, leaves, x, perm, mu, nrm, mpart,
        lpath, lplen, nleaves_dev, w;
    double max_nrm = 0.0;  // max |x|^2 (valid after dfgt_build_tree returns)
    hipStream_t stream = nullptr;  // the stream the tree was built on
    bool weighted = false;         // points carry weights (dfgt_build_tree_weighted)
    double wscale = 1.0;           // the largest weight: the tree stores w / wscale, in [0, 1]
    double wsum = 0.0;             // sum of the caller's weights (n when unweighted)
    dfgt::DevSpan view;    // a DevTree in device memory
    dfgt::DevTree host_view{};
};

namespace dfgt {

// ---------------------------------------------------------------- shared device helpers
__device__ __forceinline__ long long dbl_key(double v) {
    long long b = __double_as_longlong(v);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}
__device__ __forceinline__ double key_dbl(long long k) {
    return __longlong_as_double(k >= 0 ? k : (k ^ 0x7fffffffffffffffLL));
}

// Deterministic wave-wide sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// Load through a pointer that device code read from memory (a DevTree field):
// left to itself the compiler cannot tell that it addresses global memory and
// emits a FLAT load, whose completion also gates every later wait for LDS
// results, so a prefetch issued before LDS work would stall at its first LDS
// wait.  The cast makes it a global load.
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

// A wave-uniform load through the constant address space, which the compiler
// issues as a scalar load (s_load) into SGPRs: for data no kernel writes while
// the caller runs, at an address every lane of the wave holds (see
// uniform_ptr).
template <typename T>
__device__ __forceinline__ T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}
// The first active lane's copy of a pointer the wave's lanes share, in SGPRs.
template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (const T *)(((unsigned long long)hi << 32) | lo);
}

// DPP lane moves (GFX9 row controls: row_shr:n is 0x110 + n, row_bcast:15
// 0x142, row_bcast:31 0x143); lanes without a source lane, and rows outside
// ROWS, receive `old`.  They stay in the vector ALU: no LDS round trip, unlike
// a shuffle.  Callers run with the whole wave active.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_move64(long long old, long long v) {
    const int lo = dpp_move<CTRL, ROWS>((int)old, (int)v);
    const int hi = dpp_move<CTRL, ROWS>((int)(old >> 32), (int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Inclusive scan over the 64 lanes with an associative op: shifts by 1, 2, 4
// and 8 inside rows of 16 lanes, then row 0's last lane into row 1 and row
// 2's into row 3, then lane 31 into rows 2 and 3.  `id` is the op's identity.
template <class T, class Op>
__device__ __forceinline__ T wave_scan_dpp(T v, T id, Op op) {
    if constexpr (sizeof(T) == 8) {
        v = op(v, dpp_move64<0x111, 0xF>(id, v));
        v = op(v, dpp_move64<0x112, 0xF>(id, v));
        v = op(v, dpp_move64<0x114, 0xF>(id, v));
        v = op(v, dpp_move64<0x118, 0xF>(id, v));
        v = op(v, dpp_move64<0x142, 0xA>(id, v));
        v = op(v, dpp_move64<0x143, 0xC>(id, v));
    } else {
        v = op(v, dpp_move<0x111, 0xF>(id, v));
        v = op(v, dpp_move<0x112, 0xF>(id, v));
        v = op(v, dpp_move<0x114, 0xF>(id, v));
        v = op(v, dpp_move<0x118, 0xF>(id, v));
        v = op(v, dpp_move<0x142, 0xA>(id, v));
        v = op(v, dpp_move<0x143, 0xC>(id, v));
    }
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    v = wave_scan_dpp(v, 0, [](int a, int b) { return a + b; });
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_min_i(int v) {
    v = wave_scan_dpp(v, 0x7fffffff, [](int a, int b) { return a < b ? a : b; });
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_i(int v) {
    v = wave_scan_dpp(v, (int)0x80000000, [](int a, int b) { return a > b ? a : b; });
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v) {
    return wave_scan_dpp(v, 0, [](int a, int b) { return a + b; });
}

// ---------------------------------------------------------------- host entry points per file
// Frees the calling thread's workspace buffers of each file (dfgt_release_workspace).
void release_sum_workspace();    // dfgt.hip
void release_sweep_workspace();  // sweep.hip
void release_naive_workspace();  // naive.hip
void release_build_workspace();  // moments.hip

// naive.hip
dfgt_status launch_naive(const double *q, int64_t nq, const double *r, int64_t nr, int d,
                         const double *h, int nh, int precision, double *G, hipStream_t st);
// The same sums with every buffer carved from a fixed device region (no allocation).
dfgt_status launch_naive_noalloc(const double *q, int64_t nq, const double *r, int64_t nr, int d,
                                 const double *h, int nh, int precision, double *G, hipStream_t st);
size_t naive_noalloc_limit();  // doubles in that region
// tree.hip
dfgt_status build_tree_device(dfgt_tree_s *t, const double *pts, const double *w, hipStream_t st);
// moments.hip
dfgt_status compute_moments(dfgt_tree_s *t, hipStream_t st);
// dfgt.hip
// Gradient mode outputs (device, [n_h][N_Q] and [n_h][N_Q][d], caller order; either may be null).
struct GradOut {
    double *dGdh;
    double *dGdq;
};
// One summation problem of a call: sums over R for the queries of Q at n_h
// bandwidths, written to G ([nh][Q->n], caller order).
struct Problem {
    dfgt_tree_s *Q, *R;
    const double *h;
    int nh;
    double *G;
    int loo = 0;  // Q == R: leave each query's own point out of its sums (G - 1, computed as such)
};
// Several problems (same D and p_max) and all their bandwidths in one traversal.
dfgt_status run_gauss_multi(const Problem *pr, int np, double eps, int precision, int force, int profile,
                            double cost_e, const GradOut *grad, dfgt_stats *stats, hipStream_t st);
// Captured batches: an eager sizing run, then the launch sequence as a hipGraph.
dfgt_status batch_create(const Problem *pr, int np, double eps, int precision, int force, double cost_e,
                         dfgt_stats *stats, hipStream_t st, dfgt_batch_s **out);
dfgt_status batch_run(dfgt_batch_s *b, hipStream_t st);
dfgt_status batch_check(dfgt_batch_s *b, hipStream_t st);
// cost_e: weight of the exhaustive cost in ChooseBestMethod (1 = the paper's model).
// loo: leave-one-out sums (Q == R unweighted): G~ approximates G - 1 to eps (G - 1).
dfgt_status run_gauss_sum(dfgt_tree_s *Q, dfgt_tree_s *R, const double *h, int nh, double eps,
                          int precision, int force, int profile, double cost_e, double *G, const GradOut *grad,
                          dfgt_stats *stats, hipStream_t st, bool loo = false);

// sweep.hip
dfgt_status run_backward(dfgt_tree_s *Q, dfgt_tree_s *R, const double *h, int nh, double eps, int precision,
                         int force, double cost_e, const double *dG, double *dh_host, double *dq, hipStream_t st);
// Vector-Jacobian product of saved derivatives: dh[k] = sum_i dG[k][i] dGdh[k][i] (host),
// dq[i][c] = sum_k dG[k][i] dGdq[k][i][c]; fixed summation order.
dfgt_status run_vjp(int nh, int64_t nq, int d, const double *dG, const double *dGdh, const double *dGdq,
                    double *dh_host, double *dq, hipStream_t st);
dfgt_status run_lscv(dfgt_tree_s *R, const double *h, int nh, double eps, int precision, int force, double cost_e,
                     int variant, double *cv, double *dcv, dfgt_stats *stats, hipStream_t st);
dfgt_status run_lcv(dfgt_tree_s *R, const double *h, int nh, double eps, int precision, int force, double cost_e,
                    double *cv, double *dcv, dfgt_stats *stats, hipStream_t st);
dfgt_status run_density(dfgt_tree_s *Q, dfgt_tree_s *R, const double *h, int nh, double eps, int precision,
                        int force, double cost_e, double *p, dfgt_stats *stats, hipStream_t st);
dfgt_status run_lscv_optimize(dfgt_tree_s *R, double h_lo, double h_hi, double eps, int precision, int force,
                              double cost_e, int variant, int n_grid, double rel_tol, double *h_star,
                              double *cv_star, int *n_evals, hipStream_t st);

int default_pmax(int d);

}  // namespace dfgt
