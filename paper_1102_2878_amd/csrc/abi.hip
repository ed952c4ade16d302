// C ABI of libdfgt: argument validation, error strings, handle ownership.
// Every entry point catches C++ exceptions so none crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dfgt_internal.h"

namespace dfgt {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

namespace {
std::mutex g_hook_mu;
AllocHook g_hook;
}  // namespace

AllocHook alloc_hook() {
    std::lock_guard<std::mutex> lk(g_hook_mu);
    return g_hook;
}

int default_pmax(int d) {
    // p_max of the paper's experiments (Section 3.9)
    if (d <= 2) return 6;
    if (d == 3) return 4;
    if (d <= 5) return 2;
    return 1;
}

}  // namespace dfgt

using namespace dfgt;

#define DFGT_GUARD_BEGIN \
    clear_error();       \
    try {
#define DFGT_GUARD_END                                               \
    }                                                                \
    catch (const std::bad_alloc &) {                                 \
        set_error("host allocation failed");                         \
        return DFGT_ENOMEM;                                          \
    }                                                                \
    catch (const std::exception &e) {                                \
        set_error(std::string("internal error: ") + e.what());       \
        return DFGT_EHIP;                                            \
    }                                                                \
    catch (...) {                                                    \
        set_error("internal error");                                 \
        return DFGT_EHIP;                                            \
    }

namespace dfgt {

namespace {
struct Pooled {
    void *p;
    size_t bytes;
    hipEvent_t ev;
};
struct ArenaPool {
    std::mutex mu;
    std::vector<Pooled> items;
    std::vector<hipEvent_t> spare;  // events no pooled item holds
    size_t total = 0;
    ~ArenaPool() {
        for (auto &it : items) {
            (void)hipFree(it.p);
            (void)hipEventDestroy(it.ev);
        }
        for (auto ev : spare) (void)hipEventDestroy(ev);
    }
};
ArenaPool &arena_pool() {
    static ArenaPool pool;
    return pool;
}
constexpr size_t kPoolMaxBytes = size_t(2) << 30;
}  // namespace

void pool_put(DevBuf &b, hipStream_t st) {
    if (!b.p) return;
    if (b.hfree) {  // memory of the caller's allocator goes back to it, not to the pool
        b.release();
        return;
    }
    ArenaPool &pl = arena_pool();
    std::lock_guard<std::mutex> lk(pl.mu);
    hipEvent_t ev = nullptr;
    if (!pl.spare.empty()) {
        ev = pl.spare.back();
        pl.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    if (!ev || hipEventRecord(ev, st) != hipSuccess || pl.total + b.bytes > kPoolMaxBytes) {
        if (ev) pl.spare.push_back(ev);
        b.release();  // hipFree: synchronises, so the memory is idle before it is reused
        return;
    }
    pl.items.push_back(Pooled{b.p, b.bytes, ev});
    pl.total += b.bytes;
    b.p = nullptr;
    b.bytes = 0;
}

dfgt_status pool_get(DevBuf &b, size_t need, hipStream_t st) {
    ArenaPool &pl = arena_pool();
    std::lock_guard<std::mutex> lk(pl.mu);
    int best = -1;
    for (int i = 0; i < (int)pl.items.size(); ++i) {
        const size_t sz = pl.items[i].bytes;
        if (sz >= need && sz <= 4 * need + (size_t(1) << 20) && (best < 0 || sz < pl.items[best].bytes)) best = i;
    }
    if (best < 0) return DFGT_OK;  // the caller allocates
    Pooled it = pl.items[best];
    pl.items.erase(pl.items.begin() + best);
    pl.total -= it.bytes;
    DFGT_HIP(hipStreamWaitEvent(st, it.ev, 0));
    pl.spare.push_back(it.ev);
    b.release();
    b.p = it.p;
    b.bytes = it.bytes;
    return DFGT_OK;
}

}  // namespace dfgt

namespace dfgt {
namespace {
__global__ void k_store_view(DevTree v, DevTree *dst) { *dst = v; }

// One pass over the weights: a block-wide fold, then one atomic per block and
// quantity (same-address device atomics serialise).  flag |= 1 for a negative
// or non-finite weight; *mx = the largest weight as its bit pattern (the order
// of non-negative doubles is that of their bit patterns).
__global__ __launch_bounds__(256) void k_check_weights(const double *__restrict__ w, long long n, int *flag,
                                                       unsigned long long *mx) {
    __shared__ int fs[4];
    __shared__ unsigned long long ms[4];
    int f = 0;
    unsigned long long m = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double v = w[i];
        if (!(v >= 0.0) || !isfinite(v)) f = 1;
        else if (v > 0.0) m = max(m, (unsigned long long)__double_as_longlong(v));  // not -0.0's pattern
    }
    for (int off = 32; off >= 1; off >>= 1) {
        f |= __shfl_xor(f, off, 64);
        m = max(m, (unsigned long long)__shfl_xor((long long)m, off, 64));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        fs[wv] = f;
        ms[wv] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            f |= fs[k];
            m = max(m, ms[k]);
        }
        if (f) atomicOr(flag, f);
        if (m) atomicMax(mx, m);
    }
}
}  // namespace

// *bad: 0 fine, 1 a negative or non-finite weight, 2 all weights zero; *wmax
// the largest weight.
static thread_local DevBuf g_wcheck;  // check_weights' flag and maximum

static dfgt_status check_weights(const double *w, int64_t n, hipStream_t st, int *bad, double *wmax) {
    struct Out {
        int flag;
        int pad;
        unsigned long long mx;
    };
    static thread_local Out back;
    DFGT_TRY(g_wcheck.reserve(sizeof(Out)));
    Out *o = g_wcheck.as<Out>();
    DFGT_HIP(hipMemsetAsync(o, 0, sizeof(Out), st));
    const long long nb = std::min<long long>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_check_weights, dim3((unsigned)nb), dim3(256), 0, st, w, (long long)n, &o->flag, &o->mx);
    DFGT_HIP(hipGetLastError());
    DFGT_HIP(hipMemcpyAsync(&back, o, sizeof(Out), hipMemcpyDeviceToHost, st));
    DFGT_HIP(hipStreamSynchronize(st));
    double mxv;
    std::memcpy(&mxv, &back.mx, sizeof(double));
    *wmax = mxv;
    *bad = back.flag ? 1 : (back.mx == 0 ? 2 : 0);
    return DFGT_OK;
}

}  // namespace dfgt

extern "C" {

const char *dfgt_last_error(void) { return g_err.c_str(); }

const char *dfgt_version(void) { return "dfgt-mi355x 0.1 (gfx950)"; }

static dfgt_status build_common(const double *pts_dev, const double *w_dev, double wmax, int64_t n, int32_t d,
                                const dfgt_options *opt, void *stream, dfgt_tree *out);

dfgt_status dfgt_build_tree(const double *pts_dev, int64_t n, int32_t d, const dfgt_options *opt, void *stream,
                            dfgt_tree *out) {
    DFGT_GUARD_BEGIN
    return build_common(pts_dev, nullptr, 1.0, n, d, opt, stream, out);
    DFGT_GUARD_END
}

dfgt_status dfgt_build_tree_weighted(const double *pts_dev, const double *w_dev, int64_t n, int32_t d,
                                     const dfgt_options *opt, void *stream, dfgt_tree *out) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(out != nullptr, "dfgt_build_tree_weighted: out is NULL");
    *out = nullptr;
    DFGT_REQUIRE(w_dev != nullptr, "dfgt_build_tree_weighted: w_dev is NULL");
    DFGT_REQUIRE(n >= 1 && n < (int64_t(1) << 30), "dfgt_build_tree_weighted: n must be in [1, 2^30)");
    int bad = 0;
    double wmax = 0.0;
    DFGT_TRY(check_weights(w_dev, n, (hipStream_t)stream, &bad, &wmax));
    DFGT_REQUIRE(bad != 1, "dfgt_build_tree_weighted: a weight is negative or not finite");
    DFGT_REQUIRE(bad != 2, "dfgt_build_tree_weighted: all weights are zero");
    return build_common(pts_dev, w_dev, wmax, n, d, opt, stream, out);
    DFGT_GUARD_END
}

static dfgt_status build_common(const double *pts_dev, const double *w_dev, double wmax, int64_t n, int32_t d,
                                const dfgt_options *opt, void *stream, dfgt_tree *out) {
    DFGT_REQUIRE(out != nullptr, "dfgt_build_tree: out is NULL");
    *out = nullptr;
    DFGT_REQUIRE(pts_dev != nullptr, "dfgt_build_tree: pts_dev is NULL");
    DFGT_REQUIRE(n >= 1 && n < (int64_t(1) << 30), "dfgt_build_tree: n must be in [1, 2^30)");
    DFGT_REQUIRE(d >= 1 && d <= kMaxD, "dfgt_build_tree: d must be in [1, 32]");
    dfgt_options o{};
    if (opt) o = *opt;
    for (int i = 0; i < 2; ++i) DFGT_REQUIRE(o.reserved[i] == 0, "dfgt_build_tree: reserved option field set");
    DFGT_REQUIRE(o.leaf_size >= 0 && o.leaf_size <= 4096, "dfgt_build_tree: leaf_size must be in [0, 4096]");
    DFGT_REQUIRE(o.p_max >= 0 && o.p_max <= 16, "dfgt_build_tree: p_max must be in [0, 16]");
    DFGT_REQUIRE(o.precision == DFGT_PREC_MIXED || o.precision == DFGT_PREC_FP64,
                 "dfgt_build_tree: unknown precision");
    DFGT_REQUIRE(o.force_method >= 0 && o.force_method <= 5, "dfgt_build_tree: unknown force_method");
    const int pmax = o.p_max ? o.p_max : default_pmax(d);
    double P = std::pow((double)pmax, (double)d);
    DFGT_REQUIRE(P <= kMaxP, "dfgt_build_tree: p_max^d exceeds 8192 coefficients");
    auto *t = new dfgt_tree_s();
    t->n = n;
    t->d = d;
    t->leaf = o.leaf_size ? o.leaf_size : 32;
    t->pmax = pmax;
    t->P = (int)P;
    t->precision = o.precision;
    t->force = o.force_method;
    t->weighted = w_dev != nullptr;
    t->wscale = w_dev ? wmax : 1.0;
    hipStream_t st = (hipStream_t)stream;
    t->stream = st;
    dfgt_status s = build_tree_device(t, pts_dev, w_dev, st);
    if (s == DFGT_OK) s = compute_moments(t, st);
    if (s == DFGT_OK) {
        DevTree v{};
        v.n = (int32_t)t->n;
        v.d = t->d;
        v.m = (int32_t)t->m;
        v.pmax = t->pmax;
        v.P = t->P;
        v.depth = t->depth;
        v.nleaves = (int32_t)t->nleaves;
        v.lo = t->lo.as<double>();
        v.hi = t->hi.as<double>();
        v.ctr = t->ctr.as<double>();
        v.begin = t->begin.as<int32_t>();
        v.end = t->end.as<int32_t>();
        v.left = t->left.as<int32_t>();
        v.right = t->right.as<int32_t>();
        v.parent = t->parent.as<int32_t>();
        v.leaves = t->leaves.as<int32_t>();
        v.x = t->x.as<double>();
        v.perm = t->perm.as<int32_t>();
        v.mu = t->mu.as<double>();
        v.nrm = t->nrm.as<double>();
        v.lpath = t->lpath.as<int32_t>();
        v.lplen = t->lplen.as<int32_t>();
        v.w = t->w.as<double>();
        t->host_view = v;
        // the view's storage was carved out with the moments; it is written by
        // a kernel that takes it as its argument, so the host does not wait
        hipLaunchKernelGGL(k_store_view, dim3(1), dim3(1), 0, st, v, t->view.as<DevTree>());
        if (hipGetLastError() != hipSuccess) {
            set_error("dfgt_build_tree: writing the tree view failed");
            s = DFGT_EHIP;
        }
    }
    if (s != DFGT_OK) {
        delete t;
        return s;
    }
    *out = t;
    return DFGT_OK;
}

dfgt_status dfgt_tree_free(dfgt_tree t) {
    DFGT_GUARD_BEGIN
    if (t) {
        // the arenas go to the pool of freed trees, after the work queued on
        // the tree's stream
        pool_put(t->arena0, t->stream);
        pool_put(t->arena1, t->stream);
        pool_put(t->arena2, t->stream);
    }
    delete t;
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_tree_info(dfgt_tree t, int64_t *n, int32_t *d, int64_t *n_nodes, int32_t *depth, int32_t *p_max) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(t != nullptr, "dfgt_tree_info: tree is NULL");
    if (n) *n = t->n;
    if (d) *d = t->d;
    if (n_nodes) *n_nodes = t->m;
    if (depth) *depth = t->depth;
    if (p_max) *p_max = t->pmax;
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_tree_export(dfgt_tree t, int32_t *perm, double *lo, double *hi, int32_t *begin, int32_t *end,
                             int32_t *left, int32_t *right, int32_t *split_dim, double *split_coord) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(t != nullptr, "dfgt_tree_export: tree is NULL");
    const size_t m = (size_t)t->m, d = (size_t)t->d;
    struct Item {
        void *dst;
        const DevSpan *src;
        size_t bytes;
    } items[] = {
        {perm, &t->perm, sizeof(int32_t) * (size_t)t->n}, {lo, &t->lo, sizeof(double) * m * d},
        {hi, &t->hi, sizeof(double) * m * d},             {begin, &t->begin, sizeof(int32_t) * m},
        {end, &t->end, sizeof(int32_t) * m},              {left, &t->left, sizeof(int32_t) * m},
        {right, &t->right, sizeof(int32_t) * m},          {split_dim, &t->sdim, sizeof(int32_t) * m},
        {split_coord, &t->scoord, sizeof(double) * m},
    };
    for (auto &it : items)
        if (it.dst) DFGT_HIP(hipMemcpy(it.dst, it.src->p, it.bytes, hipMemcpyDeviceToHost));
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_tree_perm(dfgt_tree t, int32_t *perm_dev, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(t != nullptr && perm_dev != nullptr, "dfgt_tree_perm: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (t->stream != st) {  // the tree's own work first
        hipEvent_t ev;
        DFGT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        const hipError_t e1 = hipEventRecord(ev, t->stream);
        const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(st, ev, 0) : e1;
        (void)hipEventDestroy(ev);
        DFGT_HIP(e2);
    }
    DFGT_HIP(hipMemcpyAsync(perm_dev, t->perm.p, sizeof(int32_t) * (size_t)t->n, hipMemcpyDeviceToDevice, st));
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_set_allocator(dfgt_alloc_fn alloc, dfgt_free_fn free_fn, void *ctx) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE((alloc == nullptr) == (free_fn == nullptr), "dfgt_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hook.alloc = alloc;
    g_hook.free = free_fn;
    g_hook.ctx = ctx;
    g_hook.gen += 1;
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_release_workspace(void) {
    DFGT_GUARD_BEGIN
    DFGT_HIP(hipDeviceSynchronize());  // no queued work may still use the buffers
    release_sum_workspace();
    release_sweep_workspace();
    release_naive_workspace();
    release_build_workspace();
    g_wcheck.release();
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_tree_moments(dfgt_tree t, double *mu_host) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(t != nullptr && mu_host != nullptr, "dfgt_tree_moments: NULL argument");
    DFGT_HIP(hipMemcpy(mu_host, t->mu.p, sizeof(double) * (size_t)t->m * t->P, hipMemcpyDeviceToHost));
    return DFGT_OK;
    DFGT_GUARD_END
}

static dfgt_status check_bandwidths(const double *h, int32_t n_h, const char *who) {
    DFGT_REQUIRE(h != nullptr, std::string(who) + ": h_host is NULL");
    DFGT_REQUIRE(n_h >= 1 && n_h <= 65535, std::string(who) + ": n_h must be in [1, 65535]");
    for (int i = 0; i < n_h; ++i)
        DFGT_REQUIRE(std::isfinite(h[i]) && h[i] > 0.0, std::string(who) + ": bandwidths must be finite and > 0");
    return DFGT_OK;
}

dfgt_status dfgt_naive_sum(const double *q_dev, int64_t nq, const double *r_dev, int64_t nr, int32_t d,
                           const double *h_host, int32_t n_h, int32_t precision, double *G_dev, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(q_dev && r_dev && G_dev, "dfgt_naive_sum: NULL device pointer");
    DFGT_REQUIRE(nq >= 1 && nq < (int64_t(1) << 30) && nr >= 1 && nr < (int64_t(1) << 30),
                 "dfgt_naive_sum: nq and nr must be in [1, 2^30)");
    DFGT_REQUIRE(d >= 1 && d <= kMaxD, "dfgt_naive_sum: d must be in [1, 32]");
    DFGT_REQUIRE(precision == DFGT_PREC_MIXED || precision == DFGT_PREC_FP64, "dfgt_naive_sum: unknown precision");
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_naive_sum"));
    return launch_naive(q_dev, nq, r_dev, nr, d, h_host, n_h, precision, G_dev, (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_naive_sum_noalloc(const double *q_dev, int64_t nq, const double *r_dev, int64_t nr, int32_t d,
                                   const double *h_host, int32_t n_h, int32_t precision, double *G_dev,
                                   void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(q_dev && r_dev && G_dev, "dfgt_naive_sum_noalloc: NULL device pointer");
    DFGT_REQUIRE(nq >= 1 && nq < (int64_t(1) << 30) && nr >= 1 && nr < (int64_t(1) << 30),
                 "dfgt_naive_sum_noalloc: nq and nr must be in [1, 2^30)");
    DFGT_REQUIRE(d >= 1 && d <= kMaxD, "dfgt_naive_sum_noalloc: d must be in [1, 32]");
    DFGT_REQUIRE(precision == DFGT_PREC_MIXED || precision == DFGT_PREC_FP64,
                 "dfgt_naive_sum_noalloc: unknown precision");
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_naive_sum_noalloc"));
    return launch_naive_noalloc(q_dev, nq, r_dev, nr, d, h_host, n_h, precision, G_dev, (hipStream_t)stream);
    DFGT_GUARD_END
}

// Options of a summation call: precision and force default to the tree's.
static dfgt_status call_options(const dfgt_tree_s *R, const dfgt_options *opt, const char *who, int *precision,
                                int *force, int *profile, double *cost_e) {
    *precision = R->precision;
    *force = R->force;
    *profile = 0;
    *cost_e = 1.0;
    if (opt) {
        for (int i = 0; i < 2; ++i) DFGT_REQUIRE(opt->reserved[i] == 0, std::string(who) + ": reserved option field set");
        DFGT_REQUIRE(std::isfinite(opt->cost_exhaustive) && opt->cost_exhaustive >= 0.0f,
                     std::string(who) + ": cost_exhaustive must be finite and >= 0");
        if (opt->cost_exhaustive > 0.0f) *cost_e = opt->cost_exhaustive;
        DFGT_REQUIRE(opt->precision == DFGT_PREC_MIXED || opt->precision == DFGT_PREC_FP64,
                     std::string(who) + ": unknown precision");
        DFGT_REQUIRE(opt->force_method >= 0 && opt->force_method <= 5, std::string(who) + ": unknown force_method");
        *precision = opt->precision;
        *force = opt->force_method;
        *profile = opt->profile;
    }
    return DFGT_OK;
}

static dfgt_status check_pair(const dfgt_tree_s *Q, const dfgt_tree_s *R, double eps, const char *who) {
    DFGT_REQUIRE(Q->d == R->d, std::string(who) + ": query and reference dimensions differ");
    DFGT_REQUIRE(Q->pmax == R->pmax, std::string(who) + ": query and reference trees use different p_max");
    DFGT_REQUIRE(std::isfinite(eps) && eps >= 0.0 && eps < 1.0, std::string(who) + ": eps must be in [0, 1)");
    return DFGT_OK;
}

dfgt_status dfgt_gauss_sum(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                           const dfgt_options *opt, double *G_dev, dfgt_stats *stats, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(Q && R && G_dev, "dfgt_gauss_sum: NULL argument");
    DFGT_TRY(check_pair(Q, R, eps, "dfgt_gauss_sum"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_gauss_sum"));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_gauss_sum", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0 || stats != nullptr, "dfgt_gauss_sum: profile needs a stats pointer");
    return run_gauss_sum(Q, R, h_host, n_h, eps, precision, force, profile, cost_e, G_dev, nullptr, stats,
                         (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_gauss_sum_grad(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                                const dfgt_options *opt, double *G_dev, double *dGdh_dev, double *dGdq_dev,
                                dfgt_stats *stats, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(Q && R && G_dev, "dfgt_gauss_sum_grad: NULL argument");
    DFGT_REQUIRE(dGdh_dev || dGdq_dev, "dfgt_gauss_sum_grad: both derivative outputs are NULL");
    DFGT_TRY(check_pair(Q, R, eps, "dfgt_gauss_sum_grad"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_gauss_sum_grad"));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_gauss_sum_grad", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0 || stats != nullptr, "dfgt_gauss_sum_grad: profile needs a stats pointer");
    GradOut go{dGdh_dev, dGdq_dev};
    return run_gauss_sum(Q, R, h_host, n_h, eps, precision, force, profile, cost_e, G_dev, &go, stats,
                         (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_gauss_sum_backward(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                                    const dfgt_options *opt, const double *dG_dev, double *dh_host, double *dq_dev,
                                    void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(Q && R && dG_dev, "dfgt_gauss_sum_backward: NULL argument");
    DFGT_REQUIRE(dh_host || dq_dev, "dfgt_gauss_sum_backward: both gradient outputs are NULL");
    DFGT_TRY(check_pair(Q, R, eps, "dfgt_gauss_sum_backward"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_gauss_sum_backward"));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_gauss_sum_backward", &precision, &force, &profile, &cost_e));
    return run_backward(Q, R, h_host, n_h, eps, precision, force, cost_e, dG_dev, dh_host, dq_dev,
                        (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_gauss_sum_vjp(int32_t n_h, int64_t nq, int32_t d, const double *dG_dev, const double *dGdh_dev,
                               const double *dGdq_dev, double *dh_host, double *dq_dev, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(dG_dev, "dfgt_gauss_sum_vjp: NULL dG_dev");
    DFGT_REQUIRE(n_h >= 1 && nq >= 1 && nq < (int64_t(1) << 31) && d >= 1 && d <= kMaxD,
                 "dfgt_gauss_sum_vjp: n_h, nq or d out of range");
    DFGT_REQUIRE(dh_host || dq_dev, "dfgt_gauss_sum_vjp: both gradient outputs are NULL");
    DFGT_REQUIRE(!dh_host || dGdh_dev, "dfgt_gauss_sum_vjp: dh_host needs dGdh_dev");
    DFGT_REQUIRE(!dq_dev || dGdq_dev, "dfgt_gauss_sum_vjp: dq_dev needs dGdq_dev");
    return run_vjp(n_h, nq, d, dG_dev, dGdh_dev, dGdq_dev, dh_host, dq_dev, (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_lscv_score(dfgt_tree R, const double *h_host, int32_t n_h, double eps, int32_t variant,
                            const dfgt_options *opt, double *cv_host, double *dcv_host, dfgt_stats *stats,
                            void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(R && cv_host, "dfgt_lscv_score: NULL argument");
    DFGT_REQUIRE(R->n >= 2, "dfgt_lscv_score: needs at least two points");
    DFGT_REQUIRE(!R->weighted, "dfgt_lscv_score: cross-validation is defined for unweighted points");
    DFGT_REQUIRE(variant == 0 || variant == 1, "dfgt_lscv_score: variant must be 0 or 1");
    DFGT_TRY(check_pair(R, R, eps, "dfgt_lscv_score"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_lscv_score"));
    DFGT_REQUIRE(n_h <= 32767, "dfgt_lscv_score: n_h must be <= 32767");
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_lscv_score", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0, "dfgt_lscv_score: profiling is not supported here");
    return run_lscv(R, h_host, n_h, eps, precision, force, cost_e, variant, cv_host, dcv_host, stats,
                    (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_kde_density(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                             const dfgt_options *opt, double *p_dev, dfgt_stats *stats, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(Q && R && p_dev, "dfgt_kde_density: NULL argument");
    DFGT_TRY(check_pair(Q, R, eps, "dfgt_kde_density"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_kde_density"));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_kde_density", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0, "dfgt_kde_density: profiling is not supported here");
    return run_density(Q, R, h_host, n_h, eps, precision, force, cost_e, p_dev, stats, (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_lcv_score(dfgt_tree R, const double *h_host, int32_t n_h, double eps, const dfgt_options *opt,
                           double *cv_host, double *dcv_host, dfgt_stats *stats, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(R && cv_host, "dfgt_lcv_score: NULL argument");
    DFGT_REQUIRE(R->n >= 2, "dfgt_lcv_score: needs at least two points");
    DFGT_REQUIRE(!R->weighted, "dfgt_lcv_score: cross-validation is defined for unweighted points");
    DFGT_TRY(check_pair(R, R, eps, "dfgt_lcv_score"));
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_lcv_score"));
    DFGT_REQUIRE(n_h <= 32767, "dfgt_lcv_score: n_h must be <= 32767");
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_lcv_score", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0, "dfgt_lcv_score: profiling is not supported here");
    return run_lcv(R, h_host, n_h, eps, precision, force, cost_e, cv_host, dcv_host, stats, (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_lscv_optimize(dfgt_tree R, double h_lo, double h_hi, double eps, int32_t variant, int32_t n_grid,
                               double rel_tol, const dfgt_options *opt, double *h_star, double *cv_star,
                               int32_t *n_evals, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(R && h_star, "dfgt_lscv_optimize: NULL argument");
    DFGT_REQUIRE(R->n >= 2, "dfgt_lscv_optimize: needs at least two points");
    DFGT_REQUIRE(!R->weighted, "dfgt_lscv_optimize: cross-validation is defined for unweighted points");
    DFGT_REQUIRE(variant == 0 || variant == 1, "dfgt_lscv_optimize: variant must be 0 or 1");
    DFGT_REQUIRE(std::isfinite(h_lo) && std::isfinite(h_hi) && h_lo > 0.0 && h_hi > h_lo,
                 "dfgt_lscv_optimize: need 0 < h_lo < h_hi (finite)");
    DFGT_REQUIRE(n_grid >= 4 && n_grid <= 1024, "dfgt_lscv_optimize: n_grid must be in [4, 1024]");
    DFGT_REQUIRE(std::isfinite(rel_tol) && rel_tol > 0.0 && rel_tol < 1.0,
                 "dfgt_lscv_optimize: rel_tol must be in (0, 1)");
    DFGT_TRY(check_pair(R, R, eps, "dfgt_lscv_optimize"));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(R, opt, "dfgt_lscv_optimize", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0, "dfgt_lscv_optimize: profiling is not supported here");
    int ev = 0;
    DFGT_TRY(run_lscv_optimize(R, h_lo, h_hi, eps, precision, force, cost_e, variant, n_grid, rel_tol, h_star,
                               cv_star, &ev, (hipStream_t)stream));
    if (n_evals) *n_evals = ev;
    return DFGT_OK;
    DFGT_GUARD_END
}

dfgt_status dfgt_tune_leaf_size(const double *pts_dev, int64_t n, int32_t d, const double *h_host, int32_t n_h,
                                double eps, const dfgt_options *opt, int32_t reps, void *stream,
                                int32_t *leaf_out, double *ms_out) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(leaf_out != nullptr, "dfgt_tune_leaf_size: leaf_out is NULL");
    DFGT_REQUIRE(reps >= 1 && reps <= 100, "dfgt_tune_leaf_size: reps must be in [1, 100]");
    DFGT_TRY(check_bandwidths(h_host, n_h, "dfgt_tune_leaf_size"));
    DFGT_REQUIRE(n >= 1 && n < (int64_t(1) << 30), "dfgt_tune_leaf_size: n must be in [1, 2^30)");
    hipStream_t st = (hipStream_t)stream;
    // the output buffer and the two events, released on every exit
    struct Res {
        double *G = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Res() {
            if (G) (void)hipFree(G);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } res;
    DFGT_REQUIRE(hipMalloc(&res.G, sizeof(double) * (size_t)n_h * (size_t)n) == hipSuccess,
                 "dfgt_tune_leaf_size: hipMalloc of the output buffer failed");
    DFGT_HIP(hipEventCreate(&res.e0));
    DFGT_HIP(hipEventCreate(&res.e1));
    dfgt_options o{};
    if (opt) o = *opt;
    const int leaves[DFGT_N_TUNE_LEAVES] = DFGT_TUNE_LEAVES;
    constexpr double kTuneTie = 0.02;
    double med[DFGT_N_TUNE_LEAVES], best = 0.0;
    for (int c = 0; c < DFGT_N_TUNE_LEAVES; ++c) {
        o.leaf_size = leaves[c];
        std::vector<float> t;
        for (int r = 0; r <= reps; ++r) {
            DFGT_HIP(hipEventRecord(res.e0, st));
            dfgt_tree T = nullptr;
            DFGT_TRY(dfgt_build_tree(pts_dev, n, d, &o, stream, &T));
            const dfgt_status sum = dfgt_gauss_sum(T, T, h_host, n_h, eps, &o, res.G, nullptr, stream);
            if (sum != DFGT_OK) {
                (void)dfgt_tree_free(T);
                return sum;
            }
            DFGT_HIP(hipEventRecord(res.e1, st));
            DFGT_HIP(hipEventSynchronize(res.e1));
            DFGT_TRY(dfgt_tree_free(T));
            float ms = 0.0f;
            DFGT_HIP(hipEventElapsedTime(&ms, res.e0, res.e1));
            if (r > 0) t.push_back(ms);  // the first repetition sizes the workspaces
        }
        std::sort(t.begin(), t.end());
        med[c] = t.size() % 2 ? t[t.size() / 2] : 0.5 * ((double)t[t.size() / 2 - 1] + t[t.size() / 2]);
        if (ms_out) ms_out[c] = med[c];
        best = c == 0 ? med[c] : std::min(best, med[c]);
    }
    // the smallest leaf size within kTuneTie of the fastest: near-ties (timing
    // noise) resolve the same way from call to call
    for (int c = 0; c < DFGT_N_TUNE_LEAVES; ++c)
        if (med[c] <= best * (1.0 + kTuneTie)) {
            *leaf_out = leaves[c];
            break;
        }
    return DFGT_OK;
    DFGT_GUARD_END
}

static dfgt_status collect_problems(const dfgt_problem *probs, int32_t n, double eps, const char *who,
                                    std::vector<Problem> &out) {
    DFGT_REQUIRE(probs != nullptr && n >= 1, std::string(who) + ": need at least one problem");
    long long jobs = 0;
    for (int i = 0; i < n; ++i) {
        const dfgt_problem &p = probs[i];
        DFGT_REQUIRE(p.Q && p.R && p.G_dev, std::string(who) + ": NULL tree or output in a problem");
        DFGT_TRY(check_pair(p.Q, p.R, eps, who));
        DFGT_TRY(check_bandwidths(p.h_host, p.n_h, who));
        DFGT_REQUIRE(p.Q->d == probs[0].Q->d && p.Q->pmax == probs[0].Q->pmax,
                     std::string(who) + ": all problems must share the dimension and p_max");
        jobs += p.n_h;
        out.push_back(Problem{p.Q, p.R, p.h_host, p.n_h, p.G_dev});
    }
    DFGT_REQUIRE(jobs <= (1 << 20), std::string(who) + ": more than 2^20 (problem, bandwidth) jobs");
    return DFGT_OK;
}

dfgt_status dfgt_gauss_sum_batched(const dfgt_problem *probs, int32_t n_probs, double eps,
                                   const dfgt_options *opt, dfgt_stats *stats, void *stream) {
    DFGT_GUARD_BEGIN
    std::vector<Problem> pr;
    DFGT_TRY(collect_problems(probs, n_probs, eps, "dfgt_gauss_sum_batched", pr));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(probs[0].R, opt, "dfgt_gauss_sum_batched", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0 || stats != nullptr, "dfgt_gauss_sum_batched: profile needs a stats pointer");
    return run_gauss_multi(pr.data(), (int)pr.size(), eps, precision, force, profile, cost_e, nullptr, stats,
                           (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_batch_create(const dfgt_problem *probs, int32_t n_probs, double eps, const dfgt_options *opt,
                              dfgt_stats *stats, void *stream, dfgt_batch *out) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(out != nullptr, "dfgt_batch_create: out is NULL");
    *out = nullptr;
    std::vector<Problem> pr;
    DFGT_TRY(collect_problems(probs, n_probs, eps, "dfgt_batch_create", pr));
    int precision, force, profile;
    double cost_e;
    DFGT_TRY(call_options(probs[0].R, opt, "dfgt_batch_create", &precision, &force, &profile, &cost_e));
    DFGT_REQUIRE(profile == 0, "dfgt_batch_create: profiling is not supported for captured batches");
    return batch_create(pr.data(), (int)pr.size(), eps, precision, force, cost_e, stats, (hipStream_t)stream, out);
    DFGT_GUARD_END
}

dfgt_status dfgt_batch_run(dfgt_batch b, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(b != nullptr, "dfgt_batch_run: batch is NULL");
    return batch_run(b, (hipStream_t)stream);
    DFGT_GUARD_END
}

dfgt_status dfgt_batch_check(dfgt_batch b, void *stream) {
    DFGT_GUARD_BEGIN
    DFGT_REQUIRE(b != nullptr, "dfgt_batch_check: batch is NULL");
    return batch_check(b, (hipStream_t)stream);
    DFGT_GUARD_END
}

}  // extern "C"
// dfgt_batch_free is defined in dfgt.hip, where the batch type is complete.
