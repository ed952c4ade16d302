// Raw far-field moments of every node of a reference tree (Alg. DFGTInitR).
//
//   mu_alpha(N) = sum_{x in N} (x - N.c)^alpha / alpha!,   alpha < p_max
//
// These are the paper's moments of Section 3.3, eq. (far_field_moments), without
// the bandwidth: M_alpha(h) = (2h^2)^{-|alpha|/2} mu_alpha, applied on the fly by
// every consumer, so one set of moments serves a whole bandwidth sweep.
//
// Small coefficient sets (p_max^D <= 64): AccumulateFarFieldMoment at every
// node, one launch.  Otherwise leaves by AccumulateFarFieldMoment (one wave
// per leaf, one lane per coefficient, points summed in tree order) and
// internal nodes bottom-up one level per launch: TransFarToFar of both
// children, eq. (far_to_far_translation),
// applied as D one-dimensional shifts
//   mu'_{..g..} = sum_{a <= g} mu_{..a..} delta_k^{g-a} / (g-a)!,  delta = child.c - parent.c,
// which is the same operator as the paper's double loop (the coefficient
// factorises over dimensions) at D p^{D+1} instead of p^{2D} operations.
#include "series.h"

namespace dfgt {
namespace {

constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }

__global__ __launch_bounds__(64) void k_p2m(const double *__restrict__ x, const double *__restrict__ wts,
                                            const double *__restrict__ ctr, const int32_t *__restrict__ begin,
                                            const int32_t *__restrict__ end, const int32_t *__restrict__ leaves,
                                            const int *__restrict__ nleaves, int d, int pmax, int P,
                                            double *__restrict__ mu) {
    if ((int)blockIdx.x >= *nleaves) return;
    const int node = leaves[blockIdx.x];
    const int b = begin[node], e = end[node];
    const double *c = ctr + (size_t)node * d;
    for (int i = threadIdx.x; i < P; i += 64) {
        int a[kMaxD];
        int r = i;
        double fac = 1.0;
        for (int k = d - 1; k >= 0; --k) {
            a[k] = r % pmax;
            r /= pmax;
            fac *= inv_factorial(a[k]);
        }
        double s = 0.0;
        for (int j = b; j < e; ++j) {
            double term = wts ? wts[j] : 1.0;
            for (int k = 0; k < d; ++k) {
                const double dx = x[(size_t)j * d + k] - c[k];
                for (int t = 0; t < a[k]; ++t) term *= dx;
            }
            s += term;
        }
        mu[(size_t)node * P + i] = s * fac;
    }
}

// One block per internal node of one level.  buf: 2*P doubles per block (LDS
// when small, else a global scratch slice).
// skip_le > 0: nodes of at most skip_le points already hold their moments.
template <bool kLds>
__global__ __launch_bounds__(256) void k_f2f(int lb, int le, const int32_t *__restrict__ left,
                                             const int32_t *__restrict__ right, const int32_t *__restrict__ begin,
                                             const int32_t *__restrict__ end, int skip_le,
                                             const double *__restrict__ ctr, int d, int pmax, int P,
                                             double *__restrict__ mu, double *__restrict__ gscratch) {
    extern __shared__ double smem[];
    const int node = lb + blockIdx.x;
    if (node >= le || left[node] < 0) return;
    if (skip_le > 0 && end[node] - begin[node] <= skip_le) return;
    double *coef = smem;                  // pmax * pmax
    double *buf0 = kLds ? smem + pmax * pmax : gscratch + (size_t)blockIdx.x * 2 * P;
    double *buf1 = buf0 + P;
    const int kids[2] = {left[node], right[node]};
    for (int i = threadIdx.x; i < P; i += blockDim.x) mu[(size_t)node * P + i] = 0.0;
    for (int c = 0; c < 2; ++c) {
        const int ch = kids[c];
        __syncthreads();
        for (int i = threadIdx.x; i < P; i += blockDim.x) buf0[i] = mu[(size_t)ch * P + i];
        double *src = buf0, *dst = buf1;
        for (int k = 0; k < d; ++k) {
            const double delta = ctr[(size_t)ch * d + k] - ctr[(size_t)node * d + k];
            __syncthreads();
            // coef[g][a] = delta^{g-a} / (g-a)! for a <= g
            for (int i = threadIdx.x; i < pmax * pmax; i += blockDim.x) {
                const int g = i / pmax, a = i % pmax;
                double v = 0.0;
                if (a <= g) {
                    v = inv_factorial(g - a);
                    for (int t = 0; t < g - a; ++t) v *= delta;
                }
                coef[i] = v;
            }
            __syncthreads();
            mode_product(src, dst, coef, P, d, pmax, k, pmax);
            double *tmp = src;
            src = dst;
            dst = tmp;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < P; i += blockDim.x) mu[(size_t)node * P + i] += src[i];
    }
}

// Small coefficient sets (p_max^D <= 64): the moments of every node straight
// from its points, AccumulateFarFieldMoment applied at each node instead of
// TransFarToFar between levels (the same sums, one launch instead of one per
// level).  One wave per node; lane l takes the node's points l, l + 64, ... in
// tree order and keeps all P partial sums in registers; the wave adds them in
// a fixed butterfly order.  Internal nodes with more than kMomDirectMax points
// are left to TransFarToFar from their children.
constexpr int kMomDirectMax = 512;

// Sum over the 64 lanes of each of the P per-lane partials acc[i], written to
// out[i]: the partials go through LDS (row per lane, padded against bank
// conflicts) and lane i adds column i in lane order, four loads at a time.
// A butterfly per coefficient would chain 6 P dependent cross-lane steps.
template <int P>
__device__ __forceinline__ void wave_sum_rows(const double (&acc)[P], double (*red)[P + 1], double *out) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < P; ++i) red[lane][i] = acc[i];
    __syncthreads();
    for (int i = lane; i < P; i += 64) {
        double v = 0.0;
        for (int r = 0; r < 64; r += 4) {
            const double a = red[r][i], b = red[r + 1][i], c = red[r + 2][i], e = red[r + 3][i];
            v += a;
            v += b;
            v += c;
            v += e;
        }
        out[i] = v;
    }
}

template <int D, int PM>
__global__ __launch_bounds__(64) void k_moments_direct(const double *__restrict__ x, const double *__restrict__ wts,
                                                       const double *__restrict__ ctr,
                                                       const int32_t *__restrict__ begin,
                                                       const int32_t *__restrict__ end,
                                                       const int32_t *__restrict__ left, double *__restrict__ mu) {
    constexpr int P = ipow_c(PM, D);
    const int node = blockIdx.x;
    const int b = begin[node], e = end[node];
    if (e - b > kMomDirectMax && left[node] >= 0) return;
    double c[D];
#pragma unroll
    for (int k = 0; k < D; ++k) c[k] = ctr[(size_t)node * D + k];
    double acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] = 0.0;
    for (int j = b + (int)threadIdx.x; j < e; j += 64) {
        double pw[D][PM];  // (x_k - c_k)^a / a!, the point's weight on dimension 0
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double dx = x[(size_t)j * D + k] - c[k];
            pw[k][0] = k == 0 && wts ? wts[j] : 1.0;
#pragma unroll
            for (int a = 1; a < PM; ++a) pw[k][a] = pw[k][a - 1] * dx / (double)a;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double t = 1.0;
            int r = i;
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                t *= pw[k][r % PM];
                r /= PM;
            }
            acc[i] += t;
        }
    }
    __shared__ double red[64][P + 1];
    wave_sum_rows<P>(acc, red, mu + (size_t)node * P);
}

// Internal nodes above kMomDirectMax points (the top levels): the same direct
// sums over chunks of kMomDirectMax points (a wave's sums take time in
// proportion to its points, so chunks keep the launch short), one wave per (node, chunk) for all
// these levels in one launch, then one block per node adds its chunks'
// partial moments in chunk order.  Levels in the table: nodes [lb, le), nch
// chunks per node (from the level's largest node), blocks [boff, boff + (le -
// lb) nch) of the chunk launch; a node block b of the reduce launch maps the
// same way with one block per node.
constexpr int kMomLevels = 32;
struct MomLevels {
    int n;
    int lb[kMomLevels], le[kMomLevels], nch[kMomLevels], boff[kMomLevels + 1], noff[kMomLevels + 1];
};

template <int D, int PM>
__global__ __launch_bounds__(64) void k_moments_chunk(const double *__restrict__ x, const double *__restrict__ wts,
                                                      const double *__restrict__ ctr,
                                                      const int32_t *__restrict__ begin,
                                                      const int32_t *__restrict__ end,
                                                      const int32_t *__restrict__ left, MomLevels lv,
                                                      double *__restrict__ part) {
    constexpr int P = ipow_c(PM, D);
    const int blk = blockIdx.x;
    int l = 0;
    while (blk >= lv.boff[l + 1]) ++l;
    const int idx = blk - lv.boff[l], node = lv.lb[l] + idx / lv.nch[l], ch = idx % lv.nch[l];
    const int b = begin[node], e = end[node];
    if (e - b <= kMomDirectMax || left[node] < 0) return;  // k_moments_direct's node
    const int cb = b + ch * kMomDirectMax, ce = min(e, cb + kMomDirectMax);
    double c[D];
#pragma unroll
    for (int k = 0; k < D; ++k) c[k] = ctr[(size_t)node * D + k];
    double acc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) acc[i] = 0.0;
    for (int j = cb + (int)threadIdx.x; j < ce; j += 64) {
        double pw[D][PM];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double dx = x[(size_t)j * D + k] - c[k];
            pw[k][0] = k == 0 && wts ? wts[j] : 1.0;
#pragma unroll
            for (int a = 1; a < PM; ++a) pw[k][a] = pw[k][a - 1] * dx / (double)a;
        }
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double t = 1.0;
            int r = i;
#pragma unroll
            for (int k = D - 1; k >= 0; --k) {
                t *= pw[k][r % PM];
                r /= PM;
            }
            acc[i] += t;
        }
    }
    __shared__ double red[64][P + 1];
    wave_sum_rows<P>(acc, red, part + (size_t)blk * P);
}

__global__ __launch_bounds__(64) void k_moments_chunk_sum(const int32_t *__restrict__ begin,
                                                          const int32_t *__restrict__ end,
                                                          const int32_t *__restrict__ left, MomLevels lv, int P,
                                                          const double *__restrict__ part, double *__restrict__ mu) {
    const int nb = blockIdx.x;
    int l = 0;
    while (nb >= lv.noff[l + 1]) ++l;
    const int node = lv.lb[l] + (nb - lv.noff[l]);
    const int b = begin[node], e = end[node];
    if (e - b <= kMomDirectMax || left[node] < 0) return;
    const int nc = (e - b + kMomDirectMax - 1) / kMomDirectMax;  // chunks that hold points (<= nch)
    const size_t p0 = (size_t)lv.boff[l] + (size_t)(nb - lv.noff[l]) * lv.nch[l];
    for (int i = threadIdx.x; i < P; i += blockDim.x) {  // chunk order, four loads at a time
        double v = 0.0;
        for (int k0 = 0; k0 < nc; k0 += 4) {
            double t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] = k0 + u < nc ? part[(p0 + k0 + u) * P + i] : 0.0;
            v += t[0];
            v += t[1];
            v += t[2];
            v += t[3];
        }
        mu[(size_t)node * P + i] = v;
    }
}

// Launches the chunked direct kernels when (D, p_max) has an instance.
bool launch_moments_chunks(int d, int pmax, int P, const MomLevels &lv, hipStream_t st, const double *x,
                           const double *wts, const double *ctr, const int32_t *begin, const int32_t *end,
                           const int32_t *left, double *part, double *mu) {
    const unsigned nblk = (unsigned)lv.boff[lv.n], nnode = (unsigned)lv.noff[lv.n];
#define DFGT_MOMC(DV, PV)                                                                                       \
    if (d == DV && pmax == PV) {                                                                                \
        hipLaunchKernelGGL((k_moments_chunk<DV, PV>), dim3(nblk), dim3(64), 0, st, x, wts, ctr, begin, end, left, \
                           lv, part);                                                                           \
        hipLaunchKernelGGL(k_moments_chunk_sum, dim3(nnode), dim3(64), 0, st, begin, end, left, lv, P, part, mu);  \
        return true;                                                                                            \
    }
    DFGT_MOMC(1, 1) DFGT_MOMC(1, 2) DFGT_MOMC(1, 4) DFGT_MOMC(1, 6) DFGT_MOMC(1, 8)
    DFGT_MOMC(2, 1) DFGT_MOMC(2, 2) DFGT_MOMC(2, 4) DFGT_MOMC(2, 6) DFGT_MOMC(2, 8)
    DFGT_MOMC(3, 1) DFGT_MOMC(3, 2) DFGT_MOMC(3, 4)
    DFGT_MOMC(4, 1) DFGT_MOMC(4, 2)
    DFGT_MOMC(5, 1) DFGT_MOMC(5, 2)
    DFGT_MOMC(6, 1) DFGT_MOMC(6, 2)
#undef DFGT_MOMC
    return false;
}

// Whether (D, p_max) has direct-moment instances (the lists below).
bool moments_direct_available(int d, int pmax) {
    switch (d) {
    case 1:
    case 2: return pmax == 1 || pmax == 2 || pmax == 4 || pmax == 6 || pmax == 8;
    case 3: return pmax == 1 || pmax == 2 || pmax == 4;
    case 4:
    case 5:
    case 6: return pmax == 1 || pmax == 2;
    default: return false;
    }
}

// Launches the direct kernel when (D, p_max) has an instance; false otherwise.
bool launch_moments_direct(int d, int pmax, int m, hipStream_t st, const double *x, const double *wts,
                           const double *ctr, const int32_t *begin, const int32_t *end, const int32_t *left,
                           double *mu) {
#define DFGT_MOM(DV, PV)                                                                                \
    if (d == DV && pmax == PV) {                                                                        \
        hipLaunchKernelGGL((k_moments_direct<DV, PV>), dim3(m), dim3(64), 0, st, x, wts, ctr, begin, end,     \
                           left, mu);                                                                   \
        return true;                                                                                    \
    }
    DFGT_MOM(1, 1) DFGT_MOM(1, 2) DFGT_MOM(1, 4) DFGT_MOM(1, 6) DFGT_MOM(1, 8)
    DFGT_MOM(2, 1) DFGT_MOM(2, 2) DFGT_MOM(2, 4) DFGT_MOM(2, 6) DFGT_MOM(2, 8)
    DFGT_MOM(3, 1) DFGT_MOM(3, 2) DFGT_MOM(3, 4)
    DFGT_MOM(4, 1) DFGT_MOM(4, 2)
    DFGT_MOM(5, 1) DFGT_MOM(5, 2)
    DFGT_MOM(6, 1) DFGT_MOM(6, 2)
#undef DFGT_MOM
    return false;
}

}  // namespace

// Squared norms of the points (tree order) and their maximum (ordered-int max
// of non-negative doubles); the matrix-core exhaustive tiles read them.
__global__ void k_tree_sqnorm(const double *__restrict__ x, int n, int d, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int k = 0; k < d; ++k) v = fma(x[(size_t)i * d + k], x[(size_t)i * d + k], v);
    out[i] = v;
}

// Per-node F2F scratch of the moment sweep when a level's tables do not fit in
// LDS; reused across builds of a thread (freeing it would stall the device).
static thread_local DevBuf g_mscratch;

void release_build_workspace() { g_mscratch.release(); }

dfgt_status compute_moments(dfgt_tree_s *t, hipStream_t st) {
    // Levels holding a node above kMomDirectMax points take chunked direct sums
    // (up to kMomLevels of them, and when (D, p_max) has a direct instance);
    // any others translate.  The chunk partials live in the tree's own memory:
    // the build returns with this work still queued.
    const bool has_direct = moments_direct_available(t->d, t->pmax);
    std::vector<char> chunked(t->level_start.size(), 0);
    MomLevels lv{};
    size_t nblk = 0;
    for (int l = 0; has_direct && l + 1 < (int)t->level_start.size() && lv.n < kMomLevels; ++l) {
        const int lb = t->level_start[l], le = t->level_start[l + 1];
        if (le <= lb || t->level_max[l] <= kMomDirectMax) continue;
        const int nch = (t->level_max[l] + kMomDirectMax - 1) / kMomDirectMax;
        if (nblk + (size_t)(le - lb) * nch > (1u << 20)) break;  // the rest translate
        lv.lb[lv.n] = lb;
        lv.le[lv.n] = le;
        lv.nch[lv.n] = nch;
        lv.boff[lv.n] = (int)nblk;
        lv.noff[lv.n + 1] = lv.noff[lv.n] + (le - lb);
        nblk += (size_t)(le - lb) * nch;
        lv.boff[++lv.n] = (int)nblk;
        chunked[l] = 1;
    }
    {
        const int n = (int)t->n;
        DFGT_TRY(alloc_spans(t->arena2, {{&t->nrm, sizeof(double) * (size_t)n},
                                         {&t->mu, sizeof(double) * (size_t)t->m * t->P},
                                         {&t->view, sizeof(DevTree)},
                                         {&t->mpart, sizeof(double) * nblk * t->P}},
                                st, true));
        hipLaunchKernelGGL(k_tree_sqnorm, dim3((n + 255) / 256), dim3(256), 0, st, t->x.as<double>(), n, t->d,
                           t->nrm.as<double>());
        DFGT_HIP(hipGetLastError());
    }
    const int d = t->d, pmax = t->pmax, P = t->P;
    const int64_t m = t->m;
    // the build has the leaf count and the largest squared norm; only a
    // weighted tree reads a value back (the root's mu_0, its total weight)
    static thread_local HostBuf back_h;
    DFGT_TRY(back_h.reserve(sizeof(double)));
    const double *wts = t->w.as<double>();
    const bool direct = launch_moments_direct(d, pmax, (int)m, st, t->x.as<double>(), wts, t->ctr.as<double>(),
                                              t->begin.as<int32_t>(), t->end.as<int32_t>(), t->left.as<int32_t>(),
                                              t->mu.as<double>());
    if (!direct)
        hipLaunchKernelGGL(k_p2m, dim3((unsigned)((m + 1) / 2)), dim3(64), 0, st, t->x.as<double>(), wts,
                           t->ctr.as<double>(), t->begin.as<int32_t>(), t->end.as<int32_t>(), t->leaves.as<int32_t>(),
                           t->nleaves_dev.as<int>(), d, pmax, P, t->mu.as<double>());
    DFGT_HIP(hipGetLastError());
    if (direct && lv.n > 0) {
        launch_moments_chunks(d, pmax, P, lv, st, t->x.as<double>(), wts, t->ctr.as<double>(), t->begin.as<int32_t>(),
                              t->end.as<int32_t>(), t->left.as<int32_t>(), t->mpart.as<double>(), t->mu.as<double>());
        DFGT_HIP(hipGetLastError());
    }
    const int skip = direct ? kMomDirectMax : 0;
    const bool lds = (size_t)(2 * P + pmax * pmax) * sizeof(double) <= 48 * 1024;
    int maxw = 0;
    for (int l = 0; l + 1 < (int)t->level_start.size(); ++l)
        maxw = std::max(maxw, t->level_start[l + 1] - t->level_start[l]);
    if (!lds) DFGT_TRY(g_mscratch.reserve(sizeof(double) * (size_t)maxw * 2 * P));
    for (int l = t->depth - 2; l >= 0; --l) {
        const int lb = t->level_start[l], le = t->level_start[l + 1];
        if (le <= lb) continue;
        if (direct && (t->level_max[l] <= kMomDirectMax || chunked[l])) continue;
        if (lds) {
            size_t sh = sizeof(double) * (2 * P + pmax * pmax);
            hipLaunchKernelGGL(k_f2f<true>, dim3(le - lb), dim3(256), sh, st, lb, le, t->left.as<int32_t>(),
                               t->right.as<int32_t>(), t->begin.as<int32_t>(), t->end.as<int32_t>(), skip,
                               t->ctr.as<double>(), d, pmax, P, t->mu.as<double>(), (double *)nullptr);
        } else {
            size_t sh = sizeof(double) * (pmax * pmax);
            hipLaunchKernelGGL(k_f2f<false>, dim3(le - lb), dim3(256), sh, st, lb, le, t->left.as<int32_t>(),
                               t->right.as<int32_t>(), t->begin.as<int32_t>(), t->end.as<int32_t>(), skip,
                               t->ctr.as<double>(), d, pmax, P, t->mu.as<double>(), g_mscratch.as<double>());
        }
        DFGT_HIP(hipGetLastError());
    }
    // the global F2F scratch is shared by the builds of this thread: wait
    // before another build can reuse it (the large-P path only)
    bool used_scratch = false;
    for (int l = t->depth - 2; l >= 0 && !lds; --l)
        if (t->level_start[l + 1] > t->level_start[l] && !(direct && (t->level_max[l] <= kMomDirectMax || chunked[l])))
            used_scratch = true;
    if (used_scratch && !t->weighted) DFGT_HIP(hipStreamSynchronize(st));
    if (t->weighted) {
        DFGT_HIP(hipMemcpyAsync(back_h.p, t->mu.p, sizeof(double), hipMemcpyDeviceToHost, st));
        DFGT_HIP(hipStreamSynchronize(st));
        t->wsum = back_h.as<double>()[0] * t->wscale;  // root mu_0 = sum of the stored weights
    } else {
        t->wsum = (double)t->n;
    }
    return DFGT_OK;
}

}  // namespace dfgt
