// Raw far-field moments of every node of a reference tree (Alg. DFGTInitR).
//
//   mu_alpha(N) = sum_{x in N} (x - N.c)^alpha / alpha!,   alpha < p_max
//
// These are the paper's moments of Section 3.3, eq. (far_field_moments), without
// the bandwidth: M_alpha(h) = (2h^2)^{-|alpha|/2} mu_alpha, applied on the fly by
// every consumer, so one set of moments serves a whole bandwidth sweep.
//
// Leaves: AccumulateFarFieldMoment (one wave per leaf, one lane per coefficient,
// points summed in tree order).  Internal nodes, bottom-up one level per
// launch: TransFarToFar of both children, eq. (far_to_far_translation),
// applied as D one-dimensional shifts
//   mu'_{..g..} = sum_{a <= g} mu_{..a..} delta_k^{g-a} / (g-a)!,  delta = child.c - parent.c,
// which is the same operator as the paper's double loop (the coefficient
// factorises over dimensions) at D p^{D+1} instead of p^{2D} operations.
#include "series.h"

namespace dfgt {
namespace {

__global__ __launch_bounds__(64) void k_p2m(const double *__restrict__ x, const double *__restrict__ ctr,
                                            const int32_t *__restrict__ begin, const int32_t *__restrict__ end,
                                            const int32_t *__restrict__ leaves, int d, int pmax, int P,
                                            double *__restrict__ mu) {
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
            double term = 1.0;
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
template <bool kLds>
__global__ __launch_bounds__(256) void k_f2f(int lb, int le, const int32_t *__restrict__ left,
                                             const int32_t *__restrict__ right, const double *__restrict__ ctr,
                                             int d, int pmax, int P, double *__restrict__ mu,
                                             double *__restrict__ gscratch) {
    extern __shared__ double smem[];
    const int node = lb + blockIdx.x;
    if (node >= le || left[node] < 0) return;
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

}  // namespace

// Squared norms of the points (tree order) and their maximum (ordered-int max
// of non-negative doubles); the matrix-core exhaustive tiles read them.
__global__ void k_tree_sqnorm(const double *__restrict__ x, int n, int d, double *__restrict__ out,
                              unsigned long long *__restrict__ mx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        for (int k = 0; k < d; ++k) v = fma(x[(size_t)i * d + k], x[(size_t)i * d + k], v);
        out[i] = v;
    }
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(mx, (unsigned long long)__double_as_longlong(v));
}

dfgt_status compute_moments(dfgt_tree_s *t, hipStream_t st) {
    {
        const int n = (int)t->n;
        DFGT_TRY(alloc_spans(t->arena2, {{&t->nrm, sizeof(double) * (size_t)n},
                                         {&t->nrm_max, sizeof(unsigned long long)},
                                         {&t->mu, sizeof(double) * (size_t)t->m * t->P},
                                         {&t->view, sizeof(DevTree)}}));
        DFGT_HIP(hipMemsetAsync(t->nrm_max.p, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_tree_sqnorm, dim3((n + 255) / 256), dim3(256), 0, st, t->x.as<double>(), n, t->d,
                           t->nrm.as<double>(), t->nrm_max.as<unsigned long long>());
        DFGT_HIP(hipGetLastError());
        DFGT_HIP(hipMemcpyAsync(&t->max_nrm, t->nrm_max.p, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    const int d = t->d, pmax = t->pmax, P = t->P;
    const int64_t m = t->m;
    hipLaunchKernelGGL(k_p2m, dim3((unsigned)t->nleaves), dim3(64), 0, st, t->x.as<double>(), t->ctr.as<double>(),
                       t->begin.as<int32_t>(), t->end.as<int32_t>(), t->leaves.as<int32_t>(), d, pmax, P,
                       t->mu.as<double>());
    DFGT_HIP(hipGetLastError());
    const bool lds = (size_t)(2 * P + pmax * pmax) * sizeof(double) <= 48 * 1024;
    static thread_local DevBuf scratch;  // reused across builds (freeing it would stall the device)
    int maxw = 0;
    for (int l = 0; l + 1 < (int)t->level_start.size(); ++l)
        maxw = std::max(maxw, t->level_start[l + 1] - t->level_start[l]);
    if (!lds) DFGT_TRY(scratch.reserve(sizeof(double) * (size_t)maxw * 2 * P));
    for (int l = t->depth - 2; l >= 0; --l) {
        const int lb = t->level_start[l], le = t->level_start[l + 1];
        if (le <= lb) continue;
        if (lds) {
            size_t sh = sizeof(double) * (2 * P + pmax * pmax);
            hipLaunchKernelGGL(k_f2f<true>, dim3(le - lb), dim3(256), sh, st, lb, le, t->left.as<int32_t>(),
                               t->right.as<int32_t>(), t->ctr.as<double>(), d, pmax, P, t->mu.as<double>(),
                               (double *)nullptr);
        } else {
            size_t sh = sizeof(double) * (pmax * pmax);
            hipLaunchKernelGGL(k_f2f<false>, dim3(le - lb), dim3(256), sh, st, lb, le, t->left.as<int32_t>(),
                               t->right.as<int32_t>(), t->ctr.as<double>(), d, pmax, P, t->mu.as<double>(),
                               scratch.as<double>());
        }
        DFGT_HIP(hipGetLastError());
    }
    return DFGT_OK;
}

}  // namespace dfgt
