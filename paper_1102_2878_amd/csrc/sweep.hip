// Drivers built on run_gauss_sum: the vector-Jacobian product of the sums
// (backward), the least-squares cross-validation score of Section 1 (eq. of
// the LSCV score) with its bandwidth derivative, and the search for the
// bandwidth that minimises it (Section 4 sets its bandwidths relative to
// that minimiser).
//
// All reductions are deterministic: a fixed partition of each row into
// kRowBlocks chunks, a fixed-order tree inside each block, then the chunk
// partials added in order by one thread.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dfgt_internal.h"

namespace dfgt {
namespace {

constexpr int kRowBlocks = 256;
constexpr int kRedThreads = 256;

enum { ROW_DOT = 0, ROW_LOG = 1, ROW_RATIO = 2 };

// part[row][blk] = sum over the block's chunk of f(a[row][i], b[row][i]):
//   ROW_DOT    a * (b ? b : 1) - bias
//   ROW_LOG    log(a - bias)
//   ROW_RATIO  b / (a - bias)
__global__ __launch_bounds__(kRedThreads) void k_rowdot(const double *__restrict__ a, const double *__restrict__ b,
                                                        double bias, int mode, long long n,
                                                        double *__restrict__ part) {
    __shared__ double red[kRedThreads];
    const int row = blockIdx.y;
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long i0 = (long long)blockIdx.x * chunk;
    const long long i1 = i0 + chunk < n ? i0 + chunk : n;
    const double *ar = a + (size_t)row * n;
    const double *br = b ? b + (size_t)row * n : nullptr;
    double v = 0.0;
    for (long long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        if (mode == ROW_DOT) v += (br ? ar[i] * br[i] : ar[i]) - bias;
        else if (mode == ROW_LOG) v += log(ar[i] - bias);
        else v += br[i] / (ar[i] - bias);
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)row * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_rowdot_final(const double *__restrict__ part, int nblk, int rows, double *__restrict__ out) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= rows) return;
    double v = 0.0;
    for (int k = 0; k < nblk; ++k) v += part[(size_t)row * nblk + k];
    out[row] = v;
}

// dq[i][c] = sum_k dG[k][i] * J[k][i][c]  (bandwidths in order)
__global__ void k_dq(const double *__restrict__ dG, const double *__restrict__ J, int nh, long long nq, int d,
                     double *__restrict__ dq) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nq * d) return;
    const long long i = idx / d;
    double v = 0.0;
    for (int k = 0; k < nh; ++k) v = fma(dG[(size_t)k * nq + i], J[(size_t)k * nq * d + idx], v);
    dq[idx] = v;
}

// p[k][i] = G[k][i] * scale[k] (the density estimate's normalisation per bandwidth)
__global__ void k_scale_rows(double *__restrict__ p, const double *__restrict__ scale, long long n, int rows) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * rows) return;
    p[idx] *= scale[idx / n];
}

struct SweepWs {
    DevBuf G, dGdh, dGdq, part, sums, scale;
};
thread_local SweepWs g_sw;

// out_host[row] = sum_i f(a[row][i], b[row][i]) (k_rowdot's modes), deterministic.
dfgt_status row_sums(const double *a, const double *b, double bias, long long n, int rows, double *out_host,
                     hipStream_t st, int mode = ROW_DOT) {
    SweepWs &w = g_sw;
    DFGT_TRY(w.part.reserve(sizeof(double) * (size_t)rows * kRowBlocks));
    DFGT_TRY(w.sums.reserve(sizeof(double) * (size_t)rows));
    hipLaunchKernelGGL(k_rowdot, dim3(kRowBlocks, rows), dim3(kRedThreads), 0, st, a, b, bias, mode, n,
                       w.part.as<double>());
    DFGT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rowdot_final, dim3((rows + 63) / 64), dim3(64), 0, st, w.part.as<double>(), kRowBlocks,
                       rows, w.sums.as<double>());
    DFGT_HIP(hipGetLastError());
    DFGT_HIP(hipMemcpyAsync(out_host, w.sums.p, sizeof(double) * rows, hipMemcpyDeviceToHost, st));
    DFGT_HIP(hipStreamSynchronize(st));
    return DFGT_OK;
}

}  // namespace

dfgt_status run_backward(dfgt_tree_s *Q, dfgt_tree_s *R, const double *h, int nh, double eps, int precision,
                         int force, double cost_e, const double *dG, double *dh_host, double *dq, hipStream_t st) {
    SweepWs &w = g_sw;
    const size_t nq = (size_t)Q->n, d = (size_t)Q->d;
    DFGT_TRY(w.G.reserve(sizeof(double) * nh * nq));
    if (dh_host) DFGT_TRY(w.dGdh.reserve(sizeof(double) * nh * nq));
    if (dq) DFGT_TRY(w.dGdq.reserve(sizeof(double) * nh * nq * d));
    GradOut go{dh_host ? w.dGdh.as<double>() : nullptr, dq ? w.dGdq.as<double>() : nullptr};
    DFGT_TRY(run_gauss_sum(Q, R, h, nh, eps, precision, force, 0, cost_e, w.G.as<double>(), &go, nullptr, st));
    if (dq) {
        const long long tot = (long long)(nq * d);
        hipLaunchKernelGGL(k_dq, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, dG, w.dGdq.as<double>(), nh,
                           (long long)nq, (int)d, dq);
        DFGT_HIP(hipGetLastError());
    }
    if (dh_host) DFGT_TRY(row_sums(dG, w.dGdh.as<double>(), 0.0, (long long)nq, nh, dh_host, st));
    return DFGT_OK;
}

void release_sweep_workspace() {
    SweepWs &w = g_sw;
    for (DevBuf *b : {&w.G, &w.dGdh, &w.dGdq, &w.part, &w.sums, &w.scale}) b->release();
}

dfgt_status run_vjp(int nh, int64_t nq, int d, const double *dG, const double *dGdh, const double *dGdq,
                    double *dh_host, double *dq, hipStream_t st) {
    if (dq) {
        const long long tot = (long long)nq * d;
        hipLaunchKernelGGL(k_dq, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, dG, dGdq, nh, (long long)nq, d,
                           dq);
        DFGT_HIP(hipGetLastError());
    }
    if (dh_host) DFGT_TRY(row_sums(dG, dGdh, 0.0, (long long)nq, nh, dh_host, st));
    return DFGT_OK;
}

dfgt_status run_lscv(dfgt_tree_s *R, const double *h, int nh, double eps, int precision, int force, double cost_e,
                     int variant, double *cv, double *dcv, dfgt_stats *stats, hipStream_t st) {
    SweepWs &w = g_sw;
    const size_t n = (size_t)R->n;
    const int nj = 2 * nh;
    // jobs: the bandwidths h_k, then sqrt(2) h_k (the Gaussian convolved with
    // itself is a Gaussian of bandwidth sqrt(2) h)
    std::vector<double> hh(nj);
    for (int k = 0; k < nh; ++k) {
        hh[k] = h[k];
        hh[nh + k] = std::sqrt(2.0) * h[k];
    }
    DFGT_TRY(w.G.reserve(sizeof(double) * nj * n));
    if (dcv) DFGT_TRY(w.dGdh.reserve(sizeof(double) * nj * n));
    GradOut go{dcv ? w.dGdh.as<double>() : nullptr, nullptr};
    // leave-one-out sums G_j(x_i) - 1, each within eps of its own value
    DFGT_TRY(run_gauss_sum(R, R, hh.data(), nj, eps, precision, force, 0, cost_e, w.G.as<double>(),
                           dcv ? &go : nullptr, stats, st, true));
    // S_j = sum_i (G_j(x_i) - 1)
    std::vector<double> S(nj), dS(nj, 0.0);
    DFGT_TRY(row_sums(w.G.as<double>(), nullptr, 0.0, (long long)n, nj, S.data(), st));
    if (dcv) DFGT_TRY(row_sums(w.dGdh.as<double>(), nullptr, 0.0, (long long)n, nj, dS.data(), st));
    const double N = (double)n, D = (double)R->d, pi = 3.14159265358979323846;
    for (int k = 0; k < nh; ++k) {
        const double hk = h[k];
        const double S1 = S[k], S2 = S[nh + k];
        const double dS1 = dS[k], dS2 = std::sqrt(2.0) * dS[nh + k];  // d/dh of the sqrt(2) h sums
        // Gaussian normalisations at sqrt(2) h and h
        const double a = std::pow(4.0 * pi * hk * hk, -0.5 * D), b = std::pow(2.0 * pi * hk * hk, -0.5 * D);
        const double da = -D * a / hk, db = -D * b / hk;
        const double nn1 = N * (N - 1.0);
        if (variant == 0) {
            cv[k] = (a * S2 - 2.0 * b * S1) / nn1;
            if (dcv) dcv[k] = (da * S2 + a * dS2 - 2.0 * (db * S1 + b * dS1)) / nn1;
        } else {
            cv[k] = a * (N + S2) / (N * N) - 2.0 * b * S1 / nn1;
            if (dcv) dcv[k] = (da * (N + S2) + a * dS2) / (N * N) - 2.0 * (db * S1 + b * dS1) / nn1;
        }
    }
    return DFGT_OK;
}

dfgt_status run_lcv(dfgt_tree_s *R, const double *h, int nh, double eps, int precision, int force, double cost_e,
                    double *cv, double *dcv, dfgt_stats *stats, hipStream_t st) {
    SweepWs &w = g_sw;
    const size_t n = (size_t)R->n;
    DFGT_TRY(w.G.reserve(sizeof(double) * nh * n));
    if (dcv) DFGT_TRY(w.dGdh.reserve(sizeof(double) * nh * n));
    GradOut go{dcv ? w.dGdh.as<double>() : nullptr, nullptr};
    // leave-one-out sums G(r_j) - 1, each within eps of its own value
    DFGT_TRY(run_gauss_sum(R, R, h, nh, eps, precision, force, 0, cost_e, w.G.as<double>(), dcv ? &go : nullptr,
                           stats, st, true));
    // sum_j log(G(r_j) - 1)
    std::vector<double> L(nh), dL(nh, 0.0);
    DFGT_TRY(row_sums(w.G.as<double>(), nullptr, 0.0, (long long)n, nh, L.data(), st, ROW_LOG));
    if (dcv) DFGT_TRY(row_sums(w.G.as<double>(), w.dGdh.as<double>(), 0.0, (long long)n, nh, dL.data(), st, ROW_RATIO));
    const double N = (double)n, D = (double)R->d, pi = 3.14159265358979323846;
    for (int k = 0; k < nh; ++k) {
        const double logV = 0.5 * D * std::log(2.0 * pi * h[k] * h[k]);
        cv[k] = L[k] / N - std::log(N - 1.0) - logV;
        if (dcv) dcv[k] = dL[k] / N - D / h[k];
    }
    return DFGT_OK;
}

dfgt_status run_density(dfgt_tree_s *Q, dfgt_tree_s *R, const double *h, int nh, double eps, int precision,
                        int force, double cost_e, double *p, dfgt_stats *stats, hipStream_t st) {
    SweepWs &w = g_sw;
    DFGT_TRY(run_gauss_sum(Q, R, h, nh, eps, precision, force, 0, cost_e, p, nullptr, stats, st));
    const double pi = 3.14159265358979323846, D = (double)R->d, NR = R->wsum;  // W(R): n when unweighted
    std::vector<double> sc(nh);
    for (int k = 0; k < nh; ++k) sc[k] = 1.0 / (NR * std::pow(2.0 * pi * h[k] * h[k], 0.5 * D));
    DFGT_TRY(w.scale.reserve(sizeof(double) * nh));
    DFGT_HIP(hipMemcpyAsync(w.scale.p, sc.data(), sizeof(double) * nh, hipMemcpyHostToDevice, st));
    const long long tot = (long long)nh * Q->n;
    hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, p, w.scale.as<double>(),
                       (long long)Q->n, nh);
    DFGT_HIP(hipGetLastError());
    // the host vector is read by the copy: wait before it goes out of scope
    DFGT_HIP(hipStreamSynchronize(st));
    return DFGT_OK;
}

dfgt_status run_lscv_optimize(dfgt_tree_s *R, double h_lo, double h_hi, double eps, int precision, int force,
                              double cost_e, int variant, int n_grid, double rel_tol, double *h_star,
                              double *cv_star, int *n_evals, hipStream_t st) {
    // successive log-spaced grids over the bracket; each grid is one score call
    // (all its bandwidths in one traversal); the next bracket is the two cells
    // around the grid's smallest score (first one on ties)
    double a = std::log(h_lo), b = std::log(h_hi);
    const double stop = std::log1p(rel_tol);
    std::vector<double> hs(n_grid), cv(n_grid);
    double best_h = h_lo, best_cv = 0.0;
    int evals = 0;
    for (int round = 0; round < 64; ++round) {
        for (int k = 0; k < n_grid; ++k) hs[k] = std::exp(a + (b - a) * k / (n_grid - 1));
        DFGT_TRY(run_lscv(R, hs.data(), n_grid, eps, precision, force, cost_e, variant, cv.data(), nullptr,
                          nullptr, st));
        evals += n_grid;
        int kb = 0;
        for (int k = 1; k < n_grid; ++k)
            if (cv[k] < cv[kb]) kb = k;
        if (round == 0 || cv[kb] < best_cv) {
            best_cv = cv[kb];
            best_h = hs[kb];
        }
        const double na = a + (b - a) * std::max(kb - 1, 0) / (n_grid - 1);
        const double nb = a + (b - a) * std::min(kb + 1, n_grid - 1) / (n_grid - 1);
        if (nb - na <= 2.0 * stop) break;
        a = na;
        b = nb;
    }
    *h_star = best_h;
    if (cv_star) *cv_star = best_cv;
    if (n_evals) *n_evals = evals;
    return DFGT_OK;
}

}  // namespace dfgt
