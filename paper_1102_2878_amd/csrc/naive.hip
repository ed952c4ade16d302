// Brute-force Gaussian sums (Alg. NaiveKDE, Section 1) as a tiled GPU kernel.
//
// Layout: grid (query tiles, reference chunks, bandwidths).  A 256-thread block
// holds QPT queries per thread in registers, pre-scaled by sigma; reference
// points of its chunk are staged through LDS (scaled once per block) and read
// by broadcast.  Mixed precision: the squared scaled distance is formed in
// FP64 (no cancellation loss however wide the data is relative to h), rounded
// once to FP32 for the hardware exp2, summed in FP32 over at most 64 points and
// then in FP64.  Partial sums per chunk are reduced in chunk order, so results
// are bitwise reproducible.
#include "dfgt_internal.h"

namespace dfgt {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 512;   // reference points per LDS stage
constexpr int kInner = 64;   // points per FP32 partial sum

// sigma = sqrt(log2 e) / (sqrt(2) h): exp(-|q-r|^2 / 2h^2) = exp2(-|sigma (q - r)|^2).
__device__ __forceinline__ double sigma_mixed(double h) {
    return 1.2011224087864498 / (1.4142135623730951 * h);
}

template <int D, int QPT>
__global__ __launch_bounds__(kBlock) void k_naive_mixed(const double *__restrict__ q, int nq,
                                                        const double *__restrict__ r, int nr,
                                                        const double *__restrict__ hs, int chunk_len,
                                                        int nchunks, double *__restrict__ part) {
    __shared__ double tile[kTile * D];
    const int hz = blockIdx.z;
    const double sig = sigma_mixed(hs[hz]);
    double qs[QPT][D];
    double acc[QPT];
#pragma unroll
    for (int a = 0; a < QPT; ++a) {
        int qi = (blockIdx.x * QPT + a) * kBlock + threadIdx.x;
        int qc = qi < nq ? qi : nq - 1;
#pragma unroll
        for (int k = 0; k < D; ++k) qs[a][k] = q[(size_t)qc * D + k] * sig;
        acc[a] = 0.0;
    }
    const int rbeg = blockIdx.y * chunk_len;
    const int rend = min(nr, rbeg + chunk_len);
    for (int t0 = rbeg; t0 < rend; t0 += kTile) {
        const int cnt = min(kTile, rend - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * D; i += kBlock) tile[i] = r[(size_t)t0 * D + i] * sig;
        __syncthreads();
        for (int j0 = 0; j0 < cnt; j0 += kInner) {
            const int jn = min(kInner, cnt - j0);
            float ps[QPT];
#pragma unroll
            for (int a = 0; a < QPT; ++a) ps[a] = 0.0f;
            for (int j = 0; j < jn; ++j) {
                const double *rp = &tile[(j0 + j) * D];
                double rv[D];
#pragma unroll
                for (int k = 0; k < D; ++k) rv[k] = rp[k];
#pragma unroll
                for (int a = 0; a < QPT; ++a) {
                    double dd = qs[a][0] - rv[0];
                    double t = dd * dd;
#pragma unroll
                    for (int k = 1; k < D; ++k) {
                        dd = qs[a][k] - rv[k];
                        t = fma(dd, dd, t);
                    }
                    ps[a] += __builtin_amdgcn_exp2f(-(float)t);
                }
            }
#pragma unroll
            for (int a = 0; a < QPT; ++a) acc[a] += (double)ps[a];
        }
    }
#pragma unroll
    for (int a = 0; a < QPT; ++a) {
        int qi = (blockIdx.x * QPT + a) * kBlock + threadIdx.x;
        if (qi < nq) part[((size_t)hz * nchunks + blockIdx.y) * nq + qi] = acc[a];
    }
}

// Generic-dimension mixed kernel (d <= kMaxD), one query per thread.
__global__ __launch_bounds__(kBlock) void k_naive_mixed_any(const double *__restrict__ q, int nq,
                                                            const double *__restrict__ r, int nr, int d,
                                                            const double *__restrict__ hs,
                                                            int chunk_len, int nchunks,
                                                            double *__restrict__ part) {
    extern __shared__ double tile_dyn[];
    const int hz = blockIdx.z;
    const double sig = sigma_mixed(hs[hz]);
    const int qi = blockIdx.x * kBlock + threadIdx.x;
    const int qc = qi < nq ? qi : nq - 1;
    double qs[kMaxD];
    for (int k = 0; k < d; ++k) qs[k] = q[(size_t)qc * d + k] * sig;
    double acc = 0.0;
    const int tile = 4096 / d;
    const int rbeg = blockIdx.y * chunk_len;
    const int rend = min(nr, rbeg + chunk_len);
    for (int t0 = rbeg; t0 < rend; t0 += tile) {
        const int cnt = min(tile, rend - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * d; i += kBlock) tile_dyn[i] = r[(size_t)t0 * d + i] * sig;
        __syncthreads();
        for (int j0 = 0; j0 < cnt; j0 += kInner) {
            const int jn = min(kInner, cnt - j0);
            float ps = 0.0f;
            for (int j = 0; j < jn; ++j) {
                const double *rp = &tile_dyn[(j0 + j) * d];
                double t = 0.0;
                for (int k = 0; k < d; ++k) {
                    double dd = qs[k] - rp[k];
                    t = fma(dd, dd, t);
                }
                ps += __builtin_amdgcn_exp2f(-(float)t);
            }
            acc += (double)ps;
        }
    }
    if (qi < nq) part[((size_t)hz * nchunks + blockIdx.y) * nq + qi] = acc;
}

// FP64 kernel: s = 1/(sqrt(2) h), v = exp(-|s (q - r)|^2) in FP64.
__global__ __launch_bounds__(kBlock) void k_naive_fp64(const double *__restrict__ q, int nq,
                                                       const double *__restrict__ r, int nr, int d,
                                                       const double *__restrict__ hs, int chunk_len,
                                                       int nchunks, double *__restrict__ part) {
    extern __shared__ double tile_dyn[];
    const int hz = blockIdx.z;
    const double s = 1.0 / (1.4142135623730951 * hs[hz]);
    const int qi = blockIdx.x * kBlock + threadIdx.x;
    const int qc = qi < nq ? qi : nq - 1;
    double qs[kMaxD];
    for (int k = 0; k < d; ++k) qs[k] = q[(size_t)qc * d + k];
    double acc = 0.0;
    const int tile = 4096 / d;
    const int rbeg = blockIdx.y * chunk_len;
    const int rend = min(nr, rbeg + chunk_len);
    for (int t0 = rbeg; t0 < rend; t0 += tile) {
        const int cnt = min(tile, rend - t0);
        __syncthreads();
        for (int i = threadIdx.x; i < cnt * d; i += kBlock) tile_dyn[i] = r[(size_t)t0 * d + i];
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const double *rp = &tile_dyn[j * d];
            double t = 0.0;
            for (int k = 0; k < d; ++k) {
                double dd = (qs[k] - rp[k]) * s;
                t = fma(dd, dd, t);
            }
            acc += exp(-t);
        }
    }
    if (qi < nq) part[((size_t)hz * nchunks + blockIdx.y) * nq + qi] = acc;
}

__global__ void k_reduce_chunks(const double *__restrict__ part, int nq, int nchunks, int nh,
                                double *__restrict__ G) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int hz = blockIdx.y;
    if (i >= nq) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[((size_t)hz * nchunks + c) * nq + i];
    G[(size_t)hz * nq + i] = s;
}

// Workspace reused across calls on this thread (the brute force is a comparator,
// called from one host thread at a time).
thread_local DevBuf g_part, g_h;

}  // namespace

dfgt_status launch_naive(const double *q, int64_t nq64, const double *r, int64_t nr64, int d,
                         const double *h_host, int nh, int precision, double *G, hipStream_t st) {
    const int nq = (int)nq64, nr = (int)nr64;
    DFGT_TRY(g_h.reserve(sizeof(double) * nh));
    DFGT_HIP(hipMemcpyAsync(g_h.p, h_host, sizeof(double) * nh, hipMemcpyHostToDevice, st));
    int qpt = 1;
    bool specialised = precision == DFGT_PREC_MIXED && (d == 1 || d == 2 || d == 3 || d == 5);
    if (specialised) qpt = 2;
    const int bx = (nq + kBlock * qpt - 1) / (kBlock * qpt);
    // enough blocks to fill 256 CUs several times over
    int nchunks = (4096 + bx * nh - 1) / (bx * nh);
    const int max_chunks = (nr + kTile - 1) / kTile;
    if (nchunks > max_chunks) nchunks = max_chunks;
    if (nchunks < 1) nchunks = 1;
    int chunk_len = (nr + nchunks - 1) / nchunks;
    chunk_len = (chunk_len + kInner - 1) / kInner * kInner;
    nchunks = (nr + chunk_len - 1) / chunk_len;
    DFGT_TRY(g_part.reserve(sizeof(double) * (size_t)nchunks * nq * nh));
    double *part = g_part.as<double>();
    const double *hd = g_h.as<double>();
    dim3 grid(bx, nchunks, nh);
    if (precision == DFGT_PREC_FP64) {
        size_t lds = sizeof(double) * (4096 / d) * d;
        hipLaunchKernelGGL(k_naive_fp64, grid, dim3(kBlock), lds, st, q, nq, r, nr, d, hd, chunk_len,
                           nchunks, part);
    } else if (d == 1) {
        hipLaunchKernelGGL((k_naive_mixed<1, 2>), grid, dim3(kBlock), 0, st, q, nq, r, nr, hd, chunk_len,
                           nchunks, part);
    } else if (d == 2) {
        hipLaunchKernelGGL((k_naive_mixed<2, 2>), grid, dim3(kBlock), 0, st, q, nq, r, nr, hd, chunk_len,
                           nchunks, part);
    } else if (d == 3) {
        hipLaunchKernelGGL((k_naive_mixed<3, 2>), grid, dim3(kBlock), 0, st, q, nq, r, nr, hd, chunk_len,
                           nchunks, part);
    } else if (d == 5) {
        hipLaunchKernelGGL((k_naive_mixed<5, 2>), grid, dim3(kBlock), 0, st, q, nq, r, nr, hd, chunk_len,
                           nchunks, part);
    } else {
        size_t lds = sizeof(double) * (4096 / d) * d;
        hipLaunchKernelGGL(k_naive_mixed_any, grid, dim3(kBlock), lds, st, q, nq, r, nr, d, hd, chunk_len,
                           nchunks, part);
    }
    DFGT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_chunks, dim3((nq + 255) / 256, nh), dim3(256), 0, st, part, nq, nchunks, nh,
                       G);
    DFGT_HIP(hipGetLastError());
    return DFGT_OK;
}

}  // namespace dfgt
