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
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "etile.h"

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

// Matrix-core kernel for D >= 8 (see etile.h): a block of 4 waves holds 64
// queries (4 blocks of 16) as MFMA fragments; its waves take the 16-point
// reference blocks of the block's chunk round-robin.  Per lane: query
// l % 16 of each query block against references 4r + g of each reference
// block; FP32 partials over 16 reference blocks (64 terms), then FP64; the
// lane groups and the waves are added in a fixed order.
template <int NC>
__global__ __launch_bounds__(256) void k_naive_mfma(const double *__restrict__ q, const double *__restrict__ qn,
                                                    int nq, const double *__restrict__ r,
                                                    const double *__restrict__ rn, int nr, int d,
                                                    const double *__restrict__ hs, int fp64, int chunk_len,
                                                    int nchunks, double *__restrict__ part) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4;
    const int hz = blockIdx.z;
    const double s = 1.0 / (1.4142135623730951 * hs[hz]);
    const double sc = fp64 ? s : 1.2011224087864498 * s;  // mixed: 2^{-(sc |q-r|)^2}
    const double sc2 = sc * sc;
    const int q0 = blockIdx.x * 64;
    double qf[4][NC], qnv[4];
    bool qok[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int rb = q0 + 16 * b, nv = min(16, nq - rb);
        qok[b] = nv > 0;
        if (qok[b]) {
            load_frag<NC>(q, rb, nv, d, qf[b]);
            qnv[b] = qn[rb + min(lane & 15, nv - 1)];
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) qf[b][c] = 0.0;
            qnv[b] = 0.0;
        }
    }
    const int rbeg = blockIdx.y * chunk_len;
    const int rend = min(nr, rbeg + chunk_len);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    float ps[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int nblk = 0;
    for (int r0 = rbeg + 16 * wv; r0 < rend; r0 += 64) {
        const int nv = min(16, rend - r0);
        double rf[NC];
        load_frag<NC>(r, r0, nv, d, rf);
        double rnv[4];
        bool rok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int j = 4 * k + g;
            rok[k] = j < nv;
            rnv[k] = rn[r0 + min(j, nv - 1)];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (!qok[b]) continue;
            const v4d dt = block_dots<NC>(rf, qf[b]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double t = fmax(fma(-2.0, dt[k], qnv[b] + rnv[k]), 0.0) * sc2;
                if (fp64) acc[b] += rok[k] ? exp(-t) : 0.0;
                else ps[b] += rok[k] ? __builtin_amdgcn_exp2f(-(float)t) : 0.0f;
            }
        }
        if (++nblk == 16) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[b] += (double)ps[b];
                ps[b] = 0.0f;
            }
            nblk = 0;
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double v = acc[b] + (double)ps[b];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == 0) red[wv][16 * b + lane] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int qi = q0 + threadIdx.x;
        const double v = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
        if (qi < nq) part[((size_t)hz * nchunks + blockIdx.y) * nq + qi] = v;
    }
}

// Squared norms of n points and their maximum (ordered-int max of non-negative doubles).
__global__ void k_sqnorm(const double *__restrict__ x, int n, int d, double *__restrict__ out,
                         unsigned long long *__restrict__ mx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n)
        for (int k = 0; k < d; ++k) v = fma(x[(size_t)i * d + k], x[(size_t)i * d + k], v);
    if (i < n) out[i] = v;
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(mx, (unsigned long long)__double_as_longlong(v));
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
thread_local DevBuf g_part, g_h, g_qn, g_rn, g_mx;

__global__ void k_zero_u64(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Device memory of one brute-force call: chunk partials, the bandwidths, the
// norm tables of the matrix-core form and their maxima.
struct NaiveBufs {
    double *part, *h, *qn, *rn;
    unsigned long long *mx;
};

// Where a call's buffers come from: the thread's growing workspace (pool =
// null), or a fixed region of `cap` doubles carved in a fixed layout (no
// allocation).  part_doubles(n) sizes the partials for n doubles.
struct NaiveSpace {
    double *pool = nullptr;
    size_t cap = 0;
    // doubles before the partials: bandwidths, norms, maxima (256-byte aligned pieces)
    static size_t round(size_t n) { return (n + 31) / 32 * 32; }
    size_t head(int nq, int nr, int nh) const { return round(nh) + round(nq) + round(nr) + 32; }
    // the most partial doubles this space can give (SIZE_MAX: unbounded)
    size_t part_max(int nq, int nr, int nh) const {
        if (!pool) return SIZE_MAX;
        const size_t h0 = head(nq, nr, nh);
        return cap > h0 ? cap - h0 : 0;
    }
    dfgt_status get(int nq, int nr, int nh, size_t part_doubles, bool norms, NaiveBufs *b) const {
        if (!pool) {
            DFGT_TRY(g_h.reserve(sizeof(double) * nh));
            DFGT_TRY(g_part.reserve(sizeof(double) * part_doubles));
            if (norms) {
                DFGT_TRY(g_qn.reserve(sizeof(double) * nq));
                DFGT_TRY(g_rn.reserve(sizeof(double) * nr));
                DFGT_TRY(g_mx.reserve(2 * sizeof(unsigned long long)));
            }
            *b = NaiveBufs{g_part.as<double>(), g_h.as<double>(), g_qn.as<double>(), g_rn.as<double>(),
                           g_mx.as<unsigned long long>()};
            return DFGT_OK;
        }
        double *p = pool;
        b->h = p;
        p += round(nh);
        b->qn = p;
        p += round(nq);
        b->rn = p;
        p += round(nr);
        b->mx = reinterpret_cast<unsigned long long *>(p);
        p += 32;
        b->part = p;
        return DFGT_OK;
    }
};

template <int NC>
void launch_mfma(dim3 grid, hipStream_t st, const double *q, const double *qn, int nq, const double *r,
                 const double *rn, int nr, int d, const double *hd, int fp64, int chunk_len, int nchunks,
                 double *part) {
    hipLaunchKernelGGL(k_naive_mfma<NC>, grid, dim3(256), 0, st, q, qn, nq, r, rn, nr, d, hd, fp64, chunk_len,
                       nchunks, part);
}

// Norm tables for the matrix-core path (mixed precision only: FP64 sums keep
// the exact-difference VALU kernels); *use is false when s^2 (|q|^2 + |r|^2)
// could exceed 2^26 for the smallest bandwidth (rounding of the expanded
// squared distance then above ~1e-7).
bool mfma_shape(int d, int precision) { return d >= 8 && d <= 32 && precision == DFGT_PREC_MIXED; }

dfgt_status prepare_mfma(const double *q, int nq, const double *r, int nr, int d, const double *h_host, int nh,
                         int precision, const NaiveBufs &b, hipStream_t st, bool *use) {
    *use = false;
    if (!mfma_shape(d, precision)) return DFGT_OK;
    unsigned long long *mx = b.mx;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, mx, 2);
    hipLaunchKernelGGL(k_sqnorm, dim3((nq + 255) / 256), dim3(256), 0, st, q, nq, d, b.qn, mx);
    hipLaunchKernelGGL(k_sqnorm, dim3((nr + 255) / 256), dim3(256), 0, st, r, nr, d, b.rn, mx + 1);
    DFGT_HIP(hipGetLastError());
    unsigned long long hm[2];
    DFGT_HIP(hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, st));
    DFGT_HIP(hipStreamSynchronize(st));
    double hmin = h_host[0];
    for (int k = 1; k < nh; ++k) hmin = std::fmin(hmin, h_host[k]);
    double m0, m1;
    std::memcpy(&m0, &hm[0], sizeof(double));
    std::memcpy(&m1, &hm[1], sizeof(double));
    *use = (m0 + m1) / (2.0 * hmin * hmin) * 1.5 <= 67108864.0;
    return DFGT_OK;
}

// Reference chunks of one launch: enough (query tile, chunk, bandwidth) blocks
// to fill 256 CUs several times over, at most one per `unit` references and at
// most `most` (the partials' room); chunk lengths are multiples of `unit`.
// Returns the chunk count and its length in *len.
int split_chunks(int tiles, int nh, int nr, int unit, long long most, int *len) {
    int nc = (4096 + tiles * nh - 1) / (tiles * nh);
    nc = std::min(nc, (nr + unit - 1) / unit);
    if (most < nc) nc = (int)std::max<long long>(most, 1);
    nc = std::max(nc, 1);
    int cl = (nr + nc - 1) / nc;
    cl = (cl + unit - 1) / unit * unit;
    *len = cl;
    return (nr + cl - 1) / cl;
}

dfgt_status naive_run(const double *q, int64_t nq64, const double *r, int64_t nr64, int d, const double *h_host,
                      int nh, int precision, double *G, hipStream_t st, const NaiveSpace &sp) {
    const int nq = (int)nq64, nr = (int)nr64;
    const size_t pmax = sp.part_max(nq, nr, nh);
    const long long most = pmax == SIZE_MAX ? (1LL << 40) : (long long)(pmax / ((size_t)nq * nh));
    if (most < 1) {
        set_error("dfgt_naive_sum_noalloc: n_h x nq + nq + nr exceeds the scratch region");
        return DFGT_EINVAL;
    }
    int qpt = 1;
    bool specialised = precision == DFGT_PREC_MIXED && (d == 1 || d == 2 || d == 3 || d == 5);
    if (specialised) qpt = 2;
    const int bx = (nq + kBlock * qpt - 1) / (kBlock * qpt);
    int chunk_len = 0;
    const int nchunks = split_chunks(bx, nh, nr, kInner, std::min<long long>(most, (nr + kTile - 1) / kTile),
                                     &chunk_len);
    const bool norms = mfma_shape(d, precision);
    const int mbx = (nq + 63) / 64;
    int mlen = 0;
    const int mch = norms ? split_chunks(mbx, nh, nr, 64, most, &mlen) : 0;
    NaiveBufs b{};
    DFGT_TRY(sp.get(nq, nr, nh, (size_t)std::max(nchunks, mch) * nq * nh, norms, &b));
    DFGT_HIP(hipMemcpyAsync(b.h, h_host, sizeof(double) * nh, hipMemcpyHostToDevice, st));
    double *part = b.part;
    const double *hd = b.h;
    dim3 grid(bx, nchunks, nh);
    bool mfma = false;
    DFGT_TRY(prepare_mfma(q, nq, r, nr, d, h_host, nh, precision, b, st, &mfma));
    if (mfma) {
        dim3 mg(mbx, mch, nh);
        const int fp = precision == DFGT_PREC_FP64 ? 1 : 0;
        const double *qn = b.qn, *rn = b.rn;
        double *mp = b.part;
        switch ((d + 3) / 4) {
        case 2: launch_mfma<2>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        case 3: launch_mfma<3>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        case 4: launch_mfma<4>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        case 5: launch_mfma<5>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        case 6: launch_mfma<6>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        case 7: launch_mfma<7>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        default: launch_mfma<8>(mg, st, q, qn, nq, r, rn, nr, d, hd, fp, mlen, mch, mp); break;
        }
        DFGT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_reduce_chunks, dim3((nq + 255) / 256, nh), dim3(256), 0, st, mp, nq, mch, nh, G);
        DFGT_HIP(hipGetLastError());
        return DFGT_OK;
    }
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

// The no-allocation form's region: chunk partials, bandwidths and norm tables
// of the calls of every thread on this GPU (each device holds its own copy).
constexpr size_t kScratchDoubles = size_t(8) << 20;  // 64 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device, looked up once per device with
// that device current (host code never uses the symbol itself).
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

dfgt_status scratch_region(double **out) {
    int dev = 0;
    DFGT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("dfgt_naive_sum_noalloc: device index out of range");
        return DFGT_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("dfgt_naive_sum_noalloc: hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return DFGT_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double *>(g_scratch_ptr[dev]);
    return DFGT_OK;
}

}  // namespace

dfgt_status launch_naive(const double *q, int64_t nq, const double *r, int64_t nr, int d, const double *h_host,
                         int nh, int precision, double *G, hipStream_t st) {
    return naive_run(q, nq, r, nr, d, h_host, nh, precision, G, st, NaiveSpace{});
}

size_t naive_noalloc_limit() { return kScratchDoubles; }

void release_naive_workspace() {
    for (DevBuf *b : {&g_part, &g_h, &g_qn, &g_rn, &g_mx}) b->release();
}

dfgt_status launch_naive_noalloc(const double *q, int64_t nq, const double *r, int64_t nr, int d,
                                 const double *h_host, int nh, int precision, double *G, hipStream_t st) {
    NaiveSpace sp;
    DFGT_TRY(scratch_region(&sp.pool));
    sp.cap = kScratchDoubles;
    if (sp.head((int)nq, (int)nr, nh) + (size_t)nq * nh > sp.cap) {
        set_error("dfgt_naive_sum_noalloc: n_h x nq + nq + nr + n_h exceeds the " +
                  std::to_string(kScratchDoubles >> 17) + " MiB scratch region");
        return DFGT_EINVAL;
    }
    return naive_run(q, nq, r, nr, d, h_host, nh, precision, G, st, sp);
}

}  // namespace dfgt
