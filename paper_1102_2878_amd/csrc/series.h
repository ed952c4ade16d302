// Device-side series-expansion helpers shared by the moment, summarisation and
// post-processing kernels (HIP, FP64).
//
// Coefficient vectors hold p_max^D doubles, radix p_max with the last dimension
// fastest (the Appendix's linear layout).  All multi-dimensional operators of
// the method (F2F, F2L, L2L) have a coefficient that factorises over the
// dimensions, so they are applied as D one-dimensional "mode products" along
// each axis in turn.
#pragma once

#include "dfgt_internal.h"

namespace dfgt {

__device__ __forceinline__ int ipow_i(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Digit of axis k of position i (radix pmax, axis d-1 least significant).
__device__ __forceinline__ int digit(int i, int k, int d, int pmax) {
    int stride = 1;
    for (int j = d - 1; j > k; --j) stride *= pmax;
    return (i / stride) % pmax;
}

// |alpha| and whether every digit is < p.
__device__ __forceinline__ int digit_sum(int i, int d, int pmax, int p, bool *inside) {
    int s = 0;
    bool ok = true;
    for (int k = d - 1; k >= 0; --k) {
        int a = i % pmax;
        i /= pmax;
        s += a;
        ok = ok && (a < p);
    }
    *inside = ok;
    return s;
}

// out[i] = sum_j coef(a_k(i), j) * in[i with digit k replaced by j], j < p.
// coef(a, j) is given as a pmax x pmax row-major table in (LDS or global) memory.
// Every thread of the block handles positions tid, tid + nthreads, ...
__device__ __forceinline__ void mode_product(const double *in, double *out, const double *coef, int P, int d,
                                             int pmax, int k, int p) {
    int stride = 1;
    for (int j = d - 1; j > k; --j) stride *= pmax;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int a = (i / stride) % pmax;
        const int base = i - a * stride;
        double s = 0.0;
        for (int j = 0; j < p; ++j) s = fma(coef[a * pmax + j], in[base + j * stride], s);
        out[i] = s;
    }
}

// Physicists' Hermite polynomials H_0..H_{n-1} at t (h_n = e^{-t^2} H_n,
// recurrence H_{n+1} = 2t H_n - 2n H_{n-1}).
__device__ __forceinline__ void hermite_polys(double t, int n, double *H) {
    H[0] = 1.0;
    if (n > 1) H[1] = 2.0 * t;
    for (int m = 1; m + 1 < n; ++m) H[m + 1] = 2.0 * t * H[m] - 2.0 * m * H[m - 1];
}

// Digit tables for coefficient positions i < P (radix pmax <= 16, so a digit
// fits 4 bits and a position with any non-zero digit has d <= 13):
//   dg[i] = digits packed 4 bits per axis (axis k at bits 4k),
//   mt[i] = |alpha| | (max digit << 8).
__device__ __forceinline__ void build_digit_tables(unsigned long long *dg, unsigned short *mt, int P, int d,
                                                   int pmax) {
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        int rem = i, sum = 0, mx = 0;
        unsigned long long packed = 0;
        for (int k = d - 1; k >= 0; --k) {
            const int a = rem % pmax;
            rem /= pmax;
            if (a) packed |= (unsigned long long)a << (4 * k);
            sum += a;
            mx = a > mx ? a : mx;
        }
        dg[i] = packed;
        mt[i] = (unsigned short)(sum | (mx << 8));
    }
}
__device__ __forceinline__ int dig_at(unsigned long long packed, int k) {
    return k < 16 ? (int)((packed >> (4 * k)) & 15) : 0;  // k >= 16 only occurs with p_max = 1
}

__device__ __forceinline__ double inv_factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return 1.0 / f;
}

}  // namespace dfgt
