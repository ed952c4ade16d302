// Exhaustive Gaussian-sum tiles on the FP64 matrix cores (D >= 8).
//
// For a query q and reference r the squared distance is formed as
//     |q - r|^2 = |q|^2 + |r|^2 - 2 q.r
// with the dot products of a 16 x 16 block of (reference, query) pairs from
// ceil(D/4) v_mfma_f64_16x16x4f64 instructions and the squared norms taken
// from per-point tables.  In FP64 the rounding of this form is at most about
// D 2^-53 (|q|^2 + |r|^2): scaled by s^2 = 1/(2h^2) it stays below ~1e-7 as
// long as s^2 (|q|^2 + |r|^2) <= 2^26, which the host checks before choosing
// this path.  That is far inside the 1e-5 budget of the mixed-precision sums
// (FP32 exp2 and partial sums over <= 64 terms, FP64 beyond), the only mode
// that uses it: FP64 sums keep the exact-difference VALU tiles.
//
// Operand layouts of v_mfma_f64_16x16x4f64 (lane l, g = l / 16):
//   A[i][k] at lane i + 16 k,   B[k][j] at lane j + 16 k,
//   D[4 r + g][l % 16] in result register r.
// Here A = 16 references x 4 dimensions, B = 4 dimensions x 16 queries, so
// lane l ends with the dot products of query l % 16 with references 4 r + g.
// The same values, as A operands of chunk r, give E^T X (the kernel-weighted
// sums of reference coordinates that the q-gradient needs) with no data
// movement between lanes.
#pragma once

#include "dfgt_internal.h"

namespace dfgt {

typedef double v4d __attribute__((ext_vector_type(4)));

// Fragment of the 16-row block starting at row0 (rows beyond nvalid are
// clamped to the last valid one and must be masked by the caller): lane l
// holds row l % 16, dimensions 4c + l / 16 (zero beyond d).
template <int NC>
__device__ __forceinline__ void load_frag(const double *__restrict__ x, int row0, int nvalid, int d,
                                          double (&f)[NC]) {
    const int lane = threadIdx.x & 63;
    const int row = row0 + min(lane & 15, nvalid - 1);
    const double *p = x + (size_t)row * d;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int k = 4 * c + (lane >> 4);
        f[c] = k < d ? p[k] : 0.0;
    }
}

// q . r for the 16 x 16 block: acc[r] = <ref 4r + g, query l % 16>.
template <int NC>
__device__ __forceinline__ v4d block_dots(const double (&rf)[NC], const double (&qf)[NC]) {
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(rf[c], qf[c], acc, 0, 0, 0);
    return acc;
}

}  // namespace dfgt
