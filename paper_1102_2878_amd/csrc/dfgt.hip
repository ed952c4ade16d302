// The hierarchical fast Gauss transform of Section 3.9 (DFGTMain) on the GPU.
//
// Traversal.  The paper's depth-first recursion DFGT(Q, R) is unrolled into a
// level-synchronous frontier.  A "segment" is one query node Q under one job
// (a bandwidth of the sweep) together with the list of reference nodes that
// still have to be resolved against it.  All jobs share one traversal: level 0
// holds (Q_root, {R_root}) for every bandwidth.  One wave per segment:
//   1. lower bound  G^l(Q) = (pruned contributions inherited from Q and its
//      ancestors) + (min over Q's points of their exact leaf sums so far)
//      + sum over the list of |R| K(d^u(Q, R)).  Every term is a valid lower
//      bound on the part of G(q) it covers and the parts partition the
//      reference set, so G^l(Q) <= G(q) for all q in Q; the global-error
//      theorem (Section 3.10) only needs such a bound at the time of a prune.
//   2. CanSummarize / ChooseBestMethod (Sections 3.6, 3.8) per pair with
//      tau = eps' |R| G^l(Q) / |R_total|: far-field evaluation F, direct local
//      accumulation D, far-to-local translation T (including its centroid
//      form with the finite-difference bound of the global-error proof), or E.
//   3. Outputs, all contiguous per segment: pruned pairs become F or D/T op
//      groups, leaf-leaf E pairs an exhaustive group, and the rest split
//      exactly as the recursion does (Q and R both when both are internal)
//      into the next level's segments.
// Execution per level, one block per (Q, job) group, so every accumulation
// into a query's partial sums or a node's local moments happens in a fixed
// order without atomics (results are bitwise reproducible):
//   k_base    DFGTBase: exact leaf-leaf sums, and the refined lower bound
//             min_q G_E(q) for the next level;
//   k_far     EvalFarFieldExpansion for F ops;
//   k_local   AccumulateDirectLocalMoment (D) and TransFarToLocal (T) into
//             the node's local moments.
// Post-processing (DFGTPost): per (query leaf, job) the local moments of
// every node on the root-to-leaf path are shifted down by TransLocalToLocal
// and added, the result is evaluated at the leaf's points and combined with
// the far-field and exhaustive parts, in the caller's order.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "series.h"

namespace dfgt {
namespace {

enum { METH_E = 0, METH_F = 1, METH_D = 2, METH_T = 3 };

struct Job {
    double h, s, inv2h2, sig;  // s = 1/(sqrt2 h); sig = sqrt(log2 e) s
    double eps_eff;            // eps minus the rounding budget of the exhaustive sums
    double nR;                 // |R_total|
    int qt, rt;                // indices into the tree table
    long long qoff;            // offset of this job's per-query arrays
    long long noff;            // offset of this job's per-node arrays
    double *out;               // caller's output for this job (caller order)
    int mono;                  // Q and R are the same point set
    int pad;
};

struct Seg {
    int q, job, start, count;
    double gl;  // pruned lower-bound contributions inherited by Q
};

struct Group {
    int q, job, start, count;
    int flags;  // k_base: 1 = compute in FP64 (underflow guard)
    int pad;
};

struct Op {
    int r, meta;  // meta = order | (method << 8)
};

enum {
    C_SEG = 0,
    C_PAIR,
    C_EGRP,
    C_EOP,
    C_FGRP,
    C_FOP,
    C_LGRP,
    C_LOP,
    C_N
};

enum {
    S_PAIRS = 0,
    S_F,
    S_D,
    S_T,
    S_C,
    S_BLEAF,
    S_BPTS,
    S_MAXORD,
    S_FP64,
    S_N
};

// ---------------------------------------------------------------- bounds (Section 3.5)
__device__ __forceinline__ double powi(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// sum_{k<D} C(D,k) a^k b^{D-k}
__device__ double binom_mix(double a, double b, int D) {
    double c = 1.0, sum = 0.0;
    for (int k = 0; k < D; ++k) {
        sum += c * powi(a, k) * powi(b, D - k);
        c = c * (double)(D - k) / (double)(k + 1);
    }
    return sum;
}

// Far-field / local lemma bound, eqs. (error_bound_far_field), (error_bound_local).
__device__ double bound_far(double r, int p, int D, double nR) {
    const double rp = powi(r, p);
    const double b = rp * sqrt(inv_factorial(p));
    return nR * binom_mix(1.0 - rp, b, D) / powi(1.0 - r, D);
}

// Far-to-local lemma bound, eq. (error_bound_far_to_local) (its formula holds 2r).
__device__ double bound_f2l(double r, int p, int D, double nR) {
    const double tp = powi(2.0 * r, p);
    const double a = (1.0 - tp) * (1.0 - tp);
    const double b = tp * (2.0 - tp) * sqrt(inv_factorial(p));
    return nR * binom_mix(a, b, D) / powi(1.0 - 2.0 * r, 2 * D);
}

// Bounds are compared with a small relative slack on the safe side.
constexpr double kSlack = 1.0 + 1e-10;

// Alg. FarFieldOrder / LocalAccumulationOrder: r = width / (2h); 0 = infinity.
__device__ int order_far(double r, double nR, double tau, int pmax, int D) {
    if (r >= 1.0) return 0;
    for (int p = 1; p <= pmax; ++p)
        if (bound_far(r, p, D, nR) * kSlack <= tau) return p;
    return 0;
}

// Alg. ConvertFarFieldToLocalOrder, read with the lemma's radius r = width / (2h) < 1/2.
__device__ int order_f2l(double r, double nR, double tau, int pmax, int D) {
    if (r >= 0.5) return 0;
    for (int p = 1; p <= pmax; ++p)
        if (bound_f2l(r, p, D, nR) * kSlack <= tau) return p;
    return 0;
}

struct PairGeom {
    double sl, su, sc;  // squared d^l, d^u, centre distance
    double wQ, wR;
};

__device__ __forceinline__ PairGeom pair_geom(const DevTree &Q, int q, const DevTree &R, int r) {
    PairGeom g{0.0, 0.0, 0.0, 0.0, 0.0};
    const int d = Q.d;
    for (int k = 0; k < d; ++k) {
        const double ql = Q.lo[(size_t)q * d + k], qh = Q.hi[(size_t)q * d + k];
        const double rl = R.lo[(size_t)r * d + k], rh = R.hi[(size_t)r * d + k];
        const double a = rl - qh, b = ql - rh;
        const double gap = (a > 0.0 ? a : 0.0) + (b > 0.0 ? b : 0.0);
        g.sl += gap * gap;
        const double u = fmax(rh - ql, qh - rl);
        g.su += u * u;
        const double c = Q.ctr[(size_t)q * d + k] - R.ctr[(size_t)r * d + k];
        g.sc += c * c;
        g.wQ = fmax(g.wQ, qh - ql);
        g.wR = fmax(g.wR, rh - rl);
    }
    return g;
}

// ChooseBestMethod (Section 3.8) with costs c_F = D N_Q p_F^D, c_D = D N_R p_D^D,
// c_T = D p_T^{2D}, c_E = D N_Q N_R; ties F, D, T, E.  T may also be chosen at
// order 1 through the centroid bound |R| max(K(d^l)-K(d_c), K(d_c)-K(d^u)).
__device__ int choose(const PairGeom &g, double h, double inv2h2, double nQ, double nR, double tau, int pmax,
                      int D, int force, int *order) {
    int pF = 0, pD = 0, pT = 0;
    if (force != DFGT_FORCE_EXACT) {
        pF = order_far(g.wR / (2.0 * h), nR, tau, pmax, D);
        pD = order_far(g.wQ / (2.0 * h), nR, tau, pmax, D);
        pT = order_f2l(fmax(g.wQ, g.wR) / (2.0 * h), nR, tau, pmax, D);
        const double kl = exp(-g.sl * inv2h2), ku = exp(-g.su * inv2h2), kc = exp(-g.sc * inv2h2);
        const double cb = nR * (fmax(kl - kc, kc - ku) + 1e-15 * kl);
        const bool centroid = cb <= tau;
        if (centroid) pT = 1;
        if (force == DFGT_FORCE_F) pD = pT = 0;
        if (force == DFGT_FORCE_D) pF = pT = 0;
        if (force == DFGT_FORCE_T) pF = pD = 0;
        if (force == DFGT_FORCE_CENTROID) {
            pF = pD = 0;
            pT = centroid ? 1 : 0;
        }
    }
    const double inf = INFINITY;
    const double cF = pF ? D * nQ * powi((double)pF, D) : inf;
    const double cD = pD ? D * nR * powi((double)pD, D) : inf;
    const double cT = pT ? D * powi((double)pT, 2 * D) : inf;
    const double cE = D * nQ * nR;
    const double mn = fmin(fmin(cF, cD), fmin(cT, cE));
    if (pF && cF == mn) {
        *order = pF;
        return METH_F;
    }
    if (pD && cD == mn) {
        *order = pD;
        return METH_D;
    }
    if (pT && cT == mn) {
        *order = pT;
        return METH_T;
    }
    *order = 0;
    return METH_E;
}

struct TravOut {
    Seg *nsegs;
    int *npairs;
    Group *egrp;
    int *eops;
    Group *fgrp;
    Op *fops;
    Group *lgrp;
    Op *lops;
    int *cnt;
    unsigned long long *stats;
};

__device__ __forceinline__ int wave_excl(int v, int *total) {
    int inc = wave_incl_scan(v);
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

// One wave per segment.
__global__ __launch_bounds__(64) void k_traverse(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                                 const Seg *__restrict__ segs, const int *__restrict__ pairs,
                                                 const double *__restrict__ glE, int force, int *dec,
                                                 TravOut o) {
    const int lane = threadIdx.x;
    const Seg sg = segs[blockIdx.x];
    const Job jb = jobs[sg.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int D = Q.d, pmax = Q.pmax;
    const int q = sg.q;
    const bool qleaf = Q.left[q] < 0;
    const double nQ = (double)(Q.end[q] - Q.begin[q]);

    // 1. lower bound over the whole list
    double sl = 0.0;
    for (int i = lane; i < sg.count; i += 64) {
        const int r = pairs[sg.start + i];
        const PairGeom g = pair_geom(Q, q, R, r);
        sl += (double)(R.end[r] - R.begin[r]) * exp(-g.su * jb.inv2h2);
    }
    sl = wave_sum(sl);
    const double gl = (sg.gl + (qleaf ? glE[jb.noff + q] : 0.0) + sl) * (1.0 - 1e-12);

    // 2. decisions and counts
    int cE = 0, cF = 0, cL = 0, cN = 0, nT = 0, nC = 0, nD = 0, maxord = 0;
    double plo = 0.0;
    for (int i = lane; i < sg.count; i += 64) {
        const int r = pairs[sg.start + i];
        const PairGeom g = pair_geom(Q, q, R, r);
        const double nR = (double)(R.end[r] - R.begin[r]);
        const double tau = jb.eps_eff * nR * gl / jb.nR;
        int ord = 0;
        const int m = choose(g, jb.h, jb.inv2h2, nQ, nR, tau, pmax, D, force, &ord);
        const bool rleaf = R.left[r] < 0;
        if (m != METH_E) {
            plo += nR * exp(-g.su * jb.inv2h2);
            if (m == METH_F) ++cF;
            else {
                ++cL;
                if (m == METH_D) ++nD;
                else if (ord == 1) ++nC;
                else ++nT;
            }
            maxord = max(maxord, ord);
        } else if (qleaf && rleaf) {
            ++cE;
        } else {
            cN += (qleaf || !rleaf) ? 2 : 1;
        }
        dec[sg.start + i] = m | (ord << 4);
    }
    int tE, tF, tL, tN;
    wave_excl(cE, &tE);
    wave_excl(cF, &tF);
    wave_excl(cL, &tL);
    wave_excl(cN, &tN);
    plo = wave_sum(plo);
    const double gl_child = sg.gl + plo * (1.0 - 1e-12);
    const int nFp = wave_sum_i(cF), nDp = wave_sum_i(nD), nTp = wave_sum_i(nT), nCp = wave_sum_i(nC);
    int mo = maxord;
    for (int off = 32; off >= 1; off >>= 1) mo = max(mo, __shfl_xor(mo, off, 64));

    // reserve contiguous output ranges
    int ebase = 0, fbase = 0, lbase = 0, cbase = 0, egi = 0, fgi = 0, lgi = 0, sgi = 0;
    const int npair_out = qleaf ? tN : 2 * tN;
    const int nseg_out = tN > 0 ? (qleaf ? 1 : 2) : 0;
    if (lane == 0) {
        if (tE) {
            ebase = atomicAdd(&o.cnt[C_EOP], tE);
            egi = atomicAdd(&o.cnt[C_EGRP], 1);
        }
        if (tF) {
            fbase = atomicAdd(&o.cnt[C_FOP], tF);
            fgi = atomicAdd(&o.cnt[C_FGRP], 1);
        }
        if (tL) {
            lbase = atomicAdd(&o.cnt[C_LOP], tL);
            lgi = atomicAdd(&o.cnt[C_LGRP], 1);
        }
        if (npair_out) {
            cbase = atomicAdd(&o.cnt[C_PAIR], npair_out);
            sgi = atomicAdd(&o.cnt[C_SEG], nseg_out);
        }
        atomicAdd(&o.stats[S_PAIRS], (unsigned long long)sg.count);
        if (nFp) atomicAdd(&o.stats[S_F], (unsigned long long)nFp);
        if (nDp) atomicAdd(&o.stats[S_D], (unsigned long long)nDp);
        if (nTp) atomicAdd(&o.stats[S_T], (unsigned long long)nTp);
        if (nCp) atomicAdd(&o.stats[S_C], (unsigned long long)nCp);
        if (tE) atomicAdd(&o.stats[S_BLEAF], (unsigned long long)tE);
        if (mo) atomicMax(&o.stats[S_MAXORD], (unsigned long long)mo);
    }
    ebase = __shfl(ebase, 0, 64);
    fbase = __shfl(fbase, 0, 64);
    lbase = __shfl(lbase, 0, 64);
    cbase = __shfl(cbase, 0, 64);

    // 3. write outputs in pair order
    int eo = 0, fo = 0, lo = 0, no = 0;
    const int QL = qleaf ? q : Q.left[q], QR = qleaf ? q : Q.right[q];
    for (int c0 = 0; c0 < sg.count; c0 += 64) {
        const int i = c0 + lane;
        int m = METH_E, ord = 0, r = -1, e = 0, f = 0, l = 0, n = 0;
        bool rleaf = true;
        if (i < sg.count) {
            r = pairs[sg.start + i];
            const int v = dec[sg.start + i];
            m = v & 15;
            ord = v >> 4;
            rleaf = R.left[r] < 0;
            if (m == METH_F) f = 1;
            else if (m != METH_E) l = 1;
            else if (qleaf && rleaf) e = 1;
            else n = (qleaf || !rleaf) ? 2 : 1;
        }
        int te, tf, tl, tn;
        const int xe = wave_excl(e, &te), xf = wave_excl(f, &tf), xl = wave_excl(l, &tl), xn = wave_excl(n, &tn);
        if (e) o.eops[ebase + eo + xe] = r;
        if (f) o.fops[fbase + fo + xf] = Op{r, ord | (METH_F << 8)};
        if (l) o.lops[lbase + lo + xl] = Op{r, ord | (m << 8)};
        if (n) {
            const int p0 = cbase + no + xn;
            if (qleaf) {
                o.npairs[p0] = R.left[r];
                o.npairs[p0 + 1] = R.right[r];
            } else if (rleaf) {
                o.npairs[p0] = r;
                o.npairs[p0 + tN] = r;
            } else {
                o.npairs[p0] = R.left[r];
                o.npairs[p0 + 1] = R.right[r];
                o.npairs[p0 + tN] = R.left[r];
                o.npairs[p0 + tN + 1] = R.right[r];
            }
        }
        eo += te;
        fo += tf;
        lo += tl;
        no += tn;
    }
    if (lane == 0) {
        if (tE) {
            // underflow guard: FP32 exp2 flushes terms below 2^-126; keep that
            // absolute error below 2^-26 G by computing tiny sums in FP64.
            const double glb = jb.mono ? fmax(gl, 1.0) : gl;
            const int fp64 = glb < jb.nR * 0x1p-100 ? 1 : 0;
            o.egrp[egi] = Group{q, sg.job, ebase, tE, fp64, 0};
        }
        if (tF) o.fgrp[fgi] = Group{q, sg.job, fbase, tF, 0, 0};
        if (tL) o.lgrp[lgi] = Group{q, sg.job, lbase, tL, 0, 0};
        if (tN) {
            o.nsegs[sgi] = Seg{QL, sg.job, cbase, tN, gl_child};
            if (!qleaf) o.nsegs[sgi + 1] = Seg{QR, sg.job, cbase + tN, tN, gl_child};
        }
    }
}

// ---------------------------------------------------------------- DFGTBase
constexpr int kBaseBlock = 256;
constexpr int kInner = 64;

__global__ __launch_bounds__(kBaseBlock) void k_base(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                                     const Group *__restrict__ grp, const int *__restrict__ eops,
                                                     int precision, double *GE, double *glE,
                                                     unsigned long long *stats) {
    __shared__ double red[kBaseBlock];
    __shared__ double mn[kBaseBlock / 64];
    const Group g = grp[blockIdx.x];
    const Job jb = jobs[g.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int d = Q.d;
    const int qb = Q.begin[g.q], nq = Q.end[g.q] - qb;
    const bool fp64 = precision == DFGT_PREC_FP64 || g.flags;
    int slots = 1;
    while (slots < nq && slots < kBaseBlock) slots <<= 1;
    const int ngr = kBaseBlock / slots;
    const int qi = threadIdx.x % slots, gr = threadIdx.x / slots;
    double gmin = INFINITY;
    long long pts = 0;
    for (int q0 = 0; q0 < nq; q0 += slots) {
        const int qq = q0 + qi;
        const bool act = qq < nq;
        double acc = 0.0;
        if (act) {
            const double sc = fp64 ? jb.s : jb.sig;
            double qs[kMaxD];
            for (int k = 0; k < d; ++k) qs[k] = Q.x[(size_t)(qb + qq) * d + k] * sc;
            for (int e = gr; e < g.count; e += ngr) {
                const int r = eops[g.start + e];
                const int rb = R.begin[r], re = R.end[r];
                if (fp64) {
                    for (int j = rb; j < re; ++j) {
                        double t = 0.0;
                        for (int k = 0; k < d; ++k) {
                            const double dd = fma(R.x[(size_t)j * d + k], -sc, qs[k]);
                            t = fma(dd, dd, t);
                        }
                        acc += exp(-t);
                    }
                } else {
                    for (int j0 = rb; j0 < re; j0 += kInner) {
                        const int j1 = min(re, j0 + kInner);
                        float ps = 0.0f;
                        for (int j = j0; j < j1; ++j) {
                            double t = 0.0;
                            for (int k = 0; k < d; ++k) {
                                const double dd = fma(R.x[(size_t)j * d + k], -sc, qs[k]);
                                t = fma(dd, dd, t);
                            }
                            ps += __builtin_amdgcn_exp2f(-(float)t);
                        }
                        acc += (double)ps;
                    }
                }
                if (qi == 0 && q0 == 0) pts += (long long)(re - rb);
            }
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        if (gr == 0 && act) {
            double s = 0.0;
            for (int k = 0; k < ngr; ++k) s += red[k * slots + qi];
            const size_t gi = (size_t)jb.qoff + qb + qq;
            const double v = GE[gi] + s;
            GE[gi] = v;
            gmin = fmin(gmin, v);
        }
        __syncthreads();
    }
    gmin = wave_min(gmin);
    if ((threadIdx.x & 63) == 0) mn[threadIdx.x >> 6] = gmin;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = mn[0];
        for (int w = 1; w < kBaseBlock / 64; ++w) m = fmin(m, mn[w]);
        glE[jb.noff + g.q] = m;
    }
    // point pairs: lanes with qi == 0 counted |R| per exhaustive leaf they handled
    long long tot = pts;
    for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd(&stats[S_BPTS], (unsigned long long)(tot * nq));
    if (threadIdx.x == 0 && fp64 && precision != DFGT_PREC_FP64) atomicAdd(&stats[S_FP64], 1ull);
}

// ---------------------------------------------------------------- EvalFarFieldExpansion
// G_F(q) += sum_{alpha < p} M_alpha h_alpha((q - R.c) s),  M_alpha = s^|alpha| mu_alpha,
// h_alpha(t) = e^{-|t|^2} prod_k H_{alpha_k}(t_k).
__global__ __launch_bounds__(256) void k_far(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                             const Group *__restrict__ grp, const Op *__restrict__ fops,
                                             double *GF) {
    const Group g = grp[blockIdx.x];
    const Job jb = jobs[g.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int d = Q.d, pmax = Q.pmax, P = Q.P;
    const int qb = Q.begin[g.q], qe = Q.end[g.q];
    const double s = jb.s;
    for (int qi = qb + threadIdx.x; qi < qe; qi += blockDim.x) {
        double sum = 0.0;
        for (int o = 0; o < g.count; ++o) {
            const Op op = fops[g.start + o];
            const int r = op.r, p = op.meta & 255;
            double t[kMaxD], tt = 0.0;
            for (int k = 0; k < d; ++k) {
                t[k] = (Q.x[(size_t)qi * d + k] - R.ctr[(size_t)r * d + k]) * s;
                tt += t[k] * t[k];
            }
            if (tt > 745.0) continue;  // e^{-|t|^2} underflows: the expansion is 0
            double H[kMaxD * 16];
            for (int k = 0; k < d; ++k) hermite_polys(t[k], p, H + k * 16);
            const double *mu = R.mu + (size_t)r * P;
            double w = 0.0;
            const int np = ipow_i(p, d);
            for (int i = 0; i < np; ++i) {
                int rem = i, pos = 0, stride = 1, asum = 0;
                double prod = 1.0;
                for (int k = d - 1; k >= 0; --k) {
                    const int a = rem % p;
                    rem /= p;
                    pos += a * stride;
                    stride *= pmax;
                    asum += a;
                    prod *= H[k * 16 + a];
                }
                w = fma(mu[pos] * powi(s, asum), prod, w);
            }
            sum += exp(-tt) * w;
        }
        GF[(size_t)jb.qoff + qi] += sum;
    }
}

// ---------------------------------------------------------------- local moments: D and T ops
// Dynamic LDS layout: acc[P] | buf0[P] | buf1[P] | coef[pmax*pmax] | H[d * 2 pmax]
// (buf0 / buf1 / acc in a global scratch slice when P is large).
constexpr int kLocBlock = 256;

__global__ __launch_bounds__(kLocBlock) void k_local(const DevTree *__restrict__ trees,
                                                     const Job *__restrict__ jobs, const Group *__restrict__ grp,
                                                     const Op *__restrict__ lops, int use_lds,
                                                     double *__restrict__ gscratch, double *L,
                                                     unsigned char *lflag) {
    extern __shared__ double smem[];
    const Group g = grp[blockIdx.x];
    const Job jb = jobs[g.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int d = Q.d, pmax = Q.pmax, P = Q.P;
    const double s = jb.s;
    double *acc, *buf0, *buf1, *coef, *Ht;
    if (use_lds) {
        acc = smem;
        buf0 = acc + P;
        buf1 = buf0 + P;
        coef = buf1 + P;
    } else {
        acc = gscratch + (size_t)blockIdx.x * 3 * P;
        buf0 = acc + P;
        buf1 = buf0 + P;
        coef = smem;
    }
    Ht = coef + pmax * pmax;
    const double *qc = Q.ctr + (size_t)g.q * d;
    for (int i = threadIdx.x; i < P; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    for (int o = 0; o < g.count; ++o) {
        const Op op = lops[g.start + o];
        const int r = op.r, p = op.meta & 255, m = op.meta >> 8;
        if (m == METH_D) {
            // L_beta += sum_{x in R} ((-1)^|beta| / beta!) h_beta((Q.c - x) s)
            const int rb = R.begin[r], re = R.end[r];
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                bool inside;
                const int bs = digit_sum(i, d, pmax, p, &inside);
                if (!inside) continue;
                double cf = (bs & 1) ? -1.0 : 1.0;
                for (int k = 0; k < d; ++k) cf *= inv_factorial(digit(i, k, d, pmax));
                double sum = 0.0;
                for (int j = rb; j < re; ++j) {
                    double tt = 0.0, prod = 1.0;
                    for (int k = 0; k < d; ++k) {
                        const double t = (qc[k] - R.x[(size_t)j * d + k]) * s;
                        tt += t * t;
                        double Hk[16];
                        const int b = digit(i, k, d, pmax);
                        hermite_polys(t, b + 1, Hk);
                        prod *= Hk[b];
                    }
                    if (tt <= 745.0) sum = fma(exp(-tt), prod, sum);
                }
                acc[i] += cf * sum;
            }
            __syncthreads();
        } else {
            // T: L_beta += ((-1)^|beta| / beta!) sum_{alpha<p} M_alpha h_{alpha+beta}((Q.c - R.c) s)
            double tt = 0.0;
            for (int k = 0; k < d; ++k) {
                const double t = (qc[k] - R.ctr[(size_t)r * d + k]) * s;
                tt += t * t;
            }
            if (tt > 745.0) continue;  // uniform across the block
            const double e0 = exp(-tt);
            const double *mu = R.mu + (size_t)r * P;
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                bool inside;
                const int as = digit_sum(i, d, pmax, p, &inside);
                buf0[i] = inside ? mu[i] * powi(s, as) : 0.0;
            }
            // Hermite polynomials H_0 .. H_{2p-2} per dimension at t0
            for (int k = threadIdx.x; k < d; k += blockDim.x) {
                const double t = (qc[k] - R.ctr[(size_t)r * d + k]) * s;
                hermite_polys(t, 2 * p - 1, Ht + k * 2 * pmax);
            }
            __syncthreads();
            double *src = buf0, *dst = buf1;
            for (int k = 0; k < d; ++k) {
                // coef[b][a] = H_{a+b}(t0_k) for a, b < p
                for (int i = threadIdx.x; i < pmax * pmax; i += blockDim.x) {
                    const int b = i / pmax, a = i % pmax;
                    coef[i] = (a < p && b < p) ? Ht[k * 2 * pmax + a + b] : 0.0;
                }
                __syncthreads();
                mode_product(src, dst, coef, P, d, pmax, k, p);
                __syncthreads();
                double *tmp = src;
                src = dst;
                dst = tmp;
            }
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                bool inside;
                const int bs = digit_sum(i, d, pmax, p, &inside);
                if (!inside) continue;
                double cf = (bs & 1) ? -e0 : e0;
                for (int k = 0; k < d; ++k) cf *= inv_factorial(digit(i, k, d, pmax));
                acc[i] += cf * src[i];
            }
            __syncthreads();
        }
    }
    double *Lq = L + ((size_t)jb.noff + g.q) * P;
    for (int i = threadIdx.x; i < P; i += blockDim.x) Lq[i] += acc[i];
    if (threadIdx.x == 0) lflag[jb.noff + g.q] = 1;
}

// ---------------------------------------------------------------- DFGTPost
// One block per (query leaf, job).  LDS: acc[P] | tmp[P] | coef[pmax^2] (global when large).
__global__ __launch_bounds__(256) void k_post(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                              int nleaves, const double *__restrict__ L,
                                              const unsigned char *__restrict__ lflag, const double *__restrict__ GE,
                                              const double *__restrict__ GF, int use_lds,
                                              double *__restrict__ gscratch) {
    extern __shared__ double smem[];
    __shared__ int path[256];
    __shared__ int plen_s, any_s;
    const int job = blockIdx.y;
    const Job jb = jobs[job];
    const DevTree &Q = trees[jb.qt];
    const int leaf = Q.leaves[blockIdx.x];
    const int d = Q.d, pmax = Q.pmax, P = Q.P;
    const double s = jb.s;
    double *acc, *tmp, *coef;
    if (use_lds) {
        acc = smem;
        tmp = acc + P;
        coef = tmp + P;
    } else {
        const size_t slot = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        acc = gscratch + slot * 2 * P;
        tmp = acc + P;
        coef = smem;
    }
    if (threadIdx.x == 0) {
        int n = 0, v = leaf;
        int any = 0;
        while (v >= 0 && n < 256) {
            path[n++] = v;
            any |= lflag[jb.noff + v];
            v = Q.parent[v];
        }
        plen_s = (v >= 0) ? -1 : n;
        any_s = any;
    }
    __syncthreads();
    const int plen = plen_s;
    const int qb = Q.begin[leaf], qe = Q.end[leaf];
    if (plen < 0) {
        // a path deeper than 256 levels cannot be walked here; signal NaN
        for (int qi = qb + threadIdx.x; qi < qe; qi += blockDim.x) jb.out[Q.perm[qi]] = NAN;
        return;
    }
    const bool any = any_s != 0;
    if (any) {
        for (int i = threadIdx.x; i < P; i += blockDim.x) acc[i] = 0.0;
        bool nonzero = false;
        for (int pi = plen - 1; pi >= 0; --pi) {
            const int v = path[pi];
            if (pi != plen - 1 && nonzero) {
                // TransLocalToLocal from the parent path[pi+1] to v, one axis at a time:
                // child L_a += sum_{b >= a} C(b, a) L_b X^{b-a},  X = (v.c - parent.c) s
                const int u = path[pi + 1];
                double *src = acc, *dst = tmp;
                for (int k = 0; k < d; ++k) {
                    const double X = (Q.ctr[(size_t)v * d + k] - Q.ctr[(size_t)u * d + k]) * s;
                    __syncthreads();
                    for (int i = threadIdx.x; i < pmax * pmax; i += blockDim.x) {
                        const int a = i / pmax, b = i % pmax;
                        double c = 0.0;
                        if (b >= a) {
                            c = 1.0;
                            for (int t = 0; t < b - a; ++t) c *= X * (double)(b - t) / (double)(b - a - t);
                        }
                        coef[i] = c;
                    }
                    __syncthreads();
                    mode_product(src, dst, coef, P, d, pmax, k, pmax);
                    double *t2 = src;
                    src = dst;
                    dst = t2;
                }
                __syncthreads();
                if (src != acc)
                    for (int i = threadIdx.x; i < P; i += blockDim.x) acc[i] = src[i];
                __syncthreads();
            }
            if (lflag[jb.noff + v]) {
                const double *Lv = L + ((size_t)jb.noff + v) * P;
                for (int i = threadIdx.x; i < P; i += blockDim.x) acc[i] += Lv[i];
                nonzero = true;
            }
            __syncthreads();
        }
    }
    // EvalLocalExpansion at the leaf's points, then G = G_L + G_F + G_E
    const double *c = Q.ctr + (size_t)leaf * d;
    for (int qi = qb + threadIdx.x; qi < qe; qi += blockDim.x) {
        double gl = 0.0;
        if (any) {
            double y[kMaxD];
            for (int k = 0; k < d; ++k) y[k] = (Q.x[(size_t)qi * d + k] - c[k]) * s;
            for (int i = 0; i < P; ++i) {
                const double a = acc[i];
                if (a == 0.0) continue;
                int rem = i;
                double prod = 1.0;
                for (int k = d - 1; k >= 0; --k) {
                    prod *= powi(y[k], rem % pmax);
                    rem /= pmax;
                }
                gl = fma(a, prod, gl);
            }
        }
        const size_t gi = (size_t)jb.qoff + qi;
        jb.out[Q.perm[qi]] = gl + GF[gi] + GE[gi];
    }
}

// ---------------------------------------------------------------- host side
// Optional per-launch timing with HIP events on the caller's stream.
struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Rec {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    size_t used = 0;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin_call(bool enable) {
        on = enable;
        recs.clear();
        used = 0;
    }
    hipEvent_t start(hipStream_t st) {
        if (!on) return nullptr;
        hipEvent_t e = get();
        if (e) (void)hipEventRecord(e, st);
        return e;
    }
    void stop(int kind, hipEvent_t a, hipStream_t st) {
        if (!on || !a) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, st);
        recs.push_back(Rec{kind, a, b});
    }
    // Call after the stream has been synchronised.
    void collect(dfgt_stats *s) {
        for (int k = 0; k < 5; ++k) {
            s->kernel_ms[k] = 0.0;
            s->kernel_launches[k] = 0;
        }
        for (auto &r : recs) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                s->kernel_ms[r.kind] += ms;
                s->kernel_launches[r.kind] += 1;
            }
        }
    }
};
thread_local Profiler g_prof;

enum { K_TRAV = 0, K_BASE, K_FAR, K_LOCAL, K_POST };

struct Workspace {
    DevBuf jobs, trees, GE, GF, glE, L, lflag, segA, segB, pairA, pairB, dec, egrp, eops, fgrp, fops, lgrp, lops,
        cnt, stats, lscr, pscr;
};
thread_local Workspace g_ws;

template <class T> dfgt_status grow(DevBuf &b, size_t n) { return b.reserve(sizeof(T) * std::max<size_t>(n, 1)); }

}  // namespace

dfgt_status run_gauss_sum(dfgt_tree_s *Qh, dfgt_tree_s *Rh, const double *h, int nh, double eps, int precision,
                          int force, int profile, double *G, dfgt_stats *stats_out, hipStream_t st) {
    Workspace &w = g_ws;
    Profiler &prof = g_prof;
    prof.begin_call(profile != 0);
    const DevTree &Qv = Qh->host_view;
    const int NQ = (int)Qh->n, MQ = (int)Qh->m, P = Qh->P, pmax = Qh->pmax, d = Qh->d;
    const bool mono = Qh == Rh;
    // A tolerance below the mixed-precision rounding budget needs FP64 leaf sums.
    if (precision == DFGT_PREC_MIXED && eps > 0.0 && eps < 2e-5) precision = DFGT_PREC_FP64;
    // Rounding budget of the exhaustive sums (Theorem of Section 3.10 assumes
    // them exact): mixed precision <= 1e-5 relative, FP64 ~1e-13.
    const double eps_round = precision == DFGT_PREC_FP64 ? 1e-12 : 1e-5;
    const double eps_eff = eps > 2.0 * eps_round ? eps - eps_round : 0.0;

    std::vector<Job> jobs(nh);
    for (int k = 0; k < nh; ++k) {
        Job &j = jobs[k];
        j.h = h[k];
        j.s = 1.0 / (std::sqrt(2.0) * h[k]);
        j.inv2h2 = 1.0 / (2.0 * h[k] * h[k]);
        j.sig = 1.2011224087864498 * j.s;  // sqrt(log2 e) s: e^{-x^2/2h^2} = 2^{-(sig x)^2}
        j.eps_eff = eps_eff;
        j.nR = (double)Rh->n;
        j.qt = 0;
        j.rt = 1;
        j.qoff = (long long)k * NQ;
        j.noff = (long long)k * MQ;
        j.out = G + (size_t)k * NQ;
        j.mono = mono ? 1 : 0;
        j.pad = 0;
    }
    DevTree tv[2] = {Qh->host_view, Rh->host_view};
    DFGT_TRY(grow<Job>(w.jobs, nh));
    DFGT_TRY(grow<DevTree>(w.trees, 2));
    DFGT_HIP(hipMemcpyAsync(w.jobs.p, jobs.data(), sizeof(Job) * nh, hipMemcpyHostToDevice, st));
    DFGT_HIP(hipMemcpyAsync(w.trees.p, tv, sizeof(tv), hipMemcpyHostToDevice, st));
    const size_t nqa = (size_t)nh * NQ, nna = (size_t)nh * MQ;
    DFGT_TRY(grow<double>(w.GE, nqa));
    DFGT_TRY(grow<double>(w.GF, nqa));
    DFGT_TRY(grow<double>(w.glE, nna));
    DFGT_TRY(grow<double>(w.L, nna * P));
    DFGT_TRY(grow<unsigned char>(w.lflag, nna));
    DFGT_TRY(grow<int>(w.cnt, C_N));
    DFGT_TRY(grow<unsigned long long>(w.stats, S_N));
    DFGT_HIP(hipMemsetAsync(w.GE.p, 0, sizeof(double) * nqa, st));
    DFGT_HIP(hipMemsetAsync(w.GF.p, 0, sizeof(double) * nqa, st));
    DFGT_HIP(hipMemsetAsync(w.glE.p, 0, sizeof(double) * nna, st));
    DFGT_HIP(hipMemsetAsync(w.L.p, 0, sizeof(double) * nna * P, st));
    DFGT_HIP(hipMemsetAsync(w.lflag.p, 0, nna, st));
    DFGT_HIP(hipMemsetAsync(w.stats.p, 0, sizeof(unsigned long long) * S_N, st));

    // level 0: (Q_root, {R_root}) for every job
    int nseg = nh, npair = nh;
    {
        std::vector<Seg> s0(nh);
        std::vector<int> p0(nh, 0);
        for (int k = 0; k < nh; ++k) s0[k] = Seg{0, k, k, 1, 0.0};
        DFGT_TRY(grow<Seg>(w.segA, nseg));
        DFGT_TRY(grow<int>(w.pairA, npair));
        DFGT_HIP(hipMemcpyAsync(w.segA.p, s0.data(), sizeof(Seg) * nh, hipMemcpyHostToDevice, st));
        DFGT_HIP(hipMemcpyAsync(w.pairA.p, p0.data(), sizeof(int) * nh, hipMemcpyHostToDevice, st));
        DFGT_HIP(hipStreamSynchronize(st));
    }
    const size_t lds_local = sizeof(double) * (3 * (size_t)P + pmax * pmax + 2 * pmax * d);
    const bool local_lds = lds_local <= 60 * 1024;
    const size_t lds_post = sizeof(double) * (2 * (size_t)P + pmax * pmax);
    const bool post_lds = lds_post <= 60 * 1024;
    const DevTree *td = w.trees.as<DevTree>();
    const Job *jd = w.jobs.as<Job>();
    int levels = 0;
    DevBuf *segCur = &w.segA, *segNext = &w.segB, *pairCur = &w.pairA, *pairNext = &w.pairB;
    while (nseg > 0) {
        ++levels;
        DFGT_TRY(grow<Seg>(*segNext, 2 * (size_t)nseg));
        DFGT_TRY(grow<int>(*pairNext, 4 * (size_t)npair));
        DFGT_TRY(grow<int>(w.dec, npair));
        DFGT_TRY(grow<Group>(w.egrp, nseg));
        DFGT_TRY(grow<Group>(w.fgrp, nseg));
        DFGT_TRY(grow<Group>(w.lgrp, nseg));
        DFGT_TRY(grow<int>(w.eops, npair));
        DFGT_TRY(grow<Op>(w.fops, npair));
        DFGT_TRY(grow<Op>(w.lops, npair));
        DFGT_HIP(hipMemsetAsync(w.cnt.p, 0, sizeof(int) * C_N, st));
        TravOut o{segNext->as<Seg>(),       pairNext->as<int>(), w.egrp.as<Group>(), w.eops.as<int>(),
                  w.fgrp.as<Group>(),       w.fops.as<Op>(),     w.lgrp.as<Group>(), w.lops.as<Op>(),
                  w.cnt.as<int>(),          w.stats.as<unsigned long long>()};
        hipEvent_t ev = prof.start(st);
        hipLaunchKernelGGL(k_traverse, dim3(nseg), dim3(64), 0, st, td, jd, segCur->as<Seg>(), pairCur->as<int>(),
                           w.glE.as<double>(), force, w.dec.as<int>(), o);
        DFGT_HIP(hipGetLastError());
        prof.stop(K_TRAV, ev, st);
        int c[C_N];
        DFGT_HIP(hipMemcpyAsync(c, w.cnt.p, sizeof(int) * C_N, hipMemcpyDeviceToHost, st));
        DFGT_HIP(hipStreamSynchronize(st));
        if (c[C_EGRP]) {
            ev = prof.start(st);
            hipLaunchKernelGGL(k_base, dim3(c[C_EGRP]), dim3(kBaseBlock), 0, st, td, jd, w.egrp.as<Group>(),
                               w.eops.as<int>(), precision, w.GE.as<double>(), w.glE.as<double>(),
                               w.stats.as<unsigned long long>());
            prof.stop(K_BASE, ev, st);
        }
        if (c[C_FGRP]) {
            ev = prof.start(st);
            hipLaunchKernelGGL(k_far, dim3(c[C_FGRP]), dim3(256), 0, st, td, jd, w.fgrp.as<Group>(),
                               w.fops.as<Op>(), w.GF.as<double>());
            prof.stop(K_FAR, ev, st);
        }
        if (c[C_LGRP]) {
            ev = prof.start(st);
            double *scr = nullptr;
            if (!local_lds) {
                DFGT_TRY(grow<double>(w.lscr, (size_t)c[C_LGRP] * 3 * P));
                scr = w.lscr.as<double>();
            }
            const size_t sh = local_lds ? lds_local : sizeof(double) * (pmax * pmax + 2 * pmax * d);
            hipLaunchKernelGGL(k_local, dim3(c[C_LGRP]), dim3(kLocBlock), sh, st, td, jd, w.lgrp.as<Group>(),
                               w.lops.as<Op>(), local_lds ? 1 : 0, scr, w.L.as<double>(),
                               w.lflag.as<unsigned char>());
            prof.stop(K_LOCAL, ev, st);
        }
        DFGT_HIP(hipGetLastError());
        nseg = c[C_SEG];
        npair = c[C_PAIR];
        std::swap(segCur, segNext);
        std::swap(pairCur, pairNext);
    }
    {
        double *scr = nullptr;
        if (!post_lds) {
            DFGT_TRY(grow<double>(w.pscr, (size_t)Qv.nleaves * nh * 2 * P));
            scr = w.pscr.as<double>();
        }
        const size_t sh = post_lds ? lds_post : sizeof(double) * pmax * pmax;
        hipEvent_t ev = prof.start(st);
        hipLaunchKernelGGL(k_post, dim3(Qv.nleaves, nh), dim3(256), sh, st, td, jd, Qv.nleaves, w.L.as<double>(),
                           w.lflag.as<unsigned char>(), w.GE.as<double>(), w.GF.as<double>(), post_lds ? 1 : 0,
                           scr);
        DFGT_HIP(hipGetLastError());
        prof.stop(K_POST, ev, st);
    }
    if (stats_out) {
        unsigned long long sv[S_N];
        DFGT_HIP(hipMemcpyAsync(sv, w.stats.p, sizeof(sv), hipMemcpyDeviceToHost, st));
        DFGT_HIP(hipStreamSynchronize(st));
        std::memset(stats_out, 0, sizeof(*stats_out));
        stats_out->node_pairs = (int64_t)sv[S_PAIRS];
        stats_out->prune_f = (int64_t)sv[S_F];
        stats_out->prune_d = (int64_t)sv[S_D];
        stats_out->prune_t = (int64_t)sv[S_T];
        stats_out->prune_centroid = (int64_t)sv[S_C];
        stats_out->base_leaf_pairs = (int64_t)sv[S_BLEAF];
        stats_out->base_point_pairs = (int64_t)sv[S_BPTS];
        stats_out->levels = levels;
        stats_out->max_order = (int64_t)sv[S_MAXORD];
        stats_out->fp64_groups = (int64_t)sv[S_FP64];
        if (prof.on) prof.collect(stats_out);
    }
    return DFGT_OK;
}

}  // namespace dfgt
