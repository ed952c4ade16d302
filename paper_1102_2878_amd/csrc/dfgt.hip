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
// Op groups are appended to lists that persist across levels, and each (node,
// job) chains its groups (a node has at most one segment per level, so the
// chain order is fixed).  After the traversal:
//   k_local  one wave per (Q, job) with local ops: AccumulateDirectLocalMoment
//            (D) and TransFarToLocal (T) into Q's local moments;
//   k_leaf   one block per (query leaf, job) does everything its queries need:
//            the exhaustive leaf-leaf sums of its E chain (DFGTBase), the
//            far-field evaluations (EvalFarFieldExpansion) of the F chains of
//            the leaf and all its ancestors, the TransLocalToLocal walk from
//            the root to the leaf and EvalLocalExpansion (DFGTPost), and the
//            combination G = G_E + G_F + G_L in the caller's order.
// Every sum is taken in a fixed order without atomics, so results are
// bitwise reproducible and independent of the other jobs in the batch.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "etile.h"
#include "series.h"

namespace dfgt {
namespace {

enum { METH_E = 0, METH_F = 1, METH_D = 2, METH_T = 3 };

struct Job {
    double h, s, inv2h2, sig;  // s = 1/(sqrt2 h); sig = sqrt(log2 e) s
    double eps_eff;            // eps minus the rounding budget of the exhaustive sums
    double nR;                 // W(R_total): the total reference weight (|R_total| unweighted), in stored units
    double cntR;               // |R_total|
    double wscale;             // stored weights are w / wscale (1 unweighted); outputs are multiplied back
    double prior;              // a known lower bound on every G(q) (1 when Q = R: the self term)
    int qt, rt;                // indices into the tree table
    long long qoff;            // offset of this job's per-query arrays
    long long noff;            // offset of this job's per-node arrays
    double *out;               // caller's output for this job (caller order)
    double *outH, *outQ;       // gradient mode: dG/dh [N_Q] and dG/dq [N_Q][D] (caller order), or null
    double cost_e;             // weight of the exhaustive cost in ChooseBestMethod
    double wF, wD, wT;         // GPU weights of the far-field, direct-local and far-to-local costs
    int mono;                  // Q and R are the same point set
    int loo;                   // leave-one-out: Q = R and each query's own point is left out of its sum
    double a32;                // largest |a| + |b| (sig units, coordinates relative to the query
                               // leaf's centre) for which FP32 differences keep the exhaustive
                               // sums within their rounding budget; <= 0: FP64 differences only
    double r32;                // largest query-leaf half-diagonal (sig units) for which the
                               // matrix-core tiles' FP32 products keep that budget; <= 0: FP64
    double win;                // staging window of the matrix-core tiles (sig units): references
                               // farther than win from the query leaf are left out (t >= win^2)
};

struct Seg {
    int q, job, start, count;
    double gl;  // pruned lower-bound contributions inherited by Q
};

struct Group {
    int q, job, start, count;
    int flags;  // E groups: 1 = compute in FP64 (underflow guard)
    int next;   // previous group of the same (node, job), -1 = none
};

struct Op {
    int r, meta;  // meta = order | (method << 8)
};
static_assert(sizeof(Op) == 8 && offsetof(Op, meta) == 4, "k_leaf reads an Op as one 64-bit word");

// counters: the first two are reset per level, the others accumulate.  Every
// counter and statistic sits in its own 128-byte line (CP / SP stride), so the
// atomics of different counters do not serialise on one L2 channel.
constexpr int CP = 32;  // ints per counter line
constexpr int SP = 16;  // u64 per statistics line
enum {
    C_SEG = 0,  // per level: segments and pairs of the next level
    C_PAIR,
    C_EGRP,     // cumulative over the call
    C_EOP,
    C_FGRP,
    C_FOP,
    C_LGRP,
    C_LOP,
    C_LNODE,
    C_EF64,     // E groups flagged by the underflow guard (FP64 sums)
    C_EHEAVY,   // (job, query leaf) items by exhaustive work: long lists, short lists, none
    C_ENORM,
    C_EEMPTY,
    C_EWIDE,    // items left to the vector-ALU tiles by the matrix-core pass (query leaf wide against h)
    C_EHEAVY64, // items of the matrix-core pass with FP64 products: long lists, short lists
    C_ENORM64,
    C_ECH,      // entries of the flattened E chains (k_eorder)
    C_N
};

// Capacities of the traversal's output arrays.  Reservations beyond them set
// the overflow flag and write nothing; the host then grows and reruns.
struct Caps {
    int seg, pair, eop, fop, lop, grp, lnode;
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
    S_SEGS,
    S_MAXSEG,
    S_MAXLOPS,
    S_FW,  // algorithmic work of the pruned pairs: F sum N_Q p^D, D sum N_R p^D, T sum D p^2D
    S_DW,
    S_TW,
    S_EP32,  // exhaustive pairs of the matrix-core tiles with FP32 products
    S_EP64,  // ... with FP64 products
    S_N
};

// ---------------------------------------------------------------- bounds (Section 3.5)
__device__ __forceinline__ double powi(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// 1/sqrt(p!) for p = 0..16 (p_max <= 16), the factor of Szasz's inequality in
// the truncation bounds.
__constant__ double kInvSqrtFact[17] = {
    1.0, 1.0, 0.7071067811865476, 0.408248290463863, 0.2041241452319315, 0.09128709291752768,
    0.037267799624996496, 0.014085904245475277, 0.004980119205559973, 0.0016600397351866577,
    0.00052495065695726, 0.00015827857841616382, 4.569108992776174e-05, 1.2672428274337011e-05,
    3.3868489186454308e-06, 8.744806305356235e-07, 2.1862015763390587e-07};

// sum_{k<D} C(D,k) a^k b^{D-k} = (a+b)^D - a^D = b sum_{k<D} (a+b)^k a^{D-1-k},
// evaluated in the last form: positive terms only, so no cancellation when
// b << a (the bound stays an upper bound to a few ulps).
__device__ __forceinline__ double binom_tail(double a, double b, int D) {
    const double c = a + b;
    double t = 1.0, aj = 1.0;
    for (int j = 1; j < D; ++j) {
        aj *= a;
        t = fma(c, t, aj);
    }
    return b * t;
}

// Bounds are compared with a small relative slack on the safe side.
constexpr double kSlack = 1.0 + 1e-10;

// Alg. FarFieldOrder / LocalAccumulationOrder with the far-field / local lemma
// bound, eqs. (error_bound_far_field), (error_bound_local):
//   nR sum_{k<D} C(D,k) (1 - r^p)^k (r^p / sqrt(p!))^{D-k} / (1 - r)^D <= tau,
// r = width / (2h); returns the least such p <= pmax, 0 = none (r >= 1: no bound).
// r^p runs incrementally and the division is multiplied out.
__device__ int order_far(double r, double nR, double tau, int pmax, int D) {
    if (r >= 1.0) return 0;
    const double lim = tau * powi(1.0 - r, D);
    double rp = 1.0;
    for (int p = 1; p <= pmax; ++p) {
        rp *= r;
        if (nR * binom_tail(1.0 - rp, rp * kInvSqrtFact[p], D) * kSlack <= lim) return p;
    }
    return 0;
}

// Alg. ConvertFarFieldToLocalOrder with the far-to-local lemma bound, eq.
// (error_bound_far_to_local), read with the lemma's radius r = width / (2h) < 1/2
// (its formula holds 2r):
//   nR sum_{k<D} C(D,k) ((1 - (2r)^p)^2)^k ((2r)^p (2 - (2r)^p) / sqrt(p!))^{D-k} / (1 - 2r)^{2D} <= tau.
__device__ int order_f2l(double r, double nR, double tau, int pmax, int D) {
    if (r >= 0.5) return 0;
    const double lim = tau * powi(1.0 - 2.0 * r, 2 * D);
    double tp = 1.0;
    for (int p = 1; p <= pmax; ++p) {
        tp *= 2.0 * r;
        const double a = (1.0 - tp) * (1.0 - tp);
        if (nR * binom_tail(a, tp * (2.0 - tp) * kInvSqrtFact[p], D) * kSlack <= lim) return p;
    }
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
// The error bounds take wR, the weight of R (its point count |R| when the
// points carry no weights: each point's error is scaled by its weight); the
// costs take the point count nR.
// When that bound holds c_T = D, the least any method can cost; only F at
// order 1 with N_Q = 1 or D at order 1 with N_R = 1 can tie it (and win the
// tie), so the order searches are skipped.  ku = K(d^u).
// Gradient mode (gr): a local expansion truncated at order p has a q- and
// s-derivative whose truncation error is larger than the value's by about p/r
// (r the scaled node radius), and the centroid form is constant over Q.  So
// D and T use one order more than the value bound needs (at most p_max) and
// the centroid form is not used; F is unchanged (its derivative series is the
// far-field series of the derivative kernel, one Hermite index higher).
__device__ int choose(const PairGeom &g, double h, double inv2h2, double ku, double nQ, double nR, double wR,
                      double tau, int pmax, int D, int force, int gr, const Job &jb, int *order, double *kc_out) {
    const double cost_e = jb.cost_e;
    if (force == DFGT_FORCE_EXACT) {
        *order = 0;
        return METH_E;
    }
    const double kl = exp(-g.sl * inv2h2), kc = exp(-g.sc * inv2h2);
    *kc_out = kc;
    const double cb = wR * (fmax(kl - kc, kc - ku) + 1e-15 * kl);
    const bool centroid = !gr && cb <= tau;
    if (centroid && force == DFGT_FORCE_NONE) {
        if (nQ == 1.0 && order_far(g.wR / (2.0 * h), wR, tau, 1, D) == 1) {
            *order = 1;
            return METH_F;
        }
        if (nR == 1.0 && order_far(g.wQ / (2.0 * h), wR, tau, 1, D) == 1) {
            *order = 1;
            return METH_D;
        }
        *order = 1;
        return METH_T;
    }
    const int pl = gr ? pmax - 1 : pmax;  // largest value order a local expansion may need
    int pF = order_far(g.wR / (2.0 * h), wR, tau, pmax, D);
    int pD = pl > 0 ? order_far(g.wQ / (2.0 * h), wR, tau, pl, D) : 0;
    int pT = pl > 0 ? order_f2l(fmax(g.wQ, g.wR) / (2.0 * h), wR, tau, pl, D) : 0;
    if (gr) {
        pD = pD ? pD + 1 : 0;
        pT = pT ? pT + 1 : 0;
    }
    if (centroid) pT = 1;
    if (force == DFGT_FORCE_F) pD = pT = 0;
    if (force == DFGT_FORCE_D) pF = pT = 0;
    if (force == DFGT_FORCE_T) pF = pD = 0;
    if (force == DFGT_FORCE_CENTROID) {
        pF = pD = 0;
        pT = centroid ? 1 : 0;
    }
    const double inf = INFINITY;
    const double cF = pF ? jb.wF * D * nQ * powi((double)pF, D) : inf;
    const double cD = pD ? jb.wD * D * nR * powi((double)pD, D) : inf;
    const double cT = pT ? jb.wT * D * powi((double)pT, 2 * D) : inf;
    const double cE = cost_e * D * nQ * nR;
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
    int *lnodes;  // (q, job) pairs with local ops, 2 ints each
    int *headE, *headF, *headL;
    int *cnt;       // cumulative counters
    int *lvl_next;  // per-level counters written by this level
    int *overflow;
    unsigned long long *stats;
    double *cval;    // [job][node] constant local terms from order-1 translations
    unsigned char *selfE;  // [job][leaf] leave-one-out: the leaf's pair with itself is exhaustive
                           // (k_leaf adds the leaf's sums from k_selfpre)
    const double *selfmin; // [job][leaf] leave-one-out: a lower bound on the leaf's sums
    int want_stats;  // collect dfgt_stats counters
    Caps cap;
};

__device__ __forceinline__ int wave_excl(int v, int *total) {
    int inc = wave_incl_scan(v);
    *total = __builtin_amdgcn_readlane(inc, 63);
    return inc - v;
}

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// One wave per segment, kTravWaves segments per block.  Every segment appends
// to shared lists (E, F, local ops, their groups, next-level pairs and
// segments); the reservations of a block's segments are made together, one
// atomic per list per block, because same-address device atomics serialise
// (one per segment would cost ~20 ns each at thousands of segments a level).
constexpr int kTravWaves = 4;
enum { R_EOP = 0, R_EGRP, R_FOP, R_FGRP, R_LOP, R_LGRP, R_PAIR, R_SEG, R_N };
enum { T_PAIRS = 0, T_SEGS, T_F, T_D, T_T, T_C, T_BLEAF, T_BPTS, T_FW, T_DW, T_TW, T_N };  // block-summed statistics

struct TravShared {
    int req[kTravWaves][R_N];  // per-wave requests, then per-wave bases
    unsigned long long st[kTravWaves][T_N];
    unsigned long long maxseg[kTravWaves], maxord[kTravWaves];
};

// One block iteration: wave w of the block handles segment si (valid when
// si < nseg; invalid waves take part in the block's reservation with nothing).
__device__ void traverse_segment(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                 const Seg *__restrict__ segs, int si, bool valid, const int *__restrict__ pairs,
                                 int force, int gr, int leaf_local, int *dec, double *kus, const TravOut &o,
                                 TravShared &sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Seg sg{0, 0, 0, 0, 0.0};
    if (valid) sg = segs[si];
    const Job jb = jobs[sg.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int D = Q.d, pmax = Q.pmax;
    const int q = sg.q;
    const bool qleaf = valid && Q.left[q] < 0;
    const double nQ = valid ? (double)(Q.end[q] - Q.begin[q]) : 0.0;

    // 1. lower bound over the whole list.  The first 64 pairs (all of them
    // for most segments) keep their node data in registers for the passes
    // below; pairs beyond reload it.
    double sl = 0.0;
    int r0 = -1, m0 = METH_E, ord0 = 0, left0 = -1, right0 = -1;
    double nR0 = 0.0, wR0 = 0.0, ku0 = 0.0;
    PairGeom g0{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = lane; i < sg.count; i += 64) {
        const int r = pairs[sg.start + i];
        const PairGeom g = pair_geom(Q, q, R, r);
        const double ku = exp(-g.su * jb.inv2h2);
        const double nR = (double)(R.end[r] - R.begin[r]);
        const double wR = R.w ? R.mu[(size_t)r * R.P] : nR;
        // leave-one-out: the pair of a node with itself covers each query's own
        // point, which its sum leaves out
        const double wL = (jb.loo && r == q) ? wR - 1.0 : wR;
        if (i < 64) {
            r0 = r;
            g0 = g;
            ku0 = ku;
            nR0 = nR;
            wR0 = wR;
            left0 = R.left[r];
            right0 = R.right[r];
        } else {
            kus[sg.start + i] = ku;  // reused by the decisions below
        }
        sl += wL * ku;
    }
    sl = wave_sum(sl);
    double gl = fmax((sg.gl + sl) * (1.0 - 1e-12), jb.prior);
    if (jb.loo && qleaf) gl = fmax(gl, o.selfmin[(size_t)jb.noff + q]);  // the leaf's own leave-one-out sums

    // 2. decisions and counts
    int cE = 0, cF = 0, cL = 0, cN = 0, nT = 0, nC = 0, nD = 0, maxord = 0;
    double plo = 0.0, ept = 0.0, ccon = 0.0, wkF = 0.0, wkD = 0.0, wkT = 0.0;
    for (int i = lane; i < sg.count; i += 64) {
        const bool first = i < 64;
        const int r = first ? r0 : pairs[sg.start + i];
        const PairGeom g = first ? g0 : pair_geom(Q, q, R, r);
        const double nR = first ? nR0 : (double)(R.end[r] - R.begin[r]);
        const double wR = first ? wR0 : (R.w ? R.mu[(size_t)r * R.P] : nR);
        const double tau = jb.eps_eff * wR * gl / jb.nR;
        const double ku = first ? ku0 : kus[sg.start + i];
        int ord = 0;
        double kc = 0.0;
        const int m = choose(g, jb.h, jb.inv2h2, ku, nQ, nR, wR, tau, pmax, D, force, gr, jb, &ord, &kc);
        const bool rleaf = (first ? left0 : R.left[r]) < 0;
        const bool self = jb.loo && r == q;
        if (m != METH_E) {
            plo += (self ? wR - 1.0 : wR) * ku;
            // the approximation covers every query's own point (K = 1): left out here
            if (self) ccon -= 1.0;
            if (o.want_stats) {
                const double pd = powi((double)ord, D);
                if (m == METH_F) wkF += nQ * pd;
                else if (m == METH_D) wkD += nR * pd;
                else if (ord > 1) wkT += D * pd * pd;
            }
            if (m == METH_F) ++cF;
            else if (m == METH_T && ord == 1) {
                // order-1 far-to-local translation (the centroid form): its only
                // term is L_0 += mu_0 e^{-|t0|^2} = W(R) K(|Q.c - R.c|), a scalar
                // added to Q's constant term right here (no op)
                ccon += wR * kc;
                ++nC;
            } else {
                // a D op is emitted as one op per chunk of <= 64 reference points
                cL += m == METH_D ? (int)((nR + 63.0) / 64.0) : 1;
                if (m == METH_D) ++nD;
                else ++nT;
            }
            maxord = max(maxord, ord);
        } else if (qleaf && rleaf) {
            if (!self) ++cE;  // a leaf's pair with itself is summed by k_selfsum
            ept += nR;
        } else {
            cN += (qleaf || !rleaf) ? 2 : 1;
        }
        if (first) {
            m0 = m;
            ord0 = ord;
        } else {
            dec[sg.start + i] = m | (ord << 4);
        }
    }
    int tE, tF, tL, tN;
    wave_excl(cE, &tE);
    wave_excl(cF, &tF);
    wave_excl(cL, &tL);
    wave_excl(cN, &tN);
    plo = wave_sum(plo);
    ept = wave_sum(ept);
    ccon = wave_sum(ccon);
    if (o.want_stats) {
        wkF = wave_sum(wkF);
        wkD = wave_sum(wkD);
        wkT = wave_sum(wkT);
    }
    const double gl_child = sg.gl + plo * (1.0 - 1e-12);
    const int nFp = wave_sum_i(cF), nDp = wave_sum_i(nD), nTp = wave_sum_i(nT), nCp = wave_sum_i(nC);
    const int mo = wave_max_i(maxord);

    // The chain heads of (q, job): only this segment touches them at this level
    // (one segment per (node, job) per level, levels in order), so the links
    // below are a plain read and write; the read is issued here and completes
    // behind the reservation.
    const size_t hq = (size_t)jb.noff + q;
    int head0 = -1;
    if (valid && lane < 3) head0 = (lane == 0 ? o.headE : (lane == 1 ? o.headF : o.headL))[hq];

    // 3. the block's reservations: per-wave requests, one atomic per list
    const int npair_out = qleaf ? tN : 2 * tN;
    const int nseg_out = tN > 0 ? (qleaf ? 1 : 2) : 0;
    if (lane == 0) {
        int *rq = sh.req[wv];
        rq[R_EOP] = tE;
        rq[R_EGRP] = tE ? 1 : 0;
        rq[R_FOP] = tF;
        rq[R_FGRP] = tF ? 1 : 0;
        rq[R_LOP] = tL;
        rq[R_LGRP] = tL ? 1 : 0;
        rq[R_PAIR] = npair_out;
        rq[R_SEG] = nseg_out;
        if (o.want_stats) {
            unsigned long long *t = sh.st[wv];
            t[T_PAIRS] = valid ? (unsigned long long)sg.count : 0ull;
            t[T_SEGS] = valid ? 1ull : 0ull;
            t[T_F] = (unsigned long long)nFp;
            t[T_D] = (unsigned long long)nDp;
            t[T_T] = (unsigned long long)nTp;
            t[T_C] = (unsigned long long)nCp;
            t[T_BLEAF] = (unsigned long long)tE;
            t[T_BPTS] = (unsigned long long)(nQ * ept);
            t[T_FW] = (unsigned long long)wkF;
            t[T_DW] = (unsigned long long)wkD;
            t[T_TW] = (unsigned long long)wkT;
            sh.maxseg[wv] = valid ? (unsigned long long)sg.count : 0ull;
            sh.maxord[wv] = (unsigned long long)mo;
        }
    }
    __syncthreads();
    if (threadIdx.x < R_N) {
        const int c = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < kTravWaves; ++w) {
            const int v = sh.req[w][c];
            sh.req[w][c] = tot;
            tot += v;
        }
        int base = 0;
        if (tot) {
            int *ctr = c == R_EOP   ? &o.cnt[C_EOP * CP]
                       : c == R_EGRP ? &o.cnt[C_EGRP * CP]
                       : c == R_FOP  ? &o.cnt[C_FOP * CP]
                       : c == R_FGRP ? &o.cnt[C_FGRP * CP]
                       : c == R_LOP  ? &o.cnt[C_LOP * CP]
                       : c == R_LGRP ? &o.cnt[C_LGRP * CP]
                       : c == R_PAIR ? &o.lvl_next[C_PAIR * CP]
                                     : &o.lvl_next[C_SEG * CP];
            base = atomicAdd(ctr, tot);
        }
        for (int w = 0; w < kTravWaves; ++w) sh.req[w][c] += base;
    } else if (o.want_stats && threadIdx.x >= 64 && threadIdx.x < 64 + T_N) {
        const int c = threadIdx.x - 64;
        unsigned long long tot = 0;
        for (int w = 0; w < kTravWaves; ++w) tot += sh.st[w][c];
        const int sidx[T_N] = {S_PAIRS, S_SEGS, S_F, S_D, S_T, S_C, S_BLEAF, S_BPTS, S_FW, S_DW, S_TW};
        if (tot) atomicAdd(&o.stats[sidx[c] * SP], tot);
    } else if (o.want_stats && threadIdx.x == 64 + T_N) {
        unsigned long long ms = 0, mx = 0;
        for (int w = 0; w < kTravWaves; ++w) {
            ms = sh.maxseg[w] > ms ? sh.maxseg[w] : ms;
            mx = sh.maxord[w] > mx ? sh.maxord[w] : mx;
        }
        if (ms) atomicMax(&o.stats[S_MAXSEG * SP], ms);
        if (mx) atomicMax(&o.stats[S_MAXORD * SP], mx);
    }
    __syncthreads();
    const int ebase = sh.req[wv][R_EOP], gE = sh.req[wv][R_EGRP];
    const int fbase = sh.req[wv][R_FOP], gF = sh.req[wv][R_FGRP];
    const int lbase = sh.req[wv][R_LOP], gL = sh.req[wv][R_LGRP];
    const int cbase = sh.req[wv][R_PAIR], sgi = sh.req[wv][R_SEG];
    __syncthreads();  // the table is rewritten by the next iteration
    if (!valid) return;

    // 4. link the new groups into their chains, then write the group records
    const bool okE = tE && ebase + tE <= o.cap.eop && gE < o.cap.grp;
    const bool okF = tF && fbase + tF <= o.cap.fop && gF < o.cap.grp;
    const bool okL = tL && lbase + tL <= o.cap.lop && gL < o.cap.grp;
    const bool okN = npair_out && cbase + npair_out <= o.cap.pair && sgi + nseg_out <= o.cap.seg;
    if (lane == 0 && okE) o.headE[hq] = gE;
    if (lane == 1 && okF) o.headF[hq] = gF;
    if (lane == 2 && okL) o.headL[hq] = gL;
    const int prevE = __shfl(head0, 0, 64), prevF = __shfl(head0, 1, 64), prevL = __shfl(head0, 2, 64);
    if (lane == 0) {
        bool over = (tE && !okE) || (tF && !okF) || (tL && !okL) || (npair_out && !okN);
        if (okE) {
            // underflow guard: FP32 exp2 flushes terms below 2^-126 (and the
            // weighted terms w e, w <= 1 in stored units, likewise); keep that
            // absolute error, at most |R_total| 2^-126, below 2^-26 G by
            // computing tiny sums in FP64.
            const double glb = jb.mono ? fmax(gl, 1.0) : gl;  // q is one of the references: G(q) >= 1
            const int fp64 = glb < jb.cntR * 0x1p-100 ? 1 : 0;
            o.egrp[gE] = Group{q, sg.job, ebase, tE, fp64, prevE};
            if (fp64) atomicAdd(&o.cnt[C_EF64 * CP], 1);
        }
        if (okF) o.fgrp[gF] = Group{q, sg.job, fbase, tF, 0, prevF};
        if (okL) {
            o.lgrp[gL] = Group{q, sg.job, lbase, tL, 0, prevL};
            if (prevL < 0 && !(qleaf && leaf_local)) {  // a leaf's own local ops may run in k_leaf
                const int li = atomicAdd(&o.cnt[C_LNODE * CP], 1);
                if (li < o.cap.lnode) {
                    o.lnodes[2 * li] = q;
                    o.lnodes[2 * li + 1] = sg.job;
                } else {
                    over = true;
                }
            }
        }
        if (over) atomicExch(o.overflow, 1);
        // one segment per (node, job) per level and levels run in order: a
        // plain read-modify-write, deterministic
        if (ccon != 0.0) o.cval[hq] += ccon;
    }

    // 5. write outputs in pair order
    int eo = 0, fo = 0, lo = 0, no = 0;
    const int QL = qleaf ? q : Q.left[q], QR = qleaf ? q : Q.right[q];
    for (int c0 = 0; c0 < sg.count; c0 += 64) {
        const int i = c0 + lane;
        int m = METH_E, ord = 0, r = -1, e = 0, f = 0, l = 0, n = 0, rl = -1, rr = -1;
        bool rleaf = true;
        if (i < sg.count) {
            int nRi;
            if (c0 == 0) {
                r = r0;
                m = m0;
                ord = ord0;
                rl = left0;
                rr = right0;
                nRi = (int)nR0;
            } else {
                r = pairs[sg.start + i];
                const int v = dec[sg.start + i];
                m = v & 15;
                ord = v >> 4;
                rl = R.left[r];
                rr = R.right[r];
                nRi = R.end[r] - R.begin[r];
            }
            rleaf = rl < 0;
            if (m == METH_F) f = 1;
            else if (m != METH_E) l = m == METH_D ? (nRi + 63) / 64 : (ord == 1 ? 0 : 1);
            else if (qleaf && rleaf) {
                if (jb.loo && r == q) o.selfE[hq] = 1;
                else e = 1;
            } else n = (qleaf || !rleaf) ? 2 : 1;
        }
        int te, tf, tl, tn;
        const int xe = wave_excl(e, &te), xf = wave_excl(f, &tf), xl = wave_excl(l, &tl), xn = wave_excl(n, &tn);
        if (e && okE) o.eops[ebase + eo + xe] = r;
        if (f && okF) o.fops[fbase + fo + xf] = Op{r, ord | (METH_F << 8)};
        if (okL)
            for (int ch = 0; ch < l; ++ch) o.lops[lbase + lo + xl + ch] = Op{r, ord | (m << 8) | (ch << 12)};
        if (n && okN) {
            const int p0 = cbase + no + xn;
            if (qleaf) {
                o.npairs[p0] = rl;
                o.npairs[p0 + 1] = rr;
            } else if (rleaf) {
                o.npairs[p0] = r;
                o.npairs[p0 + tN] = r;
            } else {
                o.npairs[p0] = rl;
                o.npairs[p0 + 1] = rr;
                o.npairs[p0 + tN] = rl;
                o.npairs[p0 + tN + 1] = rr;
            }
        }
        eo += te;
        fo += tf;
        lo += tl;
        no += tn;
    }
    if (lane == 0 && tN && okN) {
        o.nsegs[sgi] = Seg{QL, sg.job, cbase, tN, gl_child};
        if (!qleaf) o.nsegs[sgi + 1] = Seg{QR, sg.job, cbase + tN, tN, gl_child};
    }
}

// One level of the traversal; the segment count comes from the previous
// level's counters (or nseg0 at level 0), so no host round trip is needed.
// Blocks of kTravWaves waves stride over the segments together.  Held to 168
// VGPRs (three waves per SIMD instead of two; a few spills): the kernel waits
// on chains of dependent loads, and more waves hide more of them.
__global__ __launch_bounds__(64 * kTravWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_traverse(
    const DevTree *__restrict__ trees, const Job *__restrict__ jobs, const Seg *__restrict__ segs,
    const int *__restrict__ pairs, const int *__restrict__ lvl_in, int nseg0, int force, int gr, int leaf_local,
    int *dec, double *kus, TravOut o) {
    __shared__ TravShared sh;
    if (*o.overflow) return;
    const int nseg = lvl_in ? min(lvl_in[C_SEG * CP], o.cap.seg) : nseg0;
    const int wv = threadIdx.x >> 6;
    for (int b0 = blockIdx.x * kTravWaves; b0 < nseg; b0 += gridDim.x * kTravWaves) {
        const int si = b0 + wv;
        traverse_segment(trees, jobs, segs, si, si < nseg, pairs, force, gr, leaf_local, dec, kus, o, sh);
    }
}

// ---------------------------------------------------------------- local moments: D and T ops
// One wave per (Q, job) with local ops; the node's chain of groups (all
// levels) is walked in a fixed order and accumulated in the wave's LDS:
//   D (AccumulateDirectLocalMoment):
//     L_beta += ((-1)^|beta| / beta!) sum_{x in R} e^{-|t|^2} prod_k H_{beta_k}(t_k),  t = (Q.c - x) s;
//     per chunk of 64 points each lane tabulates one point's H_b(t_k) (the
//     exponential folded into the first dimension), then lanes over beta sum
//     the chunk in point order.
//   T (TransFarToLocal):
//     L_beta += ((-1)^|beta| / beta!) e^{-|t0|^2} sum_{alpha<p} M_alpha prod_k H_{alpha_k+beta_k}(t0_k),
//     t0 = (Q.c - R.c) s, M_alpha = s^|alpha| mu_alpha; at order 1 this is
//     L_0 += |R| e^{-|t0|^2} (M_0 = mu_0 = |R|), the centroid form.
// LDS: acc[P] | Ms[P] | Ht[D][2 pmax] | Hx[64][D][pmax]
__device__ __forceinline__ double coef_beta(int i, int d, int pmax) {
    int rem = i, bs = 0;
    double f = 1.0;
    for (int k = d - 1; k >= 0; --k) {
        const int b = rem % pmax;
        rem /= pmax;
        bs += b;
        f *= inv_factorial(b);
    }
    return (bs & 1) ? -f : f;
}

// Direct local accumulation (D ops, value sums) at the default (D, p_max) of
// D = 1..5 as a contraction over points: with F_j[f] = e_j prod_{k<D-1}
// H_{f_k}(t_jk) (f the digits of axes 0..D-2) and B_j[l] = H_l(t_j,D-1), the
// coefficient beta = f p_max + l gets c_beta sum_j F_j[f] B_j[l], one
// multiply-add per point and coefficient (the general loop takes D loads and
// products).  Points go 32 at a time: lane j builds F_j and B_j in registers
// and stores them to the wave's scratch (32 (PM^(D-1) + PM) doubles plus one
// pad per row, within the general loop's 64 D PM); lanes then take
// coefficients.  The rows have odd strides in doubles: with the even strides
// PM^(D-1) and PM every lane's store of a row element hits the same LDS banks
// (32 ways at stride 16).  The products and their order per point are the
// general loop's: ((e H_0) H_1 ...) H_{D-1}.
__host__ __device__ inline int direct_kind(int d, int pmax) {
    if ((d == 1 || d == 2) && pmax == 6) return d;
    if (d == 3 && pmax == 4) return 3;
    if ((d == 4 || d == 5) && pmax == 2) return d;
    return 0;
}

template <int D, int PM>
__device__ __forceinline__ void direct_op(const DevTree &R, int p, int rb, int re, const double *qc, double s, int P,
                                          const unsigned short *mt, const double *cb, double *acc, double *Hx,
                                          int lane) {
    constexpr int NF = D == 1 ? 1 : (D == 2 ? PM : (D == 3 ? PM * PM : (D == 4 ? PM * PM * PM : PM * PM * PM * PM)));
    constexpr int NFS = NF | 1, PMS = PM | 1;  // odd row strides
    double *Fx = Hx, *Bx = Hx + 32 * NFS;
    for (int x0 = rb; x0 < re; x0 += 32) {
        const int cnt = min(32, re - x0);
        if (lane < cnt) {
            double t[D], tt = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                t[k] = (qc[k] - R.x[(size_t)(x0 + lane) * D + k]) * s;
                tt += t[k] * t[k];
            }
            const double e = (tt > 745.0 ? 0.0 : exp(-tt)) * (R.w ? R.w[x0 + lane] : 1.0);
            double H[D][PM];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                H[k][0] = 1.0;
#pragma unroll
                for (int b = 1; b < PM; ++b) {  // Hermite polynomials; orders >= p carry no term
                    const double hb = b == 1 ? 2.0 * t[k] : 2.0 * t[k] * H[k][b - 1] - 2.0 * (b - 1) * H[k][b - 2];
                    H[k][b] = hb;
                }
#pragma unroll
                for (int b = 1; b < PM; ++b)
                    if (b >= p) H[k][b] = 0.0;
            }
            double F[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                double v = e;
                int rem = f, st = NF;
#pragma unroll
                for (int k = 0; k + 1 < D; ++k) {
                    st /= PM;
                    v *= H[k][rem / st];
                    rem %= st;
                }
                F[f] = v;
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) Fx[lane * NFS + f] = F[f];
#pragma unroll
            for (int b = 0; b < PM; ++b) Bx[lane * PMS + b] = H[D - 1][b];
        }
        wave_sync();
        for (int b = lane; b < P; b += 64) {
            if ((mt[b] >> 8) >= p) continue;
            const int f = b / PM, l = b - f * PM;
            double sum = 0.0;
            for (int j = 0; j < cnt; ++j) sum = fma(Fx[j * NFS + f], Bx[j * PMS + l], sum);
            acc[b] += cb[b] * sum;
        }
        wave_sync();
    }
}

// One D or T op applied by one wave to the local moments acc[P] about qc; a D
// op covers reference points [rb, re) of node r.
// With GR the wave also accumulates the tangent moments accB[P] that carry the
// bandwidth derivative: with L' = dL/ds, accB_beta = s L'_beta + |beta| L_beta.
// (The translation and evaluation operators act on them exactly as on L, since
// s^{|beta|} accB_beta = s d(s^{|beta|} L_beta)/ds and s^{|beta|} L_beta are the
// coefficients of the same polynomial in unscaled coordinates.)  With
// h_n'(t) = -h_{n+1}(t):
//   D:  accB_beta += c_beta e^{-|t|^2} [|beta| prod_k H_{beta_k} - sum_k t_k H_{beta_k+1} prod_{j!=k} H_{beta_j}]
//   T:  accB_beta += c_beta e0 sum_alpha M_alpha [(|alpha|+|beta|) prod_k H_{alpha_k+beta_k}
//                                               - sum_k t0_k H_{alpha_k+beta_k+1} prod_{j!=k} H_{alpha_j+beta_j}]
// Wave-private scratch: Ms[P] | Ht[D][2 pmax] | T0[D] | Hx[64][D][pmax + GR] | Tx[64][D] (GR only).
template <bool GR>
__device__ void wave_local_op(const DevTree &R, int r, int p, int m, int rb, int re, const double *qc, double s,
                              int d, int pmax, int P, const unsigned long long *dg, const unsigned short *mt,
                              const double *cb, double *acc, double *accB, double *Ms, double *Ht, double *Hx,
                              int lane) {
    const int hs = pmax + (GR ? 1 : 0);  // Hermite row length per dimension
    double *T0 = Ht + 2 * d * pmax;
    double *Tx = Hx + 64 * (size_t)d * hs;
    if (m == METH_T) {
        double tt = 0.0;
        for (int k = 0; k < d; ++k) {
            const double t = (qc[k] - R.ctr[(size_t)r * d + k]) * s;
            tt += t * t;
        }
        if (tt > 745.0) return;  // e^{-|t0|^2} underflows: nothing to add
        const double e0 = exp(-tt);
        const double *mu = R.mu + (size_t)r * P;
        if (p == 1) {
            if (lane == 0) {
                acc[0] += mu[0] * e0;
                if (GR) accB[0] -= 2.0 * tt * mu[0] * e0;
            }
            return;
        }
        for (int i = lane; i < P; i += 64) {
            const int meta = mt[i];
            Ms[i] = (meta >> 8) < p ? mu[i] * powi(s, meta & 255) : 0.0;
        }
        if (lane < d) {
            const double t = (qc[lane] - R.ctr[(size_t)r * d + lane]) * s;
            hermite_polys(t, 2 * p - 1 + (GR ? 1 : 0), Ht + lane * 2 * pmax);
            T0[lane] = t;
        }
        wave_sync();
        for (int b = lane; b < P; b += 64) {
            if ((mt[b] >> 8) >= p) continue;
            const unsigned long long bd = dg[b];
            const int bs = mt[b] & 255;
            double sum = 0.0, sumB = 0.0;
            for (int a = 0; a < P; ++a) {
                if ((mt[a] >> 8) >= p) continue;
                const unsigned long long ad = dg[a];
                double pre = Ms[a], sk = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double *hk = Ht + k * 2 * pmax + dig_at(ad, k) + dig_at(bd, k);
                    if (GR) sk = sk * hk[0] + pre * T0[k] * hk[1];
                    pre *= hk[0];
                }
                sum += pre;
                if (GR) sumB += (double)((mt[a] & 255) + bs) * pre - sk;
            }
            acc[b] += cb[b] * e0 * sum;
            if (GR) accB[b] += cb[b] * e0 * sumB;
        }
        wave_sync();
        return;
    }
    if constexpr (!GR) {
        switch (direct_kind(d, pmax)) {
        case 1: direct_op<1, 6>(R, p, rb, re, qc, s, P, mt, cb, acc, Hx, lane); return;
        case 2: direct_op<2, 6>(R, p, rb, re, qc, s, P, mt, cb, acc, Hx, lane); return;
        case 3: direct_op<3, 4>(R, p, rb, re, qc, s, P, mt, cb, acc, Hx, lane); return;
        case 4: direct_op<4, 2>(R, p, rb, re, qc, s, P, mt, cb, acc, Hx, lane); return;
        case 5: direct_op<5, 2>(R, p, rb, re, qc, s, P, mt, cb, acc, Hx, lane); return;
        default: break;
        }
    }
    for (int x0 = rb; x0 < re; x0 += 64) {
        const int cnt = min(64, re - x0);
        if (lane < cnt) {
            double *row = Hx + (size_t)lane * d * hs;
            double tt = 0.0;
            for (int k = 0; k < d; ++k) {
                const double t = (qc[k] - R.x[(size_t)(x0 + lane) * d + k]) * s;
                tt += t * t;
                hermite_polys(t, p + (GR ? 1 : 0), row + k * hs);
                if (GR) Tx[lane * d + k] = t;
            }
            const double e = (tt > 745.0 ? 0.0 : exp(-tt)) * (R.w ? R.w[x0 + lane] : 1.0);
            for (int b = 0; b < p + (GR ? 1 : 0); ++b) row[b] *= e;  // the weighted exponential rides on dimension 0
        }
        wave_sync();
        for (int b = lane; b < P; b += 64) {
            if ((mt[b] >> 8) >= p) continue;
            const unsigned long long bd = dg[b];
            const double bs = (double)(mt[b] & 255);
            double sum = 0.0, sumB = 0.0;
            for (int j = 0; j < cnt; ++j) {
                const double *row = Hx + (size_t)j * d * hs;
                double pre = 1.0, sk = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double *hk = row + k * hs + dig_at(bd, k);
                    if (GR) sk = sk * hk[0] + pre * Tx[j * d + k] * hk[1];
                    pre *= hk[0];
                }
                sum += pre;
                if (GR) sumB += bs * pre - sk;
            }
            acc[b] += cb[b] * sum;
            if (GR) accB[b] += cb[b] * sumB;
        }
        wave_sync();
    }
}

// Doubles of wave-private scratch used by wave_local_op (acc and accB included).
__host__ __device__ inline size_t lop_wave_stride(int P, int d, int pmax, int gr) {
    return (size_t)(2 + gr) * P + 2 * (size_t)d * pmax + d + 64 * (size_t)d * (pmax + gr) + (gr ? 64 * (size_t)d : 0);
}

constexpr int kMaxSeg = 256;
constexpr int kMaxDepth = 256;  // deepest tree the per-leaf kernel walks

// Local ops run fully in parallel: one wave per op (a D op is one chunk of
// <= 64 reference points), each writing its contribution to Q's local
// moments into its own row of `part`; per-node sums then add the rows in
// chain order.  (Order-1 translations never reach here: the traversal adds
// their single term to the node's constant.)
// Rows hold PW = P (GR = false) or 2P doubles: L, then the tangent moments.
// LDS per block: cb[P] | dg[P] (u64) | mt[P] (u16) | per wave: lop_wave_stride doubles
template <bool GR>
__global__ __launch_bounds__(256) void k_lops(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                              const Op *__restrict__ lops, const int2 *__restrict__ lop_node,
                                              const int *__restrict__ cnt,
                                              const int *__restrict__ overflow, double *__restrict__ part) {
    extern __shared__ double smem[];
    if (*overflow) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const DevTree &Q0 = trees[jobs[0].qt];
    const int d = Q0.d, pmax = Q0.pmax, P = Q0.P;
    const size_t PW = GR ? 2 * (size_t)P : (size_t)P;
    double *cb = smem;
    unsigned long long *dg = reinterpret_cast<unsigned long long *>(cb + P);
    unsigned short *mt = reinterpret_cast<unsigned short *>(dg + P);
    double *wbase = cb + P + (10 * (size_t)P + 7) / 8 + (size_t)wv * lop_wave_stride(P, d, pmax, GR ? 1 : 0);
    double *acc = wbase, *accB = acc + P, *Ms = accB + (GR ? P : 0), *Ht = Ms + P;
    double *Hx = Ht + 2 * d * pmax + d;
    build_digit_tables(dg, mt, P, d, pmax);
    for (int i = tid; i < P; i += blockDim.x) cb[i] = coef_beta(i, d, pmax);
    __syncthreads();
    const int nops = min(cnt[C_LOP * CP], 0x7fffffff);
    const int step = gridDim.x * nwv;
    // each op's owner (node, job) comes with it, and the wave loads its next
    // op while it works on the current one
    int oi = blockIdx.x * nwv + wv;
    Op op{0, 0};
    int2 own{0, 0};
    if (oi < nops) {
        op = lops[oi];
        own = lop_node[oi];
    }
    for (; oi < nops; oi += step) {
        Op opn{0, 0};
        int2 ownn{0, 0};
        if (oi + step < nops) {
            opn = lops[oi + step];
            ownn = lop_node[oi + step];
        }
        const Job jb = jobs[own.y];
        const DevTree &Q = trees[jb.qt];
        const DevTree &R = trees[jb.rt];
        const int r = op.r, p = op.meta & 255, m = (op.meta >> 8) & 15, ch = op.meta >> 12;
        double *dst = part + (size_t)oi * PW;
        const double *qc = Q.ctr + (size_t)own.x * d;
        for (int i = lane; i < P; i += 64) {
            acc[i] = 0.0;
            if (GR) accB[i] = 0.0;
        }
        wave_sync();
        const int rb = R.begin[r] + 64 * ch, re = min(R.end[r], rb + 64);
        wave_local_op<GR>(R, r, p, m, rb, re, qc, jb.s, d, pmax, P, dg, mt, cb, acc, accB, Ms, Ht, Hx, lane);
        wave_sync();
        for (int i = lane; i < P; i += 64) {
            dst[i] = acc[i];
            if (GR) dst[P + i] = accB[i];
        }
        wave_sync();
        op = opn;
        own = ownn;
    }
}

// Adds the op rows (PW doubles, coefficient i of L at i and of the tangent at
// P + i) of one node's chain in chain order: acc += part[op].  Threads over
// the PW entries.
// Adds the partial rows of one local-op chain (every op of its groups, in
// chain order) to acc[PW], with the whole block.  Thread 0 flattens the chain
// into gs / gc (group starts, cumulative op counts; a chain has at most one
// group per level).  For PW <= the block size, G = blockDim / PW thread groups
// take ops g, g + G, ... four loads at a time, and their partials, red[G][PW],
// are added in group order: a fixed order, so the result is deterministic.
// Every thread of the block calls it; ns holds two ints.
__device__ void block_chain_parts(int head, const Group *__restrict__ lgrp, const double *__restrict__ part,
                                  int PW, double *acc, int *gs, int *gc, int *ns, double *red) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) {
        int n = 0, tot = 0;
        for (int gi = head; gi >= 0 && n < kMaxDepth; gi = lgrp[gi].next) {
            const Group g = lgrp[gi];
            gs[n] = g.start;
            tot += g.count;
            gc[n++] = tot;
        }
        ns[0] = n;
        ns[1] = tot;
    }
    __syncthreads();
    const int nops = ns[1];
    if (PW <= nthr) {
        const int G = nthr / PW, i = tid % PW, g = tid / PW;
        if (g < G) {
            double v = 0.0;
            int k = 0;
            for (int o0 = g; o0 < nops; o0 += 4 * G) {
                double t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int o = o0 + u * G;
                    t[u] = 0.0;
                    if (o < nops) {
                        while (o >= gc[k]) ++k;
                        t[u] = part[(size_t)(gs[k] + o - (k ? gc[k - 1] : 0)) * PW + i];
                    }
                }
                v += t[0];
                v += t[1];
                v += t[2];
                v += t[3];
            }
            red[g * PW + i] = v;
        }
        __syncthreads();
        if (tid < PW) {
            double sum = acc[tid];
            for (int gg = 0; gg < G; ++gg) sum += red[gg * PW + tid];
            acc[tid] = sum;
        }
    } else {
        const int ng = ns[0];
        for (int i = tid; i < PW; i += nthr) {
            double v = acc[i];
            for (int k = 0, o = 0; k < ng; ++k)
                for (; o < gc[k]; ++o) v += part[(size_t)(gs[k] + o - (k ? gc[k - 1] : 0)) * PW + i];
            acc[i] = v;
        }
    }
    __syncthreads();
}

// One block per internal (Q, job) with local ops; L rows hold PW doubles.
// Dynamic LDS: acc[PW] | red[256].
__global__ __launch_bounds__(256) void k_lreduce(const Job *__restrict__ jobs, const int *__restrict__ lnodes,
                                                 const int *__restrict__ cnt, const int *__restrict__ overflow,
                                                 const int *__restrict__ headL, const Group *__restrict__ lgrp,
                                                 const double *__restrict__ part, int PW, double *L,
                                                 unsigned char *lflag) {
    extern __shared__ double smem[];
    __shared__ int gs[kMaxDepth], gc[kMaxDepth], ns[2];
    if (*overflow) return;
    const int nl = cnt[C_LNODE * CP];
    double *acc = smem, *red = smem + PW;
    for (int li = blockIdx.x; li < nl; li += gridDim.x) {
        const int q = lnodes[2 * li], job = lnodes[2 * li + 1];
        const size_t hq = (size_t)jobs[job].noff + q;
        __syncthreads();  // the previous node's tables are no longer read
        for (int i = threadIdx.x; i < PW; i += blockDim.x) acc[i] = 0.0;
        __syncthreads();
        block_chain_parts(headL[hq], lgrp, part, PW, acc, gs, gc, ns, red);
        for (int i = threadIdx.x; i < PW; i += blockDim.x) L[hq * PW + i] = acc[i];
        if (threadIdx.x == 0) lflag[hq] = 1;
    }
}

__global__ void k_lop_owner(const Group *__restrict__ lgrp, const int *__restrict__ cnt,
                            const int *__restrict__ overflow, int2 *lop_node) {
    if (*overflow) return;
    const int ng = cnt[C_LGRP * CP];
    for (int gi = blockIdx.x; gi < ng; gi += gridDim.x) {
        const Group g = lgrp[gi];
        for (int o = threadIdx.x; o < g.count; o += blockDim.x) lop_node[g.start + o] = int2{g.q, g.job};
    }
}

// Large coefficient vectors (P > 1024): T through D one-dimensional mode
// products (block-wide, buffers in a global scratch slice), D and the order-1
// form as in k_local.  LDS: coef[pmax^2] | Ht[D][2 pmax] | Hx[64][D][pmax]
constexpr int kLocBlock = 256;

__global__ __launch_bounds__(kLocBlock) void k_local_big(const DevTree *__restrict__ trees,
                                                         const Job *__restrict__ jobs, const int *__restrict__ lnodes,
                                                         const int *__restrict__ cnt, const int *__restrict__ overflow,
                                                         const int *__restrict__ headL, const Group *__restrict__ grp,
                                                         const Op *__restrict__ lops, double *__restrict__ gscratch,
                                                         double *L, unsigned char *lflag) {
    extern __shared__ double smem[];
    if (*overflow) return;
    const int nl = cnt[C_LNODE * CP];
    for (int li = blockIdx.x; li < nl; li += gridDim.x) {
    __syncthreads();
    const int q = lnodes[2 * li], job = lnodes[2 * li + 1];
    const Job jb = jobs[job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int d = Q.d, pmax = Q.pmax, P = Q.P;
    const double s = jb.s;
    double *acc = gscratch + (size_t)blockIdx.x * 3 * P, *buf0 = acc + P, *buf1 = buf0 + P;  // one slice per block
    double *coef = smem, *Ht = coef + pmax * pmax, *Hx = Ht + 2 * d * pmax;
    const double *qc = Q.ctr + (size_t)q * d;
    for (int i = threadIdx.x; i < P; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    for (int gi = headL[(size_t)jb.noff + q]; gi >= 0; gi = grp[gi].next) {
        const Group g = grp[gi];
        for (int o = 0; o < g.count; ++o) {
            const Op op = lops[g.start + o];
            const int r = op.r, p = op.meta & 255, m = (op.meta >> 8) & 15, ch = op.meta >> 12;
            if (m == METH_T) {
                double tt = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double t = (qc[k] - R.ctr[(size_t)r * d + k]) * s;
                    tt += t * t;
                }
                if (tt > 745.0) continue;  // uniform across the block
                const double e0 = exp(-tt);
                const double *mu = R.mu + (size_t)r * P;
                if (p == 1) {
                    if (threadIdx.x == 0) acc[0] += mu[0] * e0;
                    __syncthreads();
                    continue;
                }
                for (int i = threadIdx.x; i < P; i += blockDim.x) {
                    bool inside;
                    const int as = digit_sum(i, d, pmax, p, &inside);
                    buf0[i] = inside ? mu[i] * powi(s, as) : 0.0;
                }
                for (int k = threadIdx.x; k < d; k += blockDim.x)
                    hermite_polys((qc[k] - R.ctr[(size_t)r * d + k]) * s, 2 * p - 1, Ht + k * 2 * pmax);
                __syncthreads();
                double *src = buf0, *dst = buf1;
                for (int k = 0; k < d; ++k) {
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
                    digit_sum(i, d, pmax, p, &inside);
                    if (inside) acc[i] += coef_beta(i, d, pmax) * e0 * src[i];
                }
                __syncthreads();
            } else {
                const int rb = R.begin[r] + 64 * ch, re = min(R.end[r], rb + 64);
                for (int x0 = rb; x0 < re; x0 += 64) {
                    const int cnt = min(64, re - x0);
                    if (threadIdx.x < cnt) {
                        double *row = Hx + (size_t)threadIdx.x * d * pmax;
                        double tt = 0.0;
                        for (int k = 0; k < d; ++k) {
                            const double t = (qc[k] - R.x[(size_t)(x0 + threadIdx.x) * d + k]) * s;
                            tt += t * t;
                            hermite_polys(t, p, row + k * pmax);
                        }
                        const double e =
                            (tt > 745.0 ? 0.0 : exp(-tt)) * (R.w ? R.w[x0 + threadIdx.x] : 1.0);
                        for (int b = 0; b < p; ++b) row[b] *= e;
                    }
                    __syncthreads();
                    for (int b = threadIdx.x; b < P; b += blockDim.x) {
                        // digits of b decoded once: offsets into each point's Hermite rows
                        int off[kMaxD];
                        bool inside = true;
                        for (int k = d - 1, bi = b; k >= 0; --k) {
                            const int dk = bi % pmax;
                            bi /= pmax;
                            inside = inside && dk < p;
                            off[k] = k * pmax + dk;
                        }
                        if (!inside) continue;
                        double sum = 0.0;
                        for (int j = 0; j < cnt; ++j) {
                            const double *row = Hx + (size_t)j * d * pmax;
                            double prod = row[off[d - 1]];
                            for (int k = d - 2; k >= 0; --k) prod *= row[off[k]];
                            sum += prod;
                        }
                        acc[b] += coef_beta(b, d, pmax) * sum;
                    }
                    __syncthreads();
                }
            }
        }
    }
    __syncthreads();
    double *Lq = L + ((size_t)jb.noff + q) * P;
    for (int i = threadIdx.x; i < P; i += blockDim.x) Lq[i] = acc[i];
    if (threadIdx.x == 0) lflag[jb.noff + q] = 1;
    }
}

// Flattened (job, query leaf) items: job k owns items [jlstart[k], jlstart[k+1]).
// unl > 0: every job has unl items (one query tree), no search needed.
__device__ __forceinline__ void job_leaf(const int *__restrict__ jlstart, int njobs, int unl, int item, int *job,
                                         int *li) {
    if (unl > 0) {
        *job = item / unl;
        *li = item - *job * unl;
        return;
    }
    int lo = 0, hi = njobs;  // jlstart[lo] <= item < jlstart[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jlstart[mid] <= item) lo = mid;
        else hi = mid;
    }
    *job = lo;
    *li = item - jlstart[lo];
}

// Digit tables of every coefficient position in global memory (for p_max^d
// too large for the per-leaf kernel's LDS); same layout as build_digit_tables.
__global__ void k_digits(unsigned long long *dg, unsigned short *mt, int P, int d, int pmax) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
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

// Level-0 frontier: one segment (Q root, {R root}) per job.
// Per-item record, computed once per call by k_items so that the per-item
// kernels read an item's job, query leaf and its point range with one load
// instead of a binary search over the job offsets.
struct __align__(16) ItemRec {
    int job, li, leaf, qb0;  // job, leaf rank in the query tree, leaf node, first point
    int nq, pad0, pad1, pad2;  // points of the leaf
};

__global__ __launch_bounds__(256) void k_items(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                               const int *__restrict__ jlstart, int njobs, int unl, int nitems,
                                               ItemRec *__restrict__ rec) {
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    ItemRec r;
    job_leaf(jlstart, njobs, unl, item, &r.job, &r.li);
    const DevTree &Q = trees[jobs[r.job].qt];
    r.leaf = Q.leaves[r.li];
    r.qb0 = Q.begin[r.leaf];
    r.nq = Q.end[r.leaf] - r.qb0;
    r.pad0 = r.pad1 = r.pad2 = 0;
    rec[item] = r;
}

__global__ void k_seed(Seg *__restrict__ segs, int *__restrict__ pairs, int njobs) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= njobs) return;
    segs[k] = Seg{0, k, k, 1, 0.0};
    pairs[k] = 0;
}

// Fill with a 32-bit pattern (used instead of memset nodes, so the whole
// launch sequence can be captured in a graph and replayed).
__global__ void k_fill_u32(unsigned *__restrict__ p, size_t n, unsigned v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- per query leaf
// One block per (job, query leaf).
//   1. Local moments at the leaf: every ancestor's own moments translated to
//      the leaf (TransLocalToLocal), then the leaf's own D / T ops from their
//      partial rows (chain order), and the path's constant terms.
//   2. Threads form ngr groups of `slots` lanes, one lane per query.  The F
//      chains of all path nodes are flattened into a segment table; ops are
//      processed in rounds, op = round * ngr + group, so groups sharing a
//      wave work in lock step:
//        F (EvalFarFieldExpansion): e^{-|t|^2} sum_{alpha<p} s^|alpha| mu_alpha prod_k H_{alpha_k}(t_k),
//           t = (q - R.c) s, Hermite polynomials in the lane's LDS rows.
//   3. Group partials are added in group order, the local expansion is
//      evaluated (EvalLocalExpansion) and G = G_L + G_F + G_E (G_E from the
//      exhaustive-tile kernels) is written in the caller's order.
// With GR the block also differentiates the same approximation (same ops,
// same orders) with respect to s = 1/(sqrt2 h) and the query point, per query:
//   X = s dG/ds  and  Y_k = (1/s) dG/dq_k,  written as dG/dh = -X/h, dG/dq_k = s Y_k:
//   E:  X += -2 sum_r t_r e_r,   Y_k += -2 sum_r e_r (s(q - r))_k     (t_r = s^2 |q - r|^2),
//       accumulated by the exhaustive-tile kernels
//   F:  with V_k = -sum_alpha M_alpha h_{alpha + e_k}(t):  Y_k += V_k,
//       X += sum_alpha |alpha| M_alpha h_alpha(t) + sum_k t_k V_k
//   L:  X += sum_beta B_beta y^beta (B the tangent moments), Y_k += sum_beta L_beta beta_k y^{beta - e_k}
// ln 2 and sqrt(ln 2): mixed-precision tiles work in sig = sqrt(log2 e) s units.
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kSqrtLn2 = 0.83255461115769775635;

// Far-field evaluation (EvalFarField, eq. primal) at one query for a
// dimension and p_max fixed at compile time: the Hermite rows stay in
// registers with s^a folded in (M_alpha h_alpha = mu_alpha prod_k s^{a_k}
// H_{a_k}(t_k) e^{-|t|^2}), and the sum over the p^D coefficients of order < p
// is taken one axis at a time, last axis innermost (the storage order), so a
// coefficient costs one FMA.  Returns the polynomial part; *tt = |t|^2.
// U: mu is wave-uniform (one op per wave) and read with scalar loads.
template <int D, int PM, int K, bool U = false>
struct FarAxis {
    __device__ __forceinline__ static double run(const double *__restrict__ mu, const double (&hs)[D][PM], int p,
                                                 int off) {
        double acc = 0.0;
#pragma unroll
        for (int a = PM - 1; a >= 0; --a)
            if (a < p) acc = fma(hs[K][a], FarAxis<D, PM, K + 1, U>::run(mu, hs, p, off * PM + a), acc);
        return acc;
    }
};
template <int D, int PM, bool U>
struct FarAxis<D, PM, D, U> {
    __device__ __forceinline__ static double run(const double *__restrict__ mu, const double (&)[D][PM], int,
                                                 int off) {
        if constexpr (U) return ldc(mu + off);
        else return mu[off];
    }
};

template <int D, int PM, bool U = false>
__device__ __forceinline__ double far_eval_fixed(const double *__restrict__ mu, const double *__restrict__ rc,
                                                 const double *__restrict__ q, double s, int p, double *tt) {
    double hs[D][PM];
    double t2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double t = (q[k] - (U ? ldc(rc + k) : rc[k])) * s;
        t2 += t * t;
        double h0 = 1.0, h1 = 2.0 * t, sp = s;
        hs[k][0] = 1.0;
        if (PM > 1) hs[k][1] = h1 * s;
#pragma unroll
        for (int a = 1; a + 1 < PM; ++a) {
            const double h2 = 2.0 * t * h1 - 2.0 * a * h0;
            h0 = h1;
            h1 = h2;
            sp *= s;
            hs[k][a + 1] = h2 * sp;  // sp = s^{a+1}
        }
    }
    *tt = t2;
    return FarAxis<D, PM, 0, U>::run(mu, hs, p, 0);
}

// sum over alpha in [0, p)^D of mu[alpha] prod_k Hs[k][alpha_k], for a
// dimension D fixed at compile time and a runtime p_max (<= 16, the radix of
// the storage order) and p <= p_max.  Far-field evaluation (EvalFarField, eq.
// primal): mu the op's moments, Hs the lane's Hermite rows with s^a folded
// in, p the op's order.  Local-expansion evaluation (EvalLocalExpansion): mu
// the leaf's local moments, Hs the lane's power rows, p = p_max.  The
// coefficients are visited in storage order (axis D - 1 fastest) by an
// odometer over axes 0 .. D - 2 that keeps the products of their row values
// as prefix products, so a coefficient costs one FMA; the generic loop visits
// all p_max^D positions with D LDS reads and products each.  Rows: axis k at
// Hs + k hs.
// SC: mu is read with scalar loads (an op the whole wave evaluates, moments
// no kernel writes meanwhile); otherwise with ordinary loads (the block's
// own local moments).
template <int D, bool SC = true>
__device__ __forceinline__ double far_eval_odometer(const double *__restrict__ mu, const double *Hs, int hs,
                                                    int pmax, int p) {
    const double *hl = Hs + (D - 1) * hs;  // the last axis' values
    int al[D > 1 ? D - 1 : 1], st[D > 1 ? D - 1 : 1];
    double pre[D > 1 ? D - 1 : 1];  // pre[k] = prod_{j <= k} Hs[j][al[j]]
    int stride = pmax;
#pragma unroll
    for (int k = D - 2; k >= 0; --k) {
        st[k] = stride;
        stride *= pmax;
    }
    double pr = 1.0;
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
        al[k] = 0;
        pr *= Hs[k * hs];
        pre[k] = pr;
    }
    int i = 0;
    double w = 0.0;
    for (;;) {
        double inner = 0.0;
        for (int a = 0; a < p; ++a) inner = fma(SC ? ldc(mu + i + a) : mu[i + a], hl[a], inner);
        w = D > 1 ? fma(pre[D > 1 ? D - 2 : 0], inner, w) : inner;
        // next position: the fastest of axes D - 2 .. 0 that can still advance
        // does, and the faster ones return to 0
        int kpos = -1;
#pragma unroll
        for (int k = D - 2; k >= 0; --k) {
            if (kpos < 0) {
                if (al[k] + 1 < p) {
                    ++al[k];
                    i += st[k];
                    kpos = k;
                } else {
                    i -= al[k] * st[k];
                    al[k] = 0;
                }
            }
        }
        if (kpos < 0) break;
#pragma unroll
        for (int k = 0; k < D - 1; ++k)
            if (k >= kpos) pre[k] = (k ? pre[k > 0 ? k - 1 : 0] : 1.0) * Hs[k * hs + al[k]];
    }
    return w;
}

// Local-expansion evaluation (EvalLocalExpansion) at one query for the same
// (D, p_max): sum_beta L_beta y^beta, y = (q - c) s, with the powers in
// registers and the same axis-wise contraction (every coefficient: order p_max).
template <int D, int PM>
__device__ __forceinline__ double local_eval_fixed(const double *L, const double *__restrict__ q,
                                                   const double *__restrict__ c, double s) {
    double yp[D][PM];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double y = (q[k] - c[k]) * s;
        double v = 1.0;
#pragma unroll
        for (int a = 0; a < PM; ++a) {
            yp[k][a] = v;
            v *= y;
        }
    }
    return FarAxis<D, PM, 0>::run(L, yp, PM, 0);
}

// (D, p_max) pairs with a compile-time far-field evaluation (the default p_max
// of D = 1..5); 0 = none.
__host__ __device__ inline int far_fixed_kind(int d, int pmax) {
    if (d == 1 && pmax == 6) return 1;
    if (d == 2 && pmax == 6) return 2;
    if (d == 3 && pmax == 4) return 3;
    if (d == 4 && pmax == 2) return 4;
    if (d == 5 && pmax == 2) return 5;
    return 0;
}

// Doubles of dynamic LDS k_leaf needs before the coefficient vectors; rows =
// 0 drops the per-thread Hermite rows (the compile-time (D, p_max) forms
// without gradients keep them in registers).
__host__ __device__ inline size_t leaf_lds_base(int nthr, int d, int pmax, int gr, int rows) {
    return (size_t)nthr * (1 + gr) + (size_t)d * (pmax - 1) + 1 + (size_t)rows * nthr * d * (pmax + gr) +
           (size_t)nthr * d * gr;
}

// GEN: the form for value sums at a (D, p_max) without a compile-time
// far-field evaluation (far_fixed_kind 0); its odometer evaluation would
// raise the register count of the other forms.
template <bool GR, bool GEN = false>
__global__ __launch_bounds__(256) void k_leaf(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                              const Group *__restrict__ egrp, const int *__restrict__ eops,
                                              const Group *__restrict__ fgrp, const Op *__restrict__ fops,
                                              const Group *__restrict__ lgrp, const Op *__restrict__ lops,
                                              const int *__restrict__ headE, const int *__restrict__ headF,
                                              const int *__restrict__ headL, const double *__restrict__ L,
                                              const unsigned char *__restrict__ lflag, int precision, int acc_in_lds,
                                              int leaf_local, const int *__restrict__ overflow,
                                              const double *__restrict__ part, double *__restrict__ gscratch,
                                              double *__restrict__ stG, double *__restrict__ stX,
                                              double *__restrict__ stQ, const double *__restrict__ cval,
                                              const ItemRec *__restrict__ irec,
                                              const unsigned long long *__restrict__ gdg,
                                              const unsigned short *__restrict__ gmt,
                                              const unsigned char *__restrict__ selfE,
                                              const double *__restrict__ selfG, const double *__restrict__ selfX,
                                              const double *__restrict__ selfY) {
    extern __shared__ double smem[];
    if (*overflow) return;
    __shared__ double cs_s;
    __shared__ int path[kMaxDepth];
    __shared__ double cvl[kMaxDepth];
    __shared__ unsigned char lfl[kMaxDepth];
    __shared__ int segT[kMaxSeg], segS[kMaxSeg], segE[kMaxSeg], ccnt[kMaxDepth + 1];
    __shared__ int nsg_s, nops_s, ntot_s, nops1_s, st_phase, st_gi, st_pi;
    const ItemRec ir = irec[blockIdx.x];
    const int job = ir.job, li = ir.li;
    const Job jb = jobs[job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int leaf = ir.leaf;
    const int d = Q.d, pmax = Q.pmax, P = Q.P;
    const int PW = GR ? 2 * P : P;
    const int hs = pmax + (GR ? 1 : 0);
    const int nthr = blockDim.x, tid = threadIdx.x;
    const double s = jb.s;
    const int ns = d * (pmax - 1) + 1;
    const size_t hq = (size_t)jb.noff + leaf;
    // LDS: red[nthr] | redX[nthr] (GR) | spow[ns] | Hq[nthr][D][hs] (not with fixed) | gq[nthr][D] (GR)
    //      | acc[PW] | tmp[PW] | tmp2[PW] | coef[D][pmax^2] | dg[P] (u64) | mt[P] (u16)
    //      (acc / tmp / tmp2 in a global scratch slice when P is large)
    // fixed: far-field and local evaluation in registers (no Hermite rows)
    static_assert(!(GR && GEN), "the general far-field form is for value sums");
    const int fixed = GR || GEN ? 0 : far_fixed_kind(d, pmax);
    double *red = smem;
    double *redX = red + nthr;
    double *spow = redX + (GR ? nthr : 0);
    double *Hq_all = spow + ns;
    double *Hq = Hq_all + (size_t)tid * d * hs;
    double *gq_all = Hq_all + (fixed ? 0 : (size_t)nthr * d * hs);
    double *gq = gq_all + (size_t)tid * d;
    double *tail = gq_all + (GR ? (size_t)nthr * d : 0);
    double *acc, *tmp, *tmp2, *coef;
    if (acc_in_lds) {
        acc = tail;
        tmp = acc + PW;
        tmp2 = tmp + PW;
        coef = tmp2 + PW;
    } else {
        acc = gscratch + (size_t)blockIdx.x * 3 * PW;
        tmp = acc + PW;
        tmp2 = tmp + PW;
        coef = tail;
    }
    // digit tables: in LDS, or (large P) prepared in global memory by k_digits
    const unsigned long long *dg = gdg;
    const unsigned short *mt = gmt;
    if (!gdg) {
        unsigned long long *ldg = reinterpret_cast<unsigned long long *>(coef + d * pmax * pmax);
        unsigned short *lmt = reinterpret_cast<unsigned short *>(ldg + P);
        build_digit_tables(ldg, lmt, P, d, pmax);
        dg = ldg;
        mt = lmt;
    }
    // root path (precomputed with the tree: path[0] = the leaf, path[plen-1] = the root)
    const int plen = Q.lplen[li];
    int mine = 0;
    for (int k = tid; k < plen; k += nthr) {
        const int v = Q.lpath[(size_t)li * Q.depth + k];
        path[k] = v;
        lfl[k] = lflag[jb.noff + v];
        cvl[k] = cval[jb.noff + v];
        mine |= lfl[k];
    }
    for (int i = tid; i < ns; i += nthr) spow[i] = powi(s, i);
    const int anyl = __syncthreads_or(mine);
    // constant local terms (order-1 translations) of the path nodes, root first:
    // translating a constant expansion leaves it unchanged
    if (tid == 0) {
        double c = 0.0;
        for (int k = plen - 1; k >= 0; --k) c += cvl[k];
        cs_s = c;
    }
    __syncthreads();
    const double csum = cs_s;
    const int qb = Q.begin[leaf], nq = Q.end[leaf] - qb;
    // 1. local moments at the leaf: the moments of every ancestor v that has
    //    any, translated straight to the leaf centre (TransLocalToLocal; the
    //    translation of a polynomial is exact, so one step v -> leaf equals the
    //    chain of parent -> child steps), added root first; each translation is
    //    D one-axis mode products, child L_a = sum_{b >= a} C(b, a) L_b X^{b-a},
    //    X = (leaf.c - v.c) s
    const bool any = anyl != 0 || (leaf_local && headL[hq] >= 0);
    if (any) {
        for (int i = tid; i < PW; i += nthr) acc[i] = 0.0;
        for (int pi = plen - 1; pi >= 0; --pi) {
            if (!lfl[pi]) continue;  // uniform: LDS flag
            const int v = path[pi];
            const double *Lv = L + ((size_t)jb.noff + v) * PW;
            if (pi == 0) {  // the leaf's own moments: no translation
                for (int i = tid; i < PW; i += nthr) acc[i] += Lv[i];
                __syncthreads();
                continue;
            }
            for (int i = tid; i < d * pmax * pmax; i += nthr) {
                const int k = i / (pmax * pmax), a = (i / pmax) % pmax, b = i % pmax;
                const double X = (Q.ctr[(size_t)leaf * d + k] - Q.ctr[(size_t)v * d + k]) * s;
                double c = 0.0;
                if (b >= a) {
                    c = 1.0;
                    for (int t = 0; t < b - a; ++t) c *= X * (double)(b - t) / (double)(b - a - t);
                }
                coef[i] = c;
            }
            for (int i = tid; i < PW; i += nthr) tmp[i] = Lv[i];
            __syncthreads();
            double *src = tmp, *dst = tmp2;
            for (int k = 0; k < d; ++k) {
                mode_product(src, dst, coef + k * pmax * pmax, P, d, pmax, k, pmax);
                if (GR) mode_product(src + P, dst + P, coef + k * pmax * pmax, P, d, pmax, k, pmax);
                __syncthreads();
                double *t2 = src;
                src = dst;
                dst = t2;
            }
            for (int i = tid; i < PW; i += nthr) acc[i] += src[i];
            __syncthreads();
        }
        if (leaf_local && headL[hq] >= 0) {  // the leaf's own local ops, from their partial rows
            __syncthreads();
            // the segment tables and the partial-sum rows are free until part 2
            block_chain_parts(headL[hq], lgrp, part, PW, acc, segS, segE, ccnt, red);
        }
    }
    // 2. exhaustive and far-field parts
    int slots = 1;
    while (slots < nq && slots < nthr) slots <<= 1;
    const int ngr = nthr / slots;
    const int qi = tid % slots, tg = tid / slots;
    const double *lc = Q.ctr + (size_t)leaf * d;
    // op groups: the leaf's E chain, then the F chains of the path nodes from
    // the root down, each chain in its own order.  One thread per chain counts
    // and then copies its groups; if more than kMaxSeg groups result they are
    // flattened serially in batches instead.
    // One walk: chain ch records its groups in its own region of the segment
    // tables (kMaxSeg / (plen + 1) entries) while they fit; the regions are
    // then packed in chain order.  A chain longer than its region sends the
    // block down the two-walk path (count, then copy) below.
    const int rsz = kMaxSeg / (plen + 1);
    int longch = 0;
    for (int ch = tid; ch <= plen; ch += nthr) {
        int c = 0;
        if (ch > 0) {  // chain 0 (exhaustive sums) comes from k_etile / k_emfma
            for (int gi = headF[(size_t)jb.noff + path[plen - ch]]; gi >= 0;) {
                const Group g = fgrp[gi];
                if (c < rsz) {
                    segS[ch * rsz + c] = g.start;
                    segE[ch * rsz + c] = g.count;
                }
                ++c;
                gi = g.next;
            }
        }
        ccnt[ch] = c;
        longch |= c > rsz ? 1 : 0;
    }
    const bool packed = !__syncthreads_or(longch);
    if (tid == 0) {
        int t = 0;
        for (int k = 0; k <= plen; ++k) {
            const int c = ccnt[k];
            if (packed)
                for (int j = 0; j < c; ++j) {  // forward in-place packing: t <= k * rsz + j
                    segT[t + j] = 1;
                    segS[t + j] = segS[k * rsz + j];
                    segE[t + j] = segE[k * rsz + j];
                }
            ccnt[k] = t;
            t += c;
        }
        if (packed) {
            int cum = 0;
            for (int k = 0; k < t; ++k) {
                cum += segE[k];
                segE[k] = cum;
            }
            nops1_s = cum;
        }
        ntot_s = t;
    }
    __syncthreads();
    const bool single = ntot_s <= kMaxSeg;
    if (single && !packed) {
        for (int ch = tid; ch <= plen; ch += nthr) {
            int o = ccnt[ch];
            if (ch == 0) {
                // no E chain: exhaustive sums come from k_etile / k_emfma
            } else {
                for (int gi = headF[(size_t)jb.noff + path[plen - ch]]; gi >= 0;) {
                    const Group g = fgrp[gi];
                    segT[o] = 1;
                    segS[o] = g.start;
                    segE[o++] = g.count;
                    gi = g.next;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int k = 0; k < ntot_s; ++k) {
                t += segE[k];
                segE[k] = t;
            }
            nops1_s = t;
        }
        __syncthreads();
    }
    for (int q0 = 0; q0 < nq; q0 += slots) {
        const int qq = q0 + qi;
        const bool act = qq < nq;
        const int qpos = qb + (act ? qq : 0);
        const double *qg = Q.x + (size_t)qpos * d;
        double part = 0.0, px = 0.0;
        if (GR)
            for (int k = 0; k < d; ++k) gq[k] = 0.0;
        if (tid == 0) {
            st_phase = 0;
            st_gi = -1;  // exhaustive sums come from k_etile / k_emfma
            st_pi = plen - 1;
        }
        __syncthreads();
        for (int round = 0;; ++round) {
            if (single && round > 0) break;
            if (!single && tid == 0) {
                // flatten the next batch of op groups: the leaf's E chain, then
                // the F chains of the path nodes from the root down
                int n = 0, tot = 0, ph = st_phase, gi = st_gi, pi = st_pi;
                while (n < kMaxSeg) {
                    if (ph == 0) {
                        if (gi < 0) {
                            ph = 1;
                            gi = pi >= 0 ? headF[(size_t)jb.noff + path[pi]] : -1;
                            continue;
                        }
                        const Group g = egrp[gi];
                        segT[n] = g.flags ? 2 : 0;
                        segS[n] = g.start;
                        tot += g.count;
                        segE[n++] = tot;
                        gi = g.next;
                    } else {
                        if (gi < 0) {
                            if (--pi < 0) break;
                            gi = headF[(size_t)jb.noff + path[pi]];
                            continue;
                        }
                        const Group g = fgrp[gi];
                        segT[n] = 1;
                        segS[n] = g.start;
                        tot += g.count;
                        segE[n++] = tot;
                        gi = g.next;
                    }
                }
                st_phase = ph;
                st_gi = gi;
                st_pi = pi;
                nsg_s = n;
                nops_s = tot;
            }
            __syncthreads();
            const int nops = single ? nops1_s : nops_s;
            if (!single && nsg_s == 0) break;
            int sp = 0;
            for (int base = 0; base < nops; base += ngr) {
                const int idx = base + tg;
                if (idx >= nops) continue;
                while (idx >= segE[sp]) ++sp;
                const int off = idx - (sp ? segE[sp - 1] : 0);
                const int type = segT[sp];
                if (fixed && slots >= 64) {  // one op per wave: its moments by scalar loads
                    const long long ov =
                        ldc(reinterpret_cast<const long long *>(fops) + __builtin_amdgcn_readfirstlane(segS[sp] + off));
                    const int r = (int)ov, p = (int)(ov >> 32) & 255;  // Op {r, meta}
                    const double *mu = uniform_ptr(R.mu) + (size_t)r * P;
                    const double *rc = uniform_ptr(R.ctr) + (size_t)r * d;
                    double tt = 0.0, w = 0.0;
                    switch (fixed) {
                    case 1: w = far_eval_fixed<1, 6, true>(mu, rc, qg, s, p, &tt); break;
                    case 2: w = far_eval_fixed<2, 6, true>(mu, rc, qg, s, p, &tt); break;
                    case 3: w = far_eval_fixed<3, 4, true>(mu, rc, qg, s, p, &tt); break;
                    case 4: w = far_eval_fixed<4, 2, true>(mu, rc, qg, s, p, &tt); break;
                    default: w = far_eval_fixed<5, 2, true>(mu, rc, qg, s, p, &tt); break;
                    }
                    if (act && tt <= 745.0) part = fma(exp(-tt), w, part);
                } else if (act && fixed) {  // far-field evaluation, registers only
                    const Op op = fops[segS[sp] + off];
                    const int r = op.r, p = op.meta & 255;
                    const double *mu = R.mu + (size_t)r * P;
                    const double *rc = R.ctr + (size_t)r * d;
                    double tt = 0.0, w = 0.0;
                    switch (fixed) {
                    case 1: w = far_eval_fixed<1, 6>(mu, rc, qg, s, p, &tt); break;
                    case 2: w = far_eval_fixed<2, 6>(mu, rc, qg, s, p, &tt); break;
                    case 3: w = far_eval_fixed<3, 4>(mu, rc, qg, s, p, &tt); break;
                    case 4: w = far_eval_fixed<4, 2>(mu, rc, qg, s, p, &tt); break;
                    default: w = far_eval_fixed<5, 2>(mu, rc, qg, s, p, &tt); break;
                    }
                    if (tt <= 745.0) part = fma(exp(-tt), w, part);
                } else if (GEN && slots >= 64) {  // one op per wave, general (D, p_max): moments by scalar loads
                    const long long ov =
                        ldc(reinterpret_cast<const long long *>(fops) + __builtin_amdgcn_readfirstlane(segS[sp] + off));
                    const int r = (int)ov, p = (int)(ov >> 32) & 255;  // Op {r, meta}
                    const double *mu = uniform_ptr(R.mu) + (size_t)r * P;
                    const double *rc = uniform_ptr(R.ctr) + (size_t)r * d;
                    double tt = 0.0;
                    for (int k = 0; k < d; ++k) {
                        const double t = (qg[k] - ldc(rc + k)) * s;
                        tt += t * t;
                        hermite_polys(t, p, Hq + k * hs);
                        for (int a = 1; a < p; ++a) Hq[k * hs + a] *= spow[a];  // s^a folded in
                    }
                    double w = 0.0;
                    switch (d) {
                    case 2: w = far_eval_odometer<2>(mu, Hq, hs, pmax, p); break;
                    case 3: w = far_eval_odometer<3>(mu, Hq, hs, pmax, p); break;
                    case 4: w = far_eval_odometer<4>(mu, Hq, hs, pmax, p); break;
                    case 5: w = far_eval_odometer<5>(mu, Hq, hs, pmax, p); break;
                    case 6: w = far_eval_odometer<6>(mu, Hq, hs, pmax, p); break;
                    case 7: w = far_eval_odometer<7>(mu, Hq, hs, pmax, p); break;
                    case 8: w = far_eval_odometer<8>(mu, Hq, hs, pmax, p); break;
                    default:  // every position with D LDS reads and products
                        for (int i = 0; i < P; ++i) {
                            const int meta = mt[i];
                            if ((meta >> 8) >= p) continue;
                            const unsigned long long ad = dg[i];
                            double prod = ldc(mu + i);
                            for (int k = 0; k < d; ++k) prod *= Hq[k * hs + dig_at(ad, k)];
                            w += prod;
                        }
                    }
                    if (act && tt <= 745.0) part = fma(exp(-tt), w, part);
                } else if (act) {  // every op here is a far-field evaluation
                    const Op op = fops[segS[sp] + off];
                    const int r = op.r, p = op.meta & 255;
                    const double *mu = R.mu + (size_t)r * P;
                    const double *rc = R.ctr + (size_t)r * d;
                    double tt = 0.0;
                    for (int k = 0; k < d; ++k) {
                        const double t = (qg[k] - rc[k]) * s;
                        tt += t * t;
                        hermite_polys(t, p + (GR ? 1 : 0), Hq + k * hs);
                    }
                    if (tt <= 745.0) {  // else e^{-|t|^2} underflows: the expansion is 0
                        double w = 0.0, w1 = 0.0;
                        for (int i = 0; i < P; ++i) {
                            const int meta = mt[i];
                            if ((meta >> 8) >= p) continue;
                            const unsigned long long ad = dg[i];
                            double prod = mu[i] * spow[meta & 255];
                            for (int k = 0; k < d; ++k) prod *= Hq[k * hs + dig_at(ad, k)];
                            w += prod;
                            if (GR) w1 = fma((double)(meta & 255), prod, w1);
                        }
                        const double e = exp(-tt);
                        part = fma(e, w, part);
                        if (GR) {
                            double xs_ = w1;
                            for (int k = 0; k < d; ++k) {
                                double vk = 0.0;
                                for (int i = 0; i < P; ++i) {
                                    const int meta = mt[i];
                                    if ((meta >> 8) >= p) continue;
                                    const unsigned long long ad = dg[i];
                                    double prod = mu[i] * spow[meta & 255];
                                    for (int j = 0; j < d; ++j) prod *= Hq[j * hs + dig_at(ad, j) + (j == k ? 1 : 0)];
                                    vk -= prod;
                                }
                                gq[k] = fma(e, vk, gq[k]);
                                xs_ = fma((qg[k] - rc[k]) * s, vk, xs_);
                            }
                            px = fma(e, xs_, px);
                        }
                    }
                }
            }
            __syncthreads();
        }
        red[tid] = part;
        if (GR) redX[tid] = px;
        __syncthreads();
        if (tg == 0 && act) {
            double gsum = 0.0, xsum = 0.0;
            for (int k = 0; k < ngr; ++k) gsum += red[k * slots + qi];
            if (GR) {
                for (int k = 0; k < ngr; ++k) xsum += redX[k * slots + qi];
                for (int k = 1; k < ngr; ++k)
                    for (int c = 0; c < d; ++c) gq[c] += gq_all[(size_t)(k * slots + qi) * d + c];
            }
            double gl = 0.0, xl = 0.0;
            if (any && fixed) {
                switch (fixed) {
                case 1: gl = local_eval_fixed<1, 6>(acc, qg, lc, s); break;
                case 2: gl = local_eval_fixed<2, 6>(acc, qg, lc, s); break;
                case 3: gl = local_eval_fixed<3, 4>(acc, qg, lc, s); break;
                case 4: gl = local_eval_fixed<4, 2>(acc, qg, lc, s); break;
                default: gl = local_eval_fixed<5, 2>(acc, qg, lc, s); break;
                }
            } else if (any) {
                // powers y_k^b (b < p_max) of the scaled offset from the leaf centre,
                // in this thread's Hermite rows (free here), the same products as powi
                double *yp = Hq;
                for (int k = 0; k < d; ++k) {
                    const double yk = (qg[k] - lc[k]) * s;
                    double v = 1.0;
                    for (int b = 0; b < pmax; ++b) {
                        yp[k * hs + b] = v;
                        v *= yk;
                    }
                }
                // the GEN form (value sums, D <= 8): every coefficient by the
                // odometer, one FMA each (the same polynomial, summed in
                // storage order)
                if (GEN && d >= 2 && d <= 8) {
                    switch (d) {
                    case 2: gl = far_eval_odometer<2, false>(acc, yp, hs, pmax, pmax); break;
                    case 3: gl = far_eval_odometer<3, false>(acc, yp, hs, pmax, pmax); break;
                    case 4: gl = far_eval_odometer<4, false>(acc, yp, hs, pmax, pmax); break;
                    case 5: gl = far_eval_odometer<5, false>(acc, yp, hs, pmax, pmax); break;
                    case 6: gl = far_eval_odometer<6, false>(acc, yp, hs, pmax, pmax); break;
                    case 7: gl = far_eval_odometer<7, false>(acc, yp, hs, pmax, pmax); break;
                    default: gl = far_eval_odometer<8, false>(acc, yp, hs, pmax, pmax); break;
                    }
                }
                for (int i = 0; i < P && !(GEN && d >= 2 && d <= 8); ++i) {
                    const double a = acc[i];
                    const double aB = GR ? acc[P + i] : 0.0;
                    if (a == 0.0 && aB == 0.0) continue;
                    const unsigned long long ad = dg[i];
                    double prod = a, prodB = aB;
                    for (int k = 0; k < d; ++k) {
                        const double yk = yp[k * hs + dig_at(ad, k)];
                        prod *= yk;
                        if (GR) prodB *= yk;
                    }
                    gl += prod;
                    if (GR) {
                        xl += prodB;
                        if (a != 0.0)
                            for (int c = 0; c < d; ++c) {
                                const int bc = dig_at(ad, c);
                                if (bc == 0) continue;
                                double dv = a * (double)bc;
                                for (int k = 0; k < d; ++k) dv *= yp[k * hs + dig_at(ad, k) - (k == c ? 1 : 0)];
                                gq[c] += dv;
                            }
                    }
                }
            }
            // everything but the exhaustive sums; k_leaf_finish adds those once
            // the tiles' stream has joined, and writes the caller's outputs
            const size_t ei = (size_t)jb.qoff + qpos;
            // leave-one-out: the leaf's exhaustive pair with itself (from k_selfpre)
            const bool self = selfE && selfE[hq];
            stG[ei] = (gl + csum) + gsum + (self ? selfG[ei] : 0.0);
            if (GR) {
                stX[ei] = xl + xsum + (self ? selfX[ei] : 0.0);
                for (int c = 0; c < d; ++c) stQ[ei * d + c] = gq[c] + (self ? selfY[ei * d + c] : 0.0);
            }
        }
        __syncthreads();
    }
}

// The outputs of every (job, query): k_leaf's partial sums plus the
// exhaustive leaf-leaf sums (G, and in gradient mode the dG/dh and dG/dq
// parts), scaled back by the job's weight scale, in the caller's order.
// k_leaf runs on the main stream beside the exhaustive tiles on the side
// stream (when the tiles take longer than the local moments, k_leaf fills the
// idle compute units); this pass waits for both.  One thread per query slot;
// its job is found by bisection on the slot offsets.
template <bool GR>
__global__ __launch_bounds__(256) void k_leaf_finish(const DevTree *__restrict__ trees,
                                                     const Job *__restrict__ jobs, int njobs, long long nqa,
                                                     const int *__restrict__ overflow,
                                                     const double *__restrict__ stG, const double *__restrict__ stX,
                                                     const double *__restrict__ stQ, const double *__restrict__ extE,
                                                     const double *__restrict__ extX,
                                                     const double *__restrict__ extY, int *__restrict__ sticky) {
    if (*overflow) {
        // a batch of several parts clears the flag per part: the sticky word
        // keeps whether any part overflowed
        if (blockIdx.x == 0 && threadIdx.x == 0) *sticky = 1;
        return;
    }
    const long long ei = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ei >= nqa) return;
    int lo = 0, hi = njobs;  // jobs[lo].qoff <= ei < jobs[hi].qoff
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (jobs[mid].qoff <= ei) lo = mid;
        else hi = mid;
    }
    const Job &jb = jobs[lo];
    const DevTree &Q = trees[jb.qt];
    const int qpos = (int)(ei - jb.qoff);
    const int dst = Q.perm[qpos];
    const double ws = jb.wscale;
    jb.out[dst] = (stG[ei] + extE[ei]) * ws;
    if (GR) {
        const int d = Q.d;
        if (jb.outH) jb.outH[dst] = -(stX[ei] + extX[ei]) / jb.h * ws;
        if (jb.outQ)
            for (int c = 0; c < d; ++c)
                jb.outQ[(size_t)dst * d + c] = jb.s * (stQ[ei * d + c] + extY[ei * d + c]) * ws;
    }
}

constexpr int kEChunk = 256;   // E ops flattened per chunk
constexpr int kMaxEGrp = 256;  // E groups of one (job, node) chain (at most one per level)

constexpr int kEHeavyOps = 64; // an item with at least this many E ops (mixed pass) is dispatched first

// Matrix-core exhaustive tiles (k_etile_mx*, below): block shape and the
// query-leaf and reference radii (sig units) of their two product precisions.
constexpr int kMxWaves = 4;
constexpr int kMxOps = 64 * kMxWaves;  // E ops flattened per chunk: one per thread
constexpr int kMxQ = 64 * kMxWaves;    // queries held per pass over the chain (4 blocks per wave)
constexpr int kMxSeg = 1024;           // 64-point segments of a chunk with a table entry
constexpr double kMxWideQ = 4096.0;    // 2^12
constexpr double kMxNear32 = 12.0;     // staging window when G has no lower bound (t >= 144 left out)

// Dispatch order of the mixed pass's exhaustive tiles (longest first): the
// items whose E chain holds >= kEHeavyOps ops of the mixed pass, then those
// with fewer, then those with none.  A leaf with hundreds of reference leaves
// keeps one block busy ~100 us; started in job order, such blocks began
// midway through the launch and set its end.  lists holds six lists of
// nitems entries: [0] heavy, [1] short, [2] none, and with mx (the
// matrix-core pass) [3] items whose query leaf's half-diagonal exceeds
// kMxWideQ in sig units (the vector-ALU tiles take them), [4] heavy and [5]
// short items beyond Job::r32 (FP64 products); lists 0 and 1 then hold the
// items with FP32 products.
// One thread per item counts its chain and copies the (start, count) of its
// mixed-pass groups, in chain order, to eglist at an offset reserved per block
// (ehdr[item] = (offset, groups), offset -1 when eglist is full); each block
// appends its items to the lists with one atomic per list.  Which block takes
// an item does not change its sums.
__global__ __launch_bounds__(256) void k_eorder(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                                const Group *__restrict__ egrp, const int *__restrict__ headE,
                                                const int *__restrict__ overflow, const ItemRec *__restrict__ irec,
                                                int nitems, int mx, int *cnt,
                                                int *__restrict__ lists, int2 *__restrict__ ehdr,
                                                int2 *__restrict__ eglist, int egcap) {
    constexpr int NL = 6;
    __shared__ int wc[NL][4], base[NL], wg[4], gbase;
    if (*overflow) return;
    const int item = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int cls = -1;  // no item
    int ng = 0;    // groups of the mixed pass in the item's chain
    int head = -1;
    if (item < nitems) {
        const ItemRec ir = irec[item];
        const Job jb = jobs[ir.job];
        const DevTree &Q = trees[jb.qt];
        const int leaf = ir.leaf;
        head = headE[(size_t)jb.noff + leaf];
        int ops = 0, n = 0;
        for (int gi = head; gi >= 0 && n < kMaxEGrp; ++n) {
            const Group g = egrp[gi];
            if (g.flags == 0) {
                ops += g.count;
                ++ng;
            }
            gi = g.next;
        }
        cls = ops >= kEHeavyOps ? 0 : (ops > 0 ? 1 : 2);
        if (mx && ops > 0) {  // the query leaf's half-diagonal in sig units picks the form
            double hd = 0.0;
            for (int c = 0; c < Q.d; ++c) {
                const double hw = 0.5 * (Q.hi[(size_t)leaf * Q.d + c] - Q.lo[(size_t)leaf * Q.d + c]);
                hd = fma(hw, hw, hd);
            }
            const double rho = std::sqrt(hd) * jb.sig;
            if (rho > kMxWideQ) cls = 3;
            else if (!(rho <= jb.r32)) cls += 4;
        }
    }
    int rk[NL];
    for (int c = 0; c < NL; ++c) {
        const int f = cls == c ? 1 : 0;
        const int inc = wave_incl_scan(f);
        rk[c] = inc - f;
        if (lane == 63) wc[c][wv] = inc;
    }
    const int incg = wave_incl_scan(ng);
    if (lane == 63) wg[wv] = incg;
    __syncthreads();
    if (threadIdx.x < NL) {
        const int c = threadIdx.x;
        const int tot = wc[c][0] + wc[c][1] + wc[c][2] + wc[c][3];
        base[c] = tot ? atomicAdd(&cnt[(C_EHEAVY + c) * CP], tot) : 0;
    } else if (threadIdx.x == 64) {
        const int tot = wg[0] + wg[1] + wg[2] + wg[3];
        gbase = tot ? atomicAdd(&cnt[C_ECH * CP], tot) : 0;
    }
    __syncthreads();
    if (cls >= 0) {
        int off = base[cls] + rk[cls];
        for (int w = 0; w < wv; ++w) off += wc[cls][w];
        lists[(size_t)cls * nitems + off] = item;
        // the chain's groups of the mixed pass, flattened in chain order, so
        // the tile kernels read them at once instead of following the links
        int go = gbase + incg - ng;
        for (int w = 0; w < wv; ++w) go += wg[w];
        if (go + ng <= egcap) {
            int k = 0, n = 0;
            for (int gi = head; gi >= 0 && n < kMaxEGrp; ++n) {
                const Group g = egrp[gi];
                if (g.flags == 0) eglist[go + k++] = make_int2(g.start, g.count);
                gi = g.next;
            }
            ehdr[item] = make_int2(go, ng);
        } else {
            ehdr[item] = make_int2(-1, 0);  // list full: the kernels follow the links
        }
    }
}

// Item of block b of the mixed pass in that order (order = null: in turn);
// order holds k_eorder's six lists, nitems entries each.  sel = 0 takes lists
// 0, 1, 2 in turn, sel = 1 list 3, sel = 2 lists 4, 5; -1: no item.
__device__ __forceinline__ int etile_item(int b, const int *__restrict__ cnt, const int *__restrict__ order,
                                          int nitems, int sel) {
    if (!order) return b;
    if (sel == 1) return b < cnt[C_EWIDE * CP] ? order[3 * (size_t)nitems + b] : -1;
    if (sel == 2) {
        const int nh = cnt[C_EHEAVY64 * CP], nn = cnt[C_ENORM64 * CP];
        if (b < nh) return order[4 * (size_t)nitems + b];
        return b < nh + nn ? order[5 * (size_t)nitems + b - nh] : -1;
    }
    const int nh = cnt[C_EHEAVY * CP], nn = cnt[C_ENORM * CP], ne = cnt[C_EEMPTY * CP];
    if (b < nh) return order[b];
    if (b < nh + nn) return order[nitems + b - nh];
    return b < nh + nn + ne ? order[2 * (size_t)nitems + b - nh - nn] : -1;
}

// ---------------------------------------------------------------- exhaustive tiles on the vector ALUs
// DFGTBase for every dimension (the matrix-core kernel below takes D >= 8 in
// mixed precision), in two passes over the same E lists: F64 = false takes the
// pairs summed in mixed precision and writes G_E; F64 = true takes the pairs
// summed in FP64 (precision FP64, or groups flagged by the underflow guard)
// and writes G_E (precision FP64) or adds to it (it runs after the mixed pass
// on the same stream).  Splitting them keeps FP64 exponentials out of the
// mixed kernel's registers.
// One block of kEWaves waves per (job, query leaf): the leaf's E chain is
// flattened 64 kEWaves ops at a time (reference range and point count,
// block-wide scan) into one list of reference points, which the waves take in
// rounds of RPW points, wave w rounds w, w + kEWaves, ...; each wave stages its own round in LDS (scaled
// by sig), so rounds need no block barrier.  Lanes of a wave: NG groups of
// `need` lanes; a lane holds QPT queries (ql + need a) and group g takes the
// staged points g, g + NG, ... (groups read neighbouring points: no LDS bank
// conflicts).  In the mixed pass for D <= 5 a round is padded with
// zero-weight points to 4 NG ceil(points per group / 4) entries, so every lane
// runs the same trip count, unrolled by 4.
// Mixed pairs: the FP64 scaled difference, FP32 exp2 of the rounded square,
// FP32 partial sums over <= 64 terms, FP64 beyond.  The partials of the waves
// and groups are added in a fixed order.  G_E (and with GR X_E, Y_E) are per
// query in tree order; k_leaf adds them to the rest.
constexpr int kEWaveStage = 512;  // doubles of staged reference coordinates per wave
constexpr int kEPpl = 4;          // points staged per lane and round (at most)
constexpr int kEMaxGroups = 16;   // point groups per wave (the padding is < 4 of them per group)
constexpr int kEPadPts = 4 * kEMaxGroups;
constexpr int kEUnroll = 4;
// Waves per block.  A query leaf's rounds are dealt to the block's waves, so
// a leaf with hundreds of reference leaves, which sets the end of the launch,
// finishes sooner with more waves; 8 waves with 512-double stages keep a
// block under 64 KB of LDS (two blocks per CU).
constexpr int kEWaves = 8;

template <int DT, bool F64>
struct ETileShape {
    static constexpr int DS = DT > 0 ? DT : kMaxD;        // register arrays (runtime d only in the DT = 0 form)
    static constexpr int QPT = (DT > 0 && !F64) ? 2 : 1;  // queries per lane
    static constexpr bool PAD = DT > 0 && !F64;           // padded, unrolled loop
};

template <int DT, bool F64>
__host__ __device__ constexpr int etile_rpw(int d) {
    const int n = ETileShape<DT, F64>::PAD ? kEWaveStage / d - kEPadPts : kEWaveStage / d;
    return n < 256 ? n : 256;
}

// Mixed pairs, padded rounds of t4 points per group (t4 a multiple of 4,
// weight 0 on the padding).
template <int DT, bool GR>
__device__ __forceinline__ void etile_fast(const double *__restrict__ st, const float *__restrict__ pw, int g,
                                           int ng, int t4, const double (&qs)[2][DT], double (&acc)[2],
                                           double (&xacc)[2], double (&yacc)[2][DT]) {
    for (int t0 = 0; t0 < t4; t0 += 64) {
        const int te = min(t4, t0 + 64);  // <= 64 points of this lane: one FP32 partial
        float ps[2], pt[2], py[2][DT];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            ps[a] = 0.0f;
            pt[a] = 0.0f;
#pragma unroll
            for (int c = 0; c < DT; ++c) py[a][c] = 0.0f;
        }
        for (int t = t0; t < te; t += kEUnroll) {
            double xv[kEUnroll][DT];
            float w[kEUnroll];
#pragma unroll
            for (int u = 0; u < kEUnroll; ++u) {
                const int j = g + ng * (t + u);
#pragma unroll
                for (int c = 0; c < DT; ++c) xv[u][c] = st[j * DT + c];
                w[u] = pw[j];
            }
#pragma unroll
            for (int u = 0; u < kEUnroll; ++u) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    double tt = 0.0, dd[DT];
#pragma unroll
                    for (int c = 0; c < DT; ++c) {
                        dd[c] = qs[a][c] - xv[u][c];
                        tt = fma(dd[c], dd[c], tt);
                    }
                    const float tf = (float)tt;
                    const float e = __builtin_amdgcn_exp2f(-tf);
                    if (!GR) {
                        ps[a] = fmaf(w[u], e, ps[a]);
                    } else {
                        const float ew = w[u] * e;
                        ps[a] += ew;
                        pt[a] = fmaf(tf, ew, pt[a]);
#pragma unroll
                        for (int c = 0; c < DT; ++c) py[a][c] = fmaf(ew, (float)dd[c], py[a][c]);
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            acc[a] += (double)ps[a];
            if (GR) {
                xacc[a] = fma(-2.0 * kLn2, (double)pt[a], xacc[a]);
#pragma unroll
                for (int c = 0; c < DT; ++c) yacc[a][c] = fma(-2.0 * kSqrtLn2, (double)py[a][c], yacc[a][c]);
            }
        }
    }
}

// Mixed pairs with FP32 differences: points staged as NF4 float4 each (the
// first DT components the coordinates relative to the query leaf's centre,
// scaled by sig; the last component of the last float4 the weight), padded
// rounds of t4 points per group as in etile_fast.
template <int DT, int NF4>
__device__ __forceinline__ void etile_fast32(const float4 *__restrict__ st, int g, int ng, int t4,
                                             const float (&qs)[2][DT], double (&acc)[2]) {
    for (int t0 = 0; t0 < t4; t0 += 64) {
        const int te = min(t4, t0 + 64);  // <= 64 points of this lane: one FP32 partial
        float ps[2] = {0.0f, 0.0f};
        for (int t = t0; t < te; t += kEUnroll) {
            float xv[kEUnroll][4 * NF4];
#pragma unroll
            for (int u = 0; u < kEUnroll; ++u) {
                const int j = g + ng * (t + u);
#pragma unroll
                for (int f = 0; f < NF4; ++f) {
                    const float4 v = st[j * NF4 + f];
                    xv[u][4 * f] = v.x;
                    xv[u][4 * f + 1] = v.y;
                    xv[u][4 * f + 2] = v.z;
                    xv[u][4 * f + 3] = v.w;
                }
            }
#pragma unroll
            for (int u = 0; u < kEUnroll; ++u) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float d0 = qs[a][0] - xv[u][0];
                    float tt = d0 * d0;
#pragma unroll
                    for (int c = 1; c < DT; ++c) {
                        const float dc = qs[a][c] - xv[u][c];
                        tt = fmaf(dc, dc, tt);
                    }
                    ps[a] = fmaf(xv[u][4 * NF4 - 1], __builtin_amdgcn_exp2f(-tt), ps[a]);
                }
            }
        }
        acc[0] += (double)ps[0];
        acc[1] += (double)ps[1];
    }
}

// One lane's query against the staged points g, g + ng, ... < cnt (runtime d):
// mixed pairs (F64 = false) or FP64 pairs (t in sig units, e = 2^-t), each
// term times the staged point weight sw[j] (sw null: weight 1).
template <bool GR, bool F64>
__device__ __forceinline__ void etile_strided(const double *__restrict__ st, const double *__restrict__ sw, int g,
                                              int ng, int cnt, int d, const double *qs, double &acc, double &xacc,
                                              double *yacc) {
    for (int t0 = g; t0 < cnt; t0 += 64 * ng) {
        const int te = min(cnt, t0 + 64 * ng);  // <= 64 points of this lane: one FP32 partial
        float ps = 0.0f, pt = 0.0f, py[kMaxD];
        if (GR && !F64)
            for (int c = 0; c < d; ++c) py[c] = 0.0f;
        for (int j = t0; j < te; j += ng) {
            const double *xr = st + j * d;
            double t = 0.0, dd[kMaxD];
            for (int c = 0; c < d; ++c) {
                dd[c] = qs[c] - xr[c];
                t = fma(dd[c], dd[c], t);
            }
            if (F64) {
                const double e = exp(-t * kLn2) * (sw ? sw[j] : 1.0);
                acc += e;
                if (GR) {
                    xacc = fma(-2.0 * kLn2 * t, e, xacc);
                    for (int c = 0; c < d; ++c) yacc[c] = fma(-2.0 * kSqrtLn2 * e, dd[c], yacc[c]);
                }
            } else {
                const float tf = (float)t;
                const float e = __builtin_amdgcn_exp2f(-tf) * (sw ? (float)sw[j] : 1.0f);
                ps += e;
                if (GR) {
                    pt = fmaf(tf, e, pt);
                    for (int c = 0; c < d; ++c) py[c] = fmaf(e, (float)dd[c], py[c]);
                }
            }
        }
        if (!F64) {
            acc += (double)ps;
            if (GR) {
                xacc = fma(-2.0 * kLn2, (double)pt, xacc);
                for (int c = 0; c < d; ++c) yacc[c] = fma(-2.0 * kSqrtLn2, (double)py[c], yacc[c]);
            }
        }
    }
}

template <int DT, bool GR, bool F64>
__device__ __forceinline__ void etile_body(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                           const Group *__restrict__ egrp, const int *__restrict__ eops,
                                           const int *__restrict__ headE, const int *__restrict__ cnt_dev,
                                           const int *__restrict__ overflow, const ItemRec *__restrict__ irec,
                                           int precision, const int *__restrict__ order,
                                           int nitems, int sel, double *__restrict__ GE, double *__restrict__ GX,
                                           double *__restrict__ GY) {
    using Sh = ETileShape<DT, F64>;
    constexpr int DS = Sh::DS, QPT = Sh::QPT;
    constexpr bool PAD = Sh::PAD;
    constexpr int kSP = PAD ? etile_rpw<DT, F64>(DT > 0 ? DT : 1) + kEPadPts : 1;  // padded entries per wave
    // FP32-difference form (value sums in mixed precision, D <= 5): NF4 float4
    // per staged point, RPW32 points per wave and round
    constexpr bool F32D = PAD && !GR && DT <= 3;
    constexpr int NF4 = DT <= 3 ? 1 : 2;
    constexpr int RPW32 = kEWaveStage / (2 * NF4) - kEPadPts;
    constexpr int PPL32 = (RPW32 + 63) / 64;
    __shared__ int gS[kMaxEGrp], gF[kMaxEGrp], gCum[kMaxEGrp];
    constexpr int NW = kEWaves, kCh = 64 * kEWaves;  // E ops flattened per chunk: one per thread
    __shared__ int oB[kCh], oCum[kCh];
    __shared__ int wsum[NW], nops_s, take_s;
    __shared__ double wb2[NW];
    __shared__ __align__(16) double stage[NW][kEWaveStage];
    __shared__ float pwt[NW][kSP];
    __shared__ double swt[NW][PAD ? 1 : 256];  // point weights of the strided form
    __shared__ double red[NW][64 * QPT];
    if (*overflow) return;
    const bool all64 = precision == DFGT_PREC_FP64;
    // the FP64 pass of a mixed-precision call has work only if the guard flagged a group
    if (F64 && !all64 && cnt_dev[C_EF64 * CP] == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int item = etile_item(blockIdx.x, cnt_dev, order, nitems, sel);
    if (item < 0) return;
    const ItemRec ir = irec[item];
    const Job jb = jobs[ir.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int leaf = ir.leaf;
    const int d = DT > 0 ? DT : Q.d;
    const int RPW = etile_rpw<DT, F64>(d);  // reference points per wave and round
    const int PPL = (RPW + 63) / 64;        // of which each lane stages <= PPL
    const int qb0 = Q.begin[leaf], nq = Q.end[leaf] - qb0;
    const size_t hq = (size_t)jb.noff + leaf;
    const int head = headE[hq];
    // groups of this pass: mixed pass the unflagged ones, FP64 pass the flagged
    // ones (all of them at precision FP64)
    if (tid == 0) {
        int n = 0, tot = 0, any = 0;
        for (int gi = head; gi >= 0 && n < kMaxEGrp; gi = egrp[gi].next) {
            const Group gg = egrp[gi];
            const int tk = F64 ? (all64 || gg.flags != 0) : (gg.flags == 0);
            gS[n] = gg.start;
            gF[n] = tk;
            any |= tk;
            tot += gg.count;
            gCum[n++] = tot;
        }
        nops_s = tot;
        take_s = any;
    }
    __syncthreads();
    const int nops = nops_s;
    const bool add = F64 && !all64;  // the FP64 pass of a mixed call adds to the mixed pass's G_E
    if (!take_s) {  // no pairs of this pass for this leaf
        if (!add)
            for (int i = tid; i < nq; i += blockDim.x) {
                const size_t ei = (size_t)jb.qoff + qb0 + i;
                GE[ei] = 0.0;
                if (GR) {
                    GX[ei] = 0.0;
                    for (int c = 0; c < d; ++c) GY[ei * d + c] = 0.0;
                }
            }
        return;
    }
    double *st = stage[wv];
    float4 *st4 = reinterpret_cast<float4 *>(stage[wv]);
    float *pw = pwt[wv];
    double *sw = swt[wv];
    // the query leaf's centre and half-diagonal (sig units) for the FP32 form
    const bool try32 = F32D && jb.a32 > 0.0;
    double qc[DS];
    double qhalf = 0.0;
    if (try32)
        for (int c = 0; c < d; ++c) {
            qc[c] = Q.ctr[(size_t)leaf * d + c];
            const double hw = 0.5 * (Q.hi[(size_t)leaf * d + c] - Q.lo[(size_t)leaf * d + c]);
            qhalf = fma(hw, hw, qhalf);
        }
    qhalf = std::sqrt(qhalf) * jb.sig;
    for (int qg = 0; qg < nq; qg += 64 * QPT) {
        const int nqg = min(64 * QPT, nq - qg);
        const int need = (nqg + QPT - 1) / QPT;     // lanes per group
        const int NG = min(kEMaxGroups, 64 / need);  // groups per wave
        const bool lact = lane < NG * need;
        const int ql = lact ? lane % need : 0, g = lact ? lane / need : 0;
        double qs[QPT][DS], acc[QPT], xacc[QPT], yacc[QPT][DS];
        float qs32[2][DS];
#pragma unroll
        for (int a = 0; a < QPT; ++a) {
            const int qi = ql + need * a;
            const int qpos = qb0 + qg + (qi < nqg ? qi : 0);
            for (int c = 0; c < d; ++c) qs[a][c] = Q.x[(size_t)qpos * d + c] * jb.sig;
            if (try32)
                for (int c = 0; c < d; ++c) qs32[a][c] = (float)((Q.x[(size_t)qpos * d + c] - qc[c]) * jb.sig);
            acc[a] = 0.0;
            xacc[a] = 0.0;
            if (GR)
                for (int c = 0; c < d; ++c) yacc[a][c] = 0.0;
        }
        for (int o0 = 0; o0 < nops; o0 += kCh) {
            __syncthreads();  // the previous chunk's tables are no longer read
            const int o = o0 + tid;
            int np = 0;
            double b2 = 0.0;  // squared distance of the op's farthest box corner from the leaf centre
            if (o < nops) {
                int gi = 0;
                while (o >= gCum[gi]) ++gi;
                if (gF[gi]) {  // a group of this pass
                    const int r = eops[gS[gi] + o - (gi ? gCum[gi - 1] : 0)];
                    oB[tid] = R.begin[r];
                    np = R.end[r] - R.begin[r];
                    if (try32)
                        for (int c = 0; c < d; ++c) {
                            const double l = R.lo[(size_t)r * d + c] - qc[c], h = R.hi[(size_t)r * d + c] - qc[c];
                            b2 += fmax(l * l, h * h);
                        }
                }
            }
            const int inc = wave_incl_scan(np);
            if (lane == 63) wsum[wv] = inc;
            if (try32) {
                b2 = wave_max(b2);
                if (lane == 0) wb2[wv] = b2;
            }
            __syncthreads();
            int pre = 0;
            for (int w = 0; w < wv; ++w) pre += wsum[w];
            oCum[tid] = pre + inc;
            // FP32 differences for this chunk when every pair's |a| + |b| is within the budget
            bool use32 = false;
            if (try32) {
                double m = 0.0;
                for (int w = 0; w < NW; ++w) m = fmax(m, wb2[w]);
                use32 = qhalf + std::sqrt(m) * jb.sig <= jb.a32;
            }
            __syncthreads();
            const int nopc = min(kCh, nops - o0);
            const int tot = oCum[nopc - 1];
            // rounds short enough that every wave of the block gets one (a short E list
            // would otherwise leave waves idle); multiples of 16 points
            const int RPWc = min(use32 ? RPW32 : RPW, max(16, (tot + 16 * NW - 1) / (16 * NW) * 16));
            const int PPLc = (RPWc + 63) / 64;
            for (int p0 = wv * RPWc; p0 < tot; p0 += NW * RPWc) {
                // stage the round: lane l takes points l PPL + k, k < PPL
                const int cnt = min(RPWc, tot - p0);
                int i = lane * PPLc;
                if (i < cnt) {
                    int lo = 0, hi = nopc - 1;  // first op with oCum > p0 + i
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (oCum[mid] > p0 + i) hi = mid;
                        else lo = mid + 1;
                    }
                    int op = lo;
                    for (int k = 0; k < PPLc && i < cnt; ++k, ++i) {
                        const int p = p0 + i;
                        while (oCum[op] <= p) ++op;
                        const int row = oB[op] + p - (op ? oCum[op - 1] : 0);
                        if (F32D && use32) {
                            float v[4 * NF4];
#pragma unroll
                            for (int c = 0; c < 4 * NF4; ++c)
                                v[c] = c < DS ? (float)((R.x[(size_t)row * DS + c] - qc[c]) * jb.sig) : 0.0f;
                            v[4 * NF4 - 1] = R.w ? (float)R.w[row] : 1.0f;
#pragma unroll
                            for (int f = 0; f < NF4; ++f)
                                st4[i * NF4 + f] = make_float4(v[4 * f], v[4 * f + 1], v[4 * f + 2], v[4 * f + 3]);
                        } else {
                            for (int c = 0; c < d; ++c) st[i * d + c] = R.x[(size_t)row * d + c] * jb.sig;
                            if constexpr (PAD) pw[i] = R.w ? (float)R.w[row] : 1.0f;
                            else if (R.w) sw[i] = R.w[row];
                        }
                    }
                }
                if constexpr (PAD) {
                    const int t4 = ((cnt + NG - 1) / NG + kEUnroll - 1) / kEUnroll * kEUnroll;
                    // zero-weight padding up to NG t4 entries (< cnt + 4 NG <= RPW + kEPadPts)
                    if (F32D && use32) {
                        for (int i2 = cnt + lane; i2 < NG * t4; i2 += 64)
                            for (int f = 0; f < NF4; ++f) st4[i2 * NF4 + f] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                        wave_sync();  // a wave's LDS accesses complete in order
                        if constexpr (F32D) etile_fast32<DT, NF4>(st4, g, NG, t4, qs32, acc);
                    } else {
                        for (int i2 = cnt + lane; i2 < NG * t4; i2 += 64) {
                            for (int c = 0; c < d; ++c) st[i2 * d + c] = 0.0;
                            pw[i2] = 0.0f;
                        }
                        wave_sync();  // a wave's LDS accesses complete in order
                        etile_fast<DT, GR>(st, pw, g, NG, t4, qs, acc, xacc, yacc);
                    }
                } else {
                    wave_sync();
                    etile_strided<GR, F64>(st, R.w ? sw : nullptr, g, NG, cnt, d, qs[0], acc[0], xacc[0], yacc[0]);
                }
                wave_sync();
            }
        }
        // partials of the waves and groups, added in (wave, group) order, one quantity at a time
        const int nred = GR ? 2 + d : 1;
        for (int v = 0; v < nred; ++v) {
#pragma unroll
            for (int a = 0; a < QPT; ++a)
                red[wv][lane * QPT + a] = v == 0 ? acc[a] : (v == 1 ? xacc[a] : yacc[a][v - 2]);
            __syncthreads();
            if (tid < nqg) {
                const int a = tid / need, qi = tid % need;
                double sum = 0.0;
                for (int w = 0; w < NW; ++w)
                    for (int k = 0; k < NG; ++k) sum += red[w][(k * need + qi) * QPT + a];
                const size_t ei = (size_t)jb.qoff + qb0 + qg + tid;
                double *dst = v == 0 ? &GE[ei] : (v == 1 ? &GX[ei] : &GY[ei * d + (v - 2)]);
                *dst = add ? *dst + sum : sum;
            }
            __syncthreads();
        }
    }
}

template <int DT, bool GR, bool F64>
__global__ __launch_bounds__(64 * kEWaves) void k_etile(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                                        const Group *__restrict__ egrp, const int *__restrict__ eops,
                                                        const int *__restrict__ headE, const int *__restrict__ cnt_dev,
                                                        const int *__restrict__ overflow,
                                                        const ItemRec *__restrict__ irec,
                                                        int precision, const int *__restrict__ order, int nitems,
                                                        int sel, double *__restrict__ GE, double *__restrict__ GX,
                                                        double *__restrict__ GY) {
    etile_body<DT, GR, F64>(trees, jobs, egrp, eops, headE, cnt_dev, overflow, irec, precision,
                            order, nitems, sel, GE, GX, GY);
}

// The 3-D mixed-precision value pass, held to 128 VGPRs (four waves per SIMD,
// two 8-wave blocks per CU; it fits without spills): left to itself the
// compiler takes ~165 and a CU runs one block.
template <int DT, bool GR, bool F64>
__global__ __launch_bounds__(64 * kEWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_etile_o4(
    const DevTree *__restrict__ trees, const Job *__restrict__ jobs, const Group *__restrict__ egrp,
    const int *__restrict__ eops, const int *__restrict__ headE, const int *__restrict__ cnt_dev,
    const int *__restrict__ overflow, const ItemRec *__restrict__ irec, int precision,
    const int *__restrict__ order, int nitems, int sel, double *__restrict__ GE, double *__restrict__ GX,
    double *__restrict__ GY) {
    etile_body<DT, GR, F64>(trees, jobs, egrp, eops, headE, cnt_dev, overflow, irec, precision,
                            order, nitems, sel, GE, GX, GY);
}

// ---------------------------------------------------------------- exhaustive tiles on the matrix cores, 3 <= D <= 7
// The mixed pass of the value sums (DFGTBase, Section 3.9) as a contraction.
// Coordinates are taken relative to the query leaf's box centre c and scaled
// by sig: a = sig (q - c), b = sig (r - c), so that t = |a - b|^2 and the
// kernel value is 2^-t.  With the K = 4 NC operand rows
//     A_i = (a_i, 1, 0, ...),   B_j = (2 b_j, log2 w_j - |b_j|^2, 0, ...),   C_i = -|a_i|^2
// NC v_mfma_*_16x16x4 instructions give log2 w_j - t for a block of 16
// queries x 16 references (a reference of weight 0 has -1e30 in place of
// log2 w_j - |b_j|^2).  The lanes take the hardware exp2 of it (rounded to
// FP32 once in the FP64 form), w_j 2^-t, and add it into FP32 partials of
// <= 64 terms; the partials are reduced across lanes and added in FP64, in
// a fixed order.
// Two precisions of the product, chosen per item by k_eorder from the query
// leaf's half-diagonal rho in sig units:
// Staging window W = Job::win: a reference farther than W (sig units) from
// the query leaf has t >= W^2 for every query and is left out.  W = 12 in
// general (terms below 2^-144, under the FP32 flush the mixed sums already
// allow for); when Q = R, unweighted and not leave-one-out, every G(q) >= 1
// (the self term) and the at most N_R left-out terms stay within a share
// eps_round / 50 of G(q) for W^2 = log2(N_R / (eps_round / 50)) (W ~ 6).
//   FP32 (rho <= Job::r32): a reference is staged only when |b| <= rho + W,
//     the others with weight 0.  Then A = |a| + |b| <= 2 rho + W, and the
//     FP32 rounding of the operands and of the four multiply-adds moves t by
//     at most 6.5 u A^2 (u = 2^-24); r32 keeps ln2 6.5 u A^2 + 2^-22 (exp2) +
//     68 u (weight, partials), plus the window's share and, for a weighted
//     tree, ln2 126 u for log2 w in the rounded row, within the rounding
//     budget.
//   FP64 (rho <= kMxWideQ): a reference is staged only when its distance to
//     the query leaf's bounding box is <= W.  The kept points are
//     packed at the front of each wave's 64-point region of the round (a
//     ballot gives their ranks), padded to a multiple of 16; those big leaves
//     see many such far references, which are then neither multiplied nor
//     exponentiated.  Then A <= 2 rho + W <= 2^13 + 12 and the FP64 rounding
//     of t, ~12 2^-53 A^2, stays below 1e-7, under the FP32 rounding of t
//     itself.
//   Wider leaves go to the vector-ALU tiles.
// One block of kMxWaves waves per (job, query leaf) item, taken in the order
// k_eorder made (heavy items first); the item's chain comes flattened from
// k_eorder.  The leaf's queries, kMxQ at a time, are held as operands by the
// waves: the 16-query blocks form the fewest sets of <= 4 blocks, and each
// set is held by every nsets-th wave.  The E chain is flattened
// kMxOps ops at a time into one list of reference points (only the groups of
// this pass: those the underflow guard flagged go to the FP64 pass); the
// block stages RND of them at a time in LDS as operand rows (structure of
// arrays: lane l reads row 4c + l / 16 of point l % 16, conflict-free), and
// the waves holding a set of query blocks take the round's 16-point blocks in
// turn.
// Operand layouts of v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32 (lane l,
// g = l / 16): A[i][k] at lane i + 16 k, B[k][j] at lane j + 16 k; result
// register r holds D[4 r + g][l % 16] (FP64) or D[4 g + r][l % 16] (FP32).
// Here A = 16 queries x 4 rows, B = 4 rows x 16 references.

// The operand row of a reference's weight: log2 w (0 for the unit weights
// of an unweighted tree), or kMxZeroRow for a weight of 0 or below 2^-126
// (a term under the FP32 flush), which sends the products to -1e30 and the
// exponential to 0 without an infinity.
constexpr double kMxZeroRow = -1e30;
__device__ __forceinline__ double mx_log2w(float w) {
    if (w == 1.0f) return 0.0;
    return w >= 0x1p-126f ? log2((double)w) : kMxZeroRow;
}

template <typename T, int NC>
struct MxShape {
    static constexpr int K = 4 * NC;  // operand rows
    static constexpr int DX = K - 1;  // coordinates a point can have
    // staged reference points per round (two buffers), per thread at most PPT
    static constexpr int RND = (NC == 1 ? 128 : 64) * kMxWaves * 4 / (int)sizeof(T);
    static constexpr int PPT = RND >= 64 * kMxWaves ? RND / (64 * kMxWaves) : 1;
};
template <typename T>
struct MxVec;
template <>
struct MxVec<double> {
    typedef v4d type;
    __device__ static type mfma(double a, double b, type c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int r, int g) { return 4 * r + g; }
};
template <>
struct MxVec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    __device__ static type mfma(float a, float b, type c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int r, int g) { return 4 * g + r; }
};

template <typename T, int NC>
__device__ __forceinline__ void etile_mx_body(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                              const Group *__restrict__ egrp, const int *__restrict__ eops,
                                              const int *__restrict__ headE, const int *__restrict__ cnt_dev,
                                              const int *__restrict__ overflow, const ItemRec *__restrict__ irec,
                                              const int *__restrict__ order, int nitems,
                                              int sel, const int2 *__restrict__ ehdr,
                                              const int2 *__restrict__ eglist, unsigned long long *__restrict__ npairs,
                                              double *__restrict__ GE) {
    constexpr int K = MxShape<T, NC>::K, RND = MxShape<T, NC>::RND, PPT = MxShape<T, NC>::PPT;
    constexpr int DX = MxShape<T, NC>::DX;
    typedef MxVec<T> V;
    typedef typename V::type VT;
    __shared__ int gS[kMaxEGrp], gF[kMaxEGrp], gCum[kMaxEGrp];
    __shared__ int oB[kMxOps], oCum[kMxOps];
    __shared__ unsigned char segop[kMxSeg];  // op holding the chunk's point 64 s
    __shared__ int wsum[kMxWaves], nops_s, take_s;
    __shared__ T sB[2][K][RND];           // reference operand rows of a round, two buffers (rows past D + 1 zero)
    __shared__ double sA[K][kMxQ];        // query operand rows of the pass
    __shared__ double sN[kMxQ];           // |a|^2 of the pass's queries
    __shared__ double sQ[kMxWaves][64];   // per-wave FP64 sums per query of its set
    __shared__ double sHw[K];             // FP64 form: the leaf box's half-widths in sig units
    __shared__ int sCnt[2][kMxWaves];     // FP64 form: kept points of each wave's region, padded to 16
    constexpr bool PACK = std::is_same<T, double>::value;
    static_assert(!PACK || PPT == 1, "the FP64 form stages one point per thread and round");
    if (*overflow) return;
    const int item = etile_item(blockIdx.x, cnt_dev, order, nitems, sel);
    if (item < 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, col = lane & 15;
    const ItemRec ir = irec[item];
    const int2 eh = ehdr[item];
    const Job jb = jobs[ir.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int leaf = ir.leaf;
    const int d = Q.d;
    const int qb0 = ir.qb0, nq = ir.nq;
    const size_t hq = (size_t)jb.noff + leaf;
    if (eh.x >= 0) {  // the chain's mixed-pass groups as k_eorder listed them
        const int ng = eh.y;
        if (tid < ng) {
            const int2 e = eglist[eh.x + tid];
            gS[tid] = e.x;
            gF[tid] = 1;
            gCum[tid] = e.y;
        }
        __syncthreads();
        if (ng <= 64) {
            if (wv == 0) {
                const int inc = wave_incl_scan(lane < ng ? gCum[lane] : 0);
                if (lane < ng) gCum[lane] = inc;
                if (lane == 63) {
                    nops_s = inc;
                    take_s = ng > 0;
                }
            }
        } else if (tid == 0) {
            for (int k = 1; k < ng; ++k) gCum[k] += gCum[k - 1];
            nops_s = gCum[ng - 1];
            take_s = 1;
        }
    } else if (tid == 0) {  // follow the chain's links
        int n = 0, tot = 0, any = 0;
        for (int gi = headE[hq]; gi >= 0 && n < kMaxEGrp; gi = egrp[gi].next) {
            const Group gg = egrp[gi];
            const int tk = gg.flags == 0;
            gS[n] = gg.start;
            gF[n] = tk;
            any |= tk;
            tot += gg.count;
            gCum[n++] = tot;
        }
        nops_s = tot;
        take_s = any;
    }
    __syncthreads();
    const int nops = __builtin_amdgcn_readfirstlane(nops_s);
    if (!take_s) {  // no pairs of this pass for this leaf
        for (int i = tid; i < nq; i += blockDim.x) GE[(size_t)jb.qoff + qb0 + i] = 0.0;
        return;
    }
    const double sig = jb.sig;
    double qc[K];
    double rho = 0.0;  // the leaf's half-diagonal in sig units
#pragma unroll
    for (int k = 0; k < K; ++k) {
        qc[k] = 0.0;
        if (k < d) {
            qc[k] = ldg(Q.ctr + (size_t)leaf * d + k);
            const double hw = 0.5 * (ldg(Q.hi + (size_t)leaf * d + k) - ldg(Q.lo + (size_t)leaf * d + k));
            rho = fma(hw, hw, rho);
            if (PACK && tid == 0) sHw[k] = hw * sig;
        }
    }
    rho = std::sqrt(rho) * sig;
    // squared staging radius: beyond it a term is zero to the form's precision
    const double win = jb.win;
    const double bcut = (rho + win) * (rho + win);
    for (int qs = 0; qs < nq; qs += kMxQ) {
        const int nqs = min(kMxQ, nq - qs);
        const int nqb = (nqs + 15) >> 4;  // query blocks of the pass
        // nsets sets of <= 4 query blocks, as equal as can be; wave w holds set
        // w % nsets and takes every stride-th reference block from phase on
        // (nsets divides the wave count, so every set has as many waves)
        const int nsets = nqb <= 4 ? 1 : (nqb <= 8 ? 2 : kMxWaves);
        const int set = wv % nsets;
        const int stride = (kMxWaves - set + nsets - 1) / nsets, phase = wv / nsets;
        const int bb = set * nqb / nsets;  // the set's first query block
        const int nvb = __builtin_amdgcn_readfirstlane((set + 1) * nqb / nsets - bb);
        __syncthreads();  // the previous pass's sums are read
        if (tid < kMxQ) {  // the pass's query operand rows and norms
            double nrm = 0.0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                double a = 0.0;
                if (k < d && tid < nqs) a = (ldg(Q.x + (size_t)(qb0 + qs + tid) * d + k) - qc[k]) * sig;
                if (k < d) nrm = fma(a, a, nrm);
                sA[k][tid] = k < d ? a : (k == d ? 1.0 : 0.0);
            }
            sN[tid] = nrm;
        }
        sQ[wv][lane] = 0.0;
        __syncthreads();
        T Af[4][NC];
        VT Cf[4];
        float acc[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int qb = min(bb + b, kMxQ / 16 - 1);  // blocks past the set are never used
#pragma unroll
            for (int c = 0; c < NC; ++c) Af[b][c] = (T)sA[4 * c + g][16 * qb + col];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Cf[b][r] = (T)-sN[16 * qb + V::row(r, g)];
                acc[b][r] = 0.0f;
            }
        }
        // FP32 partials into the wave's FP64 sums: across the 16 reference
        // columns (the lanes of one g, a DPP row) by an FP32 scan whose last
        // lane holds the row's sum (four more roundings per term, one
        // v_add_f32 with a DPP source each), then into LDS in FP64 by the
        // column-15 lanes
        auto flush = [&]() {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (b >= nvb) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float v = acc[b][r];
                    acc[b][r] = 0.0f;
                    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
                    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));
                    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));
                    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));
                    if (col == 15) sQ[wv][16 * b + V::row(r, g)] += (double)v;
                }
            }
        };
        int nblk = 0;  // reference blocks in the wave's current partials
        long long ptot = 0;  // reference points of the pass
        for (int o0 = 0; o0 < nops; o0 += kMxOps) {
            __syncthreads();  // the previous chunk's tables are no longer read
            const int o = o0 + tid;
            int np = 0;
            if (o < nops) {
                int gi = 0;
                while (o >= gCum[gi]) ++gi;
                if (gF[gi]) {
                    const int r = eops[gS[gi] + o - (gi ? gCum[gi - 1] : 0)];
                    const int rb0 = ldg(R.begin + r);
                    oB[tid] = rb0;
                    np = ldg(R.end + r) - rb0;
                }
            }
            const int inc = wave_incl_scan(np);
            if (lane == 63) wsum[wv] = inc;
            __syncthreads();
            int pre = 0;
            for (int w = 0; w < wv; ++w) pre += wsum[w];
            oCum[tid] = pre + inc;
            // the op of every 64-point segment's first point: op tid holds the
            // segments that start in [pre + inc - np, pre + inc)
            for (int sg = (pre + inc - np + 63) >> 6; sg < kMxSeg && (sg << 6) < pre + inc; ++sg) segop[sg] = tid;
            __syncthreads();
            const int nopc = min(kMxOps, nops - o0);
            const int tot = __builtin_amdgcn_readfirstlane(oCum[nopc - 1]);
            ptot += tot;
            // Rounds are double-buffered: a round's points are loaded into
            // registers before the previous round is computed and written to
            // the other buffer after it, so one barrier per round publishes
            // the next buffer and retires the current one.
            double px[PPT][DX];
            float pw[PPT];
            auto load_round = [&](int p0) {
                const int cnt = min(RND, tot - p0);
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    // the wave's 64 consecutive points: the op of the first from
                    // the segment table (a search beyond it), the rest by a short walk
                    const int j0 = 64 * kMxWaves * k + 64 * wv, jj = j0 + lane;
                    pw[k] = -1.0f;  // no point
#pragma unroll
                    for (int c = 0; c < DX; ++c) px[k][c] = 0.0;
                    if (j0 < cnt) {
                        int lo = 0, hi = nopc - 1;  // first op with oCum > p0 + j0
                        if (((p0 + j0) >> 6) < kMxSeg) {
                            lo = segop[(p0 + j0) >> 6];  // RND and p0 are multiples of 64
                        } else {
                            while (lo < hi) {
                                const int mid = (lo + hi) >> 1;
                                if (oCum[mid] > p0 + j0) hi = mid;
                                else lo = mid + 1;
                            }
                        }
                        if (jj < cnt) {
                            const int p = p0 + jj;
                            int op = lo;
                            while (oCum[op] <= p) ++op;
                            const int row = oB[op] + p - (op ? oCum[op - 1] : 0);
#pragma unroll
                            for (int c = 0; c < DX; ++c)
                                if (c < d) px[k][c] = ldg(R.x + (size_t)row * d + c);
                            pw[k] = R.w ? (float)ldg(R.w + row) : 1.0f;
                        }
                    }
                }
            };
            auto store_round = [&](int buf, int p0) {
                if constexpr (PACK) {  // the kept points at the front of the wave's region
                    const int j0 = 64 * wv;
                    bool keep = pw[0] >= 0.0f;
                    double bk[DX];
                    double nb = 0.0, gap = 0.0;  // |b|^2, squared distance to the leaf box
#pragma unroll
                    for (int c = 0; c < DX; ++c) {
                        bk[c] = 0.0;
                        if (c < d && keep) {
                            bk[c] = (px[0][c] - qc[c]) * sig;
                            nb = fma(bk[c], bk[c], nb);
                            const double o = fmax(0.0, fabs(bk[c]) - sHw[c]);
                            gap = fma(o, o, gap);
                        }
                    }
                    keep = keep && gap <= win * win;
                    const unsigned long long m = __ballot(keep);
                    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                    const int nk = __popcll(m), nk16 = (nk + 15) & ~15;
                    if (keep) {
                        const double nl = mx_log2w(pw[0]) - nb;
#pragma unroll
                        for (int c = 0; c < K; ++c) sB[buf][c][j0 + rank] = c < d ? 2.0 * bk[c] : (c == d ? nl : 0.0);
                    }
                    if (lane >= nk && lane < nk16) {  // zero-weight padding of the last block
#pragma unroll
                        for (int c = 0; c < K; ++c) sB[buf][c][j0 + lane] = c == d ? kMxZeroRow : 0.0;
                    }
                    if (lane == 0) sCnt[buf][wv] = nk16;
                    return;
                }
                const int cntp = (min(RND, tot - p0) + 15) & ~15;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    const int jj = 64 * kMxWaves * k + 64 * wv + lane;
                    if (jj >= cntp || jj >= RND) continue;
                    double bk[DX];
                    double nb = 0.0;
                    float w = pw[k] < 0.0f ? 0.0f : pw[k];
#pragma unroll
                    for (int c = 0; c < DX; ++c) {
                        bk[c] = 0.0;
                        if (c < d && pw[k] >= 0.0f) {
                            bk[c] = (px[k][c] - qc[c]) * sig;
                            nb = fma(bk[c], bk[c], nb);
                        }
                    }
                    if (nb > bcut) {  // a zero term
                        w = 0.0f;
                        nb = 0.0;
#pragma unroll
                        for (int c = 0; c < DX; ++c) bk[c] = 0.0;
                    }
                    const double nl = mx_log2w(w) - nb;
#pragma unroll
                    for (int c = 0; c < K; ++c) sB[buf][c][jj] = (T)(c < d ? 2.0 * bk[c] : (c == d ? nl : 0.0));
                }
            };
            load_round(0);
            store_round(0, 0);
            __syncthreads();
            int buf = 0;
            for (int p0 = 0; p0 < tot; p0 += RND, buf ^= 1) {
                // 16-point blocks of the round; the FP64 form's lie in the
                // waves' regions, nbw[w] of them from 64 w on
                int nbw[kMxWaves], nrb;
                if constexpr (PACK) {
                    nrb = 0;
#pragma unroll
                    for (int w = 0; w < kMxWaves; ++w) {
                        nbw[w] = __builtin_amdgcn_readfirstlane(sCnt[buf][w] >> 4);
                        nrb += nbw[w];
                    }
                } else {
                    nrb = (min(RND, tot - p0) + 15) >> 4;
                }
                const bool more = p0 + RND < tot;
                if (more) load_round(p0 + RND);
                // the wave's blocks of the round against its NB query blocks:
                // all NB products are issued before their exponentials
                auto blocks = [&](auto nbc) {
                    constexpr int NB = decltype(nbc)::value;
                    for (int rb = phase; rb < nrb; rb += stride) {
                        int j = 16 * rb + col;
                        if constexpr (PACK) {
                            int r = rb, w = 0;
                            bool found = false;
#pragma unroll
                            for (int q = 0; q < kMxWaves - 1; ++q) {
                                if (!found && r >= nbw[q]) {
                                    r -= nbw[q];
                                    w = q + 1;
                                } else {
                                    found = true;
                                }
                            }
                            j = 64 * w + 16 * r + col;
                        }
                        T bv[NC];
#pragma unroll
                        for (int c = 0; c < NC; ++c) bv[c] = sB[buf][4 * c + g][j];
                        VT t[NB];
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            t[b] = Cf[b];
#pragma unroll
                            for (int c = 0; c < NC; ++c) t[b] = V::mfma(Af[b][c], bv[c], t[b]);
                        }
#pragma unroll
                        for (int b = 0; b < NB; ++b)
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                acc[b][r] += __builtin_amdgcn_exp2f((float)t[b][r]);
                        if (++nblk == 64) {
                            flush();
                            nblk = 0;
                        }
                    }
                };
                switch (nvb) {
                case 1: blocks(std::integral_constant<int, 1>{}); break;
                case 2: blocks(std::integral_constant<int, 2>{}); break;
                case 3: blocks(std::integral_constant<int, 3>{}); break;
                default: blocks(std::integral_constant<int, 4>{}); break;
                }
                if (more) store_round(buf ^ 1, p0 + RND);
                __syncthreads();  // the next buffer is written, this one read
            }
        }
        flush();
        __syncthreads();
        if (tid < nqs) {  // the sums of the waves of the query's set, in wave order
            int s = 0;
            while ((s + 1) * nqb / nsets <= (tid >> 4)) ++s;
            const int lq = tid - 16 * (s * nqb / nsets);
            double sum = 0.0;
            for (int w = s; w < kMxWaves; w += nsets) sum += sQ[w][lq];
            GE[(size_t)jb.qoff + qb0 + qs + tid] = sum;
        }
        if (tid == 0 && npairs) atomicAdd(npairs, (unsigned long long)(nqs * ptot));
    }
}

// The four forms: FP32 or FP64 products, one or two operand chunks (D <= 3,
// D <= 7).  The FP64 form with one chunk is held to 128 VGPRs (four waves per
// SIMD; its few spills sit outside the block loop), with two chunks to 168
// (three waves instead of two; its spills sit outside the loops too).
#define DFGT_MX_ARGS                                                                                             \
    const DevTree *__restrict__ trees, const Job *__restrict__ jobs, const Group *__restrict__ egrp,             \
        const int *__restrict__ eops, const int *__restrict__ headE, const int *__restrict__ cnt_dev,            \
        const int *__restrict__ overflow, const ItemRec *__restrict__ irec,                                     \
        const int *__restrict__ order, int nitems, int sel, const int2 *__restrict__ ehdr,                       \
        const int2 *__restrict__ eglist, unsigned long long *__restrict__ npairs, double *__restrict__ GE
#define DFGT_MX_PASS trees, jobs, egrp, eops, headE, cnt_dev, overflow, irec, order, nitems, sel, ehdr, eglist, npairs, GE
__global__ __launch_bounds__(64 * kMxWaves) void k_etile_mx32_1(DFGT_MX_ARGS) {
    etile_mx_body<float, 1>(DFGT_MX_PASS);
}
__global__ __launch_bounds__(64 * kMxWaves) void k_etile_mx32_2(DFGT_MX_ARGS) {
    etile_mx_body<float, 2>(DFGT_MX_PASS);
}
__global__ __launch_bounds__(64 * kMxWaves) __attribute__((amdgpu_waves_per_eu(4))) void k_etile_mx64_1(DFGT_MX_ARGS) {
    etile_mx_body<double, 1>(DFGT_MX_PASS);
}
__global__ __launch_bounds__(64 * kMxWaves) __attribute__((amdgpu_waves_per_eu(3))) void k_etile_mx64_2(DFGT_MX_ARGS) {
    etile_mx_body<double, 2>(DFGT_MX_PASS);
}
#undef DFGT_MX_ARGS
#undef DFGT_MX_PASS

// Leave-one-out sums of every query leaf with itself, before the traversal:
// for each query i of the leaf, sum_{j in leaf, j != i} e^{-|x_i - x_j|^2 / 2h^2}
// in FP64 (and with GR the X_E and Y_E parts, in the exhaustive tiles' units).
// Their minimum over the leaf, scaled by (1 - 1e-12) against rounding, is a
// lower bound on every leave-one-out sum of the leaf (the other parts are
// >= 0): the traversal's G^l for the leaf's segments, where the bounds from
// box distances are weak (in high dimensions they underflow).  When the
// leaf's pair with itself ends exhaustive, k_leaf adds these sums (the pair
// is not listed as an exhaustive op).  One block per (job, query leaf), one
// thread per query; jobs without leave-one-out return at once.
template <bool GR>
__global__ __launch_bounds__(256) void k_selfpre(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                                 const ItemRec *__restrict__ irec,
                                                 double *__restrict__ selfG, double *__restrict__ selfX,
                                                 double *__restrict__ selfY, double *__restrict__ selfmin) {
    __shared__ double red[256];
    const ItemRec ir = irec[blockIdx.x];
    const Job jb = jobs[ir.job];
    if (!jb.loo) return;
    const DevTree &Q = trees[jb.qt];
    const int leaf = ir.leaf;
    const int qb = ir.qb0, nq = ir.nq, d = Q.d;
    const double sig = jb.sig;
    double mn = INFINITY;
    for (int i = threadIdx.x; i < nq; i += blockDim.x) {
        const double *xi = Q.x + (size_t)(qb + i) * d;
        double acc = 0.0, xacc = 0.0, yacc[kMaxD];
        if (GR)
            for (int c = 0; c < d; ++c) yacc[c] = 0.0;
        for (int j = 0; j < nq; ++j) {
            if (j == i) continue;
            const double *xj = Q.x + (size_t)(qb + j) * d;
            double t = 0.0, dd[kMaxD];
            for (int c = 0; c < d; ++c) {
                dd[c] = xi[c] * sig - xj[c] * sig;
                t = fma(dd[c], dd[c], t);
            }
            const double e = exp(-t * kLn2);
            acc += e;
            if (GR) {
                xacc = fma(-2.0 * kLn2 * t, e, xacc);
                for (int c = 0; c < d; ++c) yacc[c] = fma(-2.0 * kSqrtLn2 * e, dd[c], yacc[c]);
            }
        }
        const size_t ei = (size_t)jb.qoff + qb + i;
        selfG[ei] = acc;
        if (GR) {
            selfX[ei] = xacc;
            for (int c = 0; c < d; ++c) selfY[ei * d + c] = yacc[c];
        }
        mn = fmin(mn, acc);
    }
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) selfmin[(size_t)jb.noff + leaf] = nq > 1 ? red[0] * (1.0 - 1e-12) : 0.0;
}

// ---------------------------------------------------------------- exhaustive tiles on the matrix cores
// D >= 8, mixed precision (see etile.h).  One block of 4 waves per (query
// leaf, job): the leaf's E chain is flattened 256 ops at a time (in parallel,
// with a block-wide scan of their 16-point block counts); the waves take the
// reference blocks round-robin and hold up to 4 query blocks of 16 as MFMA
// fragments (larger leaves repeat the walk per group of 64 queries).  Per
// query (tree order) it writes G_E = sum e, and with GR also X_E and Y_E (the
// quantities k_leaf defines) to GE, GX, GY, which k_leaf adds to the rest.
// Groups flagged by the underflow guard are left to the FP64 pass of k_etile,
// which adds their sums afterwards.
template <bool GR, int NC>
__global__ __launch_bounds__(256) void k_emfma(const DevTree *__restrict__ trees, const Job *__restrict__ jobs,
                                               const Group *__restrict__ egrp, const int *__restrict__ eops,
                                               const int *__restrict__ headE, const int *__restrict__ overflow,
                                               const ItemRec *__restrict__ irec,
                                               double *__restrict__ GE, double *__restrict__ GX,
                                               double *__restrict__ GY) {
    constexpr int NT = (NC + 3) / 4;  // 16-dimension tiles of the gradient product
    __shared__ int gS[kMaxEGrp], gC[kMaxEGrp], gF[kMaxEGrp], gCum[kMaxEGrp];
    __shared__ int oB[kEChunk], oN[kEChunk], oCum[kEChunk];
    __shared__ int wsum[4], ngrp_s, nops_s;
    __shared__ double red[4][2][64];
    __shared__ double redY[GR ? 4 * NT * 256 : 1];
    if (*overflow) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4;
    const ItemRec ir = irec[blockIdx.x];
    const Job jb = jobs[ir.job];
    const DevTree &Q = trees[jb.qt];
    const DevTree &R = trees[jb.rt];
    const int leaf = ir.leaf;
    const int d = Q.d;
    const int qb0 = ir.qb0, nq = ir.nq;
    const size_t hq = (size_t)jb.noff + leaf;
    // fragments and norms are scaled on load (q' = sig q, |q'|^2 = sig^2 |q|^2),
    // so t = |q'|^2 + |r'|^2 - 2 q'.r' is the exponent of e = 2^-t directly
    const double sig = jb.sig, sc2 = sig * sig;
    if (tid == 0) {
        int n = 0, tot = 0;
        for (int gi = headE[hq]; gi >= 0 && n < kMaxEGrp; gi = egrp[gi].next) {
            const Group gg = egrp[gi];
            gS[n] = gg.start;
            gC[n] = gg.count;
            gF[n] = gg.flags;
            tot += gg.count;
            gCum[n++] = tot;
        }
        ngrp_s = n;
        nops_s = tot;
    }
    __syncthreads();
    const int nops = nops_s;
    for (int qg = 0; qg < nq; qg += 64) {
        double qf[4][NC], qnv[4];
        bool qok[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int nv = min(16, nq - qg - 16 * b);
            qok[b] = nv > 0;
            if (qok[b]) {
                load_frag<NC>(Q.x, qb0 + qg + 16 * b, nv, d, qf[b]);
#pragma unroll
                for (int c = 0; c < NC; ++c) qf[b][c] *= sig;
                qnv[b] = Q.nrm[qb0 + qg + 16 * b + min(lane & 15, nv - 1)] * sc2;
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) qf[b][c] = 0.0;
                qnv[b] = 0.0;
            }
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0}, at[4] = {0.0, 0.0, 0.0, 0.0};
        float ps[4] = {0.0f, 0.0f, 0.0f, 0.0f}, pt[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        v4d accY[4][NT];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) accY[b][nt] = v4d{0.0, 0.0, 0.0, 0.0};
        int nblk = 0;
        for (int o0 = 0; o0 < nops; o0 += kEChunk) {
            __syncthreads();
            // flatten ops o0 .. o0 + 255: reference range and 16-point block count
            const int o = o0 + tid;
            int nb = 0;
            if (o < nops) {
                int gi = 0;
                while (o >= gCum[gi]) ++gi;
                if (gF[gi] == 0) {  // groups flagged by the underflow guard go to the FP64 pass
                    const int r = eops[gS[gi] + o - (gi ? gCum[gi - 1] : 0)];
                    const int rb = R.begin[r], rn = R.end[r] - rb;
                    oB[tid] = rb;
                    oN[tid] = rn;
                    nb = (rn + 15) >> 4;
                }
            }
            const int inc = wave_incl_scan(nb);
            if (lane == 63) wsum[wv] = inc;
            __syncthreads();
            int pre = 0;
            for (int w = 0; w < wv; ++w) pre += wsum[w];
            oCum[tid] = pre + inc;
            __syncthreads();
            const int nopc = min(kEChunk, nops - o0);
            const int tb = oCum[nopc - 1];
            // The wave's reference blocks are software-pipelined: the next
            // block's fragment, norms and (GR) gradient operand are loaded
            // while the current one is computed.
            int op = 0;
            double nrf[NC], nrnv[4], nb2[NT][4];
            float nrw[4];
            int nnv = 0;
            auto fetch = [&](int blk) {
                while (blk >= oCum[op]) ++op;
                const int lb = blk - (op ? oCum[op - 1] : 0);
                const int r0 = oB[op] + 16 * lb;
                nnv = min(16, oN[op] - 16 * lb);
                load_frag<NC>(R.x, r0, nnv, d, nrf);
#pragma unroll
                for (int k = 0; k < 4; ++k) nrnv[k] = R.nrm[r0 + min(4 * k + g, nnv - 1)];
#pragma unroll
                for (int k = 0; k < 4; ++k) nrw[k] = R.w ? (float)R.w[r0 + min(4 * k + g, nnv - 1)] : 1.0f;
                if (GR) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int c2 = 0; c2 < 4; ++c2) {
                            const int row = r0 + min(4 * c2 + g, nnv - 1), dim = 16 * nt + (lane & 15);
                            nb2[nt][c2] = dim < d ? R.x[(size_t)row * d + dim] : 0.0;
                        }
                }
            };
            if (wv < tb) fetch(wv);
            for (int blk = wv; blk < tb; blk += 4) {
                const int nv = nnv;
                double rf[NC], rnv[4], b2[NT][4];
                float rw[4];
#pragma unroll
                for (int c = 0; c < NC; ++c) rf[c] = nrf[c] * sig;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    rnv[k] = nrnv[k] * sc2;
                    rw[k] = 4 * k + g < nv ? nrw[k] : 0.0f;  // weight 0 past the block's end
                }
                if (GR) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int c2 = 0; c2 < 4; ++c2) b2[nt][c2] = nb2[nt][c2];
                }
                if (blk + 4 < tb) fetch(blk + 4);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (!qok[b]) continue;
                    const v4d dt = block_dots<NC>(rf, qf[b]);
                    double ev[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float t = fmaxf((float)fma(-2.0, dt[k], qnv[b] + rnv[k]), 0.0f);
                        const float e = rw[k] * __builtin_amdgcn_exp2f(-t);
                        // gradient mode: the sum of the kernel values multiplies x_q
                        // in Y = x_q sum e - sum e x_r, so it is taken in FP64 like
                        // the matrix-core sums of e x_r (FP32 partials would leave a
                        // mismatch amplified by |x_q| / |q - r|)
                        if (GR) acc[b] += (double)e;
                        else ps[b] += e;
                        if (GR) pt[b] = fmaf(t, e, pt[b]);
                        ev[k] = (double)e;
                    }
                    if (GR) {
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                            for (int c2 = 0; c2 < 4; ++c2)
                                accY[b][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ev[c2], b2[nt][c2], accY[b][nt],
                                                                                   0, 0, 0);
                    }
                }
                if (++nblk == 16) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[b] += (double)ps[b];
                        ps[b] = 0.0f;
                        at[b] += (double)pt[b];
                        pt[b] = 0.0f;
                    }
                    nblk = 0;
                }
            }
        }
        // this query group: lane groups, then waves, in a fixed order
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double v = acc[b] + (double)ps[b], vt = at[b] + (double)pt[b];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            vt += __shfl_xor(vt, 16, 64);
            vt += __shfl_xor(vt, 32, 64);
            if (g == 0) {
                red[wv][0][16 * b + lane] = v;
                red[wv][1][16 * b + lane] = vt;
            }
        }
        if (GR) {
            for (int w = 0; w < 4; ++w) {
                if (wv == w) {
#pragma unroll
                    for (int b = 0; b < 4; ++b)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                double &dst = redY[(b * NT + nt) * 256 + r * 64 + lane];
                                dst = w == 0 ? accY[b][nt][r] : dst + accY[b][nt][r];
                            }
                }
                __syncthreads();
            }
        } else {
            __syncthreads();
        }
        if (tid < 64 && qg + tid < nq) {
            const int pos = qb0 + qg + tid;
            const double ge = ((red[0][0][tid] + red[1][0][tid]) + red[2][0][tid]) + red[3][0][tid];
            GE[(size_t)jb.qoff + pos] = ge;
            if (GR) {
                const double gt = ((red[0][1][tid] + red[1][1][tid]) + red[2][1][tid]) + red[3][1][tid];
                GX[(size_t)jb.qoff + pos] = -2.0 * kLn2 * gt;
                const int b = tid >> 4, i = tid & 15;
                const double *xq = Q.x + (size_t)pos * d;
                for (int k = 0; k < d; ++k) {
                    const double sy = redY[(b * NT + (k >> 4)) * 256 + (i >> 2) * 64 + 16 * (i & 3) + (k & 15)];
                    GY[((size_t)jb.qoff + pos) * d + k] = -2.0 * jb.s * fma(xq[k], ge, -sy);
                }
            }
        }
        __syncthreads();
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
        for (int k = 0; k < 6; ++k) {
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

// kernel_ms slots of dfgt_stats
enum { K_TRAV = 0, K_LEAF = 1, K_EMFMA = 2, K_LOCAL = 3, K_EF64 = 4, K_MX32 = 5 };

struct Workspace {
    DevBuf jobs, trees, jls, L, lflag, heads, segA, segB, pairA, pairB, dec, kus, egrp, eops, fgrp, fops, lgrp, lops,
        lnodes, stats, lscr, pscr, lopnode, part, extE, extX, extY, stG, stX, stQ, cval, gdg, gmt, eord, ehdr,
        eglist, irec, selfE, selfG, selfX, selfY, selfmin;
    // overflow flag, counters and per-level counts in one allocation: one fill,
    // one copy back
    DevBuf ctl;
    // set when any part of the call overflowed (cleared by the first part only)
    DevBuf sticky;
    DevSpan flag, cnt, lvl;
    // pinned staging of the plan upload and the read back; the upload's
    // copies are complete once `upev` has been reached
    HostBuf up, back;
    hipEvent_t upev = nullptr;
    Caps cap{0, 0, 0, 0, 0, 0, 0};
    int part_jobs = 0;  // jobs per part learned from the last split (0 = none yet)
    size_t part_budget = 0;  // the memory budget part_jobs was learned under
    double part_ipj = 0.0;   // (query leaf) items per job of the plan it was learned on
    // the exhaustive tiles run on a side stream beside the local-moment ops
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    dfgt_status ensure_side() {
        if (side) return DFGT_OK;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
            set_error("creating the side stream failed");
            return DFGT_EHIP;
        }
        return DFGT_OK;
    }
    ~Workspace() {
        if (upev) (void)hipEventDestroy(upev);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
    }
};
thread_local Workspace g_ws;

template <class T> dfgt_status grow(DevBuf &b, size_t n) { return b.reserve(sizeof(T) * std::max<size_t>(n, 1)); }

constexpr int kTravGrid = 8192;  // waves per traversal level (grid-stride over segments)
constexpr int kLocalGrid = 2048;

template <bool GR>
void launch_emfma(int nc, dim3 grid, hipStream_t st, const DevTree *td, const Job *jd, const Group *egrp,
                  const int *eops, const int *headE, const int *flag, const ItemRec *irec, double *GE,
                  double *GX, double *GY) {
#define DFGT_EMFMA(NCV)                                                                                     \
    hipLaunchKernelGGL((k_emfma<GR, NCV>), grid, dim3(256), 0, st, td, jd, egrp, eops, headE, flag, irec, GE, \
                       GX, GY);                                                                             \
    break;
    switch (nc) {
    case 2: DFGT_EMFMA(2)
    case 3: DFGT_EMFMA(3)
    case 4: DFGT_EMFMA(4)
    case 5: DFGT_EMFMA(5)
    case 6: DFGT_EMFMA(6)
    case 7: DFGT_EMFMA(7)
    default: DFGT_EMFMA(8)
    }
#undef DFGT_EMFMA
}

// sel (mixed pass only): 0 = every item in k_eorder's order, 1 = only the
// items it listed as wide (the rest taken by k_etile_mx).
template <bool GR>
void launch_etile(bool f64pass, int d, int nitems, hipStream_t st, const DevTree *td, const Job *jd,
                  const Group *egrp, const int *eops, const int *headE, const int *cnt, const int *flag,
                  const ItemRec *irec, int precision, const int *order, int sel, double *GE, double *GX,
                  double *GY) {
    const dim3 grid((unsigned)nitems);
#define DFGT_ETILE(DV)                                                                                            \
    if (f64pass) {                                                                                                \
        hipLaunchKernelGGL((k_etile<DV, GR, true>), grid, dim3(64 * kEWaves), 0, st, td, jd, egrp, eops, headE, cnt, flag, \
                           irec, precision, (const int *)nullptr, nitems, 0, GE, GX, GY);                          \
    } else if constexpr (DV == 3 && !GR) {                                                                        \
        hipLaunchKernelGGL((k_etile_o4<DV, GR, false>), grid, dim3(64 * kEWaves), 0, st, td, jd, egrp, eops, headE, cnt,   \
                           flag, irec, precision, order, nitems, sel, GE, GX, GY);                                \
    } else {                                                                                                      \
        hipLaunchKernelGGL((k_etile<DV, GR, false>), grid, dim3(64 * kEWaves), 0, st, td, jd, egrp, eops, headE, cnt,      \
                           flag, irec, precision, order, nitems, sel, GE, GX, GY);                                \
    }                                                                                                             \
    break;
    switch (d) {
    case 1: DFGT_ETILE(1)
    case 2: DFGT_ETILE(2)
    case 3: DFGT_ETILE(3)
    case 4: DFGT_ETILE(4)
    case 5: DFGT_ETILE(5)
    default: DFGT_ETILE(0)
    }
#undef DFGT_ETILE
}

// Everything about a call that does not depend on the traversal's output
// sizes: the job and tree tables and the launch shapes.
struct Plan {
    std::vector<Job> jobs;
    std::vector<DevTree> trees;
    std::vector<int> jls;  // per-job prefix of (job, query leaf) items
    int njobs = 0, nlev = 0, d = 0, pmax = 0, P = 0, PW = 0, precision = 0, force = 0, items = 0;
    bool gr = false, leaf_local = true, emfma = false, acc_lds = true, dig_lds = true, loo = false;
    size_t nna = 0, nqa = 0;  // node slots and query slots over all jobs
    int leaf_threads = 256, lop_waves = 4;
    size_t leaf_sh = 0, lop_sh = 0, big_sh = 0;
    size_t job_off = 0, jls_off = 0;  // where this plan's tables sit in the device arrays
    int unl = 0;                      // items per job when all jobs share one query leaf count, else 0
};

int uniform_leaves(const Plan &pl) {
    int u = -1;
    for (const Job &j : pl.jobs) {
        const int nl = pl.trees[j.qt].nleaves;
        if (u < 0) u = nl;
        else if (u != nl) return 0;
    }
    return u > 0 ? u : 0;
}

// Jobs [j0, j1) of a plan as a plan of their own (jobs are independent).
Plan sub_plan(const Plan &pl, int j0, int j1) {
    Plan sp = pl;
    sp.jobs.assign(pl.jobs.begin() + j0, pl.jobs.begin() + j1);
    sp.njobs = j1 - j0;
    sp.jls.assign(1, 0);
    long long nna = 0, nqa = 0, items = 0;
    for (Job &j : sp.jobs) {
        const DevTree &Q = pl.trees[j.qt];
        j.noff = nna;
        j.qoff = nqa;
        nna += Q.m;
        nqa += Q.n;
        items += Q.nleaves;
        sp.jls.push_back((int)items);
    }
    sp.nna = (size_t)nna;
    sp.nqa = (size_t)nqa;
    sp.items = (int)items;
    sp.job_off = sp.jls_off = 0;
    sp.unl = uniform_leaves(sp);
    return sp;
}

// Device bytes alloc_plan needs for a plan at the given capacities.
size_t plan_bytes(const Plan &pl, const Caps &c) {
    size_t b = pl.nna * (sizeof(double) * pl.PW + 1 + sizeof(double) + 3 * sizeof(int));
    if (pl.emfma) b += pl.nqa * sizeof(double) * (pl.gr ? 2 + pl.d : 1);
    b += (size_t)c.seg * 2 * sizeof(Seg) + (size_t)c.pair * (3 * sizeof(int) + sizeof(double));
    b += (size_t)c.grp * (3 * sizeof(Group) + sizeof(int2)) + (size_t)c.lnode * 2 * sizeof(int) +
         (size_t)c.eop * sizeof(int);
    b += (size_t)pl.items * (6 * sizeof(int) + sizeof(int2) + sizeof(ItemRec));
    b += (size_t)c.fop * sizeof(Op) + (size_t)c.lop * sizeof(Op);
    if (pl.leaf_local) b += (size_t)c.lop * (sizeof(int) + sizeof(double) * pl.PW);
    if (!pl.acc_lds) b += (size_t)pl.items * 3 * pl.PW * sizeof(double);
    return b;
}

// Rounding of the exhaustive sums with FP32 coordinate differences, per term
// K = 2^-t, t = |a - b|^2, where a = (q - c) sig and b = (r - c) sig are rounded
// to FP32 (c the query leaf's centre, u = 2^-24): each staged coordinate
// carries u |a_k| (u |b_k|), each difference u |a_k - b_k| more, and the
// FP32 sum of D squares D u t, so to first order
//     |dt| <= u ((D + 2) t + 2 |a - b| (|a| + |b|)).
// Terms that matter have t <= 126 (smaller ones flush, the underflow guard's
// share), so the relative error of a term is at most
//     ln2 u ((D + 2) 126 + 2 sqrt(126) A) + 2^-22 (exp2) + u (the weight),
// A = max |a| + |b| over the pairs, plus 63 u for FP32 partial sums of <= 64
// positive terms.  Returns the largest A that keeps the total within
// eps_round (<= 0: none).
double etile_a32(double eps_round, int d) {
    const double u = 0x1p-24, ln2 = 0.69314718055994530942;
    const double rest = eps_round - 0x1p-22 - 64.0 * u;
    const double a = (rest / (ln2 * u) - (d + 2) * 126.0) / (2.0 * std::sqrt(126.0));
    return a > 0.0 ? a : 0.0;
}

// Share of the rounding budget of the mixed exhaustive sums given to the
// references the matrix-core tiles leave out when G(q) >= 1.
constexpr double kMxDropShare = 1.0 / 50.0;

// Staging window (sig units) of the matrix-core tiles: with G(q) >= 1 (the
// self term of a monochromatic, unweighted sum) the at most n_r left-out
// terms, each below 2^-W^2, stay within eps_round kMxDropShare of G(q) when
// W^2 = log2(n_r / (eps_round kMxDropShare)); otherwise kMxNear32.
double mx_window(double eps_round, bool g_ge_1, double n_r) {
    if (!g_ge_1 || !(eps_round > 0.0)) return kMxNear32;
    const double w = std::sqrt(std::log2(std::max(n_r, 1.0) / (eps_round * kMxDropShare)));
    return std::min(w, kMxNear32);
}

// Largest query-leaf half-diagonal rho (sig units) for the FP32 products of
// the matrix-core tiles with staging window win: their staged pairs have
// |a| + |b| <= A = 2 rho + win, t moves by at most 6.5 u A^2 (u = 2^-24:
// operand roundings and four FP32 multiply-adds), and a term's relative
// error ln2 6.5 u A^2 + 2^-22 (exp2) + u (the weight), plus 67 u for the FP32
// partial sums (63 within a lane, 4 across the lanes of a row), plus the
// left-out terms' share when win < kMxNear32, must stay within eps_round.
// A weighted tree adds log2 w (|log2 w| <= 126) to the -|b|^2 row before it
// is rounded: ln2 126 u more.  Returns 0 when no rho > 0 does (FP64
// products).
double mx_r32(double eps_round, double win, bool weighted) {
    const double u = 0x1p-24, ln2 = 0.69314718055994530942;
    const double rest = eps_round - 0x1p-22 - 68.0 * u - (win < kMxNear32 ? eps_round * kMxDropShare : 0.0) -
                        (weighted ? ln2 * 126.0 * u : 0.0);
    if (rest <= 0.0) return 0.0;
    const double r = 0.5 * (std::sqrt(rest / (6.5 * ln2 * u)) - win);
    return r > 0.0 ? r : 0.0;
}

// Memory one call may size its traversal buffers to before it splits its jobs:
// a quarter of the device's memory, at least 1 GiB.  It depends on the device
// only, so repeated calls split the same way (a budget that followed the free
// memory changed as the workspace grew, and every change re-learnt the split
// with reruns).  An allocation that fails splits the jobs as well.
// DFGT_MEMORY_BUDGET_MB, when set to a positive number, replaces it (no
// floor): a test knob that forces the split into parts on small inputs.
size_t memory_budget() {
    if (const char *ev = std::getenv("DFGT_MEMORY_BUDGET_MB")) {
        const long long mb = std::atoll(ev);
        if (mb > 0) return (size_t)mb << 20;
    }
    static size_t total = 0;
    if (total == 0) {
        size_t fr = 0, tot = 0;
        total = hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0 ? tot : ((size_t)64 << 30);
    }
    return std::max<size_t>((size_t)1 << 30, total / 4);
}

dfgt_status make_plan(const Problem *pr, int np, double eps, int precision, int force, double cost_e,
                      const GradOut *grad, Plan &pl) {
    const dfgt_tree_s *t0 = pr[0].Q;
    pl.d = t0->d;
    pl.pmax = t0->pmax;
    pl.P = t0->P;
    pl.gr = grad != nullptr;
    pl.PW = pl.gr ? 2 * pl.P : pl.P;
    pl.force = force;
    // A tolerance below the mixed-precision rounding budget needs FP64 leaf sums.
    if (precision == DFGT_PREC_MIXED && eps > 0.0 && eps < 2e-5) precision = DFGT_PREC_FP64;
    pl.precision = precision;
    // Rounding budget of the exhaustive sums (the global-error theorem takes
    // them as exact): FP64 ~1e-13; mixed precision 1e-5 relative, or 1e-4 when
    // eps >= 2e-3 (then FP32 coordinate differences fit in it for nearby
    // leaves, see etile_a32).
    const double eps_round = precision == DFGT_PREC_FP64 ? 1e-12 : (eps >= 2e-3 ? 1e-4 : 1e-5);
    const double eps_eff = eps > 2.0 * eps_round ? eps - eps_round : 0.0;
    const double a32 = precision == DFGT_PREC_MIXED && grad == nullptr ? etile_a32(eps_round, t0->d) : 0.0;
    const bool mxr = precision == DFGT_PREC_MIXED && grad == nullptr;  // FP32 products possible
    // a query leaf's own local ops are applied inside k_leaf when its per-wave
    // scratch fits; otherwise they go through the node kernels
    pl.leaf_local = pl.P <= 512;
    // Cost of a unit of each summarisation method relative to one exhaustive
    // pair on this GPU.  calibrate_costs.py times forced-method calls with HIP
    // events over their work counters: far-field evaluation 1.9-5.7 per query x
    // coefficient, direct local accumulation 4.2-7.0 per point x coefficient
    // for p_max^D <= 512 (D = 2, 3, 5); with larger coefficient vectors (the
    // global-memory local-op kernel) 26, 163 and 23 for translation.  Those
    // per-unit times include fixed costs that do not scale with the work, and
    // whole-workload timings (2-D sweep, 3-D batch, 5-D at orders 2 and 6)
    // are fastest at about half the small-vector figures and twice the large
    // ones.  Any weights keep the error guarantee: they only choose among
    // methods whose bounds hold.
    const double wF = pl.leaf_local ? 2.0 : 50.0, wD = pl.leaf_local ? 3.0 : 320.0,
                 wT = pl.leaf_local ? 3.0 : 50.0;
    if (pl.gr && !pl.leaf_local) {
        set_error("dfgt_gauss_sum_grad: gradients need p_max^d <= 512");
        return DFGT_EINVAL;
    }
    std::vector<const dfgt_tree_s *> th;
    auto tree_index = [&](const dfgt_tree_s *t) {
        for (size_t i = 0; i < th.size(); ++i)
            if (th[i] == t) return (int)i;
        th.push_back(t);
        return (int)th.size() - 1;
    };
    pl.jls.assign(1, 0);
    long long nna = 0, nqa = 0, items = 0;
    for (int ip = 0; ip < np; ++ip) {
        const Problem &q = pr[ip];
        if (q.Q->depth > kMaxDepth) {
            set_error("dfgt_gauss_sum: query tree deeper than 256 levels");
            return DFGT_EINVAL;
        }
        const int qt = tree_index(q.Q), rt = tree_index(q.R);
        for (int k = 0; k < q.nh; ++k) {
            Job j{};
            j.h = q.h[k];
            j.s = 1.0 / (std::sqrt(2.0) * q.h[k]);
            j.inv2h2 = 1.0 / (2.0 * q.h[k] * q.h[k]);
            j.sig = 1.2011224087864498 * j.s;  // sqrt(log2 e) s: e^{-x^2/2h^2} = 2^{-(sig x)^2}
            j.eps_eff = eps_eff;
            j.nR = q.R->wsum / q.R->wscale;
            j.cntR = (double)q.R->n;
            j.wscale = q.R->wscale;
            const bool loo = q.loo && q.Q == q.R && !q.R->weighted;
            // the self term: G(q) >= 1 (left out of leave-one-out sums)
            j.prior = q.Q == q.R && !q.R->weighted && !loo ? 1.0 : 0.0;
            j.qt = qt;
            j.rt = rt;
            j.qoff = nqa;
            j.noff = nna;
            j.out = q.G + (size_t)k * q.Q->n;
            j.outH = pl.gr && grad->dGdh ? grad->dGdh + (size_t)k * q.Q->n : nullptr;
            j.outQ = pl.gr && grad->dGdq ? grad->dGdq + (size_t)k * q.Q->n * pl.d : nullptr;
            j.cost_e = cost_e;
            j.wF = wF;
            j.wD = wD;
            j.wT = wT;
            j.mono = q.Q == q.R && !q.R->weighted && !loo ? 1 : 0;  // the self term bounds G below by 1
            j.loo = loo ? 1 : 0;
            pl.loo = pl.loo || loo;
            j.a32 = a32;
            j.win = precision == DFGT_PREC_MIXED ? mx_window(eps_round, j.mono != 0, j.cntR) : kMxNear32;
            j.r32 = mxr ? mx_r32(eps_round, j.win, q.R->weighted) : 0.0;
            pl.jobs.push_back(j);
            nna += q.Q->m;
            nqa += q.Q->n;
            items += q.Q->nleaves;
            if (items >= (1LL << 31)) {
                set_error("dfgt_gauss_sum: too many (bandwidth, query leaf) items in one call");
                return DFGT_EINVAL;
            }
            pl.jls.push_back((int)items);
        }
    }
    pl.njobs = (int)pl.jobs.size();
    pl.nna = (size_t)nna;
    pl.nqa = (size_t)nqa;
    pl.items = (int)items;
    for (auto *t : th) {
        pl.trees.push_back(t->host_view);
        // every level splits Q and R wherever they can split, so no pair
        // survives more levels than the deepest tree has
        pl.nlev = std::max(pl.nlev, t->depth);
    }
    // exhaustive leaf sums on the matrix cores: mixed precision, D >= 8, and
    // s^2 (|q|^2 + |r|^2) <= 2^26 for every bandwidth (rounding of the
    // expanded squared distance below ~1e-7)
    if (pl.nlev > kMaxEGrp) {  // an E chain holds at most one group per level
        set_error("dfgt_gauss_sum: trees deeper than 256 levels");
        return DFGT_EINVAL;
    }
    pl.emfma = precision == DFGT_PREC_MIXED && pl.d >= 8 && pl.d <= 32;
    for (const Job &j : pl.jobs) {
        if (!pl.emfma) break;
        pl.emfma = j.sig * j.sig * (th[j.qt]->max_nrm + th[j.rt]->max_nrm) <= 67108864.0;
    }
    pl.unl = uniform_leaves(pl);
    // launch shapes
    const int d = pl.d, pmax = pl.pmax, P = pl.P, PW = pl.PW;
    const int g1 = pl.gr ? 1 : 0;
    if (pl.leaf_local) {
        // waves per block of k_lops: as many (up to 4) as the LDS allows
        const size_t wstride = lop_wave_stride(P, d, pmax, g1);
        int lwv = 4;
        for (;; lwv >>= 1) {
            pl.lop_sh = sizeof(double) * ((size_t)P + (10 * (size_t)P + 7) / 8 + (size_t)lwv * wstride);
            if (pl.lop_sh <= 64 * 1024 || lwv == 1) break;
        }
        if (pl.lop_sh > 64 * 1024) {
            set_error("dfgt_gauss_sum: p_max^d too large for the local-op kernel");
            return DFGT_EINVAL;
        }
        pl.lop_waves = lwv;
    } else {
        pl.big_sh = sizeof(double) * ((size_t)pmax * pmax + 2 * (size_t)d * pmax + 64 * (size_t)d * pmax);
    }
    const int rows = (!g1 && far_fixed_kind(d, pmax)) ? 0 : 1;  // per-thread Hermite rows in LDS
    int nthr = 256;
    while (nthr > 64 && sizeof(double) * leaf_lds_base(nthr, d, pmax, g1, rows) > 40 * 1024) nthr >>= 1;
    const size_t base = sizeof(double) * leaf_lds_base(nthr, d, pmax, g1, rows);
    const size_t lds_dig = (sizeof(unsigned long long) + sizeof(unsigned short)) * (size_t)P;
    const size_t lds_coef = sizeof(double) * (size_t)d * pmax * pmax;
    const size_t lds_acc = sizeof(double) * 3 * (size_t)PW + lds_coef;
    // dynamic LDS up to 56 KB: the kernel's static arrays take ~6 KB of the 64 KB
    pl.acc_lds = base + lds_acc + lds_dig <= 56 * 1024;
    pl.dig_lds = base + (pl.acc_lds ? lds_acc : lds_coef) + lds_dig <= 56 * 1024;
    pl.leaf_sh = base + (pl.acc_lds ? lds_acc : lds_coef) + (pl.dig_lds ? lds_dig : 0);
    pl.leaf_threads = nthr;
    if (pl.leaf_sh > 56 * 1024) {
        set_error("dfgt_gauss_sum: p_max^d too large for the per-leaf kernel");
        return DFGT_EINVAL;
    }
    return DFGT_OK;
}

// Device buffers for the plan and the current capacities (no-op when large enough).
dfgt_status alloc_plan(const Plan &pl, Workspace &w) {
    DFGT_TRY(w.ensure_side());
    const Caps &cap = w.cap;
    const size_t nna = pl.nna;
    DFGT_TRY(grow<Job>(w.jobs, pl.njobs));
    DFGT_TRY(grow<DevTree>(w.trees, pl.trees.size()));
    DFGT_TRY(grow<int>(w.jls, pl.jls.size()));
    DFGT_TRY(grow<double>(w.L, nna * pl.PW));
    DFGT_TRY(grow<unsigned>(w.lflag, (nna + 3) / 4));
    DFGT_TRY(grow<double>(w.cval, nna));
    if (pl.loo) {
        DFGT_TRY(grow<unsigned>(w.selfE, (nna + 3) / 4));
        DFGT_TRY(grow<double>(w.selfmin, nna));
        DFGT_TRY(grow<double>(w.selfG, pl.nqa));
        if (pl.gr) {
            DFGT_TRY(grow<double>(w.selfX, pl.nqa));
            DFGT_TRY(grow<double>(w.selfY, pl.nqa * pl.d));
        }
    }
    DFGT_TRY(grow<int>(w.heads, 3 * nna));
    DFGT_TRY(alloc_spans(w.ctl, {{&w.flag, sizeof(int) * CP},
                                 {&w.cnt, sizeof(int) * C_N * CP},
                                 {&w.lvl, sizeof(int) * (size_t)(pl.nlev + 1) * 2 * CP}}));
    DFGT_TRY(grow<unsigned long long>(w.stats, S_N * SP));
    DFGT_TRY(grow<int>(w.sticky, 64));
    // exhaustive sums per query (k_emfma or k_etile), added by k_leaf
    DFGT_TRY(grow<double>(w.extE, pl.nqa));
    DFGT_TRY(grow<double>(w.stG, pl.nqa));
    DFGT_TRY(grow<int>(w.eord, 6 * (size_t)pl.items));  // dispatch order of the exhaustive tiles
    DFGT_TRY(grow<int2>(w.ehdr, pl.items));                // and each item's flattened E chain
    DFGT_TRY(grow<ItemRec>(w.irec, pl.items));
    DFGT_TRY(grow<int2>(w.eglist, cap.grp));
    if (pl.gr) {
        DFGT_TRY(grow<double>(w.extX, pl.nqa));
        DFGT_TRY(grow<double>(w.extY, pl.nqa * pl.d));
        DFGT_TRY(grow<double>(w.stX, pl.nqa));
        DFGT_TRY(grow<double>(w.stQ, pl.nqa * pl.d));
    }
    DFGT_TRY(grow<Seg>(w.segA, cap.seg));
    DFGT_TRY(grow<Seg>(w.segB, cap.seg));
    DFGT_TRY(grow<int>(w.pairA, cap.pair));
    DFGT_TRY(grow<int>(w.pairB, cap.pair));
    DFGT_TRY(grow<int>(w.dec, cap.pair));
    DFGT_TRY(grow<double>(w.kus, cap.pair));
    DFGT_TRY(grow<Group>(w.egrp, cap.grp));
    DFGT_TRY(grow<Group>(w.fgrp, cap.grp));
    DFGT_TRY(grow<Group>(w.lgrp, cap.grp));
    DFGT_TRY(grow<int>(w.lnodes, 2 * (size_t)cap.lnode));
    DFGT_TRY(grow<int>(w.eops, cap.eop));
    DFGT_TRY(grow<Op>(w.fops, cap.fop));
    DFGT_TRY(grow<Op>(w.lops, cap.lop));
    if (pl.leaf_local) {
        DFGT_TRY(grow<int2>(w.lopnode, cap.lop));  // each local op's owner (node, job)
        DFGT_TRY(grow<double>(w.part, (size_t)cap.lop * pl.PW));
    } else {
        DFGT_TRY(grow<double>(w.lscr, (size_t)kLocalGrid * 3 * pl.P));
    }
    if (!pl.acc_lds) DFGT_TRY(grow<double>(w.pscr, (size_t)pl.items * 3 * pl.PW));
    if (!pl.dig_lds) {
        DFGT_TRY(grow<unsigned long long>(w.gdg, pl.P));
        DFGT_TRY(grow<unsigned short>(w.gmt, pl.P));
    }
    return DFGT_OK;
}

// The plan's tables go through pinned staging (the previous upload's copies
// must have left it first), so the copies do not block the host.
dfgt_status upload_plan(const Plan &pl, Workspace &w, hipStream_t st) {
    const size_t bj = sizeof(Job) * pl.njobs, bt = sizeof(DevTree) * pl.trees.size(),
                 bl = sizeof(int) * pl.jls.size();
    const size_t oj = 0, ot = (bj + 255) / 256 * 256, ol = ot + (bt + 255) / 256 * 256;
    if (!w.upev) DFGT_HIP(hipEventCreateWithFlags(&w.upev, hipEventDisableTiming));
    DFGT_HIP(hipEventSynchronize(w.upev));
    DFGT_TRY(w.up.reserve(ol + bl));
    char *h = w.up.as<char>();
    std::memcpy(h + oj, pl.jobs.data(), bj);
    std::memcpy(h + ot, pl.trees.data(), bt);
    std::memcpy(h + ol, pl.jls.data(), bl);
    DFGT_HIP(hipMemcpyAsync(w.jobs.as<Job>() + pl.job_off, h + oj, bj, hipMemcpyHostToDevice, st));
    DFGT_HIP(hipMemcpyAsync(w.trees.p, h + ot, bt, hipMemcpyHostToDevice, st));
    DFGT_HIP(hipMemcpyAsync(w.jls.as<int>() + pl.jls_off, h + ol, bl, hipMemcpyHostToDevice, st));
    DFGT_HIP(hipEventRecord(w.upev, st));
    return DFGT_OK;
}

// Several fills in one launch: region r is words[r] u32 values v[r] at p[r];
// block b takes the kFillChunk words from b * kFillChunk of the regions laid
// end to end.
constexpr int kFillN = 8, kFillChunk = 4096;
struct FillSet {
    unsigned *p[kFillN];
    unsigned long long words[kFillN], start[kFillN + 1];
    unsigned v[kFillN];
    int n;
};
__global__ void k_fill_many(FillSet fs) {
    const unsigned long long c0 = (unsigned long long)blockIdx.x * kFillChunk;
    for (int r = 0; r < fs.n; ++r) {
        const unsigned long long lo = fs.start[r], hi = fs.start[r + 1];
        if (hi <= c0 || lo >= c0 + kFillChunk) continue;
        const unsigned long long a = lo > c0 ? lo : c0, b = hi < c0 + kFillChunk ? hi : c0 + kFillChunk;
        for (unsigned long long i = a + threadIdx.x; i < b; i += blockDim.x) fs.p[r][i - lo] = fs.v[r];
    }
}
void fill_many(FillSet fs, hipStream_t st) {
    fs.start[0] = 0;
    for (int r = 0; r < fs.n; ++r) fs.start[r + 1] = fs.start[r] + fs.words[r];
    const unsigned long long tot = fs.start[fs.n];
    const unsigned blocks = (unsigned)std::max<unsigned long long>((tot + kFillChunk - 1) / kFillChunk, 1);
    hipLaunchKernelGGL(k_fill_many, dim3(blocks), dim3(256), 0, st, fs);
}

void fill_u32(void *p, size_t words, unsigned v, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(std::max(blocks, 1u)), dim3(256), 0, st, (unsigned *)p, words, v);
}

// The whole launch sequence of one call: no host synchronisation, no
// allocation, no memset or host copy, so it can be captured in a graph.
void enqueue(const Plan &pl, Workspace &w, hipStream_t st, Profiler *prof, bool first_part) {
    const size_t nna = pl.nna;
    const int nlev = pl.nlev, njobs = pl.njobs, d = pl.d, pmax = pl.pmax, P = pl.P, PW = pl.PW;
    int *headE = w.heads.as<int>(), *headF = headE + nna, *headL = headF + nna;
    const DevTree *td = w.trees.as<DevTree>();
    const Job *jd = w.jobs.as<Job>() + pl.job_off;
    const int *jls = w.jls.as<int>() + pl.jls_off;
    int *lvl = w.lvl.as<int>();
    {  // node flags, centroid scalars, chain heads (-1), flag / counters / level counts, statistics
        FillSet fs{};
        fs.n = 5;
        fs.p[0] = (unsigned *)w.lflag.p;
        fs.words[0] = (nna + 3) / 4;
        fs.p[1] = (unsigned *)w.cval.p;
        fs.words[1] = 2 * nna;
        fs.p[2] = (unsigned *)w.heads.p;
        fs.words[2] = 3 * nna;
        fs.v[2] = 0xffffffffu;
        fs.p[3] = (unsigned *)w.ctl.p;
        fs.words[3] = ((char *)w.lvl.p - (char *)w.ctl.p) / 4 + (size_t)(nlev + 1) * 2 * CP;
        fs.p[4] = (unsigned *)w.stats.p;
        fs.words[4] = 2 * S_N * SP;
        if (first_part) {
            fs.p[fs.n] = (unsigned *)w.sticky.p;
            fs.words[fs.n++] = 1;
        }
        if (pl.loo) {
            fs.p[fs.n] = (unsigned *)w.selfE.p;
            fs.words[fs.n++] = (nna + 3) / 4;
        }
        fill_many(fs, st);
    }
    const ItemRec *irec = w.irec.as<ItemRec>();
    hipLaunchKernelGGL(k_items, dim3((unsigned)((pl.items + 255) / 256)), dim3(256), 0, st, td, jd, jls, njobs, pl.unl,
                       pl.items, w.irec.as<ItemRec>());
    hipLaunchKernelGGL(k_seed, dim3((njobs + 255) / 256), dim3(256), 0, st, w.segA.as<Seg>(), w.pairA.as<int>(), njobs);
    if (pl.loo) {  // leave-one-out: every leaf's sums with itself, the traversal's lower bound for its leaves
        auto kp = pl.gr ? k_selfpre<true> : k_selfpre<false>;
        hipLaunchKernelGGL(kp, dim3((unsigned)pl.items), dim3(256), 0, st, td, jd, irec,
                           w.selfG.as<double>(), pl.gr ? w.selfX.as<double>() : nullptr,
                           pl.gr ? w.selfY.as<double>() : nullptr, w.selfmin.as<double>());
    }
    if (!pl.dig_lds)
        hipLaunchKernelGGL(k_digits, dim3((P + 255) / 256), dim3(256), 0, st, w.gdg.as<unsigned long long>(),
                           w.gmt.as<unsigned short>(), P, d, pmax);
    for (int k = 0; k < nlev; ++k) {
        DevBuf &sin = (k & 1) ? w.segB : w.segA, &sout = (k & 1) ? w.segA : w.segB;
        DevBuf &pin = (k & 1) ? w.pairB : w.pairA, &pout = (k & 1) ? w.pairA : w.pairB;
        TravOut o{sout.as<Seg>(),   pout.as<int>(),    w.egrp.as<Group>(), w.eops.as<int>(),
                  w.fgrp.as<Group>(), w.fops.as<Op>(),  w.lgrp.as<Group>(), w.lops.as<Op>(),
                  w.lnodes.as<int>(), headE,            headF,              headL,
                  w.cnt.as<int>(),  lvl + (size_t)(k + 1) * 2 * CP,         w.flag.as<int>(),
                  w.stats.as<unsigned long long>(),     w.cval.as<double>(),
                  pl.loo ? w.selfE.as<unsigned char>() : nullptr, pl.loo ? w.selfmin.as<double>() : nullptr,
                  prof ? 1 : 0, w.cap};
        hipEvent_t ev = prof ? prof->start(st) : nullptr;
        hipLaunchKernelGGL(k_traverse, dim3(kTravGrid / kTravWaves), dim3(64 * kTravWaves), 0, st, td, jd,
                           sin.as<Seg>(), pin.as<int>(),
                           k == 0 ? (const int *)nullptr : lvl + (size_t)k * 2 * CP, njobs, pl.force,
                           pl.gr ? 1 : 0, pl.leaf_local ? 1 : 0, w.dec.as<int>(), w.kus.as<double>(), o);
        if (prof) prof->stop(K_TRAV, ev, st);
    }
    // exhaustive leaf-leaf sums (DFGTBase) on the side stream, concurrent with
    // the local-moment ops and k_leaf below (they share no buffers); joined
    // before k_leaf_finish
    (void)hipEventRecord(w.fork, st);
    (void)hipStreamWaitEvent(w.side, w.fork, 0);
    {
        hipStream_t ss = w.side;
        hipEvent_t ev = prof ? prof->start(ss) : nullptr;
        double *gx = pl.gr ? w.extX.as<double>() : nullptr, *gy = pl.gr ? w.extY.as<double>() : nullptr;
        if (pl.emfma) {
            auto fn = pl.gr ? launch_emfma<true> : launch_emfma<false>;
            fn((d + 3) / 4, dim3(pl.items), ss, td, jd, w.egrp.as<Group>(), w.eops.as<int>(), headE,
               w.flag.as<int>(), irec, w.extE.as<double>(), gx, gy);
        } else if (pl.precision != DFGT_PREC_FP64) {
            // value sums with 3 <= D <= 7 on the matrix cores, but for items
            // whose query leaf is wide against h (vector-ALU tiles); with D <= 2
            // the vector-ALU tiles' 2D + 1 FMAs per pair cost less than the
            // matrix-core tiles' staging and reductions (2-D sweep: 0.29 ms
            // against 0.41 ms of tiles)
            const bool mx = !pl.gr && d >= 3 && d <= 7;
            int *ord = w.eord.as<int>();
            hipLaunchKernelGGL(k_eorder, dim3((unsigned)((pl.items + 255) / 256)), dim3(256), 0, ss, td, jd,
                               w.egrp.as<Group>(), headE, w.flag.as<int>(), irec, pl.items,
                               mx ? 1 : 0, w.cnt.as<int>(), ord, w.ehdr.as<int2>(), w.eglist.as<int2>(),
                               w.cap.grp);
            if (mx) {  // FP32 products (and the items without pairs), then FP64 products
                auto k32 = d <= 3 ? k_etile_mx32_1 : k_etile_mx32_2;
                auto k64 = d <= 3 ? k_etile_mx64_1 : k_etile_mx64_2;
                unsigned long long *sp = w.stats.as<unsigned long long>();
                for (int sel : {0, 2}) {
                    hipEvent_t e2 = prof && sel == 0 ? prof->start(ss) : nullptr;
                    hipLaunchKernelGGL(sel == 0 ? k32 : k64, dim3((unsigned)pl.items), dim3(64 * kMxWaves), 0, ss,
                                       td, jd, w.egrp.as<Group>(), w.eops.as<int>(), headE, w.cnt.as<int>(),
                                       w.flag.as<int>(), irec, ord, pl.items, sel, w.ehdr.as<int2>(),
                                       w.eglist.as<int2>(), sp + (size_t)(sel == 0 ? S_EP32 : S_EP64) * SP,
                                       w.extE.as<double>());
                    if (e2) prof->stop(K_MX32, e2, ss);
                }
            }
            auto fn = pl.gr ? launch_etile<true> : launch_etile<false>;
            fn(false, d, pl.items, ss, td, jd, w.egrp.as<Group>(), w.eops.as<int>(), headE, w.cnt.as<int>(),
               w.flag.as<int>(), irec, pl.precision, ord, mx ? 1 : 0, w.extE.as<double>(), gx, gy);
        }
        if (prof) prof->stop(K_EMFMA, ev, ss);
        {
            // the FP64 pairs (all of them at precision FP64, else the groups the
            // underflow guard flagged), added after the mixed pass
            ev = prof ? prof->start(ss) : nullptr;
            auto fn = pl.gr ? launch_etile<true> : launch_etile<false>;
            fn(true, d, pl.items, ss, td, jd, w.egrp.as<Group>(), w.eops.as<int>(), headE, w.cnt.as<int>(),
               w.flag.as<int>(), irec, pl.precision, nullptr, 0, w.extE.as<double>(), gx, gy);
            if (prof) prof->stop(K_EF64, ev, ss);
        }
    }
    (void)hipEventRecord(w.join, w.side);
    // local moments: every D / T op in parallel, then per internal node
    {
        hipEvent_t ev = prof ? prof->start(st) : nullptr;
        if (pl.leaf_local) {
            hipLaunchKernelGGL(k_lop_owner, dim3(kLocalGrid), dim3(64), 0, st, w.lgrp.as<Group>(), w.cnt.as<int>(),
                               w.flag.as<int>(), w.lopnode.as<int2>());
            auto klo = pl.gr ? k_lops<true> : k_lops<false>;
            hipLaunchKernelGGL(klo, dim3(kLocalGrid), dim3(64 * pl.lop_waves), pl.lop_sh, st, td, jd,
                               w.lops.as<Op>(), w.lopnode.as<int2>(), w.cnt.as<int>(),
                               w.flag.as<int>(), w.part.as<double>());
            hipLaunchKernelGGL(k_lreduce, dim3(kLocalGrid), dim3(256), sizeof(double) * (PW + 256), st, jd,
                               w.lnodes.as<int>(), w.cnt.as<int>(), w.flag.as<int>(), headL, w.lgrp.as<Group>(),
                               w.part.as<double>(), PW, w.L.as<double>(), w.lflag.as<unsigned char>());
        } else {
            hipLaunchKernelGGL(k_local_big, dim3(kLocalGrid), dim3(kLocBlock), pl.big_sh, st, td, jd,
                               w.lnodes.as<int>(), w.cnt.as<int>(), w.flag.as<int>(), headL, w.lgrp.as<Group>(),
                               w.lops.as<Op>(), w.lscr.as<double>(), w.L.as<double>(),
                               w.lflag.as<unsigned char>());
        }
        if (prof) prof->stop(K_LOCAL, ev, st);
    }
    // everything per (job, query leaf) but the exhaustive sums, beside the tiles
    {
        hipEvent_t ev = prof ? prof->start(st) : nullptr;
        auto kl = pl.gr ? k_leaf<true, false>
                        : (far_fixed_kind(pl.d, pl.pmax) ? k_leaf<false, false> : k_leaf<false, true>);
        hipLaunchKernelGGL(kl, dim3(pl.items), dim3(pl.leaf_threads), pl.leaf_sh, st, td, jd, w.egrp.as<Group>(),
                           w.eops.as<int>(), w.fgrp.as<Group>(), w.fops.as<Op>(), w.lgrp.as<Group>(),
                           w.lops.as<Op>(), headE, headF, headL, w.L.as<double>(), w.lflag.as<unsigned char>(),
                           pl.precision, pl.acc_lds ? 1 : 0, pl.leaf_local ? 1 : 0, w.flag.as<int>(),
                           pl.leaf_local ? w.part.as<double>() : (const double *)nullptr, w.pscr.as<double>(),
                           w.stG.as<double>(), pl.gr ? w.stX.as<double>() : nullptr,
                           pl.gr ? w.stQ.as<double>() : nullptr, w.cval.as<double>(), irec,
                           pl.dig_lds ? nullptr : w.gdg.as<unsigned long long>(),
                           pl.dig_lds ? nullptr : w.gmt.as<unsigned short>(),
                           pl.loo ? w.selfE.as<unsigned char>() : nullptr, w.selfG.as<double>(),
                           w.selfX.as<double>(), w.selfY.as<double>());
        if (prof) prof->stop(K_LEAF, ev, st);
    }
    // the outputs, once the tiles' stream has joined
    (void)hipStreamWaitEvent(st, w.join, 0);
    {
        auto kf = pl.gr ? k_leaf_finish<true> : k_leaf_finish<false>;
        hipLaunchKernelGGL(kf, dim3((unsigned)((pl.nqa + 255) / 256)), dim3(256), 0, st, td, jd, njobs,
                           (long long)pl.nqa, w.flag.as<int>(), w.stG.as<double>(),
                           pl.gr ? w.stX.as<double>() : (const double *)nullptr,
                           pl.gr ? w.stQ.as<double>() : (const double *)nullptr, w.extE.as<double>(),
                           pl.gr ? w.extX.as<double>() : (const double *)nullptr,
                           pl.gr ? w.extY.as<double>() : (const double *)nullptr, w.sticky.as<int>());
    }
}

// Reads the overflow flag and the counters (synchronises); on overflow grows
// the capacities for a rerun.
dfgt_status read_back(const Plan &pl, Workspace &w, hipStream_t st, int *overflow, int *c) {
    const int nlev = pl.nlev;
    const char *base = (const char *)w.ctl.p;
    const size_t oc = (const char *)w.cnt.p - base, ol = (const char *)w.lvl.p - base,
                 total = ol + sizeof(int) * (size_t)(nlev + 1) * 2 * CP;
    DFGT_TRY(w.back.reserve(total));
    DFGT_HIP(hipMemcpyAsync(w.back.p, w.ctl.p, total, hipMemcpyDeviceToHost, st));
    DFGT_HIP(hipStreamSynchronize(st));
    const char *hb = w.back.as<const char>();
    *overflow = *(const int *)hb;
    const int *hc = (const int *)(hb + oc), *hl = (const int *)(hb + ol);
    for (int k = 0; k < C_N; ++k) c[k] = hc[(size_t)k * CP];
    if (!*overflow && hl[((size_t)nlev * 2 + C_SEG) * CP] != 0) {
        set_error("dfgt_gauss_sum: internal error, node pairs left after the last level");
        return DFGT_EHIP;
    }
    if (*overflow) {
        Caps &cap = w.cap;
        int mseg = 0, mpair = 0;
        for (int k = 1; k <= nlev; ++k) {
            mseg = std::max(mseg, hl[((size_t)k * 2 + C_SEG) * CP]);
            mpair = std::max(mpair, hl[((size_t)k * 2 + C_PAIR) * CP]);
        }
        auto up = [](int cur, long long need) {
            long long v = std::max<long long>(2LL * cur, 2LL * need);
            return (int)std::min<long long>(v, (1LL << 30));
        };
        cap.seg = up(cap.seg, mseg);
        cap.pair = up(cap.pair, mpair);
        cap.eop = up(cap.eop, c[C_EOP]);
        cap.fop = up(cap.fop, c[C_FOP]);
        cap.lop = up(cap.lop, c[C_LOP]);
        cap.grp = up(cap.grp, std::max(c[C_EGRP], std::max(c[C_FGRP], c[C_LGRP])));
        cap.lnode = up(cap.lnode, c[C_LNODE]);
    }
    return DFGT_OK;
}

dfgt_status fill_stats(const Plan &pl, Workspace &w, const int *c, Profiler *prof, dfgt_stats *out,
                       hipStream_t st) {
    std::vector<unsigned long long> sraw((size_t)S_N * SP);
    DFGT_HIP(hipMemcpyAsync(sraw.data(), w.stats.p, sizeof(unsigned long long) * S_N * SP, hipMemcpyDeviceToHost,
                            st));
    DFGT_HIP(hipStreamSynchronize(st));
    unsigned long long sv[S_N];
    for (int k = 0; k < S_N; ++k) sv[k] = sraw[(size_t)k * SP];
    std::memset(out, 0, sizeof(*out));
    out->node_pairs = (int64_t)sv[S_PAIRS];
    out->prune_f = (int64_t)sv[S_F];
    out->prune_d = (int64_t)sv[S_D];
    out->prune_t = (int64_t)sv[S_T];
    out->prune_centroid = (int64_t)sv[S_C];
    out->base_leaf_pairs = (int64_t)sv[S_BLEAF];
    out->base_point_pairs = (int64_t)sv[S_BPTS];
    out->levels = pl.nlev;
    out->max_order = (int64_t)sv[S_MAXORD];
    out->fp64_groups = (int64_t)c[C_EF64];
    out->segments = (int64_t)sv[S_SEGS];
    out->max_segment = (int64_t)sv[S_MAXSEG];
    out->local_nodes = c[C_LNODE];
    out->max_local_ops = (int64_t)sv[S_MAXLOPS];
    out->work_f = (int64_t)sv[S_FW];
    out->work_d = (int64_t)sv[S_DW];
    out->work_t = (int64_t)sv[S_TW];
    out->e_pairs[0] = (int64_t)sv[S_EP32];
    out->e_pairs[1] = (int64_t)sv[S_EP64];
    for (int k = 0; k < 6; ++k) out->e_items[k] = (int64_t)c[C_EHEAVY + k];
    out->mfma_tiles = pl.emfma ? 1 : 0;
    if (prof && prof->on) prof->collect(out);
    return DFGT_OK;
}

// Eager run: allocate, enqueue, read back, and on overflow grow and rerun.
// When the capacities a rerun would need exceed the memory budget and the
// plan has more than one job, *too_big is set instead (capacities unchanged).
dfgt_status run_plan(const Plan &pl, Workspace &w, int profile, dfgt_stats *stats_out, hipStream_t st,
                     size_t budget, bool *too_big) {
    Profiler &prof = g_prof;
    *too_big = false;
    Caps &cap = w.cap;
    Caps least{1 << 19, 1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 18, 1 << 18};  // the starting capacities
    least.pair = std::max(least.pair, 4 * pl.njobs);
    least.seg = std::max(least.seg, 4 * pl.njobs);
    if (cap.pair == 0) cap = least;
    cap.pair = std::max(cap.pair, least.pair);
    cap.seg = std::max(cap.seg, least.seg);
    // split before running when the plan exceeds the budget even at the
    // starting capacities (capacities grown by earlier calls do not count:
    // they are what other plans needed)
    if (pl.njobs > 1 && plan_bytes(pl, least) > budget) {
        *too_big = true;
        return DFGT_OK;
    }
    int c[C_N] = {0};
    int overflow = 1;
    const Caps entry = cap;
    for (int attempt = 0; attempt < 12 && overflow; ++attempt) {
        const dfgt_status as = alloc_plan(pl, w);
        if (as == DFGT_ENOMEM && pl.njobs > 1) {  // the device cannot hold this part: split it
            clear_error();
            cap = entry;
            *too_big = true;
            return DFGT_OK;
        }
        DFGT_TRY(as);
        DFGT_TRY(upload_plan(pl, w, st));
        prof.begin_call(profile != 0);
        // stats are gathered whenever a caller asks for them
        enqueue(pl, w, st, (profile || stats_out) ? &prof : nullptr, true);
        DFGT_HIP(hipGetLastError());
        const Caps before = cap;
        DFGT_TRY(read_back(pl, w, st, &overflow, c));
        if (overflow && pl.njobs > 1 && plan_bytes(pl, cap) > budget) {
            cap = before;
            *too_big = true;
            return DFGT_OK;
        }
    }
    if (overflow) {
        set_error("dfgt_gauss_sum: the traversal's lists outgrew their buffers after 12 retries");
        return DFGT_EQUEUE;
    }
    if (stats_out) DFGT_TRY(fill_stats(pl, w, c, &prof, stats_out, st));
    return DFGT_OK;
}

void add_stats(dfgt_stats *a, const dfgt_stats &b) {
    a->node_pairs += b.node_pairs;
    a->prune_f += b.prune_f;
    a->prune_d += b.prune_d;
    a->prune_t += b.prune_t;
    a->prune_centroid += b.prune_centroid;
    a->base_leaf_pairs += b.base_leaf_pairs;
    a->base_point_pairs += b.base_point_pairs;
    a->levels = std::max(a->levels, b.levels);
    a->max_order = std::max(a->max_order, b.max_order);
    a->fp64_groups += b.fp64_groups;
    a->segments += b.segments;
    a->max_segment = std::max(a->max_segment, b.max_segment);
    a->local_nodes += b.local_nodes;
    a->max_local_ops = std::max(a->max_local_ops, b.max_local_ops);
    a->mfma_tiles += b.mfma_tiles;
    a->work_f += b.work_f;
    a->work_d += b.work_d;
    a->work_t += b.work_t;
    for (int k = 0; k < 6; ++k) a->e_items[k] += b.e_items[k];
    for (int k = 0; k < 2; ++k) a->e_pairs[k] += b.e_pairs[k];
    for (int k = 0; k < 6; ++k) {
        a->kernel_ms[k] += b.kernel_ms[k];
        a->kernel_launches[k] += b.kernel_launches[k];
    }
}

// Runs a plan, splitting its jobs in halves while a part does not fit the
// memory budget; returns the parts that ran (in order).
dfgt_status run_chunks(const Plan &full, Workspace &w, int profile, dfgt_stats *stats_out, hipStream_t st,
                       std::vector<Plan> *parts) {
    std::vector<Plan> todo;
    const size_t budget = memory_budget();
    const double ipj = (double)full.items / std::max(full.njobs, 1);
    // a part size learned under another budget, or on jobs with more items
    // (larger lists), does not apply
    if (budget != w.part_budget || ipj < 0.9 * w.part_ipj) {
        w.part_jobs = 0;
        w.part_budget = budget;
    }
    // start from the part size a previous call had to split to (a guess that
    // is only ever refined: parts that still do not fit are halved again)
    const int pj = w.part_jobs > 0 ? w.part_jobs : full.njobs;
    for (int j0 = 0; j0 < full.njobs; j0 += pj) todo.push_back(sub_plan(full, j0, std::min(full.njobs, j0 + pj)));
    if (stats_out) std::memset(stats_out, 0, sizeof(*stats_out));
    parts->clear();
    while (!todo.empty()) {
        Plan pl = std::move(todo.front());
        todo.erase(todo.begin());
        bool too_big = false;
        dfgt_stats one{};
        DFGT_TRY(run_plan(pl, w, profile, stats_out ? &one : nullptr, st, budget, &too_big));
        if (too_big) {
            const int mid = pl.njobs / 2;
            w.part_jobs = w.part_jobs > 0 ? std::min(w.part_jobs, pl.njobs - mid) : pl.njobs - mid;
            w.part_ipj = ipj;
            todo.insert(todo.begin(), sub_plan(pl, mid, pl.njobs));
            todo.insert(todo.begin(), sub_plan(pl, 0, mid));
            continue;
        }
        if (stats_out) add_stats(stats_out, one);
        parts->push_back(std::move(pl));
    }
    if (stats_out) stats_out->parts = (int64_t)parts->size();
    return DFGT_OK;
}

}  // namespace

void release_sum_workspace() {
    Workspace &w = g_ws;
    DevBuf *bufs[] = {&w.jobs, &w.trees, &w.jls, &w.L, &w.lflag, &w.heads, &w.segA, &w.segB, &w.pairA, &w.pairB,
                      &w.dec, &w.kus, &w.egrp, &w.eops, &w.fgrp, &w.fops, &w.lgrp, &w.lops, &w.lnodes, &w.stats,
                      &w.lscr, &w.pscr, &w.lopnode, &w.part, &w.extE, &w.extX, &w.extY, &w.stG, &w.stX, &w.stQ,
                      &w.cval, &w.gdg, &w.gmt, &w.eord, &w.ehdr, &w.eglist, &w.irec, &w.selfE, &w.selfG, &w.selfX, &w.selfY, &w.selfmin,
                      &w.ctl, &w.sticky};
    for (DevBuf *b : bufs) b->release();
    w.cap = Caps{0, 0, 0, 0, 0, 0, 0};
    w.part_jobs = 0;
}

dfgt_status run_gauss_multi(const Problem *pr, int np, double eps, int precision, int force, int profile,
                            double cost_e, const GradOut *grad, dfgt_stats *stats_out, hipStream_t st) {
    Plan pl;
    DFGT_TRY(make_plan(pr, np, eps, precision, force, cost_e, grad, pl));
    std::vector<Plan> parts;
    return run_chunks(pl, g_ws, profile, stats_out, st, &parts);
}

dfgt_status run_gauss_sum(dfgt_tree_s *Qh, dfgt_tree_s *Rh, const double *h, int nh, double eps, int precision,
                          int force, int profile, double cost_e, double *G, const GradOut *grad,
                          dfgt_stats *stats_out, hipStream_t st, bool loo) {
    Problem pr{Qh, Rh, h, nh, G};
    pr.loo = loo ? 1 : 0;
    return run_gauss_multi(&pr, 1, eps, precision, force, profile, cost_e, grad, stats_out, st);
}

}  // namespace dfgt

// A captured batch: the plan, its own workspace (the graph holds pointers
// into it) and the executable graph of one full launch sequence.
struct dfgt_batch_s {
    std::vector<dfgt::Plan> parts;  // the job chunks, replayed in order on one workspace
    dfgt::Workspace w;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~dfgt_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

namespace dfgt {

dfgt_status batch_create(const Problem *pr, int np, double eps, int precision, int force, double cost_e,
                         dfgt_stats *stats_out, hipStream_t st, dfgt_batch_s **out) {
    auto *b = new dfgt_batch_s();
    Plan full;
    dfgt_status s = make_plan(pr, np, eps, precision, force, cost_e, nullptr, full);
    // one eager run sizes the workspace (the inputs fix every list size) and
    // splits the jobs into parts that fit the memory budget
    if (s == DFGT_OK) s = run_chunks(full, b->w, 0, stats_out, st, &b->parts);
    if (s == DFGT_OK) {
        // every part's tables at their own offsets, uploaded once; buffers at
        // their final sizes before capture (the graph holds their addresses)
        size_t jo = 0, lo = 0;
        for (Plan &p : b->parts) {
            p.job_off = jo;
            p.jls_off = lo;
            jo += p.njobs;
            lo += p.jls.size();
        }
        for (const Plan &p : b->parts)
            if (s == DFGT_OK) s = alloc_plan(p, b->w);
        if (s == DFGT_OK) s = grow<Job>(b->w.jobs, jo);
        if (s == DFGT_OK) s = grow<int>(b->w.jls, lo);
        for (const Plan &p : b->parts)
            if (s == DFGT_OK) s = upload_plan(p, b->w, st);
    }
    if (s == DFGT_OK && hipStreamSynchronize(st) != hipSuccess) s = DFGT_EHIP;
    // capture on a stream of our own (the caller's may be the legacy default stream)
    if (s == DFGT_OK && hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) s = DFGT_EHIP;
    if (s == DFGT_OK && hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) s = DFGT_EHIP;
    if (s == DFGT_OK) {
        for (size_t k = 0; k < b->parts.size(); ++k) enqueue(b->parts[k], b->w, b->cs, nullptr, k == 0);
        const hipError_t le = hipGetLastError();
        const hipError_t ce = hipStreamEndCapture(b->cs, &b->graph);
        if (le != hipSuccess || ce != hipSuccess) s = DFGT_EHIP;
    }
    if (s == DFGT_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) s = DFGT_EHIP;
    if (s != DFGT_OK) {
        if (s == DFGT_EHIP) set_error("dfgt_batch_create: capturing the launch graph failed");
        delete b;
        return s;
    }
    *out = b;
    return DFGT_OK;
}

dfgt_status batch_run(dfgt_batch_s *b, hipStream_t st) {
    DFGT_HIP(hipGraphLaunch(b->exec, st));
    return DFGT_OK;
}

dfgt_status batch_check(dfgt_batch_s *b, hipStream_t st) {
    int overflow = 0;
    DFGT_HIP(hipMemcpyAsync(&overflow, b->w.sticky.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DFGT_HIP(hipStreamSynchronize(st));
    if (overflow) {
        set_error("dfgt_batch: the last run overflowed its traversal buffers (were the trees changed?)");
        return DFGT_EQUEUE;
    }
    return DFGT_OK;
}

}  // namespace dfgt

extern "C" dfgt_status dfgt_batch_free(dfgt_batch b) {
    try {
        delete b;
    } catch (...) {
        return DFGT_EHIP;
    }
    return DFGT_OK;
}
