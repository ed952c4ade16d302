/*
 * Plain FP64 CPU oracle for the Dual-Tree Fast Gauss Transform
 * (Lee, Gray & Moore, "Dual-Tree Fast Gauss Transforms").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library and is built by the host C
 * compiler (gcc, OpenMP for the brute-force sums only).
 *
 * Every routine follows one passage of the paper, cited by section / equation /
 * algorithm name.  Readings of passages that are garbled or ambiguous are named
 * in the comment where they are applied (A-numbers match the readings list of
 * the design notes).
 *
 * Conventions
 *   points        row-major [n][D] float64
 *   multi-index   alpha[0..D-1]; a coefficient vector of p_max^D doubles is
 *                 stored radix p_max with the LAST dimension fastest (Appendix,
 *                 "Storing the far-field/local moments as a linear array").
 *   s             1/sqrt(2 h^2), the paper's scaling of every expansion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 32

/* ------------------------------------------------------------------------ */
/* Section 1.1, eq. (gaussian_kernel_sums) and Alg. NaiveKDE (Section 1):     */
/* G(q_i, R) = sum_j exp(-||q_i - r_j||^2 / (2 h^2)), computed exactly.       */
/* The sum is Neumaier-compensated; the distance uses coordinate differences.  */
/* ------------------------------------------------------------------------ */
int oracle_naive_kde(const double *q, int64_t nq, const double *r, int64_t nr, int d,
                     double h, double *out)
{
    if (nq < 0 || nr < 0 || d < 1 || !(h > 0.0)) return 1;
    const double inv2h2 = 1.0 / (2.0 * h * h);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const double *qi = q + i * d;
        double sum = 0.0, comp = 0.0;
        for (int64_t j = 0; j < nr; ++j) {
            const double *rj = r + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = qi[k] - rj[k];
                d2 += t * t;
            }
            double v = exp(-d2 * inv2h2);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        out[i] = sum + comp;
    }
    return 0;
}

/* The same sum over a subset of query indices (sampled checks at full size). */
int oracle_naive_kde_rows(const double *q, const int64_t *rows, int64_t nrows, const double *r,
                          int64_t nr, int d, double h, double *out)
{
    if (nrows < 0 || nr < 0 || d < 1 || !(h > 0.0)) return 1;
    const double inv2h2 = 1.0 / (2.0 * h * h);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ii = 0; ii < nrows; ++ii) {
        const double *qi = q + rows[ii] * d;
        double sum = 0.0, comp = 0.0;
        for (int64_t j = 0; j < nr; ++j) {
            const double *rj = r + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = qi[k] - rj[k];
                d2 += t * t;
            }
            double v = exp(-d2 * inv2h2);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
        }
        out[ii] = sum + comp;
    }
    return 0;
}

/*
 * Derivatives of the same exact sum (not in the paper; the differentiation
 * form of the method):
 *   dG/dh   = h^-3 sum_j K_j ||q - r_j||^2
 *   dG/dq   = -h^-2 sum_j K_j (q - r_j)
 * Any of the output pointers may be NULL.
 */
int oracle_naive_kde_grad(const double *q, int64_t nq, const double *r, int64_t nr, int d,
                          double h, double *G, double *dGdh, double *dGdq)
{
    if (nq < 0 || nr < 0 || d < 1 || d > OR_MAXD || !(h > 0.0)) return 1;
    const double inv2h2 = 1.0 / (2.0 * h * h);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const double *qi = q + i * d;
        double g = 0.0, gh = 0.0, gq[OR_MAXD];
        for (int k = 0; k < d; ++k) gq[k] = 0.0;
        for (int64_t j = 0; j < nr; ++j) {
            const double *rj = r + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = qi[k] - rj[k];
                d2 += t * t;
            }
            double v = exp(-d2 * inv2h2);
            g += v;
            gh += v * d2;
            for (int k = 0; k < d; ++k) gq[k] += v * (qi[k] - rj[k]);
        }
        if (G) G[i] = g;
        if (dGdh) dGdh[i] = gh / (h * h * h);
        if (dGdq)
            for (int k = 0; k < d; ++k) dGdq[i * d + k] = -gq[k] / (h * h);
    }
    return 0;
}

/*
 * Scale of the query gradient (not in the paper; the differentiation form of
 * the method): the sum of the norms of the terms of dG/dq,
 *   out(q) = h^-2 sum_j K_j ||q - r_j||,
 * which bounds ||dG/dq|| from above (triangle inequality) and is the unit in
 * which the relative error of a computed dG/dq is measured.
 */
int oracle_naive_kde_qscale(const double *q, int64_t nq, const double *r, int64_t nr, int d, double h,
                            double *out)
{
    if (nq < 0 || nr < 0 || d < 1 || d > OR_MAXD || !(h > 0.0)) return 1;
    const double inv2h2 = 1.0 / (2.0 * h * h);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const double *qi = q + i * d;
        double acc = 0.0;
        for (int64_t j = 0; j < nr; ++j) {
            const double *rj = r + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = qi[k] - rj[k];
                d2 += t * t;
            }
            acc += exp(-d2 * inv2h2) * sqrt(d2);
        }
        out[i] = acc / (h * h);
    }
    return 0;
}

/*
 * Weighted kernel sums (the sums of Section 1 with a weight per reference
 * point, as a weighted density estimate takes them), computed exactly:
 *   G_w(q)    = sum_j w_j K_j,  K_j = exp(-||q - r_j||^2 / (2 h^2))
 *   dG_w/dh   = h^-3 sum_j w_j K_j ||q - r_j||^2
 *   dG_w/dq   = -h^-2 sum_j w_j K_j (q - r_j)
 * The value sum is Neumaier-compensated.  Any output pointer may be NULL.
 */
int oracle_naive_kde_weighted(const double *q, int64_t nq, const double *r, const double *w, int64_t nr,
                              int d, double h, double *G, double *dGdh, double *dGdq)
{
    if (nq < 0 || nr < 0 || d < 1 || d > OR_MAXD || !(h > 0.0)) return 1;
    const double inv2h2 = 1.0 / (2.0 * h * h);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nq; ++i) {
        const double *qi = q + i * d;
        double sum = 0.0, comp = 0.0, gh = 0.0, gq[OR_MAXD];
        for (int k = 0; k < d; ++k) gq[k] = 0.0;
        for (int64_t j = 0; j < nr; ++j) {
            const double *rj = r + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = qi[k] - rj[k];
                d2 += t * t;
            }
            const double v = w[j] * exp(-d2 * inv2h2);
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
            else comp += (v - t) + sum;
            sum = t;
            gh += v * d2;
            for (int k = 0; k < d; ++k) gq[k] += v * (qi[k] - rj[k]);
        }
        if (G) G[i] = sum + comp;
        if (dGdh) dGdh[i] = gh / (h * h * h);
        if (dGdq)
            for (int k = 0; k < d; ++k) dGdq[i * d + k] = -gq[k] / (h * h);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 2.1, Alg. BuildKdTree: recursive mid-point kd-tree.                */
/*   box     b[d].l = min, b[d].u = max over the node's points (A1: the text   */
/*           writes "min" twice; the algorithm's max is taken)                */
/*   split   sd = argmax width (lowest dimension on ties, A3),                */
/*           sc = (l + u) / 2 in FP64 (A6); points with x[sd] <= sc go left.  */
/*   order   stable partition: relative order is kept on each side (A5).     */
/*   leaf    n <= leaf_size, zero width, or an empty side (A2, A4).           */
/* Nodes are numbered in pre-order; perm[k] = original index of the k-th      */
/* point in tree order.                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *x;
    int d, leaf;
    int32_t *perm, *tmp;
    double *lo, *hi;
    int64_t *begin, *end;
    int32_t *left, *right, *sdim;
    double *scoord;
    int64_t count, cap;
} kd_ctx;

static int64_t kd_build(kd_ctx *c, int64_t b, int64_t e)
{
    if (c->count >= c->cap) return -1;
    int64_t id = c->count++;
    int d = c->d;
    double *lo = c->lo + id * d, *hi = c->hi + id * d;
    for (int k = 0; k < d; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int64_t i = b; i < e; ++i) {
        const double *p = c->x + (int64_t)c->perm[i] * d;
        for (int k = 0; k < d; ++k) {
            if (p[k] < lo[k]) lo[k] = p[k];
            if (p[k] > hi[k]) hi[k] = p[k];
        }
    }
    c->begin[id] = b;
    c->end[id] = e;
    c->left[id] = -1;
    c->right[id] = -1;
    c->sdim[id] = -1;
    c->scoord[id] = 0.0;
    if (e - b <= c->leaf) return id;
    int sd = 0;
    double wmax = hi[0] - lo[0];
    for (int k = 1; k < d; ++k)
        if (hi[k] - lo[k] > wmax) {
            wmax = hi[k] - lo[k];
            sd = k;
        }
    if (!(wmax > 0.0)) return id;
    double sc = (lo[sd] + hi[sd]) / 2.0;
    int64_t nl = 0;
    for (int64_t i = b; i < e; ++i)
        if (c->x[(int64_t)c->perm[i] * d + sd] <= sc) ++nl;
    if (nl == 0 || nl == e - b) return id;
    int64_t wl = b, wr = b + nl;
    for (int64_t i = b; i < e; ++i) {
        int32_t pi = c->perm[i];
        if (c->x[(int64_t)pi * d + sd] <= sc) c->tmp[wl++] = pi;
        else c->tmp[wr++] = pi;
    }
    memcpy(c->perm + b, c->tmp + b, (size_t)(e - b) * sizeof(int32_t));
    c->sdim[id] = sd;
    c->scoord[id] = sc;
    int64_t l = kd_build(c, b, b + nl);
    if (l < 0) return -1;
    int64_t r = kd_build(c, b + nl, e);
    if (r < 0) return -1;
    c->left[id] = (int32_t)l;
    c->right[id] = (int32_t)r;
    return id;
}

int oracle_build_kdtree(const double *x, int64_t n, int d, int leaf_size, int64_t max_nodes,
                        int32_t *perm, double *lo, double *hi, int64_t *begin, int64_t *end,
                        int32_t *left, int32_t *right, int32_t *sdim, double *scoord,
                        int64_t *n_nodes)
{
    if (n < 1 || d < 1 || leaf_size < 1) return 1;
    kd_ctx c;
    c.x = x;
    c.d = d;
    c.leaf = leaf_size;
    c.perm = perm;
    c.tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!c.tmp) return 2;
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    c.lo = lo;
    c.hi = hi;
    c.begin = begin;
    c.end = end;
    c.left = left;
    c.right = right;
    c.sdim = sdim;
    c.scoord = scoord;
    c.count = 0;
    c.cap = max_nodes;
    int64_t root = kd_build(&c, 0, n);
    free(c.tmp);
    if (root < 0) return 3;
    *n_nodes = c.count;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.1, multi-index notation, and the Appendix's linear layout.       */
/* ------------------------------------------------------------------------ */

/* Appendix, MultiIndexToPosition: radix-p number, alpha[D-1] least significant. */
int64_t oracle_mi_to_pos(const int *alpha, int d, int p)
{
    int64_t x = 0, f = 1;
    for (int k = d - 1; k >= 0; --k) {
        x += f * alpha[k];
        f *= p;
    }
    return x;
}

/* Appendix, PositionToMultiindex, as the inverse of MultiIndexToPosition
 * (A14: the printed digit extraction is garbled; the last dimension is taken
 * as the least significant digit). */
void oracle_pos_to_mi(int64_t i, int d, int p, int *alpha)
{
    for (int k = d - 1; k >= 0; --k) {
        alpha[k] = (int)(i % p);
        i /= p;
    }
}

static int64_t ipow64(int b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

static double mi_factorial(const int *a, int d)
{
    double f = 1.0;
    for (int k = 0; k < d; ++k) f *= factorial(a[k]);
    return f;
}

static int mi_abs(const int *a, int d)
{
    int s = 0;
    for (int k = 0; k < d; ++k) s += a[k];
    return s;
}

/* Appendix, MultiIndexExpansion: out = { x^alpha }_{alpha < p}, each entry
 * obtained from a direct ancestor (alpha with one unit removed from its first
 * non-zero digit) by one multiplication.  Entry alpha is written at radix-pmax
 * position (A15); the loop starts at the first non-zero position (A16). */
void oracle_mi_expansion(const double *x, int d, int p, int pmax, double *out)
{
    int a[OR_MAXD], ap[OR_MAXD];
    int64_t n = ipow64(p, d);
    memset(a, 0, sizeof(a));
    out[0] = 1.0;
    for (int64_t i = 1; i < n; ++i) {
        oracle_pos_to_mi(i, d, p, a);
        int j = 0;
        while (a[j] < 1) ++j;
        memcpy(ap, a, sizeof(int) * d);
        ap[j] -= 1;
        out[oracle_mi_to_pos(a, d, pmax)] = out[oracle_mi_to_pos(ap, d, pmax)] * x[j];
    }
}

/* Section 3.1, Hermite functions h_n(t) = e^{-t^2} H_n(t), by the recurrence
 * h_{n+1} = 2 t h_n - 2 n h_{n-1}; Appendix, ComputePartialDerivatives:
 * H[k*n + m] = h_m(a[k]) for m < n. */
void oracle_hermite_table(const double *a, int d, int n, double *H)
{
    for (int k = 0; k < d; ++k) {
        double *row = H + (int64_t)k * n;
        double e = exp(-a[k] * a[k]);
        row[0] = e;
        if (n > 1) row[1] = 2.0 * a[k] * e;
        for (int m = 1; m + 1 < n; ++m) row[m + 1] = 2.0 * a[k] * row[m] - 2.0 * m * row[m - 1];
    }
}

/* Appendix, ComputeHermiteFunction: h_alpha = prod_d h_{alpha[d]}(a[d]). */
static double hermite_fn(const double *H, int n, const int *alpha, int d)
{
    double f = 1.0;
    for (int k = 0; k < d; ++k) f *= H[(int64_t)k * n + alpha[k]];
    return f;
}

/* ------------------------------------------------------------------------ */
/* Section 3.3, eq. (far_field_moments); Appendix, AccumulateFarFieldMoment: */
/*   M_alpha(R, c) = sum_{r in R} (1/alpha!) ((r - c) s)^alpha,  alpha < p.   */
/* Adds into M (radix pmax).                                                  */
/* ------------------------------------------------------------------------ */
int oracle_p2m(const double *pts, int64_t n, int d, const double *c, double h, int p, int pmax,
               double *M)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int64_t np = ipow64(pmax, d);
    double *acc = (double *)calloc((size_t)np, sizeof(double));
    double *mp = (double *)calloc((size_t)np, sizeof(double));
    if (!acc || !mp) {
        free(acc);
        free(mp);
        return 2;
    }
    double x[OR_MAXD] = {0};
    int a[OR_MAXD];
    int64_t nsub = ipow64(p, d);
    for (int64_t j = 0; j < n; ++j) {
        for (int k = 0; k < d; ++k) x[k] = (pts[j * d + k] - c[k]) * s;
        oracle_mi_expansion(x, d, p, pmax, mp);
        for (int64_t i = 0; i < nsub; ++i) {
            oracle_pos_to_mi(i, d, p, a);
            int64_t pos = oracle_mi_to_pos(a, d, pmax);
            acc[pos] += mp[pos];
        }
    }
    for (int64_t i = 0; i < nsub; ++i) {
        oracle_pos_to_mi(i, d, p, a);
        int64_t pos = oracle_mi_to_pos(a, d, pmax);
        M[pos] += acc[pos] / mi_factorial(a, d);
    }
    free(acc);
    free(mp);
    return 0;
}

/* Section 3.7, F2F lemma, eq. (far_to_far_translation); Appendix,
 * TransFarToFar.  Shifts the child's moments (about cc) to the parent centre
 * cp and adds them into Mp:
 *   Mp_gamma += sum_{alpha <= gamma} Mc_alpha ((cc - cp) s)^{gamma-alpha} / (gamma-alpha)!   */
int oracle_f2f(const double *Mc, const double *cc, const double *cp, int d, double h, int pmax,
               double *Mp)
{
    if (d < 1 || d > OR_MAXD) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int64_t np = ipow64(pmax, d);
    double *C = (double *)calloc((size_t)np, sizeof(double));
    if (!C) return 2;
    double x[OR_MAXD] = {0};
    for (int k = 0; k < d; ++k) x[k] = (cc[k] - cp[k]) * s;
    oracle_mi_expansion(x, d, pmax, pmax, C);
    int g[OR_MAXD], a[OR_MAXD], ga[OR_MAXD];
    for (int64_t i = 0; i < np; ++i) {
        oracle_pos_to_mi(i, d, pmax, g);
        double acc = 0.0;
        for (int64_t j = 0; j < np; ++j) {
            oracle_pos_to_mi(j, d, pmax, a);
            int le = 1;
            for (int k = 0; k < d; ++k)
                if (a[k] > g[k]) le = 0;
            if (!le) continue;
            for (int k = 0; k < d; ++k) ga[k] = g[k] - a[k];
            acc += Mc[j] * C[oracle_mi_to_pos(ga, d, pmax)] / mi_factorial(ga, d);
        }
        Mp[i] += acc;
    }
    free(C);
    return 0;
}

/* Section 3.3 (far-field expansion) and Appendix, EvalFarFieldExpansion:
 *   out[i] += sum_{alpha < p} M_alpha h_alpha((q_i - c) s).                  */
int oracle_far_eval(const double *M, const double *c, int d, double h, int p, int pmax,
                    const double *q, int64_t nq, double *out)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    double *H = (double *)malloc(sizeof(double) * (size_t)d * p);
    if (!H) return 2;
    double t[OR_MAXD] = {0};
    int a[OR_MAXD];
    int64_t nsub = ipow64(p, d);
    for (int64_t i = 0; i < nq; ++i) {
        for (int k = 0; k < d; ++k) t[k] = (q[i * d + k] - c[k]) * s;
        oracle_hermite_table(t, d, p, H);
        double w = 0.0;
        for (int64_t j = 0; j < nsub; ++j) {
            oracle_pos_to_mi(j, d, p, a);
            w += M[oracle_mi_to_pos(a, d, pmax)] * hermite_fn(H, p, a, d);
        }
        out[i] += w;
    }
    free(H);
    return 0;
}

/* Section 3.4, F2L lemma, eq. (farfield_to_local_formula); Appendix,
 * TransFarToLocal.  Converts R's moments (about cr) into local moments about
 * cq and adds them into L:
 *   L_beta += ((-1)^|beta| / beta!) sum_{alpha < p} M_alpha h_{alpha+beta}((cq - cr) s)   */
int oracle_f2l(const double *M, const double *cr, const double *cq, int d, double h, int p,
               int pmax, double *L)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int n = 2 * p - 1;
    double *H = (double *)malloc(sizeof(double) * (size_t)d * n);
    if (!H) return 2;
    double t[OR_MAXD] = {0};
    for (int k = 0; k < d; ++k) t[k] = (cq[k] - cr[k]) * s;
    oracle_hermite_table(t, d, n, H);
    int b[OR_MAXD], a[OR_MAXD], ab[OR_MAXD];
    int64_t nsub = ipow64(p, d);
    for (int64_t i = 0; i < nsub; ++i) {
        oracle_pos_to_mi(i, d, p, b);
        double acc = 0.0;
        for (int64_t j = 0; j < nsub; ++j) {
            oracle_pos_to_mi(j, d, p, a);
            for (int k = 0; k < d; ++k) ab[k] = a[k] + b[k];
            acc += M[oracle_mi_to_pos(a, d, pmax)] * hermite_fn(H, n, ab, d);
        }
        double sign = (mi_abs(b, d) & 1) ? -1.0 : 1.0;
        L[oracle_mi_to_pos(b, d, pmax)] += sign / mi_factorial(b, d) * acc;
    }
    free(H);
    return 0;
}

/* Section 3.3, eq. (local_moments); Appendix, AccumulateDirectLocalMoment
 * (A17: the Hermite function is taken at beta):
 *   L_beta += sum_{r in R} ((-1)^|beta| / beta!) h_beta((cq - r) s),  beta < p.   */
int oracle_direct_local(const double *pts, int64_t n, const double *cq, int d, double h, int p,
                        int pmax, double *L)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int64_t nsub = ipow64(p, d);
    double *acc = (double *)calloc((size_t)nsub, sizeof(double));
    double *H = (double *)malloc(sizeof(double) * (size_t)d * p);
    if (!acc || !H) {
        free(acc);
        free(H);
        return 2;
    }
    double t[OR_MAXD] = {0};
    int b[OR_MAXD];
    for (int64_t j = 0; j < n; ++j) {
        for (int k = 0; k < d; ++k) t[k] = (cq[k] - pts[j * d + k]) * s;
        oracle_hermite_table(t, d, p, H);
        for (int64_t i = 0; i < nsub; ++i) {
            oracle_pos_to_mi(i, d, p, b);
            acc[i] += hermite_fn(H, p, b, d);
        }
    }
    for (int64_t i = 0; i < nsub; ++i) {
        oracle_pos_to_mi(i, d, p, b);
        double sign = (mi_abs(b, d) & 1) ? -1.0 : 1.0;
        L[oracle_mi_to_pos(b, d, pmax)] += sign / mi_factorial(b, d) * acc[i];
    }
    free(acc);
    free(H);
    return 0;
}

/* Section 3.7, L2L lemma, eq. (local_to_local_translation); Appendix,
 * TransLocalToLocal (A10, A19: parent Q' -> child Q, left-hand side indexed by
 * alpha, no extra final add):
 *   Lc_alpha += sum_{alpha <= beta < p} C(beta, alpha) Lp_beta ((cc - cp) s)^{beta - alpha}   */
int oracle_l2l(const double *Lp, const double *cp, const double *cc, int d, double h, int p,
               int pmax, double *Lc)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int64_t np = ipow64(pmax, d);
    double *X = (double *)calloc((size_t)np, sizeof(double));
    if (!X) return 2;
    double x[OR_MAXD] = {0};
    for (int k = 0; k < d; ++k) x[k] = (cc[k] - cp[k]) * s;
    oracle_mi_expansion(x, d, p, pmax, X);
    int a[OR_MAXD], b[OR_MAXD], ba[OR_MAXD];
    int64_t nsub = ipow64(p, d);
    for (int64_t j = 0; j < nsub; ++j) {
        oracle_pos_to_mi(j, d, p, a);
        double acc = 0.0;
        for (int64_t k2 = 0; k2 < nsub; ++k2) {
            oracle_pos_to_mi(k2, d, p, b);
            int ge = 1;
            for (int k = 0; k < d; ++k)
                if (b[k] < a[k]) ge = 0;
            if (!ge) continue;
            for (int k = 0; k < d; ++k) ba[k] = b[k] - a[k];
            double binom = mi_factorial(b, d) / (mi_factorial(a, d) * mi_factorial(ba, d));
            acc += binom * Lp[oracle_mi_to_pos(b, d, pmax)] * X[oracle_mi_to_pos(ba, d, pmax)];
        }
        Lc[oracle_mi_to_pos(a, d, pmax)] += acc;
    }
    free(X);
    return 0;
}

/* Section 3.3 (local expansion) and Appendix, EvalLocalExpansion (A18: outer
 * loop over query points; z accumulates L_beta times the expansion term):
 *   out[i] += sum_{beta < p} L_beta ((q_i - c) s)^beta.                      */
int oracle_local_eval(const double *L, const double *c, int d, double h, int p, int pmax,
                      const double *q, int64_t nq, double *out)
{
    if (d < 1 || d > OR_MAXD || p < 1 || p > pmax) return 1;
    const double s = 1.0 / sqrt(2.0 * h * h);
    int64_t np = ipow64(pmax, d);
    double *X = (double *)calloc((size_t)np, sizeof(double));
    if (!X) return 2;
    double x[OR_MAXD] = {0};
    int b[OR_MAXD];
    int64_t nsub = ipow64(p, d);
    for (int64_t i = 0; i < nq; ++i) {
        for (int k = 0; k < d; ++k) x[k] = (q[i * d + k] - c[k]) * s;
        oracle_mi_expansion(x, d, p, pmax, X);
        double z = 0.0;
        for (int64_t j = 0; j < nsub; ++j) {
            oracle_pos_to_mi(j, d, p, b);
            int64_t pos = oracle_mi_to_pos(b, d, pmax);
            z += L[pos] * X[pos];
        }
        out[i] += z;
    }
    free(X);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 3.5, truncation error bounds.                                      */
/* ------------------------------------------------------------------------ */
static double binom_d(int n, int k)
{
    return factorial(n) / (factorial(k) * factorial(n - k));
}

/* Lemma (truncated far-field), eq. (error_bound_far_field); the local lemma,
 * eq. (error_bound_local), has the same right-hand side with r taken from Q:
 *   |R| (1-r)^-D sum_{k<D} C(D,k) (1-r^p)^k (r^p / sqrt(p!))^{D-k}.         */
double oracle_bound_far(double r, int p, int d, double nR)
{
    double rp = pow(r, (double)p);
    double a = 1.0 - rp, b = rp / sqrt(factorial(p));
    double sum = 0.0;
    for (int k = 0; k < d; ++k) sum += binom_d(d, k) * pow(a, (double)k) * pow(b, (double)(d - k));
    return nR / pow(1.0 - r, (double)d) * sum;
}

double oracle_bound_local(double r, int p, int d, double nR)
{
    return oracle_bound_far(r, p, d, nR);
}

/* Lemma (far-to-local), eq. (error_bound_far_to_local):
 *   |R| (1-2r)^-2D sum_{k<D} C(D,k) ((1-(2r)^p)^2)^k ((2r)^p (2-(2r)^p) / sqrt(p!))^{D-k}.   */
double oracle_bound_f2l(double r, int p, int d, double nR)
{
    double tp = pow(2.0 * r, (double)p);
    double a = (1.0 - tp) * (1.0 - tp), b = tp * (2.0 - tp) / sqrt(factorial(p));
    double sum = 0.0;
    for (int k = 0; k < d; ++k) sum += binom_d(d, k) * pow(a, (double)k) * pow(b, (double)(d - k));
    return nR / pow(1.0 - 2.0 * r, (double)(2 * d)) * sum;
}

/* ------------------------------------------------------------------------ */
/* Section 2.2, node-pair distance bounds (eqs. 5-6):                         */
/*   d^l = sqrt(sum_k (max(R.l-Q.u, 0) + max(Q.l-R.u, 0))^2)                  */
/*   d^u = sqrt(sum_k max(R.u-Q.l, Q.u-R.l)^2)                                */
/* ------------------------------------------------------------------------ */
void oracle_dist_bounds(const double *qlo, const double *qhi, const double *rlo,
                        const double *rhi, int d, double *dl, double *du)
{
    double sl = 0.0, su = 0.0;
    for (int k = 0; k < d; ++k) {
        double a = rlo[k] - qhi[k], b = qlo[k] - rhi[k];
        double g = (a > 0 ? a : 0.0) + (b > 0 ? b : 0.0);
        sl += g * g;
        double u1 = rhi[k] - qlo[k], u2 = qhi[k] - rlo[k];
        double u = u1 > u2 ? u1 : u2;
        su += u * u;
    }
    *dl = sqrt(sl);
    *du = sqrt(su);
}

/* ------------------------------------------------------------------------ */
/* Section 3.6, order selection; Section 3.8, ChooseBestMethod.               */
/* A return of 0 means "infinity" (no admissible order <= p_max).            */
/* ------------------------------------------------------------------------ */
static double max_width(const double *lo, const double *hi, int d)
{
    double w = 0.0;
    for (int k = 0; k < d; ++k)
        if (hi[k] - lo[k] > w) w = hi[k] - lo[k];
    return w;
}

/* Alg. FarFieldOrder: r = max width of R / (2h); least p with bound <= tau.
 * Comparisons are inclusive (A29) so an exactly-zero bound prunes at tau = 0. */
int oracle_far_field_order(double wR, double h, int d, double nR, double tau, int pmax)
{
    double r = wR / (2.0 * h);
    if (r >= 1.0) return 0;
    for (int p = 1; p <= pmax; ++p)
        if (oracle_bound_far(r, p, d, nR) <= tau) return p;
    return 0;
}

/* Alg. LocalAccumulationOrder: r = max width of Q / (2h). */
int oracle_local_order(double wQ, double h, int d, double nR, double tau, int pmax)
{
    double r = wQ / (2.0 * h);
    if (r >= 1.0) return 0;
    for (int p = 1; p <= pmax; ++p)
        if (oracle_bound_local(r, p, d, nR) <= tau) return p;
    return 0;
}

/* Alg. ConvertFarFieldToLocalOrder, conservative reading (A11): the lemma
 * needs every point within r h of its centre in each dimension with r < 1/2,
 * i.e. r = max(width_Q, width_R) / (2h) ("side length less than h"), and its
 * bound is evaluated with that r (the formula itself contains 2r).
 * literal != 0 selects the printed radius width/(4h) instead (for tests). */
int oracle_f2l_order(double wQ, double wR, double h, int d, double nR, double tau, int pmax,
                     int literal)
{
    double w = wQ > wR ? wQ : wR;
    double r = literal ? w / (4.0 * h) : w / (2.0 * h);
    if (r >= 0.5) return 0;
    for (int p = 1; p <= pmax; ++p)
        if (oracle_bound_f2l(r, p, d, nR) <= tau) return p;
    return 0;
}

/* Centroid approximation T(c, 1) with the finite-difference bound used in the
 * proof of the global-error theorem (Section 3.10; A13):
 *   |R| max(K(d^l) - K(d_c), K(d_c) - K(d^u)),  d_c = ||Q.c - R.c||.        */
double oracle_centroid_bound(double dl, double du, double dc, double h, double nR)
{
    double inv2h2 = 1.0 / (2.0 * h * h);
    double kl = exp(-dl * dl * inv2h2), ku = exp(-du * du * inv2h2), kc = exp(-dc * dc * inv2h2);
    double a = kl - kc, b = kc - ku;
    return nR * (a > b ? a : b);
}

enum { OR_E = 0, OR_F = 1, OR_D = 2, OR_T = 3 };

/* Alg. ChooseBestMethod with the cost reading A12:
 *   c_F = D N_Q p_F^D,  c_D = D N_R p_D^D,  c_T = D p_T^{2D},  c_E = D N_Q N_R,
 * an order of 0 (infinity) meaning infinite cost; ties go F, D, T, E.  The
 * T order is 1 whenever the centroid bound meets tau (A13).
 * force: 0 = best method; 1/2/3 = only F/D/T may be chosen (operator tests);
 *        4 = only the centroid form of T (ablation).                        */
int oracle_choose_method(const double *qlo, const double *qhi, const double *rlo,
                         const double *rhi, int d, double nQ, double nR, double h, double tau,
                         int pmax, int force, int literal_f2l, int *order)
{
    double wQ = max_width(qlo, qhi, d), wR = max_width(rlo, rhi, d);
    int pF = oracle_far_field_order(wR, h, d, nR, tau, pmax);
    int pD = oracle_local_order(wQ, h, d, nR, tau, pmax);
    int pT = oracle_f2l_order(wQ, wR, h, d, nR, tau, pmax, literal_f2l);
    double qc[OR_MAXD], rc[OR_MAXD];
    for (int k = 0; k < d; ++k) {
        qc[k] = (qlo[k] + qhi[k]) / 2.0;
        rc[k] = (rlo[k] + rhi[k]) / 2.0;
    }
    double dl, du, dc2 = 0.0;
    oracle_dist_bounds(qlo, qhi, rlo, rhi, d, &dl, &du);
    for (int k = 0; k < d; ++k) dc2 += (qc[k] - rc[k]) * (qc[k] - rc[k]);
    if (oracle_centroid_bound(dl, du, sqrt(dc2), h, nR) <= tau) pT = 1;
    if (force == 1) pD = pT = 0;
    if (force == 2) pF = pT = 0;
    if (force == 3) pF = pD = 0;
    if (force == 4) {
        pF = pD = 0;
        pT = (oracle_centroid_bound(dl, du, sqrt(dc2), h, nR) <= tau) ? 1 : 0;
    }
    double cF = pF ? d * nQ * pow((double)pF, (double)d) : INFINITY;
    double cD = pD ? d * nR * pow((double)pD, (double)d) : INFINITY;
    double cT = pT ? d * pow((double)pT, (double)(2 * d)) : INFINITY;
    double cE = d * nQ * nR;
    double m = cF;
    if (cD < m) m = cD;
    if (cT < m) m = cT;
    if (cE < m) m = cE;
    if (cF == m && pF) {
        *order = pF;
        return OR_F;
    }
    if (cD == m && pD) {
        *order = pD;
        return OR_D;
    }
    if (cT == m && pT) {
        *order = pT;
        return OR_T;
    }
    *order = 0;
    return OR_E;
}

/* ------------------------------------------------------------------------ */
/* Section 3.9, the hierarchical FGT: DFGTMain, DFGTInitQ, DFGTInitR, DFGT,  */
/* CanSummarize, Summarize, DFGTBase, DFGTPost, in the paper's order.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d, pmax, force, literal_f2l;
    double h, eps, NR;
    int64_t np; /* pmax^d */
    /* query tree (tree order) */
    const double *qx; /* permuted query points [nq][d] */
    double *qlo, *qhi, *qc;
    int64_t *qb, *qe;
    int32_t *ql, *qr;
    double *Gl, *Gu, *Dl, *Du, *L;
    int *pL;
    int64_t *covN;
    /* per query point */
    double *Glp, *Gup, *GE, *GF, *GL;
    int64_t *covp;
    /* reference tree */
    const double *rx;
    double *rlo, *rhi, *rc;
    int64_t *rb, *re;
    int32_t *rl, *rr;
    double *M;
    /* optional exact sums (tree order) for invariant checks */
    const double *Gexact;
    int64_t *stats;
} dfgt_ctx;

/* stats layout */
enum {
    ST_PAIRS = 0,     /* node pairs visited */
    ST_PRUNE_F = 1,
    ST_PRUNE_D = 2,
    ST_PRUNE_T = 3,
    ST_PRUNE_C = 4,   /* T prunes with order 1 */
    ST_BASE = 5,      /* leaf-leaf base cases */
    ST_BASE_PAIRS = 6, /* point pairs evaluated exhaustively */
    ST_VIOL = 7,      /* bound-invariant violations observed */
    ST_MAXORD = 8,
    ST_COUNT = 16
};

static int is_leaf_q(dfgt_ctx *c, int64_t n) { return c->ql[n] < 0; }
static int is_leaf_r(dfgt_ctx *c, int64_t n) { return c->rl[n] < 0; }

static double kern(double dist, double h) { return exp(-dist * dist / (2.0 * h * h)); }

/* DFGTInitR: far-field moments at leaves by AccumulateFarFieldMoment, at
 * internal nodes by TransFarToFar from both children (post-order). */
static void dfgt_init_r(dfgt_ctx *c, int64_t R)
{
    double *MR = c->M + R * c->np;
    memset(MR, 0, sizeof(double) * (size_t)c->np);
    if (is_leaf_r(c, R)) {
        oracle_p2m(c->rx + c->rb[R] * c->d, c->re[R] - c->rb[R], c->d, c->rc + R * c->d, c->h,
                   c->pmax, c->pmax, MR);
    } else {
        int64_t a = c->rl[R], b = c->rr[R];
        dfgt_init_r(c, a);
        dfgt_init_r(c, b);
        oracle_f2f(c->M + a * c->np, c->rc + a * c->d, c->rc + R * c->d, c->d, c->h, c->pmax, MR);
        oracle_f2f(c->M + b * c->np, c->rc + b * c->d, c->rc + R * c->d, c->d, c->h, c->pmax, MR);
    }
}

/* DFGTInitQ: G^l = 0, G^u = |R|, Delta = 0, L = 0 on every node; per-point
 * bounds and the three partial sums at leaves. */
static void dfgt_init_q(dfgt_ctx *c, int64_t Q)
{
    c->Gl[Q] = 0.0;
    c->Gu[Q] = c->NR;
    c->Dl[Q] = 0.0;
    c->Du[Q] = 0.0;
    c->covN[Q] = 0;
    c->pL[Q] = 0;
    memset(c->L + Q * c->np, 0, sizeof(double) * (size_t)c->np);
    if (is_leaf_q(c, Q)) {
        for (int64_t i = c->qb[Q]; i < c->qe[Q]; ++i) {
            c->Glp[i] = 0.0;
            c->Gup[i] = c->NR;
            c->GE[i] = c->GF[i] = c->GL[i] = 0.0;
            c->covp[i] = 0;
        }
    } else {
        dfgt_init_q(c, c->ql[Q]);
        dfgt_init_q(c, c->qr[Q]);
    }
}

static void check_point_bounds(dfgt_ctx *c, int64_t i)
{
    if (!c->Gexact) return;
    double g = c->Gexact[i], tol = 1e-9 * (1.0 + g);
    if (c->Glp[i] > g + tol || c->Gup[i] < g - tol) c->stats[ST_VIOL]++;
}

static void check_node_bounds(dfgt_ctx *c, int64_t Q, double gl, double gu)
{
    if (!c->Gexact) return;
    for (int64_t i = c->qb[Q]; i < c->qe[Q]; ++i) {
        double g = c->Gexact[i], tol = 1e-9 * (1.0 + g);
        if (gl > g + tol || gu < g - tol) {
            c->stats[ST_VIOL]++;
            return;
        }
    }
}

/* DFGTBase: exact contribution of leaf R to leaf Q; per-point bounds absorb
 * the postponed changes, then the node's bounds are refined to the min/max
 * over its points and the postponed changes are cleared. */
static void dfgt_base(dfgt_ctx *c, int64_t Q, int64_t R)
{
    int d = c->d;
    double gl = INFINITY, gu = -INFINITY;
    c->stats[ST_BASE]++;
    for (int64_t i = c->qb[Q]; i < c->qe[Q]; ++i) {
        c->Glp[i] += c->Dl[Q];
        c->Gup[i] += c->Du[Q];
        c->covp[i] += c->covN[Q] + (c->re[R] - c->rb[R]);
        const double *q = c->qx + i * d;
        for (int64_t j = c->rb[R]; j < c->re[R]; ++j) {
            const double *r = c->rx + j * d;
            double d2 = 0.0;
            for (int k = 0; k < d; ++k) d2 += (q[k] - r[k]) * (q[k] - r[k]);
            double v = exp(-d2 / (2.0 * c->h * c->h));
            c->Glp[i] += v;
            c->GE[i] += v;
            c->Gup[i] += v - 1.0;
        }
        c->stats[ST_BASE_PAIRS] += c->re[R] - c->rb[R];
        if (c->Glp[i] < gl) gl = c->Glp[i];
        if (c->Gup[i] > gu) gu = c->Gup[i];
    }
    c->Gl[Q] = gl;
    c->Gu[Q] = gu;
    c->Dl[Q] = 0.0;
    c->Du[Q] = 0.0;
    c->covN[Q] = 0;
}

/* Summarize: add the bound changes of the pair, then evaluate the far field
 * (F), accumulate direct local moments (D) or translate far field to local
 * (T) at the chosen order. */
static void dfgt_summarize(dfgt_ctx *c, int64_t Q, int64_t R, int method, int p, double dlo,
                           double dup)
{
    int d = c->d;
    c->Dl[Q] += dlo;
    c->Du[Q] += dup;
    c->covN[Q] += c->re[R] - c->rb[R];
    if (p > c->stats[ST_MAXORD]) c->stats[ST_MAXORD] = p;
    if (method == OR_F) {
        c->stats[ST_PRUNE_F]++;
        oracle_far_eval(c->M + R * c->np, c->rc + R * d, d, c->h, p, c->pmax, c->qx + c->qb[Q] * d,
                        c->qe[Q] - c->qb[Q], c->GF + c->qb[Q]);
    } else if (method == OR_D) {
        c->stats[ST_PRUNE_D]++;
        oracle_direct_local(c->rx + c->rb[R] * d, c->re[R] - c->rb[R], c->qc + Q * d, d, c->h, p,
                            c->pmax, c->L + Q * c->np);
        if (p > c->pL[Q]) c->pL[Q] = p;
    } else {
        c->stats[p == 1 ? ST_PRUNE_C : ST_PRUNE_T]++;
        oracle_f2l(c->M + R * c->np, c->rc + R * d, c->qc + Q * d, d, c->h, p, c->pmax,
                   c->L + Q * c->np);
        if (p > c->pL[Q]) c->pL[Q] = p;
    }
}

/* DFGT(Q, R): the core recursion. */
static void dfgt_rec(dfgt_ctx *c, int64_t Q, int64_t R)
{
    int d = c->d;
    double nR = (double)(c->re[R] - c->rb[R]), nQ = (double)(c->qe[Q] - c->qb[Q]);
    double dl, du;
    c->stats[ST_PAIRS]++;
    oracle_dist_bounds(c->qlo + Q * d, c->qhi + Q * d, c->rlo + R * d, c->rhi + R * d, d, &dl, &du);
    double dlo = nR * kern(du, c->h);
    double dup = nR * (kern(dl, c->h) - 1.0);
    double glnew = c->Gl[Q] + c->Dl[Q] + dlo;
    double gunew = c->Gu[Q] + c->Du[Q] + dup;
    check_node_bounds(c, Q, glnew, gunew);
    /* CanSummarize: ChooseBestMethod(Q, R, eps |R| G^{l,new}(Q) / |R_total|) != E */
    int p = 0;
    int method = oracle_choose_method(c->qlo + Q * d, c->qhi + Q * d, c->rlo + R * d, c->rhi + R * d,
                                      d, nQ, nR, c->h, c->eps * nR * glnew / c->NR, c->pmax,
                                      c->force, c->literal_f2l, &p);
    if (method != OR_E) {
        dfgt_summarize(c, Q, R, method, p, dlo, dup);
        return;
    }
    if (is_leaf_q(c, Q)) {
        if (is_leaf_r(c, R)) {
            dfgt_base(c, Q, R);
        } else {
            dfgt_rec(c, Q, c->rl[R]);
            dfgt_rec(c, Q, c->rr[R]);
        }
        return;
    }
    int64_t QL = c->ql[Q], QR = c->qr[Q];
    c->Dl[QL] += c->Dl[Q];
    c->Dl[QR] += c->Dl[Q];
    c->Du[QL] += c->Du[Q];
    c->Du[QR] += c->Du[Q];
    c->covN[QL] += c->covN[Q];
    c->covN[QR] += c->covN[Q];
    c->Dl[Q] = 0.0;
    c->Du[Q] = 0.0;
    c->covN[Q] = 0;
    if (is_leaf_r(c, R)) {
        dfgt_rec(c, QL, R);
        dfgt_rec(c, QR, R);
    } else {
        dfgt_rec(c, QL, c->rl[R]);
        dfgt_rec(c, QL, c->rr[R]);
        dfgt_rec(c, QR, c->rl[R]);
        dfgt_rec(c, QR, c->rr[R]);
    }
    double a = c->Gl[QL] + c->Dl[QL], b = c->Gl[QR] + c->Dl[QR];
    c->Gl[Q] = a < b ? a : b;
    a = c->Gu[QL] + c->Du[QL];
    b = c->Gu[QR] + c->Du[QR];
    c->Gu[Q] = a > b ? a : b;
    check_node_bounds(c, Q, c->Gl[Q], c->Gu[Q]);
}

/* DFGTPost: L2L to both children at the largest order used so far (A21),
 * push postponed changes, recurse; at a leaf add the postponed changes to the
 * points, evaluate the local expansion (the D-and-T part, A20) and combine the
 * three partial sums. */
static void dfgt_post(dfgt_ctx *c, int64_t Q)
{
    int d = c->d;
    if (is_leaf_q(c, Q)) {
        double gl = INFINITY, gu = -INFINITY;
        for (int64_t i = c->qb[Q]; i < c->qe[Q]; ++i) {
            c->Glp[i] += c->Dl[Q];
            c->Gup[i] += c->Du[Q];
            c->covp[i] += c->covN[Q];
            if (c->Glp[i] < gl) gl = c->Glp[i];
            if (c->Gup[i] > gu) gu = c->Gup[i];
            check_point_bounds(c, i);
        }
        if (c->pL[Q] > 0)
            oracle_local_eval(c->L + Q * c->np, c->qc + Q * d, d, c->h, c->pL[Q], c->pmax,
                              c->qx + c->qb[Q] * d, c->qe[Q] - c->qb[Q], c->GL + c->qb[Q]);
        c->Gl[Q] = gl;
        c->Gu[Q] = gu;
        c->Dl[Q] = c->Du[Q] = 0.0;
        c->covN[Q] = 0;
        memset(c->L + Q * c->np, 0, sizeof(double) * (size_t)c->np);
        return;
    }
    int64_t ch[2] = {c->ql[Q], c->qr[Q]};
    for (int t = 0; t < 2; ++t) {
        int64_t C = ch[t];
        if (c->pL[Q] > 0) {
            oracle_l2l(c->L + Q * c->np, c->qc + Q * d, c->qc + C * d, d, c->h, c->pL[Q], c->pmax,
                       c->L + C * c->np);
            if (c->pL[Q] > c->pL[C]) c->pL[C] = c->pL[Q];
        }
        c->Dl[C] += c->Dl[Q];
        c->Du[C] += c->Du[Q];
        c->covN[C] += c->covN[Q];
    }
    memset(c->L + Q * c->np, 0, sizeof(double) * (size_t)c->np);
    c->Dl[Q] = c->Du[Q] = 0.0;
    c->covN[Q] = 0;
    dfgt_post(c, ch[0]);
    dfgt_post(c, ch[1]);
    c->Gl[Q] = c->Gl[ch[0]] < c->Gl[ch[1]] ? c->Gl[ch[0]] : c->Gl[ch[1]];
    c->Gu[Q] = c->Gu[ch[0]] > c->Gu[ch[1]] ? c->Gu[ch[0]] : c->Gu[ch[1]];
}

typedef struct {
    int32_t *perm;
    double *lo, *hi, *c;
    int64_t *b, *e;
    int32_t *l, *r, *sd;
    double *sc;
    double *x;
    int64_t m;
} tree_tmp;

static int tree_alloc_build(const double *x, int64_t n, int d, int leaf, tree_tmp *t)
{
    int64_t cap = 2 * n + 1;
    t->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    t->lo = (double *)malloc(sizeof(double) * (size_t)(cap * d));
    t->hi = (double *)malloc(sizeof(double) * (size_t)(cap * d));
    t->c = (double *)malloc(sizeof(double) * (size_t)(cap * d));
    t->b = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    t->e = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    t->l = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    t->r = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    t->sd = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    t->sc = (double *)malloc(sizeof(double) * (size_t)cap);
    t->x = (double *)malloc(sizeof(double) * (size_t)(n * d));
    if (!t->perm || !t->lo || !t->hi || !t->c || !t->b || !t->e || !t->l || !t->r || !t->sd ||
        !t->sc || !t->x)
        return 2;
    int rc = oracle_build_kdtree(x, n, d, leaf, cap, t->perm, t->lo, t->hi, t->b, t->e, t->l, t->r,
                                 t->sd, t->sc, &t->m);
    if (rc) return rc;
    for (int64_t i = 0; i < t->m; ++i)
        for (int k = 0; k < d; ++k) t->c[i * d + k] = (t->lo[i * d + k] + t->hi[i * d + k]) / 2.0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) t->x[i * d + k] = x[(int64_t)t->perm[i] * d + k];
    return 0;
}

static void tree_free(tree_tmp *t)
{
    free(t->perm);
    free(t->lo);
    free(t->hi);
    free(t->c);
    free(t->b);
    free(t->e);
    free(t->l);
    free(t->r);
    free(t->sd);
    free(t->sc);
    free(t->x);
}

/* DFGTMain: build both trees, initialise, run the recursion from the roots,
 * post-process.  Outputs (user query order):
 *   G      the approximation G~(q_i, R)
 *   Gl, Gu the final per-point lower/upper bounds (may be NULL)
 *   cov    reference points accounted per query (may be NULL)
 *   stats  ST_COUNT counters (may be NULL)
 * Gexact (user order, may be NULL) enables the bound-invariant checks.
 * force / literal_f2l: see oracle_choose_method.                            */
int oracle_dfgt(const double *q, int64_t nq, const double *r, int64_t nr, int d, double h,
                double eps, int leaf, int pmax, int force, int literal_f2l, const double *Gexact,
                double *G, double *Glo, double *Gup, int64_t *cov, int64_t *stats)
{
    if (nq < 1 || nr < 1 || d < 1 || d > OR_MAXD || !(h > 0) || pmax < 1 || leaf < 1) return 1;
    tree_tmp tq, tr;
    memset(&tq, 0, sizeof(tq));
    memset(&tr, 0, sizeof(tr));
    int rc = tree_alloc_build(q, nq, d, leaf, &tq);
    if (!rc) rc = tree_alloc_build(r, nr, d, leaf, &tr);
    int64_t st_local[ST_COUNT];
    memset(st_local, 0, sizeof(st_local));
    dfgt_ctx c;
    memset(&c, 0, sizeof(c));
    double *Gx = NULL;
    if (!rc) {
        c.d = d;
        c.pmax = pmax;
        c.force = force;
        c.literal_f2l = literal_f2l;
        c.h = h;
        c.eps = eps;
        c.NR = (double)nr;
        c.np = ipow64(pmax, d);
        c.qx = tq.x;
        c.qlo = tq.lo;
        c.qhi = tq.hi;
        c.qc = tq.c;
        c.qb = tq.b;
        c.qe = tq.e;
        c.ql = tq.l;
        c.qr = tq.r;
        c.rx = tr.x;
        c.rlo = tr.lo;
        c.rhi = tr.hi;
        c.rc = tr.c;
        c.rb = tr.b;
        c.re = tr.e;
        c.rl = tr.l;
        c.rr = tr.r;
        int64_t mq = tq.m, mr = tr.m;
        c.Gl = (double *)malloc(sizeof(double) * (size_t)mq);
        c.Gu = (double *)malloc(sizeof(double) * (size_t)mq);
        c.Dl = (double *)malloc(sizeof(double) * (size_t)mq);
        c.Du = (double *)malloc(sizeof(double) * (size_t)mq);
        c.L = (double *)malloc(sizeof(double) * (size_t)(mq * c.np));
        c.pL = (int *)malloc(sizeof(int) * (size_t)mq);
        c.covN = (int64_t *)malloc(sizeof(int64_t) * (size_t)mq);
        c.Glp = (double *)malloc(sizeof(double) * (size_t)nq);
        c.Gup = (double *)malloc(sizeof(double) * (size_t)nq);
        c.GE = (double *)malloc(sizeof(double) * (size_t)nq);
        c.GF = (double *)malloc(sizeof(double) * (size_t)nq);
        c.GL = (double *)malloc(sizeof(double) * (size_t)nq);
        c.covp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nq);
        c.M = (double *)malloc(sizeof(double) * (size_t)(mr * c.np));
        c.stats = stats ? stats : st_local;
        if (stats) memset(stats, 0, sizeof(int64_t) * ST_COUNT);
        if (Gexact) {
            Gx = (double *)malloc(sizeof(double) * (size_t)nq);
            if (Gx)
                for (int64_t i = 0; i < nq; ++i) Gx[i] = Gexact[tq.perm[i]];
            c.Gexact = Gx;
        }
        if (!c.Gl || !c.Gu || !c.Dl || !c.Du || !c.L || !c.pL || !c.covN || !c.Glp || !c.Gup ||
            !c.GE || !c.GF || !c.GL || !c.covp || !c.M || (Gexact && !Gx)) {
            rc = 2;
        } else {
            dfgt_init_q(&c, 0);
            dfgt_init_r(&c, 0);
            dfgt_rec(&c, 0, 0);
            dfgt_post(&c, 0);
            for (int64_t i = 0; i < nq; ++i) {
                int64_t u = tq.perm[i];
                G[u] = c.GL[i] + c.GF[i] + c.GE[i];
                if (Glo) Glo[u] = c.Glp[i];
                if (Gup) Gup[u] = c.Gup[i];
                if (cov) cov[u] = c.covp[i];
            }
        }
    }
    free(Gx);
    free(c.Gl);
    free(c.Gu);
    free(c.Dl);
    free(c.Du);
    free(c.L);
    free(c.pL);
    free(c.covN);
    free(c.Glp);
    free(c.Gup);
    free(c.GE);
    free(c.GF);
    free(c.GL);
    free(c.covp);
    free(c.M);
    tree_free(&tq);
    tree_free(&tr);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Section 1, eq. (4): least-squares cross-validation score from exact sums.  */
/* The convolution K_h * K_h of two normalised Gaussians is the normalised    */
/* Gaussian of bandwidth sqrt(2) h (A7; the text's "2h" is taken as sqrt 2 h). */
/*   S_h   = sum_j (G_h(r_j) - 1)       (leave-one-out: the self term removed) */
/*   variant 0 (eq. 4 literally, both terms leave-one-out):                   */
/*     CV = [(4 pi h^2)^{-D/2} S_{sqrt2 h} - 2 (2 pi h^2)^{-D/2} S_h] / (N (N-1))  */
/*   variant 1 (integral of the squared estimate keeps its diagonal):         */
/*     CV = (4 pi h^2)^{-D/2} (N + S_{sqrt2 h}) / N^2 - 2 (2 pi h^2)^{-D/2} S_h / (N (N-1))  */
/* dcv (may be NULL) receives dCV/dh.                                         */
/* ------------------------------------------------------------------------ */
int oracle_lscv(const double *x, int64_t n, int d, const double *hs, int nh, int variant,
                double *cv, double *dcv)
{
    if (n < 2 || d < 1 || d > OR_MAXD || nh < 1) return 1;
    double *G1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *G2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *H1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *H2 = (double *)malloc(sizeof(double) * (size_t)n);
    if (!G1 || !G2 || !H1 || !H2) {
        free(G1);
        free(G2);
        free(H1);
        free(H2);
        return 2;
    }
    const double PI = 3.14159265358979323846;
    double N = (double)n;
    for (int k = 0; k < nh; ++k) {
        double h = hs[k], h2 = sqrt(2.0) * h;
        oracle_naive_kde_grad(x, n, x, n, d, h, G1, H1, NULL);
        oracle_naive_kde_grad(x, n, x, n, d, h2, G2, H2, NULL);
        double S1 = 0.0, S2 = 0.0, dS1 = 0.0, dS2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            S1 += G1[i] - 1.0;
            S2 += G2[i] - 1.0;
            dS1 += H1[i];
            dS2 += H2[i] * sqrt(2.0); /* d/dh of G at sqrt(2) h, chain rule */
        }
        double a = pow(4.0 * PI * h * h, -d / 2.0), b = pow(2.0 * PI * h * h, -d / 2.0);
        double da = -d * a / h, db = -d * b / h;
        double v, dv;
        if (variant == 0) {
            v = (a * S2 - 2.0 * b * S1) / (N * (N - 1.0));
            dv = (da * S2 + a * dS2 - 2.0 * (db * S1 + b * dS1)) / (N * (N - 1.0));
        } else {
            v = a * (N + S2) / (N * N) - 2.0 * b * S1 / (N * (N - 1.0));
            dv = (da * (N + S2) + a * dS2) / (N * N) - 2.0 * (db * S1 + b * dS1) / (N * (N - 1.0));
        }
        cv[k] = v;
        if (dcv) dcv[k] = dv;
    }
    free(G1);
    free(G2);
    free(H1);
    free(H2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 1, the kernel density estimate: p_h(q) = G(q, R) / (|R| V_Dh), with */
/* V_Dh the integral of the kernel, (2 pi h^2)^{D/2} for the Gaussian.        */
/* ------------------------------------------------------------------------ */
int oracle_kde_density(const double *q, int64_t nq, const double *r, int64_t nr, int d, double h, double *out)
{
    if (nr < 1) return 1;
    int rc = oracle_naive_kde(q, nq, r, nr, d, h, out);
    if (rc) return rc;
    const double PI = 3.14159265358979323846;
    const double V = pow(2.0 * PI * h * h, d / 2.0);
    for (int64_t i = 0; i < nq; ++i) out[i] /= (double)nr * V;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section 1, likelihood cross-validation score:                              */
/*   CV_LK(h) = (1/N) sum_j log p_{h,-j}(r_j),                                 */
/*   p_{h,-j}(r_j) = S_j / ((N-1) V_Dh),  S_j = sum_{i != j} K_h(|r_j - r_i|)  */
/* (the estimate from all points but r_j).  S_j is summed directly over        */
/* i != j (Neumaier), not as G - 1.  dcv (may be NULL) receives dCV_LK/dh =    */
/* (1/N) sum_j S_j'/S_j - D/h with S_j' = sum_{i != j} K |r_j - r_i|^2 / h^3.  */
/* A point with S_j = 0 (underflow at tiny h) gives -inf.                      */
/* ------------------------------------------------------------------------ */
int oracle_lcv(const double *x, int64_t n, int d, const double *hs, int nh, double *cv, double *dcv)
{
    if (n < 2 || d < 1 || d > OR_MAXD || nh < 1) return 1;
    const double PI = 3.14159265358979323846;
    for (int k = 0; k < nh; ++k) {
        const double h = hs[k];
        if (!(h > 0.0)) return 1;
        const double inv2h2 = 1.0 / (2.0 * h * h);
        double acc = 0.0, dacc = 0.0;
        int neg_inf = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : acc, dacc) reduction(| : neg_inf)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0, c = 0.0, ds = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                if (i == j) continue;
                double t = 0.0;
                for (int m = 0; m < d; ++m) {
                    double v = x[j * d + m] - x[i * d + m];
                    t += v * v;
                }
                double kv = exp(-t * inv2h2);
                double y = kv, u = s + y; /* Neumaier */
                c += fabs(s) >= fabs(y) ? (s - u) + y : (y - u) + s;
                s = u;
                ds += kv * t / (h * h * h);
            }
            s += c;
            if (s > 0.0) {
                acc += log(s);
                dacc += ds / s;
            } else {
                neg_inf = 1;
            }
        }
        const double N = (double)n;
        const double logV = 0.5 * d * log(2.0 * PI * h * h);
        cv[k] = neg_inf ? -INFINITY : acc / N - log(N - 1.0) - logV;
        if (dcv) dcv[k] = neg_inf ? NAN : dacc / N - d / h;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
