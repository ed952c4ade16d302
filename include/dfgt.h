/*
 * dfgt.h - C ABI of the MI355X dual-tree fast Gauss transform library (libdfgt.so).
 *
 * The library computes the Gaussian kernel sums of Section 1.1,
 * eq. (gaussian_kernel_sums), of "Dual-Tree Fast Gauss Transforms"
 * (Lee, Gray, Moore):
 *
 *     G(q_i, R) = sum_{r_j in R} exp(-||q_i - r_j||^2 / (2 h^2))
 *
 * with the hard per-query relative error bound |G~ - G| <= eps * G of the
 * paper's Definition (bounding the relative error) and its global-error
 * theorem (Section 3.10), by the hierarchical DFGT of Section 3.9.
 *
 * Conventions shared by every entry point
 *   - Plain C types only.  Pointers named *_dev are device (HIP) pointers,
 *     *_host are host pointers.  The caller owns every buffer it passes; the
 *     library owns tree handles and its internal workspace.
 *   - Points are float64, row-major [n][d].
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on that stream.  Entry points that return host results
 *     (lscv, backward h-gradients, stats, exports) synchronise the stream.
 *   - Every call returns a dfgt_status; on failure dfgt_last_error() returns a
 *     message for the calling thread.  No C++ exception crosses the ABI.
 *   - Handles are not thread-safe: use one handle from one thread at a time.
 */
#ifndef DFGT_H
#define DFGT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dfgt_status {
    DFGT_OK = 0,
    DFGT_EINVAL = 1, /* an argument is out of range (message says which) */
    DFGT_ENOMEM = 2, /* device or host allocation failed */
    DFGT_EHIP = 3,   /* a HIP runtime call failed */
    DFGT_EQUEUE = 4, /* the traversal's lists outgrew their buffers after every retry
                        (eager calls grow and rerun up to 12 times), or a captured
                        batch's replay overflowed them (dfgt_batch_check) */
    DFGT_EBOUND = 5  /* the error guarantee cannot be certified for this input */
} dfgt_status;

/* Precision of the exhaustive leaf-leaf sums (DFGTBase, Section 3.9). */
enum {
    DFGT_PREC_MIXED = 0, /* FP64 coordinate differences, FP32 exp, FP64 per-query sums */
    DFGT_PREC_FP64 = 1   /* FP64 throughout */
};

/* Restriction of the summarisation methods (Section 3.2's E, F(c,p), D(c,p),
 * T(c,p)); anything other than DFGT_FORCE_NONE is a test and ablation knob. */
enum {
    DFGT_FORCE_NONE = 0,
    DFGT_FORCE_F = 1,        /* only far-field evaluation may prune */
    DFGT_FORCE_D = 2,        /* only direct local accumulation */
    DFGT_FORCE_T = 3,        /* only far-to-local translation (incl. centroid form) */
    DFGT_FORCE_CENTROID = 4, /* only the centroid T(c,1) with the finite-difference bound */
    DFGT_FORCE_EXACT = 5     /* no pruning at all: every leaf pair is exhaustive */
};

typedef struct dfgt_options {
    int32_t leaf_size;    /* kd-tree leaf threshold (Alg. BuildKdTree); 0 = 32 */
    int32_t p_max;        /* terms per dimension kept in every expansion; 0 = the
                             paper's experimental table (Section 3.9): 6 for D<=2,
                             4 for D=3, 2 for D=4,5, 1 for D>=6 */
    int32_t precision;    /* DFGT_PREC_* */
    int32_t force_method; /* DFGT_FORCE_* */
    int32_t profile;      /* 1: gauss_sum records HIP events around its kernel
                             launches on the caller's stream and reports the
                             per-kernel time in dfgt_stats (adds a few us per
                             launch); 0: off */
    float cost_exhaustive; /* multiplier of the exhaustive cost c_E = D N_Q N_R in
                              ChooseBestMethod (Section 3.8); 0 = 1.  The series
                              costs carry this GPU's measured weights per unit
                              (far-field 2, direct local 3, far-to-local 3 in
                              exhaustive pairs; 50, 320, 50 when p_max^D > 512);
                              with all weights 1 the model is the paper's.
                              Smaller values choose exhaustive sums more often.
                              Any value keeps the error guarantee (it only picks
                              among methods whose bounds hold) */
    int32_t reserved[2];  /* must be zero */
} dfgt_options;

/* Counters of one gauss_sum call (summed over its bandwidths). */
typedef struct dfgt_stats {
    int64_t node_pairs;     /* node pairs visited by the traversal */
    int64_t prune_f;        /* pairs summarised by far-field evaluation */
    int64_t prune_d;        /* ... by direct local accumulation */
    int64_t prune_t;        /* ... by far-to-local translation, order >= 2 */
    int64_t prune_centroid; /* ... by the centroid form T(c,1) */
    int64_t base_leaf_pairs;  /* exhaustive leaf-leaf pairs */
    int64_t base_point_pairs; /* exhaustive point pairs */
    int64_t levels;         /* traversal levels executed */
    int64_t max_order;      /* largest expansion order used */
    int64_t fp64_groups;    /* exhaustive groups computed in FP64 by the underflow guard */
    int64_t segments;       /* (query node, bandwidth) segments processed by the traversal */
    int64_t max_segment;    /* most reference nodes in one segment */
    int64_t local_nodes;    /* internal (node, bandwidth) pairs with local-moment ops */
    int64_t max_local_ops;  /* most local-moment ops of one (node, bandwidth) */
    int64_t mfma_tiles;     /* parts of the call whose exhaustive sums ran on the
                               matrix cores (D >= 8, mixed precision), else 0 */
    int64_t parts;          /* job parts the call ran in turn (the jobs of a call
                               whose traversal buffers would exceed the memory
                               budget are split; 1 = not split) */
    int64_t work_f;         /* algorithmic work of the pruned pairs (the cost
                               formulas of ChooseBestMethod, Section 3.8, without
                               their factor D): far-field sum N_Q p^D, */
    int64_t work_d;         /* direct local sum N_R p^D, */
    int64_t work_t;         /* far-to-local sum D p^2D (order >= 2) */
    int64_t e_items[6];     /* (query leaf, bandwidth) items of the mixed exhaustive
                               pass: [0] >= 64 reference leaves in the E list,
                               [1] fewer, [2] none; for value sums with 3 <= D <= 7
                               (matrix-core tiles) [0], [1] count the items with
                               FP32 products, [4], [5] those with FP64 products
                               and [3] those whose query leaf is too wide against
                               h for either (vector-ALU tiles); all 0 at
                               precision FP64 or with D >= 8 */
    int64_t e_pairs[2];     /* exhaustive point pairs of the matrix-core tiles with
                               FP32 [0] and FP64 [1] products (value sums, 3 <= D <= 7),
                               counting the references the tiles leave out as beyond
                               their staging window (terms below the rounding budget) */
    /* With dfgt_options.profile = 1: summed event time (ms) and launch count
     * per kernel: [0] traversal (bounds, ChooseBestMethod, list emission),
     * [1] per-query-leaf kernel (far-field evaluation, local-to-local walk,
     * local evaluation, combine),
     * [2] the mixed-precision pass of the exhaustive leaf-leaf sums of
     * DFGTBase (its dispatch order and every tile launch of the pass: matrix
     * cores for value sums with 3 <= D <= 7 or D >= 8, else the vector ALUs; [1]
     * adds their results), [3] local-moment accumulation (D and T ops),
     * [4] the exhaustive pairs summed in FP64 on the vector ALUs (all of them
     * at precision FP64, else those the underflow guard flags),
     * [5] of [2], the launch of the matrix-core tiles with FP32 products alone
     * (the e_pairs[0] pairs). */
    double kernel_ms[6];
    int64_t kernel_launches[6];
} dfgt_stats;

typedef struct dfgt_tree_s *dfgt_tree;

/* Last error message of the calling thread ("" if none). */
const char *dfgt_last_error(void);

/* Library version string. */
const char *dfgt_version(void);

/*
 * Builds the mid-point kd-tree of Section 2.1, Alg. BuildKdTree, on the GPU.
 *   pts_dev  n x d float64, row-major; read during the call only (the tree
 *            keeps its own permuted copy).
 *   opt      NULL for defaults.  leaf_size and the tree's permutation follow
 *            the algorithm exactly: boxes are the exact min/max of the node's
 *            points, the split dimension is the widest one (lowest index on
 *            ties), the split coordinate is the FP64 mid-point, points with
 *            x[sd] <= sc go left, the partition is stable, and a node is a leaf
 *            when it holds <= leaf_size points, has zero width, or one side
 *            would be empty.
 *   out      receives the handle; free it with dfgt_tree_free.
 * The call also computes the node's raw far-field moments (Alg. DFGTInitR:
 * AccumulateFarFieldMoment at leaves, TransFarToFar upwards).
 * Errors: n < 1, d < 1 or d > 32, p_max^d > 8192, non-finite input, a
 * non-zero reserved field -> DFGT_EINVAL.  The call waits for the tree's
 * structure (it reads the levels back); the moments and the device view are
 * still queued on the stream when it returns.  Work on the same stream sees
 * them; work on another stream must wait for this one.  pts_dev is no longer
 * read after the call returns.
 */
dfgt_status dfgt_build_tree(const double *pts_dev, int64_t n, int32_t d, const dfgt_options *opt,
                            void *stream, dfgt_tree *out);

/*
 * Builds a reference tree whose points carry weights, for the weighted sums
 * G_w(q) = sum_j w_j exp(-|q - r_j|^2 / 2h^2) (the kernel sums of Section 1
 * with a weight per reference point; the moments of Section 3.3 take w_j as
 * a factor of each point's term).  The per-query guarantee is unchanged:
 * |G~_w(q) - G_w(q)| <= eps G_w(q), the bounds of Sections 3.4-3.7 taken with
 * the node's weight W(R) = sum_{j in R} w_j in place of its point count.
 *   w_dev    n float64 weights in the order of pts_dev, device memory, read
 *            during the call only; every w_j >= 0 and finite, not all zero.
 * Other arguments as dfgt_build_tree.  A weighted tree is a reference tree
 * for dfgt_gauss_sum, dfgt_gauss_sum_grad, dfgt_gauss_backward, the batches
 * and dfgt_kde_density (which then divides by W(R) instead of N_R); as a
 * query tree its weights are ignored.  The cross-validation calls
 * (dfgt_lscv_score, dfgt_lcv_score, dfgt_lscv_optimize) reject it.
 * Errors: those of dfgt_build_tree; w_dev NULL, a negative or non-finite
 * weight, or all weights zero -> DFGT_EINVAL.  Waits for the stream twice
 * more than dfgt_build_tree (the weights' maximum, then their total), so
 * w_dev is no longer read after the call returns.
 */
dfgt_status dfgt_build_tree_weighted(const double *pts_dev, const double *w_dev, int64_t n, int32_t d,
                                     const dfgt_options *opt, void *stream, dfgt_tree *out);

/* Frees a tree handle (NULL is allowed).  Work already queued on the stream the
 * tree was built on may still use it: its device memory is kept by the library
 * and handed to a later build only after that stream reaches this point.  Work
 * that uses the tree on other streams must have completed before the call. */
dfgt_status dfgt_tree_free(dfgt_tree t);

/* Sizes of a tree: points, dimension, nodes, levels, p_max. Any pointer may be NULL. */
dfgt_status dfgt_tree_info(dfgt_tree t, int64_t *n, int32_t *d, int64_t *n_nodes, int32_t *depth,
                           int32_t *p_max);

/*
 * Copies the tree to host arrays (test hook).  Nodes are in breadth-first
 * order (root = 0; children of level-l nodes follow level l in parent order,
 * left before right).  Sizes: perm[n]; lo, hi[n_nodes*d] (node-major);
 * begin, end, left, right, split_dim[n_nodes]; split_coord[n_nodes].
 * perm[k] is the caller's index of the k-th point in tree order; begin/end
 * index tree order; left/right are -1 for leaves, split_dim is -1 for leaves.
 * Any pointer may be NULL.
 */
dfgt_status dfgt_tree_export(dfgt_tree t, int32_t *perm_host, double *lo_host, double *hi_host,
                             int32_t *begin_host, int32_t *end_host, int32_t *left_host,
                             int32_t *right_host, int32_t *split_dim_host,
                             double *split_coord_host);

/*
 * The tree's permutation on the device: perm_dev[k] = the caller's index of
 * the k-th point in tree order (n int32, caller-allocated device memory).
 * Enqueued on stream after the tree's own work (the tree's build stream
 * is made to wait first when it differs).  Errors: NULL argument -> EINVAL.
 */
dfgt_status dfgt_tree_perm(dfgt_tree t, int32_t *perm_dev, void *stream);

/*
 * Device memory from the caller's allocator.  With alloc != NULL, the
 * library's growing workspaces (traversal lists, per-node and per-query
 * buffers, brute-force partials) and tree arenas come from
 * alloc(bytes, ctx) and return through free(ptr, bytes, ctx) instead of
 * hipMalloc / hipFree, e.g. torch's caching allocator, so that a caller's
 * steady state allocates nothing from the runtime.  alloc must return device
 * memory of the current device, 256-byte aligned, or NULL (-> DFGT_ENOMEM);
 * both must be callable from any thread that calls the library.
 * dfgt_set_allocator(NULL, NULL, NULL) goes back to hipMalloc for new
 * buffers.  A buffer goes back through the free of the setting that made it
 * only while that setting is still the current one: after any later
 * dfgt_set_allocator call it is dropped without a free call, since the old
 * allocator may no longer exist.  So call dfgt_release_workspace, and free
 * trees built under the hook, before changing it.  dfgt_release_workspace
 * waits for the device, then frees the calling thread's workspace buffers
 * (traversal, sweep, brute-force and tree-build scratch); later calls
 * allocate again.  Trees keep their own memory until dfgt_tree_free.
 */
typedef void *(*dfgt_alloc_fn)(size_t bytes, void *ctx);
typedef void (*dfgt_free_fn)(void *ptr, size_t bytes, void *ctx);
dfgt_status dfgt_set_allocator(dfgt_alloc_fn alloc, dfgt_free_fn free_fn, void *ctx);
dfgt_status dfgt_release_workspace(void);

/*
 * Raw (bandwidth-free) far-field moments of every node (test hook):
 *     mu_alpha(N) = sum_{x in N} (x - N.c)^alpha / alpha!,  alpha < p_max,
 * N.c the box centre.  The paper's moments of Section 3.3,
 * eq. (far_field_moments), are M_alpha = (2h^2)^(-|alpha|/2) mu_alpha.
 * mu_host: n_nodes x p_max^d float64, breadth-first node order, each vector
 * radix p_max with the last dimension fastest (Appendix, linear layout).
 */
dfgt_status dfgt_tree_moments(dfgt_tree t, double *mu_host);

/*
 * Brute-force Gaussian sums, Alg. NaiveKDE (Section 1), as a tiled GPU kernel:
 *     G_dev[k*nq + i] = sum_j exp(-||q_i - r_j||^2 / (2 h_k^2)).
 *   q_dev nq x d, r_dev nr x d (float64 row-major), h_host[n_h] > 0,
 *   precision DFGT_PREC_*, G_dev n_h x nq float64 (caller-allocated).
 * Asynchronous on stream.
 */
dfgt_status dfgt_naive_sum(const double *q_dev, int64_t nq, const double *r_dev, int64_t nr,
                           int32_t d, const double *h_host, int32_t n_h, int32_t precision,
                           double *G_dev, void *stream);

/*
 * dfgt_naive_sum without any device allocation, for callers that cannot
 * allocate (code running under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * dfgt_naive_sum; the chunk partials, the bandwidth table and the norm tables
 * of the matrix-core form live in one fixed 64 MiB device region that the
 * library holds on every GPU it runs on until the process ends.  Limit:
 *   n_h * nq + nq + nr + n_h (rounded up to 32 each, + 32) <= 8 * 2^20 doubles,
 * else DFGT_EINVAL without touching the device.  Below the limit the
 * reference points are split into as many chunks as fit (as many as
 * dfgt_naive_sum takes when they fit, and then the result is bitwise the
 * same).  The region is shared by every call on that GPU and keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Asynchronous on the
 * stream, except that d >= 8 in mixed precision waits for the stream once
 * (the norm maxima decide whether the matrix-core form is exact enough).
 */
dfgt_status dfgt_naive_sum_noalloc(const double *q_dev, int64_t nq, const double *r_dev, int64_t nr,
                                   int32_t d, const double *h_host, int32_t n_h, int32_t precision,
                                   double *G_dev, void *stream);

/*
 * Dual-tree fast Gauss transform, Section 3.9 (DFGTMain):
 *     G_dev[k*NQ + i] ~= sum_j exp(-||q_i - r_j||^2 / (2 h_k^2))
 * for every query i in the caller's order, with |G~ - G| <= eps * G for every
 * i and k (the global-error theorem of Section 3.10).
 *   Q, R     tree handles of the same dimension (Q == R is the monochromatic
 *            cross-validation case; the self term is included).
 *   h_host   n_h bandwidths > 0; all are processed in one traversal.
 *   eps      in [0, 1).  eps = 0 prunes only where the bound is exactly zero.
 *   opt      NULL for the options R was built with (precision, force_method
 *            are read from here; leaf_size / p_max are the trees').
 *   G_dev    n_h x NQ float64, caller-allocated.
 *   stats    NULL, or counters (forces a stream synchronisation).
 * Errors: mismatched dimensions or p_max, h <= 0, eps outside [0,1) -> EINVAL.
 */
dfgt_status dfgt_gauss_sum(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                           const dfgt_options *opt, double *G_dev, dfgt_stats *stats, void *stream);

/*
 * Gradient mode of dfgt_gauss_sum (an extension: the paper has no gradients).
 * Returns sums G~ with the same guarantee |G~ - G| <= eps * G and the exact
 * derivatives of that approximation, per query:
 *     dGdh_dev[k*NQ + i]       = d G~_k(q_i) / d h_k          (may be NULL)
 *     dGdq_dev[(k*NQ + i)*d+c] = d G~_k(q_i) / d q_{i,c}      (may be NULL)
 * with the reference points held fixed.  Exhaustive leaf pairs contribute
 * the exact terms h^-3 sum_j K_ij |q_i - r_j|^2 and -h^-2 sum_j K_ij (q_i - r_j);
 * far-field, direct-local, far-to-local and local-to-local terms are
 * differentiated through their Hermite functions (d/dt h_n(t) = -h_{n+1}(t))
 * and the s^|alpha| moment scaling.  So that these derivatives approximate the
 * true ones about as well as the values do, the traversal of this mode uses
 * local expansions (direct local, far-to-local) one order above what the value
 * bound needs and does not use the centroid form (which is constant in q);
 * G~ may therefore differ from dfgt_gauss_sum's within the guarantee.  The
 * derivative error has no certified bound; measured on clustered 2-D and 3-D
 * data it stays below a few eps * G / h.
 * Buffers are caller-allocated device memory; G_dev is required.
 * Errors as dfgt_gauss_sum; p_max^d > 512 -> DFGT_EINVAL.
 */
dfgt_status dfgt_gauss_sum_grad(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                                const dfgt_options *opt, double *G_dev, double *dGdh_dev, double *dGdq_dev,
                                dfgt_stats *stats, void *stream);

/*
 * Vector-Jacobian product of dfgt_gauss_sum (the backward pass of the sums
 * as a differentiable function of the bandwidths and the query points):
 *     dh_host[k] = sum_i dG_dev[k*NQ + i] * dG~_k(q_i)/dh_k           (may be NULL)
 *     dq_dev[i*d + c] = sum_k dG_dev[k*NQ + i] * dG~_k(q_i)/dq_{i,c}   (may be NULL)
 * The derivatives are those of dfgt_gauss_sum_grad with the same arguments
 * (deterministic: repeated calls return the same bits).  Sums over queries and
 * bandwidths are taken in a fixed order.
 * dG_dev: n_h x NQ float64 device; dq_dev: NQ x d float64 device.
 * Synchronises the stream when dh_host is given.
 */
dfgt_status dfgt_gauss_sum_backward(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                                    const dfgt_options *opt, const double *dG_dev, double *dh_host,
                                    double *dq_dev, void *stream);

/*
 * Vector-Jacobian product of derivatives already computed by
 * dfgt_gauss_sum_grad (the saved context of a forward pass in gradient mode):
 *     dh_host[k] = sum_i dG_dev[k*nq + i] * dGdh_dev[k*nq + i]              (may be NULL)
 *     dq_dev[i*d + c] = sum_k dG_dev[k*nq + i] * dGdq_dev[(k*nq + i)*d + c]  (may be NULL)
 * So a caller that keeps the forward's G~ and derivatives differentiates
 * exactly the approximation it returned (the same traversal, the same
 * interaction lists), with no second traversal.  Layouts as in
 * dfgt_gauss_sum_grad; all device buffers caller-owned.  Sums are taken in a
 * fixed order (repeated calls give the same bits).  Synchronises the stream
 * when dh_host is given.  Errors: NULL dG_dev, both outputs NULL, an output
 * without its derivative array, n_h < 1, nq < 1 or d outside [1, 32] ->
 * DFGT_EINVAL.
 */
dfgt_status dfgt_gauss_sum_vjp(int32_t n_h, int64_t nq, int32_t d, const double *dG_dev, const double *dGdh_dev,
                               const double *dGdq_dev, double *dh_host, double *dq_dev, void *stream);

/*
 * Least-squares cross-validation score of Section 1 (the LSCV criterion used
 * to choose h), for every bandwidth h_k of h_host, from DFGT sums over R at
 * h_k and at sqrt(2) h_k (a Gaussian convolved with itself has bandwidth
 * sqrt(2) h), all 2 n_h of them in one traversal.  With
 *     S(h) = sum_i (G~(x_i, R; h) - 1),  a = (4 pi h^2)^(-D/2),  b = (2 pi h^2)^(-D/2):
 *   variant 0 (leave-one-out in both terms, the paper's formula):
 *     cv = (a S(sqrt2 h) - 2 b S(h)) / (N (N-1))
 *   variant 1 (the standard score: integral of the squared estimate keeps its
 *              diagonal terms):
 *     cv = a (N + S(sqrt2 h)) / N^2 - 2 b S(h) / (N (N-1))
 * cv_host[n_h] receives the scores; dcv_host[n_h] (may be NULL) receives
 * d cv / d h from the gradient mode.  The sums G~(x_i) - 1 are computed as
 * leave-one-out sums (each point's own term left out, the pruning tolerance
 * scaled by a lower bound on G - 1), each within eps of its own value, so
 * each S carries an error of at most eps * S.  N >= 2 and n_h <= 32767.
 * Synchronises the stream.
 */
dfgt_status dfgt_lscv_score(dfgt_tree R, const double *h_host, int32_t n_h, double eps, int32_t variant,
                            const dfgt_options *opt, double *cv_host, double *dcv_host, dfgt_stats *stats,
                            void *stream);

/*
 * Kernel density estimate of Section 1: p[k][i] = G~(q_i, R; h_k) / (N_R V_k),
 * V_k = (2 pi h_k^2)^(D/2) the integral of the Gaussian kernel (for a weighted
 * R: G~_w / (W(R) V_k), W(R) the sum of its weights).  Same
 * arguments, layout ([n_h][N_Q], user query order, FP64, caller-owned device
 * memory) and per-query relative error bound eps as dfgt_gauss_sum.
 */
dfgt_status dfgt_kde_density(dfgt_tree Q, dfgt_tree R, const double *h_host, int32_t n_h, double eps,
                             const dfgt_options *opt, double *p_dev, dfgt_stats *stats, void *stream);

/*
 * Likelihood cross-validation score of Section 1 for every bandwidth h_k:
 *     CV_LK(h) = (1/N) sum_j log p_{h,-j}(r_j),
 *     p_{h,-j}(r_j) = (G~(r_j, R; h) - 1) / ((N - 1) (2 pi h^2)^(D/2)),
 * the estimate at r_j from all points but r_j (G includes the self term 1).
 * dcv_host (may be NULL) receives dCV_LK/dh from the gradient mode:
 * (1/N) sum_j G'(r_j) / (G(r_j) - 1) - D/h.  The leave-one-out sums are
 * computed as such (each point's own term left out, the pruning tolerance
 * scaled by a lower bound on G - 1), each within eps of its own value however
 * isolated the point, so each log term is within -log(1 - eps).  A
 * leave-one-out sum that underflows FP64 to 0 makes the score -inf.
 * N >= 2, n_h <= 32767.
 * Synchronises the stream.  The bandwidth maximising CV_LK is the
 * likelihood-optimal one.
 */
dfgt_status dfgt_lcv_score(dfgt_tree R, const double *h_host, int32_t n_h, double eps, const dfgt_options *opt,
                           double *cv_host, double *dcv_host, dfgt_stats *stats, void *stream);

/*
 * The bandwidth that minimises the LSCV score above over [h_lo, h_hi]
 * (Section 4 sweeps its bandwidths around this minimiser h*, taking it from
 * the least-squares cross-validation score).  Search: n_grid log-spaced
 * bandwidths over the bracket, scored in one dfgt_lscv_score call (all 2 n_grid
 * sums in one traversal); the bracket becomes the two grid cells around the
 * smallest score (the first one on ties) and the search repeats until the
 * bracket spans at most a factor (1 + rel_tol)^2.  The score is not convex in
 * general: the grid finds the smallest score on the grid, and a minimiser at an
 * end of [h_lo, h_hi] means the bracket should be widened.
 *   h_star  receives the best bandwidth evaluated, cv_star (may be NULL) its
 *           score, n_evals (may be NULL) the number of bandwidths scored.
 * 0 < h_lo < h_hi, 4 <= n_grid <= 1024, 0 < rel_tol < 1, variant 0 or 1 (as in
 * dfgt_lscv_score).  Synchronises the stream after every grid.
 */
dfgt_status dfgt_lscv_optimize(dfgt_tree R, double h_lo, double h_hi, double eps, int32_t variant, int32_t n_grid,
                               double rel_tol, const dfgt_options *opt, double *h_star, double *cv_star,
                               int32_t *n_evals, void *stream);

/* One problem of a batch: the sums over R for the queries of Q at n_h
 * bandwidths, into G_dev (n_h x NQ float64, caller-allocated, caller order). */
typedef struct dfgt_problem {
    dfgt_tree Q;
    dfgt_tree R;          /* Q == R: the monochromatic case, self terms included */
    const double *h_host; /* n_h bandwidths > 0 */
    int32_t n_h;
    double *G_dev;
} dfgt_problem;

/*
 * Several problems of the same dimension and p_max, every bandwidth of each,
 * in one traversal (Alg. DFGTMain per (problem, bandwidth); the jobs share the
 * level-synchronous launches).  Same guarantee as dfgt_gauss_sum for every
 * query of every problem and bandwidth; results do not depend on the other
 * jobs of the batch (bitwise).  Options and errors as dfgt_gauss_sum; at most
 * 2^20 (problem, bandwidth) jobs.
 * Memory: when the traversal buffers of all jobs would exceed a budget of a
 * quarter of the device's memory (at least 1 GiB), or cannot be allocated,
 * the jobs are split into parts that run in turn on the same buffers
 * (stats->parts).  The
 * environment variable DFGT_MEMORY_BUDGET_MB, when set to a positive number of
 * MiB, replaces that budget (a test knob that forces the split; results are
 * bitwise the same however the jobs are split).
 */
dfgt_status dfgt_gauss_sum_batched(const dfgt_problem *probs, int32_t n_probs, double eps,
                                   const dfgt_options *opt, dfgt_stats *stats, void *stream);

/*
 * Leaf-size tuning: the kd-tree leaf threshold of Alg. BuildKdTree trades
 * tree depth (traversal levels, build levels, expansions) against exhaustive
 * leaf-leaf work (DFGTBase), and the best value depends on the data, D and the
 * bandwidths.  For each candidate in DFGT_TUNE_LEAVES the call times, with HIP
 * events on the stream, `reps` repetitions of a tree build on pts_dev (n x d,
 * float64, device) plus the monochromatic sums dfgt_gauss_sum(T, T, h_host,
 * n_h, eps) (after one untimed repetition), and returns in *leaf_out the
 * smallest candidate whose median time is within 2% of the fastest one (so
 * near-ties resolve the same way from call to call).  ms_out (may be NULL) receives the
 * DFGT_N_TUNE_LEAVES medians in milliseconds, in the order of the list.  opt
 * supplies the other build and sum options (its leaf_size is ignored).  The
 * sums of every candidate satisfy the same error bound; the choice only
 * affects time, and timing noise can make it differ between calls.  Allocates
 * an n_h x n output buffer for the duration of the call and synchronises the
 * stream after every repetition.  1 <= reps <= 100; other errors as those of
 * dfgt_build_tree and dfgt_gauss_sum.
 */
#define DFGT_N_TUNE_LEAVES 5
#define DFGT_TUNE_LEAVES {16, 32, 64, 128, 256}
dfgt_status dfgt_tune_leaf_size(const double *pts_dev, int64_t n, int32_t d, const double *h_host, int32_t n_h,
                                double eps, const dfgt_options *opt, int32_t reps, void *stream,
                                int32_t *leaf_out, double *ms_out);

/*
 * A batch captured as a HIP graph, for callers that repeat the same sweep (or
 * must not pay per-launch host overhead): dfgt_batch_create runs the batch
 * once eagerly (which sizes every internal buffer; stats, if given, are that
 * run's), then captures the whole launch sequence of one run into a graph
 * that owns its workspace.  dfgt_batch_run replays it asynchronously on
 * stream, rewriting every G_dev.  The trees, bandwidths and output buffers are
 * fixed at creation: keep them alive and unchanged until dfgt_batch_free.
 * dfgt_batch_check synchronises the stream and reports DFGT_EQUEUE if any part
 * of the last run overflowed its buffers (which unchanged inputs cannot cause).
 */
typedef struct dfgt_batch_s *dfgt_batch;
dfgt_status dfgt_batch_create(const dfgt_problem *probs, int32_t n_probs, double eps, const dfgt_options *opt,
                              dfgt_stats *stats, void *stream, dfgt_batch *out);
dfgt_status dfgt_batch_run(dfgt_batch b, void *stream);
dfgt_status dfgt_batch_check(dfgt_batch b, void *stream);
dfgt_status dfgt_batch_free(dfgt_batch b);

#ifdef __cplusplus
}
#endif

#endif /* DFGT_H */
