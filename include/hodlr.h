/*
 * hodlr.h -- C ABI of libhodlrgp, a HODLR (hierarchical off-diagonal
 * low-rank) factorization of Gaussian-process covariance matrices for AMD
 * MI355X (gfx950).
 *
 * Problem (Ambikasaran et al., "Fast Direct Methods for Gaussian Processes",
 * §1 Eq. (1) and §2.1): data x_1..x_n in R^dim, observations y, covariance
 * C = sigma^2 I + K with K_ij = k(x_i, x_j; theta).  The library factors C
 * as a product of a block-diagonal matrix and block-diagonal low-rank updates
 * of the identity (§3.2), reads log det C off that factorization by
 * Sylvester's determinant theorem (§4), and applies C^{-1} through it
 * (§3.2, inverse of the factor list).  Two user knobs follow the paper: the
 * compression tolerance epsilon and the leaf (smallest diagonal block) size
 * p_max (§3.2 pseudo-code; §5.6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns hodlr_status; HODLR_OK = 0.  On any other status
 *    no output is written (except where a function says otherwise), nothing
 *    is printed and nothing aborts; hodlr_last_error() returns a message for
 *    the calling thread's last failure.
 *  - Host-pointer entry points (hodlr_build, hodlr_solve, gp_loglik,
 *    hodlr_order) take points point-major (x[i*dim + d]) in the caller's
 *    order; vectors are in the caller's order.  The library orders points
 *    internally (sort in 1-D, count-median k-d split in 2-D/3-D) and keeps the
 *    permutation.  The caller owns all its buffers; the library keeps no
 *    caller pointer after a call returns.
 *  - Device entry points (suffix _dev) take device pointers to points that
 *    are ALREADY in tree order (see hodlr_order), stored coordinate-major
 *    (x[d*n + i]), plus a caller-provided device workspace and a hipStream_t
 *    passed as void*.  They enqueue work on that stream and may synchronize
 *    it internally while the cross-approximation runs.
 *  - Precision: FP64 everywhere by default.  HODLR_MIXED stores the applied
 *    bases W~ = (block inverses) W and the solve vector in FP32; every
 *    arithmetic operation (kernel evaluation, compression, leaf factors,
 *    level products, coupling LU, log-det sums) stays FP64, loaded FP32
 *    values are widened in registers and results rounded on store.  The
 *    host solve recovers full accuracy by iterative refinement against an
 *    exact FP64 matrix-vector product (see hodlr_opts.precision).  The log
 *    det is held to a relative error of 1e-8: each mixed likelihood (or
 *    factor) computes the error estimate 4 eps_32 sqrt(sum over split nodes
 *    of det M_tau^-2) (the FP32 rounding of W~, amplified at most by
 *    1 / det M_tau at each node, the nodes' independent roundings adding as
 *    a root sum of squares), and one whose estimate exceeds
 *    1e-8 max(|log det|, 1) is computed again with FP64 panels (counted in
 *    hodlr_info.fp64_fallback; the workspace sizes of mixed plans leave room
 *    for it).  The estimate is calibrated, not proven: on seeded settings of
 *    the 1-D hyperparameter box the error stayed below a third of it.
 *  - Thread safety: distinct factors/plans may be used concurrently; one
 *    workspace must not be used by two calls at once.
 */
#ifndef HODLR_H
#define HODLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HODLR_OK = 0,
    HODLR_EINVAL = 1,   /* bad argument: n < 1, dim not in {1,2,3}, leaf < 1, tol <= 0,
                           sigma2 < 0, a <= 0 or l <= 0, NaN/Inf input, workspace too small */
    HODLR_ENOTSPD = 2,  /* a leaf Cholesky pivot or a coupling determinant was not positive */
    HODLR_ENOMEM = 3,   /* device or host allocation failed */
    HODLR_EDEVICE = 4,  /* a HIP runtime call failed */
    HODLR_ENOCONV = 5   /* refined solve: refinement missed refine_tol within max_refine
                           steps (outputs ARE written with the best iterate) */
} hodlr_status;

/* Covariance kernels (Table 1 and §5 of the paper, amplitude/length-scale form),
 * r = Euclidean distance, theta = {a, l}. */
typedef enum {
    HODLR_K_SE = 0,        /* a^2 exp(-r^2 / (2 l^2))                      */
    HODLR_K_MATERN32 = 1,  /* a^2 (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)  */
    HODLR_K_EXP = 2,       /* a^2 exp(-r / l)  (Ornstein-Uhlenbeck)         */
    HODLR_K_CONST = 3,     /* a^2  (rank one; for tests)                    */
    HODLR_K_IMQ = 4        /* a^2 / sqrt(1 + r^2 / l^2)  (inverse
                              multiquadric, §5)                             */
} hodlr_kernel;

enum { HODLR_FP64 = 0, HODLR_MIXED = 1 };
enum { HODLR_COMPRESS_ACA = 0, HODLR_COMPRESS_SKETCH = 1 };

typedef struct {
    int32_t max_rank;    /* per off-diagonal block rank cap in [0, 512] (default 64); a
                            hit cap is counted in hodlr_info, not an error.  Levels
                            whose rank is above 64 keep their coupling matrices in
                            device memory instead of LDS (slower node solves)        */
    int32_t precision;   /* HODLR_FP64 (default) or HODLR_MIXED: the applied bases
                            W~ = (block inverses) W and the solve vector stored in
                            FP32 (updates computed in FP64 registers, rounded on
                            store); compression, bases W,
                            leaf Cholesky factors, coupling-matrix LU and every log-det
                            sum in FP64.  hodlr_solve and gp_loglik then refine against
                            the exact FP64 product (hodlr_matvec_dev) by conjugate
                            gradients preconditioned with the factor; gp_loglik_dev and
                            the batched form return the unrefined quadratic form      */
    double refine_tol;   /* refined solves: stop at ||y - C x|| / ||y|| <= refine_tol,
                            the true residual (default 1e-10)                         */
    int32_t max_refine;  /* refined solves: at most 1 + max_refine preconditioned steps,
                            each one exact product and one factor solve (default 8;
                            0 allows the first step only)                             */
    int32_t presorted;   /* 1: the points are already in tree order; skip ordering     */
    const double *noise; /* optional per-point noise variances sigma_i^2 (host memory,
                            n entries in the caller's point order, each >= 0 and
                            finite; §5 writes the diagonal of C as sigma_i^2): the
                            diagonal of C becomes sigma2 + noise[i].  Read during the
                            call only (the factor keeps its own copy).  Taken by
                            hodlr_build and gp_loglik; the plan-based, batched,
                            uneven-size and autotuning entry points reject a non-NULL
                            value with HODLR_EINVAL.  Default NULL                    */
    int32_t refine;      /* 1: FP64 factors also refine every hodlr_solve / hodlr_predict
                            solve and the host gp_loglik quadratic form against the
                            exact FP64 product, as the mixed form always does (to
                            refine_tol within max_refine steps; ENOCONV otherwise).
                            0 (default): an FP64 factor is applied once, whose
                            residual is about tol ||K|| / sigma2                      */
    int32_t mixed_unchecked; /* HODLR_MIXED only.  0 (default): every likelihood or
                            factor tests its log-det error estimate (see Precision
                            at the top) and is redone with FP64 panels when the
                            estimate misses 1e-8.  1: keep the FP32-panel result
                            untested (the caller measures its error)               */
    int32_t compressor;  /* How the off-diagonal blocks K(alpha, beta) are compressed
                            (§3.1 lists both kinds).  HODLR_COMPRESS_ACA (default):
                            adaptive cross approximation, O(r^2 (m + n)) work per
                            block.  HODLR_COMPRESS_SKETCH: a randomized two-sided
                            sketch (generalized Nystrom): random-sign matrices X and
                            Y of s = min(max_rank + 16, m, n) and s + 8 columns,
                            A X and A^T Y evaluated entry by entry (every entry of
                            every block twice: O(n^2) work in all), the core
                            Y^T A X factored by a Jacobi SVD and its pseudo-inverse
                            truncated at tol / 10 of its largest singular value.  It
                            needs no pivoting heuristic, so it also holds where
                            cross approximation can stall, at the price of the
                            quadratic work (moderate n).  Needs max_rank <= 64;
                            taken by hodlr_build, gp_loglik, gp_loglik_dev and
                            gp_loglik_grad_dev (the batched, uneven-size and
                            autotuning entry points reject it with HODLR_EINVAL)  */
    int32_t speculate;   /* gp_loglik_dev with cross approximation only.  0 (default):
                            after the compression the call waits for the block ranks
                            to lay out the panel columns.  1: a call on a plan whose
                            previous gp_loglik_dev completed assumes that call's
                            panel widths and large-block step count and runs on
                            without waiting; a device check after the compression
                            compares the actual ranks and convergence with them,
                            and a call whose ranks exceed a width or whose blocks
                            did not converge is redone the ordinary way (same
                            results; when every rank fits but some width shrank,
                            the padding columns change the rounding of the coupling
                            solves at the 1e-15 level).  Meant for repeated
                            likelihoods of nearby hyperparameters on one plan     */
    int32_t level_form;  /* How a likelihood (a call given a right-hand side y) runs
                            the levels.  0 (default): projected when it fits (panel
                            columns <= 128, widths <= 32 per depth, each level's
                            coupling solve within 60 KB of LDS): the bases'
                            projections G = Z^T K^{-1} Z (Z: y and the bases on a
                            node's rows) go up the tree and C^{-1} y comes down it,
                            with the same coupling matrices and determinants as the
                            level-by-level factorization (§3.2, §4) and O(n r)
                            panel traffic instead of O(n r L^2).  1: always the
                            level-by-level updates of every applied basis.  A kept
                            factor (hodlr_build) always takes the latter          */
} hodlr_opts;          /* pass NULL for all defaults */

typedef struct hodlr_factor_s *hodlr_factor;   /* opaque; factors fixed after build; one
                                                  solve at a time per factor (it uses the
                                                  factor's own solve vector)           */
typedef struct hodlr_plan_s *hodlr_plan;       /* opaque; tree + workspace layout */

#define HODLR_MAX_LEVELS 40

typedef struct {
    int64_t n;
    int32_t dim;
    int32_t levels;                            /* L: depth of the leaves           */
    int32_t leaf_max;                          /* largest leaf size                */
    int32_t max_rank_used;
    int32_t capped_blocks;                     /* blocks whose ACA hit max_rank    */
    int32_t rank_max[HODLR_MAX_LEVELS];        /* per depth d of the split node    */
    double rank_mean[HODLR_MAX_LEVELS];
    int64_t device_bytes;                      /* device memory held by the factor */
    int32_t precision;
    int32_t refine_steps;                      /* mixed form, last solve           */
    double refine_residual;                    /* mixed form, last solve           */
    int32_t fp64_fallback;                     /* mixed form: factors (or likelihoods
                                                  of the last plan call) redone with
                                                  FP64 panels (see HODLR_MIXED)    */
    int32_t speculated;                        /* plans: 1 if the last gp_loglik_dev
                                                  ran on the assumed panel widths
                                                  without a redo (hodlr_opts.speculate) */
    int32_t projected;                         /* plans: 1 if the last gp_loglik_dev
                                                  ran the projected levels
                                                  (hodlr_opts.level_form)          */
} hodlr_info_t;

/* ------------------------------------------------------------------ ordering */

/* Tree ordering of the points (§3: k-d sorting; node = contiguous index range,
 * left child = floor(m/2) points).  perm[k] = caller index of the k-th ordered
 * point (int64[n], caller-allocated).  1-D: stable sort.  dim > 1: at depth d
 * the node is sorted along coordinate (d mod dim), ties in input order.
 * Errors: EINVAL (bad sizes, NaN/Inf).                                       */
hodlr_status hodlr_order(const double *x, int64_t n, int32_t dim, int32_t leaf,
                         int64_t *perm);

/* Number of levels L used for n points and leaf size `leaf`: the smallest L
 * with ceil(n / 2^L) <= leaf (the paper's kappa, §3.2 pseudo-code).         */
int32_t hodlr_num_levels(int64_t n, int32_t leaf);

/* ----------------------------------------------------------- host interface */

/* Factor C = sigma2 I + K(x; theta) (§3.1 compression, §3.2 factorization).
 * x: point-major n*dim doubles, caller order.  theta = {a, l}.  tol: relative
 * per-block compression tolerance (epsilon).  On success *out holds a new
 * factor that owns its device memory until hodlr_free.
 * Errors: EINVAL, ENOTSPD, ENOMEM, EDEVICE.                                  */
hodlr_status hodlr_build(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                         const double theta[2], double sigma2, int32_t leaf, double tol,
                         const hodlr_opts *opts, hodlr_factor *out);

/* log det C from the factorization (§4: Sylvester + multiplicativity).      */
hodlr_status hodlr_logdet(hodlr_factor f, double *logdet);

/* x = C^{-1} y for nrhs right-hand sides (§3.2, inverse of the factor list).
 * y, x: column-major n x nrhs host arrays in the caller's order; x may alias
 * y.  Mixed-precision factors, and FP64 factors built with opts.refine = 1,
 * refine each column to refine_tol (ENOCONV if not reached; x still holds
 * the best iterate).                                                        */
hodlr_status hodlr_solve(hodlr_factor f, const double *y, double *x, int64_t nrhs);

/* Prediction at m new inputs through the factor (§2.1, predictive mean and
 * variance of f, mean function 0):
 *   mean_j = k(xt_j, x) C^{-1} y,
 *   var_j  = k(xt_j, xt_j) - k(xt_j, x) C^{-1} k(x, xt_j)
 * (the variance of the latent f; add sigma2 for a new noisy observation).
 * y: n doubles in the caller's order (the observations the factor's x
 * belongs to); xt: point-major m*dim doubles, any order; mean, var: m
 * doubles (var may be NULL: the mean needs one solve, each variance one
 * solve more).  Every kernel entry is evaluated exactly; the solves are the
 * factor's (mixed factors refine them as hodlr_solve does: ENOCONV if a solve
 * misses refine_tol, with all outputs written; hodlr_info reports the largest
 * step count and residual).  m = 0 is a no-op.
 * Errors: EINVAL (NULL with m > 0, m < 0, non-finite y or xt), ENOMEM,
 * EDEVICE, ENOCONV.                                                         */
hodlr_status hodlr_predict(hodlr_factor f, const double *y, const double *xt, int64_t m,
                           double *mean, double *var);

/* Gaussian log-likelihood of y (Eq. (1) with the normal constant, mean 0):
 *   loglik = -y^T C^{-1} y / 2 - log det C / 2 - (n/2) log(2 pi).
 * logdet and quad (= y^T C^{-1} y) are optional outputs (NULL to skip).     */
hodlr_status gp_loglik(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                       const double theta[2], double sigma2, const double *y, int32_t leaf,
                       double tol, const hodlr_opts *opts, double *loglik, double *logdet,
                       double *quad);

hodlr_status hodlr_info(hodlr_factor f, hodlr_info_t *out);
void hodlr_free(hodlr_factor f);
const char *hodlr_last_error(void);

/* --------------------------------------------------------- device interface */

/* A plan fixes n, dim, leaf and options; it precomputes the tree and the
 * work tables and uploads them to the current device.  Plans are reusable
 * across hyperparameters and right-hand sides.                               */
hodlr_status hodlr_plan_create(int64_t n, int32_t dim, int32_t leaf, const hodlr_opts *opts,
                               hodlr_plan *out);
void hodlr_plan_destroy(hodlr_plan p);

/* Launch shape chosen by the autotuner: the leaf size (any leaf <= 256) and
 * the level stage's tiles, rows per chunk (256, 512 or 1024), columns per
 * reduction step (4 or 8) and columns per reduction work-group (8 or 64).  The method's result does not depend on the tiles;
 * the leaf size changes the tree (and so the approximation) within the
 * compression tolerance.                                                     */
typedef struct {
    int32_t leaf;
    int32_t level_rows;
    int32_t reduce_cols;
    int32_t reduce_group;
} hodlr_tune_t;

/* As hodlr_plan_create, with the leaf size and tiles from `tune`.           */
hodlr_status hodlr_plan_tuned_create(int64_t n, int32_t dim, const hodlr_opts *opts,
                                     const hodlr_tune_t *tune, hodlr_plan *out);

/* Times the whole likelihood on the caller's problem (host arrays as for
 * gp_loglik) for each leaf size in leaf_cands (NULL/0: 32, 64, 96, 128) with
 * the default tiles (512, 4, 8), then the twelve tile shapes at the fastest
 * leaf (rows outer, then columns per step, then group); keeps the best of
 * `reps` runs after a warm-up per candidate.  *best receives the fastest
 * shape; times_ms (nullable, nleaf + 12 doubles, 4 + 12 for the defaults) the
 * per-candidate times in that order.  The result is also cached
 * per (ceil log2 n, dim, kernel, precision) for hodlr_tune_lookup.  Allocates
 * and frees device memory per candidate.  Errors: EINVAL, ENOTSPD, ENOMEM,
 * EDEVICE.                                                                   */
hodlr_status hodlr_autotune(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                            const double theta[2], double sigma2, const double *y, double tol,
                            const hodlr_opts *opts, const int32_t *leaf_cands, int32_t nleaf,
                            int32_t reps, hodlr_tune_t *best, double *times_ms);
/* The cached result of an earlier hodlr_autotune for this problem class in
 * this process; EINVAL if there is none.                                    */
hodlr_status hodlr_tune_lookup(int64_t n, int32_t dim, hodlr_kernel k, int32_t precision,
                               hodlr_tune_t *out);

/* Bytes of device workspace one gp_loglik_dev call needs (256-byte aligned).*/
hodlr_status hodlr_plan_workspace_size(hodlr_plan p, size_t *bytes);

/* The plan's tree (n, dim, levels, largest leaf; device_bytes = workspace plus
 * tables) and the block ranks of the last call on it: after gp_loglik_dev
 * (when it completed) the per-depth maximum and mean and the capped count;
 * after gp_loglik_batch_dev the per-depth maxima over its items (the column
 * layout every item was padded to; means 0) and the capped count summed over
 * items.  Zeros before the first call.  Errors: EINVAL (NULL).               */
hodlr_status hodlr_plan_info(hodlr_plan p, hodlr_info_t *out);

/* Log-likelihood with every input already resident on the device.
 * d_x: tree-ordered points, coordinate-major (d_x[d*n + i]); d_y: n doubles
 * in the same order; d_work: workspace of >= hodlr_plan_workspace_size bytes;
 * stream: hipStream_t as void* (NULL = default stream).  d_out receives three
 * doubles {loglik, logdet, quad} in device memory; d_z (nullable) receives
 * C^{-1} y in tree order.  Errors: EINVAL, ENOTSPD (reported after the call
 * synchronizes the stream), EDEVICE.                                         */
hodlr_status gp_loglik_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                           const double theta[2], double sigma2, const double *d_y, double tol,
                           void *d_work, size_t work_bytes, void *stream, double *d_out,
                           double *d_z);

/* Batched log-likelihoods (many hyperparameter settings on shared points):
 * item b uses (a, l, sigma2) = d_params[3b .. 3b+2] (device memory) and the
 * right-hand side d_y + b * y_stride (y_stride = 0 shares one y).  Every stage
 * is one launch over all items; after the compression the library reads the
 * batch-wide rank maxima once (one synchronization) to fix a common column
 * layout, and with use_graph != 0 (and a non-NULL stream) the remaining stages
 * run as a hipGraph captured once per layout and buffer set and replayed.
 * d_out receives 3 doubles per item {loglik, logdet, quad}; an item whose
 * factorization fails (non-positive pivot or coupling determinant, or
 * non-positive parameters) gets NaNs and does not stop the batch.
 * Workspace: hodlr_plan_batch_workspace_size(plan, nitems).  The call returns
 * without synchronizing (results are ready when the stream is), except for
 * mixed plans: they synchronize at the end to read each item's log-det error
 * estimate and redo the items that miss the bar with FP64 panels, one at a
 * time (see Precision above).                                              */
hodlr_status hodlr_plan_batch_workspace_size(hodlr_plan p, int32_t nitems, size_t *bytes);
hodlr_status gp_loglik_batch_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                                 const double *d_params, int32_t nitems, const double *d_y,
                                 int64_t y_stride, double tol, void *d_work, size_t work_bytes,
                                 void *stream, double *d_out, int32_t use_graph);

/* Gradient of the log-likelihood in the hyperparameters (a, l, sigma2) --
 * what the hyperparameter fits of §2.3 iterate on.  The paper gives no
 * formula for it; this entry point takes the central difference of the
 * likelihood the factorization computes,
 *   dL/dp = (L(p + h_p) - L(p - h_p)) / (2 h_p),  h_p = rel_step * p,
 * for p = a, l, sigma2: 7 likelihoods (the point and the six shifted ones),
 * each through the single-likelihood pipeline on the workspace; on FP64
 * plans the two sigma2 items reuse the point's compression (the off-diagonal
 * blocks do not depend on sigma2).  The error is O(h^2) from the difference
 * plus about
 * eps_L |L| / h from the likelihood's own error eps_L (~1e-13 FP64, ~1e-9
 * mixed); rel_step <= 0 takes 1e-4 (FP64 plans) or 1e-3 (mixed plans).
 * Arguments as gp_loglik_dev; sigma2 must be positive (the step below it
 * must stay a valid noise variance) and rel_step below 0.5.  d_out (device)
 * receives 6 doubles {loglik, logdet, quad, dL/da, dL/dl, dL/dsigma2}, the
 * first three at the unshifted point.  Workspace:
 * hodlr_plan_grad_workspace_size.  The call synchronizes the stream (it
 * reads the items' status).  Errors: EINVAL, ENOTSPD (any of the 7
 * factorizations failed), EDEVICE.                                         */
hodlr_status hodlr_plan_grad_workspace_size(hodlr_plan p, size_t *bytes);
hodlr_status gp_loglik_grad_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                                const double theta[2], double sigma2, const double *d_y,
                                double tol, double rel_step, void *d_work, size_t work_bytes,
                                void *stream, double *d_out);

/* Log-likelihoods (Eq. (1), as gp_loglik) of m independent problems of
 * uneven size.  Item i has ns[i] points xs[i] (point-major ns[i]*dim host
 * doubles, caller order), observations ys[i] (ns[i] host doubles) and
 * hyperparameters {a, l, sigma2} = params[3i .. 3i+2]; dim, kernel, leaf,
 * tol and opts are shared.  nworkers host threads (<= 0: 8) each own a
 * stream and one device arena sized for the largest item, and take items
 * largest first.  out receives 3 doubles per item {loglik, logdet, quad}; an
 * item that is invalid or whose factorization fails gets NaNs and does not
 * stop the others (mixed precision: the quadratic form is unrefined, as in
 * gp_loglik_dev).  All pointers are host memory owned by the caller; the
 * call returns when every item is done.  Errors: EINVAL (shared arguments),
 * EDEVICE (the device failed; items not reached hold NaN or are untouched). */
hodlr_status gp_loglik_ragged(int32_t m, const int64_t *ns, const double *const *xs,
                              const double *const *ys, int32_t dim, hodlr_kernel k,
                              const double *params, int32_t leaf, double tol,
                              const hodlr_opts *opts, int32_t nworkers, double *out);

/* Exact FP64 product out = C v evaluated entry by entry on the device
 * (O(n^2), nothing stored): the operator used by iterative refinement and for
 * residual checks.  Same layout rules as gp_loglik_dev; no workspace.       */
hodlr_status hodlr_matvec_dev(int64_t n, int32_t dim, const double *d_x, hodlr_kernel k,
                              const double theta[2], double sigma2, const double *d_v,
                              double *d_out, void *stream);

/* ------------------------------------------- surrogate of the likelihood */

/* The paper's outer loop needs the likelihood at many hyperparameters (§1,
 * Eq. (1), posterior over theta).  A small network l~(theta) screens
 * proposals before the exact HODLR likelihood is paid for:
 *   u = (log theta - mu_in) / sd_in;  h1 = tanh(W1 u + b1);
 *   h2 = tanh(W2 h1 + b2);  o = W3 . h2 + b3;  l~ = mu_out + sd_out * o.
 * Parameters: one flat vector of HODLR_MLP_NPARAM numbers in the order
 * W1 (128 x 3, row = unit), b1 (128), W2 (128 x 128, row = output unit), b2,
 * W3 (128), b3 (1).  The optimizer owns an FP32 master copy; products use a
 * BF16 copy (uint16 bit patterns, round to nearest even) and accumulate in
 * FP32.  log theta rows are (log a, log l, log sigma2), FP64, row-major. */
#define HODLR_MLP_NPARAM 17153
typedef struct {
    float mu_in[3], sd_in[3]; /* input standardization (sd > 0)            */
    float mu_out, sd_out;     /* output scale: l~ = mu_out + sd_out * o     */
} hodlr_mlp_norm;

/* Workspace bytes for a training or gradient call on `batch` samples.      */
hodlr_status hodlr_mlp_workspace_size(int32_t batch, size_t *bytes);
/* d_wbf16[p] = BF16(d_master[p]) for all parameters (device arrays).       */
hodlr_status hodlr_mlp_cast_dev(const float *d_master, uint16_t *d_wbf16, void *stream);
/* d_out[s] = l~(d_logtheta[3s .. 3s+2]) for s < batch (device memory).     */
hodlr_status hodlr_mlp_forward_dev(const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                                   const double *d_logtheta, int32_t batch, double *d_out,
                                   void *stream);
/* Loss mean_s (o_s - (t_s - mu_out)/sd_out)^2 over the batch and its
 * gradient with respect to the parameters (FP32, HODLR_MLP_NPARAM floats),
 * evaluated with the BF16 weights.  d_loss (device float) may be NULL.     */
hodlr_status hodlr_mlp_grad_dev(const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                                const double *d_logtheta, const double *d_target, int32_t batch,
                                void *d_work, size_t work_bytes, float *d_grad, float *d_loss,
                                void *stream);
/* One training step: gradient as above, then Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, step number `step` >= 1 for the bias correction) on the master
 * copy and moments d_m, d_v (FP32, zero before step 1), and the BF16 copy
 * refreshed.  Sample s of the batch is row d_index[s] of d_logtheta and
 * d_target (d_index NULL: row s).  Nothing is synchronized.
 * Errors: EINVAL, EDEVICE.                                                  */
hodlr_status hodlr_mlp_train_step_dev(float *d_master, uint16_t *d_wbf16, float *d_m, float *d_v,
                                      int32_t step, float lr, const hodlr_mlp_norm *norm,
                                      const double *d_logtheta, const double *d_target,
                                      const int32_t *d_index, int32_t batch, void *d_work,
                                      size_t work_bytes, float *d_loss, void *stream);
/* The training step above without a workspace argument, for callers that
 * cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc): the per-tile gradient slots live in a
 * fixed array of the library in device memory (one per GPU, held until the
 * process ends; 4 * 17154 * ceil(HODLR_MLP_NOALLOC_MAX_BATCH / 32) bytes, about
 * 8.4 MiB).  batch must be <= HODLR_MLP_NOALLOC_MAX_BATCH (EINVAL otherwise).
 * The call allocates nothing; every slot it reads is written earlier in the
 * same call.  Calls on one GPU share that array, so calls that overlap in time
 * on one GPU (different streams or threads) race and give wrong results;
 * serialize them.  Results equal hodlr_mlp_train_step_dev's.  The first call
 * on a device looks up the array's device address (EDEVICE if that fails). */
#define HODLR_MLP_NOALLOC_MAX_BATCH 4096
hodlr_status hodlr_mlp_train_step_noalloc_dev(float *d_master, uint16_t *d_wbf16, float *d_m,
                                              float *d_v, int32_t step, float lr,
                                              const hodlr_mlp_norm *norm,
                                              const double *d_logtheta, const double *d_target,
                                              const int32_t *d_index, int32_t batch,
                                              float *d_loss, void *stream);
/* `epochs` passes over n training pairs in minibatches of `batch` (the last
 * one of an epoch may be smaller), epoch e visiting rows in the order
 * d_perm[e*n .. e*n+n-1]; Adam step numbers start at step0.  d_loss_hist
 * (nullable, device) receives one loss per minibatch.  The workspace must
 * hold hodlr_mlp_workspace_size(batch).                                    */
hodlr_status hodlr_mlp_fit_dev(float *d_master, uint16_t *d_wbf16, float *d_m, float *d_v,
                               int32_t step0, float lr, const hodlr_mlp_norm *norm,
                               const double *d_logtheta, const double *d_target, int32_t n,
                               const int32_t *d_perm, int32_t epochs, int32_t batch, void *d_work,
                               size_t work_bytes, float *d_loss_hist, void *stream);

/* ------------------------------------------------------------- sampling */

/* Random-walk Metropolis over log theta = (log a, log l, log sigma2) for the
 * posterior exp(l(theta)) p(theta) that the paper's likelihood serves (§1,
 * Eq. (1)), with a uniform prior on a box in log theta.  The delayed form
 * (Christen and Fox, 2005) screens each proposal with the surrogate l~:
 *   stage 1: survive if log u1 < l~(theta') - l~(theta);
 *   stage 2: accept if log u2 < [l(theta') - l(theta)] - [l~(theta') - l~(theta)],
 * which leaves the exact posterior invariant for any surrogate.  The plain
 * form accepts if log u1 < l(theta') - l(theta).  Proposals leave the box
 * rejected, with no likelihood evaluated.  Random numbers are inputs.
 * Walker arrays are device memory: theta W x 3 row-major, lp and sur W.     */
typedef struct {
    int32_t walkers;    /* W in [1, 1024]                                  */
    int32_t steps;      /* steps per call                                  */
    double lo[3], hi[3];/* prior box in log theta                          */
    double chol[9];     /* proposal theta' = theta + L eps, L row-major    */
    int32_t init_state; /* 1: evaluate lp (and sur) at theta before step 1 */
} hodlr_sampler_cfg;
typedef struct {
    int64_t proposals, survivors, exact_evals, accepted;
} hodlr_sampler_stats;

/* prop = theta + eps L^T row by row (chol: host, 9 doubles, row-major).     */
hodlr_status hodlr_mh_propose_dev(int32_t w, const double *d_theta, const double chol[9],
                                  const double *d_eps, double *d_prop, void *stream);
/* Stage 1.  d_sur_prop NULL: plain form (box test only).  Writes slot[i]
 * (position of walker i among the survivors, walker order, or -1), the
 * survivor count (one int) and the survivors' (a, l, sigma2) = exp(prop)
 * rows, ready for gp_loglik_batch_dev.  lo/hi: host arrays.                 */
hodlr_status hodlr_da_screen_dev(int32_t w, const double *d_prop, const double lo[3],
                                 const double hi[3], const double *d_sur, const double *d_sur_prop,
                                 const double *d_u1, int32_t *d_slot, int32_t *d_count,
                                 double *d_params, void *stream);
/* Stage 2 (delayed != 0) or the plain decision, for walkers with a slot:
 * d_exact holds rows {loglik, ...} (3 doubles) of the survivors in slot
 * order; d_u is u2 (delayed) or u1 (plain).  Accepted walkers take prop, the
 * exact value and (delayed) the surrogate value.  d_accepted nullable.      */
hodlr_status hodlr_da_accept_dev(int32_t w, int32_t delayed, const int32_t *d_slot,
                                 const double *d_exact, const double *d_u, const double *d_prop,
                                 const double *d_sur_prop, double *d_theta, double *d_lp,
                                 double *d_sur, int32_t *d_accepted, void *stream);
/* Workspace of gp_sample_dev for W walkers on plan p.                      */
hodlr_status hodlr_sampler_workspace_size(hodlr_plan p, int32_t walkers, size_t *bytes);
/* cfg->steps steps of all walkers on the shared points d_x / observations
 * d_y of plan p (kernel k, tolerance tol).  d_wbf16 non-NULL selects the
 * delayed form with that network; NULL the plain form.  Step t uses
 * d_eps[3Wt ..], d_u1[Wt ..], d_u2[Wt ..]; d_chain (nullable) receives theta
 * after each step (steps x W x 3).  One host synchronization per step reads
 * the survivor count.  stats (host, nullable) gets the tallies.
 * Errors: EINVAL, EDEVICE; a failed exact evaluation rejects its move.     */
hodlr_status gp_sample_dev(hodlr_plan p, const double *d_x, hodlr_kernel k, const double *d_y,
                           double tol, const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                           const hodlr_sampler_cfg *cfg, double *d_theta, double *d_lp,
                           double *d_sur, const double *d_eps, const double *d_u1,
                           const double *d_u2, void *d_work, size_t work_bytes, void *stream,
                           double *d_chain, hodlr_sampler_stats *stats);

/* ------------------------------------------------------------ profiling */

#define HODLR_PROF_STAGES 16

/* Per-kernel timing with HIP events recorded on the stream each kernel is
 * launched on (tracing aid; not part of the method).  Stage names are
 * NUL-terminated; ms is the summed event time and launches the number of
 * timed launches since the last reset.                                      */
typedef struct {
    int32_t nstages;
    char name[HODLR_PROF_STAGES][32];
    double ms[HODLR_PROF_STAGES];
    int64_t launches[HODLR_PROF_STAGES];
} hodlr_profile_t;

/* on = 1 starts timing (and clears the counters), 0 stops.  Process-wide.  */
hodlr_status hodlr_profile_enable(int32_t on);
/* Bit s of mask (stage s in the order hodlr_profile_read reports them)
 * selects which kinds are timed; default: all.  Timing only the kernel of
 * interest keeps the event overhead out of a throughput measurement.        */
hodlr_status hodlr_profile_select(uint32_t mask);
/* Copies the counters of every timed launch so far (waits for the events of
 * launches still in flight).                                               */
hodlr_status hodlr_profile_read(hodlr_profile_t *out);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H */
