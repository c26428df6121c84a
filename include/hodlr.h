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
 *  - Precision: FP64 everywhere by default.  HODLR_MIXED evaluates kernel
 *    entries, compresses and runs the level updates in FP32, keeps leaf
 *    factorizations and determinants in FP64, and recovers the solve by
 *    iterative refinement against an exact FP64 matrix-vector product.
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
    HODLR_ENOCONV = 5   /* mixed form: refinement missed refine_tol within max_refine steps
                           (outputs ARE written with the best iterate) */
} hodlr_status;

/* Covariance kernels (Table 1 and §5 of the paper, amplitude/length-scale form),
 * r = Euclidean distance, theta = {a, l}. */
typedef enum {
    HODLR_K_SE = 0,        /* a^2 exp(-r^2 / (2 l^2))                      */
    HODLR_K_MATERN32 = 1,  /* a^2 (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)  */
    HODLR_K_EXP = 2,       /* a^2 exp(-r / l)  (Ornstein-Uhlenbeck)         */
    HODLR_K_CONST = 3      /* a^2  (rank one; for tests)                    */
} hodlr_kernel;

enum { HODLR_FP64 = 0, HODLR_MIXED = 1 };

typedef struct {
    int32_t max_rank;    /* per off-diagonal block rank cap (default 64); a hit cap is
                            counted in hodlr_info, not an error                       */
    int32_t precision;   /* HODLR_FP64 (default) or HODLR_MIXED                        */
    double refine_tol;   /* mixed form: stop at ||y - C x|| / ||y|| <= refine_tol
                            (default 1e-10)                                           */
    int32_t max_refine;  /* mixed form: at most this many refinement steps (default 8) */
    int32_t presorted;   /* 1: the points are already in tree order; skip ordering     */
} hodlr_opts;          /* pass NULL for all defaults */

typedef struct hodlr_factor_s *hodlr_factor;   /* opaque; immutable after build */
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
 * y.  Mixed-precision factors refine each column to refine_tol (ENOCONV if
 * not reached; x still holds the best iterate).                             */
hodlr_status hodlr_solve(hodlr_factor f, const double *y, double *x, int64_t nrhs);

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

/* Bytes of device workspace one gp_loglik_dev call needs (256-byte aligned).*/
hodlr_status hodlr_plan_workspace_size(hodlr_plan p, size_t *bytes);

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
 * without synchronizing; results are ready when the stream is.             */
hodlr_status hodlr_plan_batch_workspace_size(hodlr_plan p, int32_t nitems, size_t *bytes);
hodlr_status gp_loglik_batch_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                                 const double *d_params, int32_t nitems, const double *d_y,
                                 int64_t y_stride, double tol, void *d_work, size_t work_bytes,
                                 void *stream, double *d_out, int32_t use_graph);

/* Log-likelihoods (Eq. (1), as gp_loglik) of m independent problems of
 * uneven size.  Item i has ns[i] points xs[i] (point-major ns[i]*dim host
 * doubles, caller order), observations ys[i] (ns[i] host doubles) and
 * hyperparameters {a, l, sigma2} = params[3i .. 3i+2]; dim, kernel, leaf,
 * tol and opts are shared.  nworkers host threads (<= 0: 8) each own a
 * stream and one device arena sized for the largest item, and take items
 * largest first.  out receives 3 doubles per item {loglik, logdet, quad}; an
 * item that is invalid or whose factorization fails gets NaNs and does not
 * stop the others.  All pointers are host memory owned by the caller; the
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
/* Copies the counters accumulated by completed calls.                      */
hodlr_status hodlr_profile_read(hodlr_profile_t *out);

#ifdef __cplusplus
}
#endif
#endif /* HODLR_H */
