// Internal definitions shared by the HIP translation units of libhodlrgp.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "hodlr.h"

namespace hodlr {

// ------------------------------------------------------------- constants
constexpr int ZERO_RETRY = 8;     // consecutive zero-pivot rows before a block stops
// block entries per work-group and pass of the large blocks' cross
// approximation.  1-D (ranks ~3) measured at n = 2^20: 512 0.52 ms, 1024 0.39,
// 2048 0.37, 4096 0.39 per likelihood.  2-D SE at n = 2^18 (ranks up to 64,
// about 130 passes, each entry subtracting up to 64 earlier terms):
// 256 -> 30.0, 512 -> 35.6, 1024 -> 33.2, 2048 -> 19.8 likelihoods/s (short
// work-groups shorten every pass until the per-pass record sums dominate).
constexpr int ACA_CHUNK_1D = 2048;
constexpr int ACA_CHUNK_ND = 512;
constexpr int ACA_SMALL = 2048;   // blocks with both sides <= this run in one work-group
constexpr int ACA_TINY = 256;     // ... and on a single wave when both sides are <= this
constexpr int ACA_THREADS = 256;
// sketch compressor: oversampling of X (beyond the cap) and of Y (beyond X),
// the largest cap, and the sketch widths it implies
constexpr int SK_OVER_X = 16, SK_OVER_Y = 8;
constexpr int SK_CAP_MAX = 64;
constexpr int SK_SMAX = SK_CAP_MAX + SK_OVER_X;    // 80 columns of X
constexpr int SK_SPMAX = SK_SMAX + SK_OVER_Y;      // 88 columns of Y
constexpr int SK_ROWS = 64;                        // rows per sketch work-group
constexpr int LVL_ROWS = 512;     // default rows per level work-group
constexpr int LEAF_LDS_MAX = 128; // leaves up to this size are factored wholly in LDS
constexpr int LEAF_MAX = 256;     // larger leaves (up to this) keep their off-diagonal half in HBM
constexpr int RMAX_ABS = 512;     // upper bound on max_rank
constexpr int RMAX_LDS = 64;      // ranks up to this: coupling matrices in LDS, narrow kernels
// rows a block may try as pivots: every accepted term can follow ZERO_RETRY zero rows
constexpr int used_max(int rb) { return (rb + 1) * (ZERO_RETRY + 1) + 2; }
constexpr int USED_MAX = used_max(RMAX_ABS);

enum AcaDone { ACA_ACTIVE = 0, ACA_CONVERGED = 1, ACA_CAPPED = 2, ACA_EXHAUSTED = 3 };

// Cross-approximation state of one large block (device resident, moved
// between launches only).
struct BigState {
    int k;          // terms accepted so far
    int istar;      // current pivot row (local index in alpha)
    int jstar;      // pivot column of the current term (local index in beta)
    int zeros;      // consecutive zero-pivot rows
    int nused;      // rows used as pivots so far
    int cap;        // min(max_rank, |alpha|, |beta|)
    int usercap;    // 1 if cap came from max_rank (a hit counts as "capped")
    int done;       // AcaDone
    int phase;      // which pass results are pending
    int pad_;
    double delta;   // pivot value of the current term
    double v2;      // ||v_k||^2 of the current term
    double s2;      // ||S_k||_F^2 running estimate
};

// One work-group's slice of a block or of a level.
struct Chunk {
    int node;       // heap index of the split node tau
    int side;       // 0: rows of alpha (left child), 1: rows of beta (right child)
    int64_t lo, hi; // global row range (tree order)
    int part;       // partial-result slot (unique within its launch table)
    int pad_;
};

// Kernel parameters: k(r) from r^2, with c the scale of the kernel:
//   SE: a2 exp(-c r^2), c = 1/(2 l^2);  Matern-3/2: s = c r, a2 (1+s) e^{-s},
//   c = sqrt(3)/l;  exponential: a2 exp(-c r), c = 1/l;  constant: a2.
struct KParams {
    int kind;
    int dim;
    double a2;
    double c;
    double sigma2;
    const double *noise = nullptr;   // per-point variances added to sigma2, tree order
};

inline KParams make_kparams(int kind, int dim, const double theta[2], double sigma2)
{
    KParams k;
    k.kind = kind;
    k.dim = dim;
    k.a2 = theta[0] * theta[0];
    double l = theta[1];
    switch (kind) {
    case HODLR_K_SE: k.c = 1.0 / (2.0 * l * l); break;
    case HODLR_K_MATERN32: k.c = std::sqrt(3.0) / l; break;
    case HODLR_K_EXP: k.c = 1.0 / l; break;
    case HODLR_K_IMQ: k.c = 1.0 / (l * l); break;
    default: k.c = 0.0; break;
    }
    k.sigma2 = sigma2;
    k.noise = nullptr;
    return k;
}

template <typename T>
__device__ __forceinline__ T kfun_r2(int kind, T a2, T c, T r2)
{
    switch (kind) {
    case HODLR_K_SE:
        return a2 * exp(-c * r2);
    case HODLR_K_MATERN32: {
        T s = c * sqrt(r2);
        return a2 * (T(1) + s) * exp(-s);
    }
    case HODLR_K_EXP:
        return a2 * exp(-c * sqrt(r2));
    case HODLR_K_IMQ:
        return a2 / sqrt(T(1) + c * r2);
    default:
        return a2;
    }
}

// Squared distance between ordered points i and j; coordinates are
// coordinate-major (x[d*n + i]).
// dim is 1, 2 or 3 (checked at every entry point).  All coordinate loads are
// issued without a condition (dimensions past dim read coordinate 0 and add
// nothing), so none waits in a branch of its own; the sum is the same.
__device__ __forceinline__ double dist2(const double *__restrict__ x, int64_t n, int dim, int64_t i,
                                        int64_t j)
{
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int64_t o = (d < dim ? d : 0) * n;
        const double t = x[o + i] - x[o + j];
        r2 += d < dim ? t * t : 0.0;
    }
    return r2;
}

// ----------------------------------------------------------- batching
// A batch of items shares one plan: item b's workspace starts b * istride
// bytes after item 0's, its kernel parameters (a, l, sigma^2) are
// params[3b .. 3b+2] when params is given, and its right-hand side starts
// b * ystride doubles after item 0's.  Kernels take the item from blockIdx.z.
struct BatchArgs {
    int64_t istride = 0;
    const double *params = nullptr;
    int64_t ystride = 0;
};

template <typename T>
__device__ __forceinline__ T *ioff(T *p, const BatchArgs &B, int item)
{
    return p ? (T *)((char *)p + B.istride * item) : p;
}

__device__ __forceinline__ KParams item_kp(KParams kp, const BatchArgs &B, int item)
{
    if (B.params) {
        const double a = B.params[3 * item], l = B.params[3 * item + 1];
        kp.a2 = a * a;
        kp.c = (kp.kind == HODLR_K_SE) ? 1.0 / (2.0 * l * l)
             : (kp.kind == HODLR_K_MATERN32) ? 1.7320508075688772 / l
             : (kp.kind == HODLR_K_EXP) ? 1.0 / l
             : (kp.kind == HODLR_K_IMQ) ? 1.0 / (l * l) : 0.0;
        kp.sigma2 = B.params[3 * item + 2];
    }
    return kp;
}

__device__ __forceinline__ double kentry(const KParams &kp, const double *__restrict__ x, int64_t n,
                                         int64_t i, int64_t j)
{
    return kfun_r2<double>(kp.kind, kp.a2, kp.c, dist2(x, n, kp.dim, i, j));
}

// ------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// argmax of |value| with ties to the smaller index
__device__ __forceinline__ void wave_argmax(double &v, int64_t &idx)
{
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off, 64);
        int64_t oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

// same, carrying a payload (the signed value at the winning index)
__device__ __forceinline__ void wave_argmax_signed(double &v, int64_t &idx, double &pay)
{
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off, 64);
        int64_t oi = __shfl_xor(idx, off, 64);
        double op = __shfl_xor(pay, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
            pay = op;
        }
    }
}

__device__ __forceinline__ double ld_coherent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_coherent(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------- host helpers
struct Error {
    hodlr_status st;
    std::string msg;
};

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::hodlr::Error{HODLR_EDEVICE, std::string(#expr) + ": " +               \
                                                    hipGetErrorString(e_)};               \
    } while (0)

// Status bits written by kernels into the workspace.
enum DevStatus { DS_NOTSPD_LEAF = 1, DS_NOTSPD_NODE = 2, DS_NONFINITE = 4, DS_SPEC_MISS = 8 };

// ----------------------------------------------------------- the plan
// Tree, per-depth column layout and launch tables for one (n, dim, leaf, cap).
struct Plan {
    int64_t n = 0;
    int dim = 1;
    int leaf = 1;
    int L = 0;
    int cap = 64;
    int precision = HODLR_FP64;
    int lvl_rows = LVL_ROWS;   // rows per level-stage chunk (256, 512 or 1024)
    int red_cols = 4;          // columns per iteration of the small-rank reduction (4 or 8)
    int red_grp = 8;           // columns per work-group of the small-rank reduction (8 or 64)
    double refine_tol = 1e-10;
    int max_refine = 8;
    bool refine = false;       // host solves refine against the exact product (always when mixed)
    bool mixed_check = false;  // mixed form: test the log-det error bound, redo in FP64 if missed
    int compressor = HODLR_COMPRESS_ACA;
    int level_form = 0;        // 0: projected levels for a likelihood when they fit; 1: never
    // sketch compressor tables, per depth d: 64-row chunks of both children of
    // every depth-d node (alpha chunks of a node first; an alpha chunk's part
    // is its partial-core slot, contiguous per node), and per node the first
    // alpha slot and the alpha chunk count
    std::vector<std::vector<Chunk>> sk;
    std::vector<std::vector<int>> sk_abase, sk_acnt;
    int64_t nint = 0;    // internal (split) nodes 2^L - 1
    int64_t nleaf = 1;   // 2^L
    int leafmax = 0;
    std::vector<int64_t> start, end;   // per heap node (2^(L+1) - 1)
    std::vector<int> capj;             // per depth j = 1..L: columns reserved
    std::vector<int64_t> cofa;         // per depth j: first column of the panel; [L+1] = total
    int64_t ncol = 1;                  // columns of W / Xt (column 0 is the solve vector)
    // cross-approximation tables
    std::vector<int> aca_small;            // heap indices of blocks done by one work-group
    int aca_small_wide = 0;                // the first ones, with a side above ACA_TINY
    mutable int aca_iters = 0;             // large-block steps the last call took (poll hint;
                                           // relaxed atomic accesses, plans may be shared)
    std::vector<int> aca_big;              // heap indices of multi-work-group blocks
    int aca_big_active = 0;                // big blocks with a positive rank cap
    std::vector<Chunk> aca_row, aca_col;   // big blocks: chunks over beta / alpha
    std::vector<int> aca_rowidx, aca_colidx;   // per chunk: big-block index
    std::vector<int> aca_nrow, aca_ncol;   // per big block: chunk counts
    std::vector<int> aca_rowbase, aca_colbase;
    std::vector<Chunk> pad_chunks;         // all blocks, both sides
    int aca_pw = 0;                        // doubles per ACA partial record
    int aca_chunk = ACA_CHUNK_1D;          // block entries per large-block pass work-group
    // level tables: per depth d, chunks over rows of the children of depth-d nodes
    std::vector<std::vector<Chunk>> lvl;
    std::vector<std::vector<int>> lvl_nch;   // per depth, per node: chunks (both sides)
    std::vector<std::vector<int>> lvl_base;  // per depth, per node: first partial slot
    std::vector<int> lvl_maxlen;             // per depth: rows of the longest chunk
    // offsets of the device tables inside their image
    struct TableOffsets {
        size_t start, end, ar, ac, pc, nr, nc, rb, cb, bg, sm, ri, ci;
        std::vector<size_t> l, ln, lb, k, ka, kc;
    } tbl;
    // device copies of the tables
    void *dev_tables = nullptr;
    size_t dev_tables_bytes = 0;
    int64_t *d_start = nullptr, *d_end = nullptr;
    Chunk *d_aca_row = nullptr, *d_aca_col = nullptr, *d_pad_chunks = nullptr;
    int *d_aca_nrow = nullptr, *d_aca_ncol = nullptr, *d_aca_rowbase = nullptr,
        *d_aca_colbase = nullptr, *d_aca_small = nullptr, *d_aca_big = nullptr,
        *d_aca_rowidx = nullptr, *d_aca_colidx = nullptr;
    std::vector<Chunk *> d_lvl;
    std::vector<int *> d_lvl_nch, d_lvl_base;
    std::vector<Chunk *> d_sk;
    std::vector<int *> d_sk_abase, d_sk_acnt;
    int device = 0;

    int depth_of(int64_t h) const
    {
        int d = 0;
        while (((int64_t)2 << d) - 1 <= h)
            ++d;
        return d;
    }
    int64_t first_at(int d) const { return ((int64_t)1 << d) - 1; }
    // the mixed form keeps the applied-basis panel W~ (and the solve vector) in
    // FP32; the compressed bases W stay FP64
    bool f32() const { return precision == HODLR_MIXED; }
    size_t panel_bytes() const { return f32() ? sizeof(float) : sizeof(double); }
};

// byte offset in the workspace's misc area of the mixed form's log-det error
// estimate (one double per item, written by the finish kernel)
constexpr size_t MISC_BOUND = 3072;
constexpr size_t MISC_SPEC = 2048;   // 64 ints: a speculative call's actual rank statistics

// Workspace layout (byte offsets into one device buffer).
struct Layout {
    size_t W, Xt, G, L21;
    size_t aca_state, aca_used, aca_vdots, aca_part, aca_status;
    size_t rank, leaf_ld, node_ld;
    size_t lvl_part, Tbuf, Sbuf, small;
    size_t dot_part, out, status, cols, misc;
    size_t sk_buf, sk_part, sk_core, sk_fac;   // sketch compressor (8 bytes otherwise)
    size_t total;
    int64_t small_stride;   // doubles per internal node in the small-factor store
    int64_t T_stride;       // doubles per node in Tbuf/Sbuf
    int64_t lvl_part_cap;   // doubles in lvl_part
    bool store_leaf;
};

Layout make_layout(const Plan &p, bool store_leaf);

// Build the plan (host); upload tables to the current device.
void plan_build(Plan &p, int64_t n, int dim, int leaf, const hodlr_opts *opts,
                int lvl_rows = LVL_ROWS, int red_cols = 4, int red_grp = 8);
void plan_upload(Plan &p);
void plan_release(Plan &p);
size_t plan_image(Plan &p, std::vector<char> &host);   // table image + offsets
void plan_bind(Plan &p, char *dev);                    // point the tables at dev

// k-d / sort ordering of caller points (point-major) -> perm
void order_points(const double *x, int64_t n, int dim, int leaf, int64_t *perm);
int num_levels(int64_t n, int leaf);

// ------------------------------------------------------ device pipeline
struct Pipeline {
    const Plan *plan;
    Layout lay;
    char *ws;
    hipStream_t stream;
    const double *x;      // ordered, coordinate-major
    KParams kp;
    double tol;
    int nitems = 1;       // batch size (all items share the plan)
    BatchArgs batch;      // istride = lay.total rounded, params per item
    bool capturing = false;
    bool side_stream = true;  // small-block compression on a second stream of this thread
    int *host_ints = nullptr; // 64 host ints for the compression's statistics (nullptr:
                              // this thread's pinned buffer, allocated on first use)
    // host-side results of the compression
    std::vector<int> rmax;    // per depth j (1..L), used columns of the panel
    std::vector<int> cols;    // used column indices, depth-ascending, cols[0] = 0
    std::vector<int> cnt;     // cnt[d] = 1 + sum_{j<=d} rmax[j]
    int capped = 0;
    std::vector<int> ranks;   // per internal node
    // speculation (gp_loglik_dev): panel widths per depth index (as rmax) to
    // assume instead of waiting for the compression's statistics; spec_run
    // tells whether the compression actually ran that way
    const std::vector<int> *spec = nullptr;
    bool spec_run = false;
    const double *rhs = nullptr;   // the right-hand side the leaf factor was given
    bool proj_run = false;         // the last run_levels_factor took the projected form
};

// ------------------------------------------------------------ profiling
// Optional HIP-event timing of every launch, per kernel kind (tracing aid).
enum ProfStage {
    PS_ACA_ROW = 0, PS_ACA_COL, PS_ACA_SMALL, PS_ACA_MISC, PS_LEAF, PS_LEAF_SOLVE, PS_LVL_REDUCE, PS_LVL_SOLVE,
    PS_LVL_UPDATE, PS_FINISH, PS_MATVEC, PS_PREDICT, PS_SKETCH, PS_SKETCH_CORE, PS_COUNT
};
bool prof_on(int stage);
void prof_suspend(bool on);   // no event recording (e.g. while a stream is captured)
int prof_begin(hipStream_t s);
void prof_end(int slot, hipStream_t s, int stage);
void prof_collect();   // after the stream has been synchronized
struct ProfScope {
    int slot;
    hipStream_t s;
    int stage;
    ProfScope(hipStream_t s_, int st) : slot(-1), s(s_), stage(st)
    {
        if (prof_on(st))
            slot = prof_begin(s);
    }
    ~ProfScope()
    {
        if (slot >= 0)
            prof_end(slot, s, stage);
    }
};

// Stages (implemented in the .hip files)
void run_aca(Pipeline &P);                                   // fills W panels, ranks
void run_aca_batched(Pipeline &P);                           // every block of every item
void run_leaf_factor(Pipeline &P, const double *y);          // leaves: G, log-dets, Xt
void run_levels_factor(Pipeline &P);                         // coupling matrices, Xt, z
// projected levels (log det and C^{-1} y from the bases' projections)
constexpr int PJ_MMAX = 128;   // panel columns (y and the bases of all depths)
constexpr int PJ_WMAX = 32;    // columns of one depth
bool proj_fits(const Pipeline &P);
void run_levels_projected(Pipeline &P);
void run_solve(Pipeline &P, double *z);                      // z := C^{-1} z using a built factor
void run_finish(Pipeline &P, const double *y, double *d_out, int ostride = 8);  // log det, quad, loglik
// refinement helpers (misc.hip); z is the panel-typed solve vector
void run_cast_scaled(const double *r, double inv, void *z, bool f32, int64_t n, hipStream_t s);
void run_axpy(double *x, double a, const void *z, bool f32, int64_t n, hipStream_t s);
void run_widen(const void *z, bool f32, double *out, int64_t n, hipStream_t s,
               double scale = 1.0);
void run_xpby(const double *z, double beta, double *p, int64_t n, hipStream_t s);   // p = z + beta p
double run_dot(const double *a, const double *b, int64_t n, double *part, hipStream_t s);
// prediction (predict.hip): the mean k(xt, x) alpha (part holds
// predict_slices(n, m) x m doubles) and columns of k(x, xt)
int predict_slices(int64_t n, int64_t m);
void run_predict_mean(int64_t n, const KParams &kp, const double *x, const double *alpha,
                      int64_t m, const double *xt, double *part, double *mean, hipStream_t s);
void run_kcross(int64_t n, const KParams &kp, const double *x, int64_t m, const double *xt,
                int64_t j0, int nb, double *out, hipStream_t s);
void run_sub(const double *y, const double *cx, double *r, int64_t n, hipStream_t s);
double run_sumsq(const double *v, int64_t n, double *part, hipStream_t s);
void run_matvec(int64_t n, const KParams &kp, const double *x, const double *v, double *out,
                hipStream_t s);
void make_columns(Pipeline &P);                                // column list after compression
int read_status(Pipeline &P);                                  // synchronizes the stream
void raise_status(int st);
void factor_pipeline(Pipeline &P, const double *d_y, double *d_out);
// mixed form: true if the log-det error bound of batch item `item` (written by
// the finish kernel) exceeds the 1e-8 bar for this log det (synchronizes)
bool mixed_estimate_missed(const Pipeline &P, double logdet, int item);
bool mixed_estimate_exceeds(double estimate, double logdet);
double *queue_mixed_check(const Pipeline &P, const double *d_out);
int *pinned_scratch();                                         // per-thread pinned ints
int *pinned_ints(size_t n, int slot);   // per-thread growable pinned ints, slots 0-3 (0: ranks, 1: column list, 2: statistics, 3: end-of-call values)
void host_wait(hipStream_t s);                                 // poll the stream to completion

template <typename T>
inline T *wsp(const Pipeline &P, size_t off)
{
    return reinterpret_cast<T *>(P.ws + off);
}

}  // namespace hodlr
