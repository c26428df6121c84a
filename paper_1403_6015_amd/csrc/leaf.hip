// Leaf stage: the dense diagonal blocks C_lambda = K(lambda, lambda) +
// sigma^2 I of the finest level (the factor K_kappa of §3.2), their Cholesky
// factors and log-dets, and the application of C_lambda^{-1} to the rows of
// every off-diagonal basis that covers the leaf ("a p x p inverse ... applied
// to all left low-rank factors", §3.3) together with the right-hand side.
//
// One work-group per leaf.  The block is evaluated on the fly from the
// ordered coordinates straight into LDS (packed lower triangle), factored
// there, and the basis columns stream through LDS in batches.
#include "common.h"

namespace hodlr {

constexpr int LEAF_THREADS = 256;
constexpr int LEAF_XB = 32;   // columns per batch of the triangular solves

struct LeafArgs {
    const double *x;
    int64_t n;
    KParams kp;
    const int64_t *start, *end;
    int64_t leaf0;          // heap index of the first leaf
    const double *W;        // original bases (source columns)
    double *Xt;             // destination columns
    const double *y;        // right-hand side for column 0 (nullable)
    const int *cols;
    int ncols, cbeg;
    double *G;              // packed Cholesky factors (nullable)
    int64_t gstride;
    double *leaf_ld;
    int *status;
};

__device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__device__ __forceinline__ int tri_row(int idx)
{
    int i = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (tri(i + 1) <= idx)
        ++i;
    while (tri(i) > idx)
        --i;
    return i;
}

// Forward and backward substitution with the packed factor in LDS on nb
// columns of Xs (row stride LEAF_XB + 1): Xs <- C^{-1} Xs.
__device__ void leaf_trsm(const double *Ap, double *Xs, int m, int nb)
{
    const int tid = threadIdx.x;
    const int ld = LEAF_XB + 1;
    for (int j = 0; j < m; ++j) {
        double g = Ap[tri(j) + j];
        for (int c = tid; c < nb; c += LEAF_THREADS)
            Xs[j * ld + c] /= g;
        __syncthreads();
        int rows = m - j - 1;
        for (int idx = tid; idx < rows * nb; idx += LEAF_THREADS) {
            int i = j + 1 + idx / nb, c = idx % nb;
            Xs[i * ld + c] -= Ap[tri(i) + j] * Xs[j * ld + c];
        }
        __syncthreads();
    }
    for (int j = m - 1; j >= 0; --j) {
        double g = Ap[tri(j) + j];
        for (int c = tid; c < nb; c += LEAF_THREADS)
            Xs[j * ld + c] /= g;
        __syncthreads();
        for (int idx = tid; idx < j * nb; idx += LEAF_THREADS) {
            int i = idx / nb, c = idx % nb;
            Xs[i * ld + c] -= Ap[tri(j) + i] * Xs[j * ld + c];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(LEAF_THREADS) void leaf_factor_kernel(LeafArgs A)
{
    __shared__ double Ap[LEAF_LDS_MAX * (LEAF_LDS_MAX + 1) / 2];
    __shared__ double Xs[LEAF_LDS_MAX * (LEAF_XB + 1)];
    __shared__ double xc[3][LEAF_LDS_MAX];
    __shared__ double colj[LEAF_LDS_MAX];
    __shared__ double red[4];
    __shared__ int sfail;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    const int64_t n = A.n;
    if (m == 0) {
        if (tid == 0)
            A.leaf_ld[b] = 0.0;
        return;
    }
    for (int idx = tid; idx < m * A.kp.dim; idx += LEAF_THREADS) {
        int d = idx / m, i = idx % m;
        xc[d][i] = A.x[d * n + s + i];
    }
    if (tid == 0)
        sfail = 0;
    __syncthreads();
    const int np = tri(m);
    for (int idx = tid; idx < np; idx += LEAF_THREADS) {
        int i = tri_row(idx), k = idx - tri(i);
        double r2 = 0.0;
        for (int d = 0; d < A.kp.dim; ++d) {
            double t = xc[d][i] - xc[d][k];
            r2 += t * t;
        }
        double v = kfun_r2<double>(A.kp.kind, A.kp.a2, A.kp.c, r2);
        if (i == k)
            v += A.kp.sigma2;
        Ap[idx] = v;
    }
    __syncthreads();
    // right-looking Cholesky in the packed lower triangle
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            double d = Ap[tri(j) + j];
            if (!(d > 0.0))
                sfail = 1;
            else
                Ap[tri(j) + j] = sqrt(d);
        }
        __syncthreads();
        if (sfail)
            break;
        double g = Ap[tri(j) + j];
        for (int i = j + 1 + tid; i < m; i += LEAF_THREADS) {
            double v = Ap[tri(i) + j] / g;
            Ap[tri(i) + j] = v;
            colj[i] = v;
        }
        __syncthreads();
        for (int i = j + 1 + wid; i < m; i += 4) {
            double ci = colj[i];
            int base = tri(i);
            for (int k = j + 1 + lane; k <= i; k += 64)
                Ap[base + k] -= ci * colj[k];
        }
        __syncthreads();
    }
    if (sfail) {
        if (tid == 0) {
            atomicOr(A.status, DS_NOTSPD_LEAF);
            A.leaf_ld[b] = __builtin_nan("");
        }
        return;
    }
    double lg = 0.0;
    for (int i = tid; i < m; i += LEAF_THREADS)
        lg += log(Ap[tri(i) + i]);
    lg = wave_sum(lg);
    if (lane == 0)
        red[wid] = lg;
    if (A.G) {
        double *g = A.G + b * A.gstride;
        for (int idx = tid; idx < np; idx += LEAF_THREADS)
            g[idx] = Ap[idx];
    }
    __syncthreads();
    if (tid == 0)
        A.leaf_ld[b] = 2.0 * ((red[0] + red[1]) + (red[2] + red[3]));
    // C_lambda^{-1} on the leaf rows of every column of the list
    for (int c0 = A.cbeg; c0 < A.ncols; c0 += LEAF_XB) {
        int nb = min(LEAF_XB, A.ncols - c0);
        for (int idx = tid; idx < nb * m; idx += LEAF_THREADS) {
            int c = idx / m, i = idx % m;
            int col = A.cols[c0 + c];
            double v = (col == 0) ? A.y[s + i] : A.W[(int64_t)col * n + s + i];
            Xs[i * (LEAF_XB + 1) + c] = v;
        }
        __syncthreads();
        leaf_trsm(Ap, Xs, m, nb);
        for (int idx = tid; idx < nb * m; idx += LEAF_THREADS) {
            int c = idx / m, i = idx % m;
            int col = A.cols[c0 + c];
            A.Xt[(int64_t)col * n + s + i] = Xs[i * (LEAF_XB + 1) + c];
        }
        __syncthreads();
    }
}

// z <- C_lambda^{-1} z on each leaf with the stored packed factors
__global__ __launch_bounds__(LEAF_THREADS) void leaf_solve_kernel(LeafArgs A, double *z)
{
    __shared__ double Ap[LEAF_LDS_MAX * (LEAF_LDS_MAX + 1) / 2];
    __shared__ double Xs[LEAF_LDS_MAX * (LEAF_XB + 1)];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t h = A.leaf0 + b;
    const int64_t s = A.start[h];
    const int m = (int)(A.end[h] - s);
    if (m == 0)
        return;
    const double *g = A.G + b * A.gstride;
    for (int idx = tid; idx < tri(m); idx += LEAF_THREADS)
        Ap[idx] = g[idx];
    for (int i = tid; i < m; i += LEAF_THREADS)
        Xs[i * (LEAF_XB + 1)] = z[s + i];
    __syncthreads();
    leaf_trsm(Ap, Xs, m, 1);
    for (int i = tid; i < m; i += LEAF_THREADS)
        z[s + i] = Xs[i * (LEAF_XB + 1)];
}

static LeafArgs leaf_args(Pipeline &P)
{
    const Plan &p = *P.plan;
    LeafArgs A;
    A.x = P.x;
    A.n = p.n;
    A.kp = P.kp;
    A.start = p.d_start;
    A.end = p.d_end;
    A.leaf0 = p.nint;
    A.W = wsp<double>(P, P.lay.W);
    A.Xt = wsp<double>(P, P.lay.Xt);
    A.y = nullptr;
    A.cols = wsp<int>(P, P.lay.cols);
    A.ncols = 0;
    A.cbeg = 1;
    A.G = P.lay.store_leaf ? wsp<double>(P, P.lay.G) : nullptr;
    A.gstride = (int64_t)p.leafmax * (p.leafmax + 1) / 2;
    A.leaf_ld = wsp<double>(P, P.lay.leaf_ld);
    A.status = wsp<int>(P, P.lay.status);
    return A;
}

void run_leaf_factor(Pipeline &P, const double *y)
{
    const Plan &p = *P.plan;
    if (p.leafmax > LEAF_LDS_MAX)
        throw Error{HODLR_EINVAL, "leaf size above 128 is not supported by this build"};
    LeafArgs A = leaf_args(P);
    A.y = y;
    A.cbeg = y ? 0 : 1;
    A.ncols = P.cnt[p.L];
    ProfScope ps(P.stream, PS_LEAF);
    leaf_factor_kernel<<<(unsigned)p.nleaf, LEAF_THREADS, 0, P.stream>>>(A);
    HIP_TRY(hipGetLastError());
}

void run_leaf_solve(Pipeline &P, double *z)
{
    const Plan &p = *P.plan;
    LeafArgs A = leaf_args(P);
    ProfScope ps(P.stream, PS_LEAF_SOLVE);
    leaf_solve_kernel<<<(unsigned)p.nleaf, LEAF_THREADS, 0, P.stream>>>(A, z);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
