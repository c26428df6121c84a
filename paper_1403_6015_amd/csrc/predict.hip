// Prediction through the factor (§2.1, the predictive mean and variance of
// f at new inputs): the mean is the kernel product k(xt, x) alpha with
// alpha = C^{-1} y, the variance k(xt, xt) - k(xt, x) C^{-1} k(x, xt) needs
// the columns k(x, xt_j), which are built here and solved by the factor.
//
// Both products evaluate every kernel entry exactly (no truncation of small
// entries): one test point per thread, the training points streamed through
// LDS in tiles, and the training points split into slices over a second grid
// dimension so that a few hundred test points still fill the chip; the slices'
// partial sums are added in slice order, so the result does not depend on
// the launch.
#include <type_traits>

#include "common.h"

namespace hodlr {

constexpr int PR_T = 256;   // test points per work-group, training points per LDS tile

// k / a^2 between a test point and a training point, specialized on the kernel
// and the dimension (in 1-D the distance is |d|, no square root of d^2); the
// amplitude a^2 multiplies whole sums and columns instead of every entry
template <int KIND, int DIM>
__device__ __forceinline__ double kshape(const KParams &kp, const double (&a)[3], const double *b)
{
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double q = a[d] - b[d];
        r2 += q * q;
    }
    if constexpr (KIND == HODLR_K_SE) {
        return exp(-kp.c * r2);
    } else if constexpr (KIND == HODLR_K_MATERN32 || KIND == HODLR_K_EXP) {
        const double r = DIM == 1 ? fabs(a[0] - b[0]) : sqrt(r2);
        const double s = kp.c * r;
        return KIND == HODLR_K_MATERN32 ? (1.0 + s) * exp(-s) : exp(-s);
    } else if constexpr (KIND == HODLR_K_IMQ) {
        return 1.0 / sqrt(1.0 + kp.c * r2);
    } else {
        return 1.0;
    }
}

// part[s * m + j] = sum over slice s of the training points of k(xt_j, x_i) alpha_i
// (a^2 times the sum of the shape products)
template <int KIND, int DIM>
__global__ __launch_bounds__(PR_T) void predict_part_kernel(int64_t n, KParams kp,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ alpha,
                                                            int64_t m, const double *__restrict__ xt,
                                                            int64_t slice, double *__restrict__ part)
{
    __shared__ double sx[PR_T][DIM];
    __shared__ double sa[PR_T];
    const int tid = threadIdx.x;
    const int64_t j = blockIdx.x * (int64_t)PR_T + tid;
    double xj[3] = {0.0, 0.0, 0.0};
    if (j < m)
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            xj[d] = xt[d * m + j];
    const int64_t i0 = blockIdx.y * slice;
    const int64_t i1 = min(n, i0 + slice);
    double acc = 0.0;
    for (int64_t c0 = i0; c0 < i1; c0 += PR_T) {
        const int64_t i = c0 + tid;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            sx[tid][d] = (i < i1) ? x[d * n + i] : 0.0;
        sa[tid] = (i < i1) ? alpha[i] : 0.0;
        __syncthreads();
        const int cnt = (int)min<int64_t>(PR_T, i1 - c0);
        for (int t = 0; t < cnt; ++t)
            acc += kshape<KIND, DIM>(kp, xj, sx[t]) * sa[t];
        __syncthreads();
    }
    if (j < m)
        part[blockIdx.y * m + j] = kp.a2 * acc;
}

__global__ void predict_sum_kernel(const double *__restrict__ part, int nslice, int64_t m,
                                   double *__restrict__ mean)
{
    for (int64_t j = blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int q = 0; q < nslice; ++q)
            s += part[(int64_t)q * m + j];
        mean[j] = s;
    }
}

// out[c * n + i] = k(x_i, xt_{j0 + c}) for c < nb (columns of k(x, xt))
template <int KIND, int DIM>
__global__ void kcross_kernel(int64_t n, KParams kp, const double *__restrict__ x, int64_t m,
                              const double *__restrict__ xt, int64_t j0, int nb,
                              double *__restrict__ out)
{
    const int64_t total = n * nb;
    for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t c = idx / n, i = idx - c * n;
        double a[3] = {0.0, 0.0, 0.0}, b[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            a[d] = xt[d * m + j0 + c];
            b[d] = x[d * n + i];
        }
        out[idx] = kp.a2 * kshape<KIND, DIM>(kp, a, b);
    }
}

// the instantiation for a (kind, dim) pair
template <template <int, int> class Launch, typename... Args>
static void by_kind_dim(int kind, int dim, Args &&...args)
{
    auto go = [&](auto kd) {
        constexpr int K = decltype(kd)::value;
        if (dim == 1)
            Launch<K, 1>::run(args...);
        else if (dim == 2)
            Launch<K, 2>::run(args...);
        else
            Launch<K, 3>::run(args...);
    };
    switch (kind) {
    case HODLR_K_SE: go(std::integral_constant<int, HODLR_K_SE>{}); break;
    case HODLR_K_MATERN32: go(std::integral_constant<int, HODLR_K_MATERN32>{}); break;
    case HODLR_K_EXP: go(std::integral_constant<int, HODLR_K_EXP>{}); break;
    case HODLR_K_IMQ: go(std::integral_constant<int, HODLR_K_IMQ>{}); break;
    default: go(std::integral_constant<int, HODLR_K_CONST>{}); break;
    }
}

template <int K, int D>
struct PartLaunch {
    static void run(dim3 grid, hipStream_t s, int64_t n, const KParams &kp, const double *x,
                    const double *alpha, int64_t m, const double *xt, int64_t slice, double *part)
    {
        predict_part_kernel<K, D><<<grid, PR_T, 0, s>>>(n, kp, x, alpha, m, xt, slice, part);
    }
};

template <int K, int D>
struct CrossLaunch {
    static void run(unsigned blocks, hipStream_t s, int64_t n, const KParams &kp, const double *x,
                    int64_t m, const double *xt, int64_t j0, int nb, double *out)
    {
        kcross_kernel<K, D><<<blocks, 256, 0, s>>>(n, kp, x, m, xt, j0, nb, out);
    }
};

int predict_slices(int64_t n, int64_t m)
{
    const int64_t nbx = (m + PR_T - 1) / PR_T;
    const int64_t want = (2048 + nbx - 1) / nbx;   // about 2048 work-groups in all
    const int64_t most = (n + PR_T - 1) / PR_T;    // at least one tile per slice
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, most));
}

void run_predict_mean(int64_t n, const KParams &kp, const double *x, const double *alpha,
                      int64_t m, const double *xt, double *part, double *mean, hipStream_t s)
{
    const int nslice = predict_slices(n, m);
    int64_t slice = (n + nslice - 1) / nslice;
    slice = (slice + PR_T - 1) / PR_T * PR_T;
    const dim3 grid((unsigned)((m + PR_T - 1) / PR_T), (unsigned)nslice);
    {
        ProfScope ps(s, PS_PREDICT);   // the product kernel alone
        by_kind_dim<PartLaunch>(kp.kind, kp.dim, grid, s, n, kp, x, alpha, m, xt, slice, part);
    }
    const unsigned nb = (unsigned)std::min<int64_t>((m + 255) / 256, 1024);
    predict_sum_kernel<<<nb, 256, 0, s>>>(part, nslice, m, mean);
    HIP_TRY(hipGetLastError());
}

void run_kcross(int64_t n, const KParams &kp, const double *x, int64_t m, const double *xt,
                int64_t j0, int nb, double *out, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<int64_t>((n * nb + 255) / 256, 4096);
    ProfScope ps(s, PS_PREDICT);
    by_kind_dim<CrossLaunch>(kp.kind, kp.dim, blocks, s, n, kp, x, m, xt, j0, nb, out);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
