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
#include "common.h"

namespace hodlr {

constexpr int PR_T = 256;   // test points per work-group, training points per LDS tile

// part[s * m + j] = sum over slice s of the training points of k(xt_j, x_i) alpha_i
__global__ __launch_bounds__(PR_T) void predict_part_kernel(int64_t n, KParams kp,
                                                            const double *__restrict__ x,
                                                            const double *__restrict__ alpha,
                                                            int64_t m, const double *__restrict__ xt,
                                                            int64_t slice, double *__restrict__ part)
{
    __shared__ double sx[3][PR_T];
    __shared__ double sa[PR_T];
    const int tid = threadIdx.x;
    const int64_t j = blockIdx.x * (int64_t)PR_T + tid;
    double xj[3] = {0.0, 0.0, 0.0};
    if (j < m)
        for (int d = 0; d < kp.dim; ++d)
            xj[d] = xt[d * m + j];
    const int64_t i0 = blockIdx.y * slice;
    const int64_t i1 = min(n, i0 + slice);
    double acc = 0.0;
    for (int64_t c0 = i0; c0 < i1; c0 += PR_T) {
        const int64_t i = c0 + tid;
        for (int d = 0; d < kp.dim; ++d)
            sx[d][tid] = (i < i1) ? x[d * n + i] : 0.0;
        sa[tid] = (i < i1) ? alpha[i] : 0.0;
        __syncthreads();
        const int cnt = (int)min<int64_t>(PR_T, i1 - c0);
        for (int t = 0; t < cnt; ++t) {
            double r2 = 0.0;
            for (int d = 0; d < kp.dim; ++d) {
                const double q = xj[d] - sx[d][t];
                r2 += q * q;
            }
            acc += kfun_r2<double>(kp.kind, kp.a2, kp.c, r2) * sa[t];
        }
        __syncthreads();
    }
    if (j < m)
        part[blockIdx.y * m + j] = acc;
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
__global__ void kcross_kernel(int64_t n, KParams kp, const double *__restrict__ x, int64_t m,
                              const double *__restrict__ xt, int64_t j0, int nb,
                              double *__restrict__ out)
{
    const int64_t total = n * nb;
    for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t c = idx / n, i = idx - c * n;
        double r2 = 0.0;
        for (int d = 0; d < kp.dim; ++d) {
            const double q = x[d * n + i] - xt[d * m + j0 + c];
            r2 += q * q;
        }
        out[idx] = kfun_r2<double>(kp.kind, kp.a2, kp.c, r2);
    }
}

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
    ProfScope ps(s, PS_PREDICT);
    predict_part_kernel<<<grid, PR_T, 0, s>>>(n, kp, x, alpha, m, xt, slice, part);
    const unsigned nb = (unsigned)std::min<int64_t>((m + 255) / 256, 1024);
    predict_sum_kernel<<<nb, 256, 0, s>>>(part, nslice, m, mean);
    HIP_TRY(hipGetLastError());
}

void run_kcross(int64_t n, const KParams &kp, const double *x, int64_t m, const double *xt,
                int64_t j0, int nb, double *out, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<int64_t>((n * nb + 255) / 256, 4096);
    ProfScope ps(s, PS_PREDICT);
    kcross_kernel<<<blocks, 256, 0, s>>>(n, kp, x, m, xt, j0, nb, out);
    HIP_TRY(hipGetLastError());
}

}  // namespace hodlr
