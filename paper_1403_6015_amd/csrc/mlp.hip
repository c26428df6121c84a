// Surrogate network of the log-likelihood over log-hyperparameters:
// 3 -> 128 -> 128 -> 1 with tanh hidden units.  Weights are held in BF16 for
// the products (an FP32 master copy is what the optimizer updates); every
// product accumulates in FP32.  The two 128-wide contractions per tile of 32
// samples (forward h1 -> z2, backward z2 -> h1 and the weight gradient
// z2^T h1) run on the matrix cores as 16x16x16 BF16 MFMA tiles with operands
// staged in LDS; the 3-wide first layer and the 128 -> 1 head are plain FP32.
//
// Training is deterministic: each work-group writes its tile's gradient to
// its own slot of the workspace, and the optimizer kernel sums the slots in
// a fixed order before the Adam update (Kingma and Ba, Algorithm 1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>
#include <mutex>

#include <string>

#include "hodlr.h"

namespace hodlr {
hodlr_status report(hodlr_status st, const std::string &msg);   // sets hodlr_last_error
}

namespace {

constexpr int NIN = 3, NH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH,
              NPARAM = OFF_B3 + 1;
static_assert(NPARAM == HODLR_MLP_NPARAM, "parameter count");

constexpr int TS = 32;           // samples per work-group
constexpr int THREADS = 256;     // 4 waves
constexpr int SW = NH + 4;       // bf16 row stride of [.][128] tiles (66 words: conflict-free b64)
constexpr int ST = TS + 4;       // bf16 row stride of [128][32] tiles (18 words)
constexpr int SF = NH + 1;       // fp32 row stride

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ v4s ld4(const uint16_t *p)   // 8-byte LDS read
{
    return *reinterpret_cast<const v4s *>(p);
}

struct Norm {
    float mu_in[3], sd_in[3], mu_out, sd_out;
};

struct Smem {
    uint16_t w2[NH * SW];      // W2[o][i]              (forward B operand)
    uint16_t w2t[NH * SW];     // W2^T[i][o]            (backward B operand)
    uint16_t h1b[TS * SW];     // h1[s][i] bf16         (forward A operand)
    uint16_t h1t[NH * ST];     // h1^T[i][s] bf16       (weight-gradient B operand)
    uint16_t g2b[TS * SW];     // dz2[s][o] bf16        (backward A operand)
    uint16_t g2t[NH * ST];     // dz2^T[o][s] bf16      (weight-gradient A operand)
    float h1[TS * SF];         // h1 fp32, later dz1 in place
    float h2[TS * SF];         // h2 fp32
    float u[TS][4];
    float o[TS];
    float go[TS];
};

// Forward over one tile of 32 samples; with TRAIN the backward pass follows
// and the tile's gradient and squared-residual sum go to part (NPARAM + 1
// floats).  Without TRAIN, out[s] = mu_out + sd_out * o_s.
template <bool TRAIN>
__global__ __launch_bounds__(THREADS) void mlp_tile_kernel(
    const uint16_t *__restrict__ wb, Norm nm, const double *__restrict__ lt,
    const int32_t *__restrict__ idx, int B, const double *__restrict__ target,
    double *__restrict__ out, float *__restrict__ part)
{
    extern __shared__ __align__(16) char smem_raw[];
    Smem &S = *reinterpret_cast<Smem *>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s0 = blockIdx.x * TS;

    // stage W2 (and its transpose for the backward pass)
    for (int e = tid; e < NH * NH; e += THREADS) {
        const int o = e / NH, i = e % NH;
        const uint16_t w = wb[OFF_W2 + e];
        S.w2[o * SW + i] = w;
        if (TRAIN)
            S.w2t[i * SW + o] = w;
    }
    if (tid < TS) {
        const int s = s0 + tid;
        const size_t row = s < B ? (size_t)(idx ? idx[s] : s) : 0;
        for (int k = 0; k < NIN; ++k)
            S.u[tid][k] = s < B ? ((float)lt[row * NIN + k] - nm.mu_in[k]) / nm.sd_in[k] : 0.f;
    }
    __syncthreads();

    // layer 1: h1 = tanh(W1 u + b1), FP32
    for (int e = tid; e < TS * NH; e += THREADS) {
        const int s = e / NH, i = e % NH;
        float z = from_bf16(wb[OFF_B1 + i]);
        for (int k = 0; k < NIN; ++k)
            z = fmaf(from_bf16(wb[OFF_W1 + i * NIN + k]), S.u[s][k], z);
        const float h = tanhf(z);
        S.h1[s * SF + i] = h;
        const uint16_t hb = to_bf16(h);
        S.h1b[s * SW + i] = hb;
        if (TRAIN)
            S.h1t[i * ST + s] = hb;
    }
    __syncthreads();

    // layer 2 on MFMA: z2[s][o] = sum_i h1[s][i] W2[o][i]; 2 x 8 tiles, 4 per wave
    const int r16 = lane & 15, q4 = (lane >> 4) * 4;
    for (int t = wave; t < (TS / 16) * (NH / 16); t += 4) {
        const int ts = (t / (NH / 16)) * 16, to = (t % (NH / 16)) * 16;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < NH; k0 += 16) {
            const v4s a = ld4(&S.h1b[(ts + r16) * SW + k0 + q4]);
            const v4s b = ld4(&S.w2[(to + r16) * SW + k0 + q4]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        const int o = to + r16;
        const float bo = from_bf16(wb[OFF_B2 + o]);
        for (int v = 0; v < 4; ++v)
            S.h2[(ts + q4 + v) * SF + o] = tanhf(acc[v] + bo);
    }
    __syncthreads();

    // head: o_s = W3 . h2_s + b3 (8 lanes per sample, 16 units each)
    {
        const int s = tid >> 3, part8 = tid & 7;
        float a = 0.f;
        for (int j = 0; j < 16; ++j) {
            const int o = part8 * 16 + j;
            a = fmaf(from_bf16(wb[OFF_W3 + o]), S.h2[s * SF + o], a);
        }
        a += __shfl_xor(a, 1);
        a += __shfl_xor(a, 2);
        a += __shfl_xor(a, 4);
        if (part8 == 0) {
            a += from_bf16(wb[OFF_B3]);
            S.o[s] = a;
            if (!TRAIN && s0 + s < B)
                out[s0 + s] = (double)nm.mu_out + (double)nm.sd_out * (double)a;
        }
    }
    if (!TRAIN)
        return;
    __syncthreads();

    float *P = part + (size_t)blockIdx.x * (NPARAM + 1);
    if (tid < TS) {
        const int s = s0 + tid;
        float g = 0.f, r2 = 0.f;
        if (s < B) {
            const float t = (float)target[idx ? idx[s] : s];
            const float r = S.o[tid] - (t - nm.mu_out) / nm.sd_out;
            g = 2.f * r / (float)B;
            r2 = r * r;
        }
        S.go[tid] = g;
        // squared residuals of the tile (lanes 0..31 of wave 0)
        for (int m = 16; m >= 1; m >>= 1)
            r2 += __shfl_xor(r2, m);
        if (tid == 0)
            P[NPARAM] = r2;
    }
    __syncthreads();

    // head gradients and dz2 = g_o W3 (1 - h2^2)
    if (tid < NH) {
        const int o = tid;
        float gw = 0.f, gb = 0.f;
        const float w3 = from_bf16(wb[OFF_W3 + o]);
        for (int s = 0; s < TS; ++s) {
            const float h = S.h2[s * SF + o];
            gw = fmaf(S.go[s], h, gw);
            const float d = S.go[s] * w3 * (1.f - h * h);
            gb += d;
            const uint16_t db = to_bf16(d);
            S.g2b[s * SW + o] = db;
            S.g2t[o * ST + s] = db;
        }
        P[OFF_W3 + o] = gw;
        P[OFF_B2 + o] = gb;
    }
    if (tid == NH) {
        float g = 0.f;
        for (int s = 0; s < TS; ++s)
            g += S.go[s];
        P[OFF_B3] = g;
    }
    __syncthreads();

    // weight gradient on MFMA: gW2[o][i] = sum_s dz2[s][o] h1[s][i]; 8 x 8 tiles
    for (int t = wave; t < (NH / 16) * (NH / 16); t += 4) {
        const int to = (t / (NH / 16)) * 16, ti = (t % (NH / 16)) * 16;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < TS; k0 += 16) {
            const v4s a = ld4(&S.g2t[(to + r16) * ST + k0 + q4]);
            const v4s b = ld4(&S.h1t[(ti + r16) * ST + k0 + q4]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int v = 0; v < 4; ++v)
            P[OFF_W2 + (to + q4 + v) * NH + ti + r16] = acc[v];
    }
    // input-side gradient on MFMA: dh1[s][i] = sum_o dz2[s][o] W2[o][i]; then dz1 in place
    for (int t = wave; t < (TS / 16) * (NH / 16); t += 4) {
        const int ts = (t / (NH / 16)) * 16, ti = (t % (NH / 16)) * 16;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < NH; k0 += 16) {
            const v4s a = ld4(&S.g2b[(ts + r16) * SW + k0 + q4]);
            const v4s b = ld4(&S.w2t[(ti + r16) * SW + k0 + q4]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int v = 0; v < 4; ++v) {
            float *h = &S.h1[(ts + q4 + v) * SF + ti + r16];
            *h = acc[v] * (1.f - *h * *h);
        }
    }
    __syncthreads();

    // first-layer gradients: gW1[i][k] = sum_s dz1[s][i] u[s][k], gb1[i] = sum_s dz1[s][i]
    if (tid < NH) {
        const int i = tid;
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, gb = 0.f;
        for (int s = 0; s < TS; ++s) {
            const float d = S.h1[s * SF + i];
            g0 = fmaf(d, S.u[s][0], g0);
            g1 = fmaf(d, S.u[s][1], g1);
            g2 = fmaf(d, S.u[s][2], g2);
            gb += d;
        }
        P[OFF_W1 + i * NIN + 0] = g0;
        P[OFF_W1 + i * NIN + 1] = g1;
        P[OFF_W1 + i * NIN + 2] = g2;
        P[OFF_B1 + i] = gb;
    }
}

// Sum the per-tile gradients in tile order; optionally export the gradient,
// then (if adam) update master, moments and the BF16 copy.  The loss (mean
// squared standardized residual) is summed by the first thread.
__global__ __launch_bounds__(256) void mlp_update_kernel(const float *__restrict__ part, int ntile,
                                                        int B, float *__restrict__ master,
                                                        uint16_t *__restrict__ wb, float *m,
                                                        float *v, int adam, int t, float lr,
                                                        float *grad_out, float *loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        float l = 0.f;
        for (int w = 0; w < ntile; ++w)
            l += part[(size_t)w * (NPARAM + 1) + NPARAM];
        *loss_out = l / (float)B;
    }
    if (p >= NPARAM)
        return;
    float g = 0.f;
    for (int w = 0; w < ntile; ++w)
        g += part[(size_t)w * (NPARAM + 1) + p];
    if (grad_out)
        grad_out[p] = g;
    if (!adam)
        return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)t));
    const float vh = vv / (1.f - powf(b2, (float)t));
    const float w = master[p] - lr * mh / (sqrtf(vh) + eps);
    master[p] = w;
    wb[p] = to_bf16(w);
}

__global__ void mlp_cast_kernel(const float *__restrict__ master, uint16_t *__restrict__ wb)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM)
        wb[p] = to_bf16(master[p]);
}

hodlr_status bad(const char *m) { return hodlr::report(HODLR_EINVAL, m); }

bool norm_ok(const hodlr_mlp_norm *n)
{
    if (!n)
        return false;
    for (int k = 0; k < 3; ++k)
        if (!(n->sd_in[k] > 0.f) || !std::isfinite(n->mu_in[k]) || !std::isfinite(n->sd_in[k]))
            return false;
    return n->sd_out > 0.f && std::isfinite(n->sd_out) && std::isfinite(n->mu_out);
}

Norm to_norm(const hodlr_mlp_norm *n)
{
    Norm r;
    for (int k = 0; k < 3; ++k) {
        r.mu_in[k] = n->mu_in[k];
        r.sd_in[k] = n->sd_in[k];
    }
    r.mu_out = n->mu_out;
    r.sd_out = n->sd_out;
    return r;
}

int ntiles(int B) { return (B + TS - 1) / TS; }

hodlr_status launch_status()
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HODLR_OK
                           : hodlr::report(HODLR_EDEVICE, std::string("launch: ") +
                                                              hipGetErrorString(e));
}

bool g_attr_done = false;

hodlr_status set_attr()
{
    if (g_attr_done)
        return HODLR_OK;
    if (hipFuncSetAttribute((const void *)mlp_tile_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(Smem)) != hipSuccess ||
        hipFuncSetAttribute((const void *)mlp_tile_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(Smem)) != hipSuccess)
        return hodlr::report(HODLR_EDEVICE, "cannot raise the LDS limit of the network kernels");
    g_attr_done = true;
    return HODLR_OK;
}

hodlr_status grad_pass(const uint16_t *wb, const hodlr_mlp_norm *norm, const double *lt,
                       const int32_t *idx, const double *target, int B, void *work,
                       size_t work_bytes, hipStream_t s)
{
    if (!wb || !lt || !target || B < 1 || !work)
        return bad("NULL argument or empty batch");
    if (!norm_ok(norm))
        return bad("normalization scales must be positive and finite");
    size_t need = 0;
    hodlr_mlp_workspace_size(B, &need);
    if (work_bytes < need)
        return bad("workspace too small");
    if (hodlr_status st = set_attr())
        return st;
    hipLaunchKernelGGL(mlp_tile_kernel<true>, dim3(ntiles(B)), dim3(THREADS), sizeof(Smem), s,
                       wb, to_norm(norm), lt, idx, B, target, (double *)nullptr, (float *)work);
    return launch_status();
}

// ----------------------------------------------- allocation-free train step
// Per-tile gradient slots for callers that cannot allocate: a fixed array in
// device memory, one copy per GPU for the life of the process.  In host code
// the array's name only stands for it; kernels receive the device address
// that hipGetSymbolAddress returns, taken once per device (with that device
// current) on the entry point's first call there.
constexpr int NOALLOC_MAX_BATCH = HODLR_MLP_NOALLOC_MAX_BATCH;
constexpr size_t NOALLOC_FLOATS = (size_t)((NOALLOC_MAX_BATCH + TS - 1) / TS) * (NPARAM + 1);
__device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

hodlr_status scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return hodlr::report(HODLR_EDEVICE, "no current device for the network scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hodlr::report(HODLR_EDEVICE, std::string("address of the network scratch: ") +
                                                    hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HODLR_OK;
}

}  // namespace

extern "C" {

hodlr_status hodlr_mlp_workspace_size(int32_t batch, size_t *bytes)
{
    if (batch < 1 || !bytes)
        return bad("batch must be >= 1");
    *bytes = sizeof(float) * (size_t)ntiles(batch) * (NPARAM + 1);
    return HODLR_OK;
}

hodlr_status hodlr_mlp_cast_dev(const float *d_master, uint16_t *d_wbf16, void *stream)
{
    if (!d_master || !d_wbf16)
        return bad("NULL argument");
    hipLaunchKernelGGL(mlp_cast_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, d_master, d_wbf16);
    return launch_status();
}

hodlr_status hodlr_mlp_forward_dev(const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                                   const double *d_logtheta, int32_t batch, double *d_out,
                                   void *stream)
{
    if (!d_wbf16 || !d_logtheta || !d_out || batch < 1)
        return bad("NULL argument or empty batch");
    if (!norm_ok(norm))
        return bad("normalization scales must be positive and finite");
    if (hodlr_status st = set_attr())
        return st;
    hipLaunchKernelGGL(mlp_tile_kernel<false>, dim3(ntiles(batch)), dim3(THREADS), sizeof(Smem),
                       (hipStream_t)stream, d_wbf16, to_norm(norm), d_logtheta,
                       (const int32_t *)nullptr, (int)batch, (const double *)nullptr, d_out,
                       (float *)nullptr);
    return launch_status();
}

hodlr_status hodlr_mlp_grad_dev(const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                                const double *d_logtheta, const double *d_target, int32_t batch,
                                void *d_work, size_t work_bytes, float *d_grad, float *d_loss,
                                void *stream)
{
    if (!d_grad)
        return bad("NULL gradient");
    hipStream_t s = (hipStream_t)stream;
    hodlr_status st =
        grad_pass(d_wbf16, norm, d_logtheta, nullptr, d_target, batch, d_work, work_bytes, s);
    if (st)
        return st;
    hipLaunchKernelGGL(mlp_update_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s,
                       (const float *)d_work, ntiles(batch), (int)batch, (float *)nullptr,
                       (uint16_t *)nullptr, (float *)nullptr, (float *)nullptr, 0, 0, 0.f, d_grad,
                       d_loss);
    return launch_status();
}

hodlr_status hodlr_mlp_train_step_dev(float *d_master, uint16_t *d_wbf16, float *d_m, float *d_v,
                                      int32_t step, float lr, const hodlr_mlp_norm *norm,
                                      const double *d_logtheta, const double *d_target,
                                      const int32_t *d_index, int32_t batch, void *d_work,
                                      size_t work_bytes, float *d_loss, void *stream)
{
    if (!d_master || !d_m || !d_v || step < 1 || !(lr > 0.f))
        return bad("NULL state, step < 1 or lr <= 0");
    hipStream_t s = (hipStream_t)stream;
    hodlr_status st =
        grad_pass(d_wbf16, norm, d_logtheta, d_index, d_target, batch, d_work, work_bytes, s);
    if (st)
        return st;
    hipLaunchKernelGGL(mlp_update_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, s,
                       (const float *)d_work, ntiles(batch), (int)batch, d_master, d_wbf16, d_m,
                       d_v, 1, (int)step, lr, (float *)nullptr, d_loss);
    return launch_status();
}

hodlr_status hodlr_mlp_train_step_noalloc_dev(float *d_master, uint16_t *d_wbf16, float *d_m,
                                              float *d_v, int32_t step, float lr,
                                              const hodlr_mlp_norm *norm,
                                              const double *d_logtheta, const double *d_target,
                                              const int32_t *d_index, int32_t batch,
                                              float *d_loss, void *stream)
{
    if (batch < 1 || batch > NOALLOC_MAX_BATCH)
        return bad("batch must be in [1, HODLR_MLP_NOALLOC_MAX_BATCH]");
    void *work = nullptr;
    if (hodlr_status st = scratch_address(&work))
        return st;
    // every slot the update kernel reads is written by this call's tile kernel
    return hodlr_mlp_train_step_dev(d_master, d_wbf16, d_m, d_v, step, lr, norm, d_logtheta,
                                    d_target, d_index, batch, work,
                                    sizeof(float) * NOALLOC_FLOATS, d_loss, stream);
}

hodlr_status hodlr_mlp_fit_dev(float *d_master, uint16_t *d_wbf16, float *d_m, float *d_v,
                               int32_t step0, float lr, const hodlr_mlp_norm *norm,
                               const double *d_logtheta, const double *d_target, int32_t n,
                               const int32_t *d_perm, int32_t epochs, int32_t batch, void *d_work,
                               size_t work_bytes, float *d_loss_hist, void *stream)
{
    if (n < 1 || epochs < 1 || batch < 1 || !d_perm || step0 < 1)
        return bad("bad fit sizes");
    const int per_epoch = (n + batch - 1) / batch;
    int step = step0;
    for (int e = 0; e < epochs; ++e)
        for (int b = 0; b < per_epoch; ++b, ++step) {
            const int b0 = b * batch, nb = std::min(batch, n - b0);
            hodlr_status st = hodlr_mlp_train_step_dev(
                d_master, d_wbf16, d_m, d_v, step, lr, norm, d_logtheta, d_target,
                d_perm + (size_t)e * n + b0, nb, d_work, work_bytes,
                d_loss_hist ? d_loss_hist + (size_t)e * per_epoch + b : nullptr, stream);
            if (st)
                return st;
        }
    return HODLR_OK;
}

}  // extern "C"
