// Random-walk Metropolis over log-hyperparameters, plain or with delayed
// acceptance (Christen and Fox, 2005): the surrogate network screens every
// proposal, and only the survivors pay for an exact HODLR likelihood, taken
// for all of them at once by the batched entry point.  The second-stage
// ratio corrects for the surrogate, so the chain keeps the exact posterior
// exp(l(theta)) p(theta) of the paper's outer loop (§1, Eq. (1)) as its
// stationary law whatever the surrogate's error.
//
// Walker state (device, FP64): log theta (W x 3), exact log-likelihood lp
// and surrogate value sur at log theta.  Random numbers are inputs: eps
// (W x 3 standard normals), u1 and u2 (W uniforms in (0, 1)) per step.  The
// prior is uniform on a box in log theta, so it cancels everywhere except the
// box test.  One step issues: propose, surrogate forward (delayed form),
// screen + compaction (one work-group), a read of the survivor count, the
// batched exact likelihood of the survivors, accept.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "hodlr.h"

namespace hodlr {
hodlr_status report(hodlr_status st, const std::string &msg);   // sets hodlr_last_error
}

namespace {

constexpr int MAXW = 1024;   // walkers per call (one work-group screens them all)

struct Box {
    double lo[3], hi[3];
};
struct Chol {
    double l[9];
};

__global__ void propose_kernel(int w, const double *__restrict__ th, Chol L,
                               const double *__restrict__ eps, double *__restrict__ prop)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w)
        return;
    const double e0 = eps[3 * i], e1 = eps[3 * i + 1], e2 = eps[3 * i + 2];
    prop[3 * i + 0] = th[3 * i + 0] + L.l[0] * e0 + L.l[1] * e1 + L.l[2] * e2;
    prop[3 * i + 1] = th[3 * i + 1] + L.l[3] * e0 + L.l[4] * e1 + L.l[5] * e2;
    prop[3 * i + 2] = th[3 * i + 2] + L.l[6] * e0 + L.l[7] * e1 + L.l[8] * e2;
}

// Survivors: in the prior box and (delayed form) log u1 < sur' - sur.  The
// survivors keep walker order in the compacted list; slot[i] is walker i's
// position there or -1.  params receives (a, l, sigma2) = exp(log theta').
__global__ __launch_bounds__(MAXW) void screen_kernel(
    int w, const double *__restrict__ prop, Box box, const double *__restrict__ sur,
    const double *__restrict__ sur_prop, const double *__restrict__ u1, int *__restrict__ slot,
    int *__restrict__ count, double *__restrict__ params)
{
    __shared__ int scan[MAXW];
    const int i = threadIdx.x;
    int keep = 0;
    if (i < w) {
        keep = 1;
        for (int k = 0; k < 3; ++k) {
            const double v = prop[3 * i + k];
            if (!(v >= box.lo[k] && v <= box.hi[k]))
                keep = 0;
        }
        if (keep && sur_prop) {
            const double d = sur_prop[i] - sur[i];
            keep = (log(u1[i]) < d) ? 1 : 0;   // NaN surrogate values reject
        }
    }
    scan[i] = keep;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {   // inclusive Hillis-Steele scan
        const int v = i >= off ? scan[i - off] : 0;
        __syncthreads();
        scan[i] += v;
        __syncthreads();
    }
    if (i < w) {
        const int pos = scan[i] - 1;
        slot[i] = keep ? pos : -1;
        if (keep)
            for (int k = 0; k < 3; ++k)
                params[3 * pos + k] = exp(prop[3 * i + k]);
    }
    if (i == (int)blockDim.x - 1)
        *count = scan[i];
}

// Exact stage for every walker with a slot.  Delayed form: accept if
// log u < (lp' - lp) - (sur' - sur); plain form: log u < lp' - lp.  A NaN
// exact value (failed factorization) rejects.
__global__ void accept_kernel(int w, int delayed, const int *__restrict__ slot,
                              const double *__restrict__ exact, const double *__restrict__ u,
                              const double *__restrict__ prop, const double *__restrict__ sur_prop,
                              double *__restrict__ th, double *__restrict__ lp,
                              double *__restrict__ sur, int *__restrict__ accepted,
                              double *__restrict__ chain_row)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w)
        return;
    const int j = slot[i];
    int acc = 0;
    if (j >= 0) {
        const double l1 = exact[3 * j];
        double ratio = l1 - lp[i];
        if (delayed)
            ratio -= sur_prop[i] - sur[i];
        acc = (log(u[i]) < ratio) ? 1 : 0;
        if (acc) {
            th[3 * i + 0] = prop[3 * i + 0];
            th[3 * i + 1] = prop[3 * i + 1];
            th[3 * i + 2] = prop[3 * i + 2];
            lp[i] = l1;
            if (sur_prop)
                sur[i] = sur_prop[i];
        }
    }
    if (accepted)
        accepted[i] = acc;
    if (chain_row)
        for (int k = 0; k < 3; ++k)
            chain_row[3 * i + k] = th[3 * i + k];
}

__global__ void exp_kernel(int n, const double *__restrict__ a, double *__restrict__ b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        b[i] = exp(a[i]);
}

__global__ void copy_exact_kernel(int w, const double *__restrict__ exact, double *__restrict__ lp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < w)
        lp[i] = exact[3 * i];
}

__global__ void count_kernel(int w, const int *__restrict__ accepted, const int *__restrict__ count,
                             long long *__restrict__ tallies)
{
    // tallies: [0] accepted moves, [1] stage-1 survivors (exact evaluations)
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long a = 0;
        for (int i = 0; i < w; ++i)
            a += accepted[i];
        tallies[0] += a;
        tallies[1] += *count;
    }
}

hodlr_status bad(const char *m) { return hodlr::report(HODLR_EINVAL, m); }

hodlr_status launched()
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HODLR_OK
                           : hodlr::report(HODLR_EDEVICE, std::string("launch: ") +
                                                              hipGetErrorString(e));
}

int screen_threads(int w)
{
    int t = 64;
    while (t < w)
        t <<= 1;
    return t;
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// workspace carve-up of the driver: [batch likelihood workspace | small buffers]
struct Carve {
    size_t batch, prop, params, exact, sur_prop, slot, count, acc, tallies, total;
};

Carve carve(size_t batch_bytes, int w)
{
    Carve c;
    size_t off = 0;
    c.batch = off;
    off += a256(batch_bytes);
    c.prop = off;
    off += a256(sizeof(double) * 3 * w);
    c.params = off;
    off += a256(sizeof(double) * 3 * w);
    c.exact = off;
    off += a256(sizeof(double) * 3 * w);
    c.sur_prop = off;
    off += a256(sizeof(double) * w);
    c.slot = off;
    off += a256(sizeof(int) * w);
    c.count = off;
    off += 256;
    c.acc = off;
    off += a256(sizeof(int) * w);
    c.tallies = off;
    off += 256;
    c.total = off;
    return c;
}

}  // namespace

extern "C" {

hodlr_status hodlr_mh_propose_dev(int32_t w, const double *d_theta, const double chol[9],
                                  const double *d_eps, double *d_prop, void *stream)
{
    if (w < 1 || !d_theta || !chol || !d_eps || !d_prop)
        return bad("NULL argument or no walkers");
    Chol L;
    for (int k = 0; k < 9; ++k)
        L.l[k] = chol[k];
    hipLaunchKernelGGL(propose_kernel, dim3((w + 255) / 256), dim3(256), 0, (hipStream_t)stream, w,
                       d_theta, L, d_eps, d_prop);
    return launched();
}

hodlr_status hodlr_da_screen_dev(int32_t w, const double *d_prop, const double lo[3],
                                 const double hi[3], const double *d_sur, const double *d_sur_prop,
                                 const double *d_u1, int32_t *d_slot, int32_t *d_count,
                                 double *d_params, void *stream)
{
    if (w < 1 || w > MAXW)
        return bad("walkers must be in [1, 1024]");
    if (!d_prop || !lo || !hi || !d_slot || !d_count || !d_params)
        return bad("NULL argument");
    if (d_sur_prop && (!d_sur || !d_u1))
        return bad("the delayed screen needs sur and u1");
    Box b;
    for (int k = 0; k < 3; ++k) {
        if (!(lo[k] <= hi[k]))
            return bad("prior box must have lo <= hi");
        b.lo[k] = lo[k];
        b.hi[k] = hi[k];
    }
    hipLaunchKernelGGL(screen_kernel, dim3(1), dim3(screen_threads(w)), 0, (hipStream_t)stream, w,
                       d_prop, b, d_sur, d_sur_prop, d_u1, d_slot, d_count, d_params);
    return launched();
}

hodlr_status hodlr_da_accept_dev(int32_t w, int32_t delayed, const int32_t *d_slot,
                                 const double *d_exact, const double *d_u, const double *d_prop,
                                 const double *d_sur_prop, double *d_theta, double *d_lp,
                                 double *d_sur, int32_t *d_accepted, void *stream)
{
    if (w < 1 || !d_slot || !d_exact || !d_u || !d_prop || !d_theta || !d_lp)
        return bad("NULL argument or no walkers");
    if (delayed && (!d_sur_prop || !d_sur))
        return bad("the delayed form needs sur and sur_prop");
    hipLaunchKernelGGL(accept_kernel, dim3((w + 255) / 256), dim3(256), 0, (hipStream_t)stream, w,
                       delayed ? 1 : 0, d_slot, d_exact, d_u, d_prop,
                       delayed ? d_sur_prop : nullptr, d_theta, d_lp, d_sur, d_accepted,
                       (double *)nullptr);
    return launched();
}

hodlr_status hodlr_sampler_workspace_size(hodlr_plan p, int32_t walkers, size_t *bytes)
{
    if (!p || !bytes || walkers < 1 || walkers > MAXW)
        return bad("NULL argument or walkers outside [1, 1024]");
    size_t b = 0;
    if (hodlr_status st = hodlr_plan_batch_workspace_size(p, walkers, &b))
        return st;
    *bytes = carve(b, walkers).total;
    return HODLR_OK;
}

hodlr_status gp_sample_dev(hodlr_plan p, const double *d_x, hodlr_kernel k, const double *d_y,
                           double tol, const uint16_t *d_wbf16, const hodlr_mlp_norm *norm,
                           const hodlr_sampler_cfg *cfg, double *d_theta, double *d_lp,
                           double *d_sur, const double *d_eps, const double *d_u1,
                           const double *d_u2, void *d_work, size_t work_bytes, void *stream,
                           double *d_chain, hodlr_sampler_stats *stats)
{
    if (!p || !d_x || !d_y || !cfg || !d_theta || !d_lp || !d_eps || !d_u1)
        return bad("NULL argument");
    const int w = cfg->walkers;
    const bool delayed = d_wbf16 != nullptr;
    if (w < 1 || w > MAXW || cfg->steps < 0)
        return bad("walkers outside [1, 1024] or negative steps");
    if (delayed && (!norm || !d_sur || !d_u2))
        return bad("the delayed form needs the network, its scales, sur and u2");
    size_t bb = 0;
    if (hodlr_status st = hodlr_plan_batch_workspace_size(p, w, &bb))
        return st;
    const Carve c = carve(bb, w);
    if (work_bytes < c.total)
        return bad("workspace too small (hodlr_sampler_workspace_size)");
    hipStream_t s = (hipStream_t)stream;
    char *W = (char *)d_work;
    double *prop = (double *)(W + c.prop), *params = (double *)(W + c.params);
    double *exact = (double *)(W + c.exact), *sur_prop = (double *)(W + c.sur_prop);
    int *slot = (int *)(W + c.slot), *count = (int *)(W + c.count), *acc = (int *)(W + c.acc);
    long long *tallies = (long long *)(W + c.tallies);
    if (hipMemsetAsync(tallies, 0, 2 * sizeof(long long), s) != hipSuccess)
        return launched();
    int64_t exact_evals = 0;
    const int g = (w + 255) / 256;

    if (cfg->init_state) {   // lp (and sur) at the starting points
        hipLaunchKernelGGL(exp_kernel, dim3((3 * w + 255) / 256), dim3(256), 0, s, 3 * w,
                           (const double *)d_theta, params);
        if (hodlr_status st = gp_loglik_batch_dev(p, d_x, k, params, w, d_y, 0, tol, W + c.batch,
                                                  bb, stream, exact, 0))
            return st;
        exact_evals += w;
        hipLaunchKernelGGL(copy_exact_kernel, dim3(g), dim3(256), 0, s, w, (const double *)exact,
                           d_lp);
        if (delayed)
            if (hodlr_status st = hodlr_mlp_forward_dev(d_wbf16, norm, d_theta, w, d_sur, stream))
                return st;
    }
    int host_count = 0;
    for (int t = 0; t < cfg->steps; ++t) {
        const size_t o3 = (size_t)t * w * 3, o1 = (size_t)t * w;
        if (hodlr_status st = hodlr_mh_propose_dev(w, d_theta, cfg->chol, d_eps + o3, prop, stream))
            return st;
        if (delayed)
            if (hodlr_status st = hodlr_mlp_forward_dev(d_wbf16, norm, prop, w, sur_prop, stream))
                return st;
        if (hodlr_status st = hodlr_da_screen_dev(w, prop, cfg->lo, cfg->hi, d_sur,
                                                  delayed ? sur_prop : nullptr, d_u1 + o1, slot,
                                                  count, params, stream))
            return st;
        if (hipMemcpyAsync(&host_count, count, sizeof(int), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return hodlr::report(HODLR_EDEVICE, "reading the survivor count failed");
        if (host_count > 0) {
            if (hodlr_status st = gp_loglik_batch_dev(p, d_x, k, params, host_count, d_y, 0, tol,
                                                      W + c.batch, bb, stream, exact, 0))
                return st;
            exact_evals += host_count;
        }
        hipLaunchKernelGGL(accept_kernel, dim3(g), dim3(256), 0, s, w, delayed ? 1 : 0,
                           (const int *)slot, (const double *)exact,
                           delayed ? d_u2 + o1 : d_u1 + o1, (const double *)prop,
                           delayed ? (const double *)sur_prop : nullptr, d_theta, d_lp, d_sur, acc,
                           d_chain ? d_chain + o3 : nullptr);
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(64), 0, s, w, (const int *)acc,
                           (const int *)count, tallies);
        if (hodlr_status st = launched())
            return st;
    }
    if (stats) {
        long long h[2];
        if (hipMemcpyAsync(h, tallies, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return hodlr::report(HODLR_EDEVICE, "reading the sampler tallies failed");
        stats->accepted = h[0];
        stats->survivors = h[1];
        stats->exact_evals = exact_evals;
        stats->proposals = (int64_t)cfg->steps * w;
    }
    return HODLR_OK;
}

}  // extern "C"
