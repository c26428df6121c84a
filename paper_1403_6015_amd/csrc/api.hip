// C ABI of libhodlrgp: argument checks, ordering, device memory for the
// host-pointer entry points, and the order of the device stages.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>

#include "plan_handle.h"

namespace hodlr {
void run_leaf_solve(Pipeline &P, void *z);
void run_levels_apply(Pipeline &P);
void prime_level_attributes();
}  // namespace hodlr

using namespace hodlr;

namespace {

thread_local std::string g_err;

hodlr_status fail(hodlr_status st, const std::string &m)
{
    g_err = m;
    return st;
}

template <typename F>
hodlr_status guarded(F &&f)
{
    try {
        return f();
    } catch (const Error &e) {
        return fail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(HODLR_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(HODLR_EDEVICE, "unexpected exception");
    }
}

hodlr_opts default_opts()
{
    hodlr_opts o;
    o.max_rank = 64;
    o.precision = HODLR_FP64;
    o.refine_tol = 1e-10;
    o.max_refine = 8;
    o.presorted = 0;
    o.noise = nullptr;
    o.refine = 0;
    o.mixed_unchecked = 0;
    o.compressor = HODLR_COMPRESS_ACA;
    o.speculate = 0;
    o.level_form = 0;
    return o;
}

// per-point variances: finite and >= 0
void check_noise(const double *noise, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!(noise[i] >= 0.0) || !std::isfinite(noise[i]))
            throw Error{HODLR_EINVAL, "noise variances must be >= 0 and finite"};
}

// entry points that take no per-point noise
void no_noise(const hodlr_opts &o)
{
    if (o.noise)
        throw Error{HODLR_EINVAL, "per-point noise is taken by hodlr_build and gp_loglik only"};
}

void check_sizes(int64_t n, int32_t dim, int32_t leaf)
{
    if (n < 1)
        throw Error{HODLR_EINVAL, "n must be >= 1"};
    if (dim < 1 || dim > 3)
        throw Error{HODLR_EINVAL, "dim must be 1, 2 or 3"};
    if (leaf < 1)
        throw Error{HODLR_EINVAL, "leaf must be >= 1"};
}

void check_opts(const hodlr_opts &o)
{
    if (o.max_rank < 0 || o.max_rank > RMAX_ABS)
        throw Error{HODLR_EINVAL, "max_rank must be in [0, " + std::to_string(RMAX_ABS) + "]"};
    if (o.precision != HODLR_FP64 && o.precision != HODLR_MIXED)
        throw Error{HODLR_EINVAL, "unknown precision"};
    if (o.max_refine < 0)
        throw Error{HODLR_EINVAL, "max_refine must be >= 0"};
    if (!(o.refine_tol > 0.0) || !std::isfinite(o.refine_tol))
        throw Error{HODLR_EINVAL, "refine_tol must be positive"};
    if (o.refine != 0 && o.refine != 1)
        throw Error{HODLR_EINVAL, "refine must be 0 or 1"};
    if (o.mixed_unchecked != 0 && o.mixed_unchecked != 1)
        throw Error{HODLR_EINVAL, "mixed_unchecked must be 0 or 1"};
    if (o.compressor != HODLR_COMPRESS_ACA && o.compressor != HODLR_COMPRESS_SKETCH)
        throw Error{HODLR_EINVAL, "unknown compressor"};
    if (o.speculate != 0 && o.speculate != 1)
        throw Error{HODLR_EINVAL, "speculate must be 0 or 1"};
    if (o.level_form != 0 && o.level_form != 1)
        throw Error{HODLR_EINVAL, "level_form must be 0 or 1"};
    if (o.compressor == HODLR_COMPRESS_SKETCH && o.max_rank > SK_CAP_MAX)
        throw Error{HODLR_EINVAL, "the sketch compressor needs max_rank <= " +
                                      std::to_string(SK_CAP_MAX)};
}

void check_finite(const double *v, int64_t m, const char *what)
{
    if (!v)
        throw Error{HODLR_EINVAL, std::string(what) + " is NULL"};
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(v[i]))
            throw Error{HODLR_EINVAL, std::string(what) + " has a NaN or Inf entry"};
}

// RAII device buffer
struct DevBuf {
    void *p = nullptr;
    explicit DevBuf(size_t bytes)
    {
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
            p = nullptr;
            throw Error{HODLR_ENOMEM, "device allocation of " + std::to_string(bytes) +
                                          " bytes failed"};
        }
    }
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            if (p)
                (void)hipFree(p);
            p = o.p;
            o.p = nullptr;
        }
        return *this;
    }
    void *release()
    {
        void *q = p;
        p = nullptr;
        return q;
    }
};

// the per-point variances in tree order into d (n doubles; nothing without)
void upload_noise(DevBuf &d, const double *noise, const std::vector<int64_t> &perm)
{
    if (!noise)
        return;
    const int64_t n = (int64_t)perm.size();
    std::vector<double> ns(n);
    for (int64_t i = 0; i < n; ++i)
        ns[i] = noise[perm[i]];
    HIP_TRY(hipMemcpy(d.p, ns.data(), sizeof(double) * n, hipMemcpyHostToDevice));
}

// ordered, coordinate-major copy of caller points
std::vector<double> ordered_soa(const double *x, int64_t n, int dim, const std::vector<int64_t> &perm)
{
    std::vector<double> xs((size_t)n * dim);
    for (int d = 0; d < dim; ++d)
        for (int64_t k = 0; k < n; ++k)
            xs[(size_t)d * n + k] = x[perm[k] * dim + d];
    return xs;
}

}  // namespace

namespace hodlr {
void check_params(int k, const double theta[2], double sigma2, double tol)
{
    if (k < HODLR_K_SE || k > HODLR_K_IMQ)
        throw Error{HODLR_EINVAL, "unknown kernel"};
    if (!theta)
        throw Error{HODLR_EINVAL, "theta is NULL"};
    if (!(theta[0] > 0.0) || !std::isfinite(theta[0]) || !(theta[1] > 0.0) ||
        !std::isfinite(theta[1]))
        throw Error{HODLR_EINVAL, "theta = {a, l} must be positive and finite"};
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2))
        throw Error{HODLR_EINVAL, "sigma2 must be >= 0 and finite"};
    if (!(tol > 0.0) || !std::isfinite(tol))
        throw Error{HODLR_EINVAL, "tol must be positive and finite"};
}

void make_columns(Pipeline &P)
{
    const Plan &p = *P.plan;
    P.cols.assign(1, 0);
    P.cnt.assign(p.L + 1, 1);
    for (int j = 1; j <= p.L; ++j) {
        for (int c = 0; c < P.rmax[j]; ++c)
            P.cols.push_back((int)(p.cofa[j] + c));
        P.cnt[j] = (int)P.cols.size();
    }
    if (P.spec_run)
        return;   // the speculation check wrote the same list on the device
    int *hc = pinned_ints(P.cols.size(), 1);
    std::memcpy(hc, P.cols.data(), sizeof(int) * P.cols.size());
    HIP_TRY(hipMemcpyAsync(wsp<int>(P, P.lay.cols), hc, sizeof(int) * P.cols.size(),
                           hipMemcpyHostToDevice, P.stream));
}

// The status word through this thread's pinned slot 3 (ints 8 on; the mixed
// check's values take ints 0-3), the stream polled to completion: a plain
// synchronization wakes the host tens of microseconds later.
int read_status(Pipeline &P)
{
    int *hs = pinned_ints(16, 3) + 8;
    HIP_TRY(hipMemcpyAsync(hs, wsp<int>(P, P.lay.status), sizeof(int), hipMemcpyDeviceToHost,
                           P.stream));
    host_wait(P.stream);
    prof_collect();
    return *hs;
}

void raise_status(int st)
{
    if (st & DS_NOTSPD_LEAF)
        throw Error{HODLR_ENOTSPD, "a leaf block is not positive definite"};
    if (st & DS_NOTSPD_NODE)
        throw Error{HODLR_ENOTSPD, "a coupling determinant is not positive"};
}

// The mixed form's log-det bar: relative error at most 1e-8 of max(|log det|, 1).
// Its FP32 storage of the applied bases W~ perturbs each coupling matrix
// I - QP by about the FP32 unit roundoff u, which its inverse amplifies by at
// most 1 / det M_tau; the finish kernel writes the estimate
// 4 u sqrt(sum_tau det M_tau^-2) of the log-det error (independent roundings
// at the nodes add as a root sum of squares; on seeded problems of the batched
// hyperparameter box the error stayed below a third of it).  A likelihood
// whose estimate exceeds the bar is redone with FP64 panels.
constexpr double MIXED_LOGDET_BAR = 1e-8;

bool mixed_estimate_exceeds(double estimate, double logdet)
{
    return !(estimate <= MIXED_LOGDET_BAR * std::max(std::fabs(logdet), 1.0));
}

// The end of a likelihood call: the status word, and when asked a speculative
// call's rank statistics and ranks and a mixed call's log det and error
// estimate, written by one kernel straight into this thread's pinned buffers
// (device addresses of the same memory) instead of one copy each.
struct EndArgs {
    const int *status = nullptr, *stats = nullptr, *ranks = nullptr;
    int64_t nint = 0;
    const double *ld = nullptr, *est = nullptr;
    int *h_status = nullptr, *h_stats = nullptr, *h_ranks = nullptr;
    double *h_vals = nullptr;
};

__global__ __launch_bounds__(256) void end_read_kernel(EndArgs E)
{
    for (int64_t i = threadIdx.x; i < E.nint; i += 256)
        E.h_ranks[i] = E.ranks[i];
    if (E.stats)
        for (int i = threadIdx.x; i < 64; i += 256)
            E.h_stats[i] = E.stats[i];
    if (threadIdx.x == 0) {
        *E.h_status = *E.status;
        if (E.ld) {
            E.h_vals[0] = *E.ld;
            E.h_vals[1] = *E.est;
        }
    }
}

template <typename T>
T *device_alias(T *host)
{
    void *d = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&d, (void *)host, 0));
    return (T *)d;
}

// Enqueues on P's stream the copies of a mixed likelihood's log det (d_out[1])
// and error estimate into this thread's pinned slot 3: {log det, estimate},
// valid after the stream's next synchronization (the read of the status).
double *queue_mixed_check(const Pipeline &P, const double *d_out)
{
    double *hv = (double *)pinned_ints(4, 3);
    HIP_TRY(hipMemcpyAsync(hv, d_out + 1, sizeof(double), hipMemcpyDeviceToHost, P.stream));
    HIP_TRY(hipMemcpyAsync(hv + 1, wsp<double>(P, P.lay.misc + MISC_BOUND), sizeof(double),
                           hipMemcpyDeviceToHost, P.stream));
    return hv;
}

bool mixed_estimate_missed(const Pipeline &P, double logdet, int item)
{
    double est = 0.0;
    const char *src = P.ws + (size_t)P.batch.istride * item + P.lay.misc + MISC_BOUND;
    HIP_TRY(hipMemcpy(&est, src, sizeof(double), hipMemcpyDeviceToHost));
    return mixed_estimate_exceeds(est, logdet);
}

// compression, leaves, levels, finish: everything for one likelihood
void factor_pipeline(Pipeline &P, const double *d_y, double *d_out)
{
    run_aca(P);   // its first launch also zeroes the status words
    make_columns(P);
    if (!d_y)
        HIP_TRY(hipMemsetAsync(P.ws + P.lay.Xt, 0, P.plan->panel_bytes() * P.plan->n, P.stream));
    run_leaf_factor(P, d_y);
    run_levels_factor(P);
    run_finish(P, d_y, d_out);
}

}  // namespace hodlr

namespace {
__global__ void zero_status_kernel(int *status0, BatchArgs B)
{
    if (threadIdx.x == 0)
        *ioff(status0, B, blockIdx.x) = 0;
}
size_t item_stride(const Layout &lay) { return (lay.total + 255) & ~(size_t)255; }
}  // namespace

struct hodlr_factor_s {
    Plan plan;
    Layout lay;
    hodlr_opts opts;
    void *ws = nullptr;
    double *dx = nullptr;
    double *dnoise = nullptr;   // per-point variances in tree order (or none)
    std::vector<int64_t> perm;
    KParams kp;
    double tol = 0;
    double logdet = 0;
    std::vector<int> rmax, cols, cnt, ranks;
    int capped = 0;
    int device = 0;
    int fp64_fallback = 0;         // a mixed factor rebuilt with FP64 panels
    int refine_steps = 0;          // largest refinement count of the last solve
    double refine_residual = 0.0;  // largest final relative residual of the last solve
    ~hodlr_factor_s()
    {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        if (ws)
            (void)hipFree(ws);
        if (dx)
            (void)hipFree(dx);
        if (dnoise)
            (void)hipFree(dnoise);
        plan_release(plan);
        (void)hipSetDevice(cur);
    }
};

namespace {

// Pipeline view of a stored factor
Pipeline factor_pipeline_of(hodlr_factor_s *f)
{
    Pipeline P;
    P.plan = &f->plan;
    P.lay = f->lay;
    P.ws = (char *)f->ws;
    P.stream = nullptr;
    P.x = f->dx;
    P.kp = f->kp;
    P.tol = f->tol;
    P.rmax = f->rmax;
    P.cols = f->cols;
    P.cnt = f->cnt;
    P.ranks = f->ranks;
    return P;
}

struct Refined {
    int steps;
    double residual;   // ||y - C x|| / ||y||; -1 when not measured (FP64 factor)
    bool converged;
};

// d_x = C^{-1} d_y in tree order (device FP64 vectors).  An FP64 factor
// applies its inverse once unless refinement was asked for.  A refined solve
// (always for a mixed factor) iterates against the exact FP64 product by
// conjugate gradients preconditioned with the factor (flexible form, since
// the FP32 factor is only nearly symmetric): with an accurate
// factor this converges like x_{k+1} = x_k + H^{-1}(y - C x_k), and it still
// converges when rank caps make the factor too rough for that stationary
// iteration.  Stops at ||y - C x|| <= refine_tol ||y|| (true residual) or
// after 1 + max_refine products.
struct Work {
    double *r, *q, *z, *p, *part;
};

Refined solve_tree(hodlr_factor_s *f, Pipeline &P, const double *d_y, double *d_x, const Work &w)
{
    const int64_t n = f->plan.n;
    const bool f32 = f->plan.f32();
    void *zp = P.ws + P.lay.Xt;   // column 0 of the panel carries the vector
    hipStream_t s = P.stream;
    if (!f->plan.refine) {
        HIP_TRY(hipMemcpyAsync(zp, d_y, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        run_leaf_solve(P, zp);
        run_levels_apply(P);
        HIP_TRY(hipMemcpyAsync(d_x, zp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        return {0, -1.0, true};
    }
    // z = H^{-1} v, the vector scaled to unit norm through the FP32 panel
    auto precond = [&](const double *v, double vnorm, double *out) {
        run_cast_scaled(v, 1.0 / vnorm, zp, f32, n, s);
        run_leaf_solve(P, zp);
        run_levels_apply(P);
        run_widen(zp, f32, out, n, s, vnorm);
    };
    const double ynorm = std::sqrt(run_sumsq(d_y, n, w.part, s));
    HIP_TRY(hipMemsetAsync(d_x, 0, sizeof(double) * n, s));
    if (ynorm == 0.0)
        return {0, 0.0, true};
    const double tol = f->plan.refine_tol;
    const int maxit = 1 + f->plan.max_refine;
    HIP_TRY(hipMemcpyAsync(w.r, d_y, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    double rnorm = ynorm;
    precond(w.r, rnorm, w.z);
    HIP_TRY(hipMemcpyAsync(w.p, w.z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    double rz = run_dot(w.r, w.z, n, w.part, s);
    double rel = 1.0;
    for (int it = 0; it < maxit; ++it) {
        run_matvec(n, f->kp, f->dx, w.p, w.q, s);
        const double pq = run_dot(w.p, w.q, n, w.part, s);
        if (!(pq > 0.0) || !std::isfinite(rz))
            return {it, rel, false};
        const double alpha = rz / pq;
        run_axpy(d_x, alpha, w.p, false, n, s);
        run_axpy(w.r, -alpha, w.q, false, n, s);
        rnorm = std::sqrt(run_sumsq(w.r, n, w.part, s));
        const bool last = it + 1 == maxit;
        if (rnorm <= tol * ynorm || last) {
            // confirm with the true residual y - C x (the recurrence drifts)
            run_matvec(n, f->kp, f->dx, d_x, w.q, s);
            run_sub(d_y, w.q, w.r, n, s);
            rnorm = std::sqrt(run_sumsq(w.r, n, w.part, s));
            rel = rnorm / ynorm;
            if (!std::isfinite(rel))
                return {it, rel, false};
            if (rel <= tol)
                return {it, rel, true};
            if (last)
                return {it, rel, false};
            // restart from the true residual
            precond(w.r, rnorm, w.z);
            HIP_TRY(hipMemcpyAsync(w.p, w.z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            rz = run_dot(w.r, w.z, n, w.part, s);
            continue;
        }
        rel = rnorm / ynorm;
        const double rzold = run_dot(w.r, w.z, n, w.part, s);   // r_{k+1} . z_k
        precond(w.r, rnorm, w.z);
        const double rznew = run_dot(w.r, w.z, n, w.part, s);
        const double beta = (rznew - rzold) / rz;
        rz = rznew;
        run_xpby(w.z, beta, w.p, n, s);
    }
    return {maxit - 1, rel, false};
}

}  // namespace

extern "C" {

const char *hodlr_last_error(void) { return g_err.c_str(); }

int32_t hodlr_num_levels(int64_t n, int32_t leaf) { return num_levels(n, leaf); }

hodlr_status hodlr_order(const double *x, int64_t n, int32_t dim, int32_t leaf, int64_t *perm)
{
    return guarded([&]() {
        check_sizes(n, dim, leaf);
        check_finite(x, n * dim, "x");
        if (!perm)
            throw Error{HODLR_EINVAL, "perm is NULL"};
        order_points(x, n, dim, leaf, perm);
        return HODLR_OK;
    });
}

hodlr_status hodlr_build(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                         const double theta[2], double sigma2, int32_t leaf, double tol,
                         const hodlr_opts *opts, hodlr_factor *out)
{
    return guarded([&]() {
        hodlr_opts o = opts ? *opts : default_opts();
        check_sizes(n, dim, leaf);
        check_opts(o);
        check_params(k, theta, sigma2, tol);
        check_finite(x, n * dim, "x");
        if (o.noise)
            check_noise(o.noise, n);
        if (!out)
            throw Error{HODLR_EINVAL, "out is NULL"};
        auto f = std::make_unique<hodlr_factor_s>();
        HIP_TRY(hipGetDevice(&f->device));
        f->opts = o;
        f->opts.noise = nullptr;   // the caller's array is not kept
        f->perm.resize(n);
        if (o.presorted)
            for (int64_t i = 0; i < n; ++i)
                f->perm[i] = i;
        else
            order_points(x, n, dim, leaf, f->perm.data());
        plan_build(f->plan, n, dim, leaf, &o);
        plan_upload(f->plan);
        f->lay = make_layout(f->plan, true);
        DevBuf ws(f->lay.total), dxb(sizeof(double) * n * dim);
        DevBuf dnz(o.noise ? sizeof(double) * n : 8);
        upload_noise(dnz, o.noise, f->perm);
        std::vector<double> xs = ordered_soa(x, n, dim, f->perm);
        HIP_TRY(hipMemcpy(dxb.p, xs.data(), sizeof(double) * xs.size(), hipMemcpyHostToDevice));
        Pipeline P;
        P.plan = &f->plan;
        P.lay = f->lay;
        P.ws = (char *)ws.p;
        P.stream = nullptr;
        P.x = (const double *)dxb.p;
        P.kp = make_kparams(k, dim, theta, sigma2);
        P.kp.noise = o.noise ? (const double *)dnz.p : nullptr;
        P.tol = tol;
        double *d_out = wsp<double>(P, P.lay.out);
        factor_pipeline(P, nullptr, d_out);
        double hout[8];
        HIP_TRY(hipMemcpyAsync(hout, d_out, sizeof(double) * 8, hipMemcpyDeviceToHost, P.stream));
        raise_status(read_status(P));
        if (f->plan.mixed_check && mixed_estimate_missed(P, hout[1], 0)) {
            // FP64 panels for this factor (solves still refine, as for mixed)
            f->plan.precision = HODLR_FP64;
            f->lay = make_layout(f->plan, true);
            DevBuf ws64(f->lay.total);
            ws = std::move(ws64);
            P.lay = f->lay;
            P.ws = (char *)ws.p;
            d_out = wsp<double>(P, P.lay.out);
            factor_pipeline(P, nullptr, d_out);
            HIP_TRY(hipMemcpyAsync(hout, d_out, sizeof(double) * 8, hipMemcpyDeviceToHost,
                                   P.stream));
            raise_status(read_status(P));
            f->fp64_fallback = 1;
        }
        f->logdet = hout[1];
        f->kp = P.kp;
        f->tol = tol;
        f->rmax = P.rmax;
        f->cols = P.cols;
        f->cnt = P.cnt;
        f->ranks = P.ranks;
        f->capped = P.capped;
        f->ws = ws.release();
        f->dx = (double *)dxb.release();
        if (o.noise)
            f->dnoise = (double *)dnz.release();
        *out = f.release();
        return HODLR_OK;
    });
}

hodlr_status hodlr_logdet(hodlr_factor f, double *logdet)
{
    if (!f || !logdet)
        return fail(HODLR_EINVAL, "NULL argument");
    *logdet = f->logdet;
    return HODLR_OK;
}

hodlr_status hodlr_solve(hodlr_factor f, const double *y, double *x, int64_t nrhs)
{
    return guarded([&]() {
        if (!f || !y || !x || nrhs < 0)
            throw Error{HODLR_EINVAL, "bad argument"};
        const int64_t n = f->plan.n;
        check_finite(y, n * nrhs, "y");
        HIP_TRY(hipSetDevice(f->device));
        Pipeline P = factor_pipeline_of(f);
        const bool refined = f->plan.refine;
        DevBuf dy(sizeof(double) * n), dx(sizeof(double) * n);
        const size_t vb = refined ? sizeof(double) * n : 8;
        DevBuf dr(vb), dq(vb), dz(vb), dp(vb), part(sizeof(double) * 512);
        const Work w{(double *)dr.p, (double *)dq.p, (double *)dz.p, (double *)dp.p,
                     (double *)part.p};
        std::vector<double> buf(n), res(n);
        int steps = 0;
        double worst = refined ? 0.0 : -1.0;
        bool all_ok = true;
        for (int64_t c = 0; c < nrhs; ++c) {
            const double *yc = y + c * n;
            for (int64_t k = 0; k < n; ++k)
                buf[k] = yc[f->perm[k]];
            HIP_TRY(hipMemcpy(dy.p, buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
            Refined r = solve_tree(f, P, (const double *)dy.p, (double *)dx.p, w);
            HIP_TRY(hipMemcpy(buf.data(), dx.p, sizeof(double) * n, hipMemcpyDeviceToHost));
            prof_collect();
            steps = std::max(steps, r.steps);
            if (refined)
                worst = std::max(worst, r.residual);
            all_ok = all_ok && r.converged;
            for (int64_t k = 0; k < n; ++k)
                res[f->perm[k]] = buf[k];
            std::memcpy(x + c * n, res.data(), sizeof(double) * n);
        }
        f->refine_steps = steps;
        f->refine_residual = worst;
        if (!all_ok)
            throw Error{HODLR_ENOCONV, "refinement did not reach refine_tol within max_refine "
                                       "steps (the best iterate was written)"};
        return HODLR_OK;
    });
}

hodlr_status hodlr_predict(hodlr_factor f, const double *y, const double *xt, int64_t m,
                           double *mean, double *var)
{
    return guarded([&]() {
        if (!f || !y || m < 0 || (m > 0 && (!xt || !mean)))
            throw Error{HODLR_EINVAL, "bad argument"};
        const int64_t n = f->plan.n;
        const int dim = f->plan.dim;
        check_finite(y, n, "y");
        check_finite(xt, m * dim, "xt");
        if (m == 0)
            return HODLR_OK;
        HIP_TRY(hipSetDevice(f->device));
        Pipeline P = factor_pipeline_of(f);
        hipStream_t s = P.stream;
        const bool refined = f->plan.refine;
        DevBuf dy(sizeof(double) * n), da(sizeof(double) * n);
        const size_t vb = refined ? sizeof(double) * n : 8;
        DevBuf dr(vb), dq(vb), dz(vb), dp(vb), part(sizeof(double) * 512);
        const Work w{(double *)dr.p, (double *)dq.p, (double *)dz.p, (double *)dp.p,
                     (double *)part.p};
        // alpha = C^{-1} y in tree order
        std::vector<double> buf(n);
        for (int64_t k = 0; k < n; ++k)
            buf[k] = y[f->perm[k]];
        HIP_TRY(hipMemcpy(dy.p, buf.data(), sizeof(double) * n, hipMemcpyHostToDevice));
        Refined ra = solve_tree(f, P, (const double *)dy.p, (double *)da.p, w);
        int steps = ra.steps;
        double worst = refined ? ra.residual : -1.0;
        bool all_ok = ra.converged;
        // test points, coordinate-major
        std::vector<double> xs((size_t)m * dim);
        for (int d = 0; d < dim; ++d)
            for (int64_t j = 0; j < m; ++j)
                xs[(size_t)d * m + j] = xt[j * dim + d];
        DevBuf dxt(sizeof(double) * xs.size()), dmean(sizeof(double) * m);
        DevBuf dpart(sizeof(double) * (size_t)predict_slices(n, m) * m);
        HIP_TRY(hipMemcpy(dxt.p, xs.data(), sizeof(double) * xs.size(), hipMemcpyHostToDevice));
        run_predict_mean(n, f->kp, f->dx, (const double *)da.p, m, (const double *)dxt.p,
                         (double *)dpart.p, (double *)dmean.p, s);
        HIP_TRY(hipMemcpyAsync(mean, dmean.p, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (var) {
            // var_j = k(xt_j, xt_j) - k_j . C^{-1} k_j with k_j = k(x, xt_j) in tree
            // order; k(r = 0) = a^2 for every kernel here
            const int nb = (int)std::min<int64_t>(m, 16);
            DevBuf dk(sizeof(double) * n * nb), dv(sizeof(double) * n);
            for (int64_t j0 = 0; j0 < m; j0 += nb) {
                const int cnt = (int)std::min<int64_t>(nb, m - j0);
                run_kcross(n, f->kp, f->dx, m, (const double *)dxt.p, j0, cnt, (double *)dk.p, s);
                for (int c = 0; c < cnt; ++c) {
                    const double *kc = (const double *)dk.p + (int64_t)c * n;
                    Refined rv = solve_tree(f, P, kc, (double *)dv.p, w);
                    steps = std::max(steps, rv.steps);
                    if (refined)
                        worst = std::max(worst, rv.residual);
                    all_ok = all_ok && rv.converged;
                    var[j0 + c] = f->kp.a2 - run_dot(kc, (const double *)dv.p, n, w.part, s);
                }
            }
        }
        prof_collect();
        f->refine_steps = steps;
        f->refine_residual = worst;
        if (!all_ok)
            throw Error{HODLR_ENOCONV, "refinement did not reach refine_tol within max_refine "
                                       "steps (the outputs were written)"};
        return HODLR_OK;
    });
}

hodlr_status gp_loglik(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                       const double theta[2], double sigma2, const double *y, int32_t leaf,
                       double tol, const hodlr_opts *opts, double *loglik, double *logdet,
                       double *quad)
{
    return guarded([&]() {
        hodlr_opts o = opts ? *opts : default_opts();
        check_sizes(n, dim, leaf);
        check_opts(o);
        check_params(k, theta, sigma2, tol);
        check_finite(x, n * dim, "x");
        check_finite(y, n, "y");
        if (o.noise)
            check_noise(o.noise, n);
        if (!loglik)
            throw Error{HODLR_EINVAL, "loglik is NULL"};
        if (o.precision == HODLR_MIXED || o.refine) {
            // factor once, then the refined solve for the quadratic form
            hodlr_factor f = nullptr;
            hodlr_status st = hodlr_build(x, n, dim, k, theta, sigma2, leaf, tol, &o, &f);
            if (st != HODLR_OK)
                return st;
            std::unique_ptr<hodlr_factor_s> own(f);
            std::vector<double> z(n);
            st = hodlr_solve(f, y, z.data(), 1);
            if (st != HODLR_OK && st != HODLR_ENOCONV)
                return st;   // ENOCONV: the best iterate still gives the outputs
            double q = 0.0;
            for (int64_t i = 0; i < n; ++i)
                q += y[i] * z[i];
            const double ld = f->logdet;
            *loglik = -0.5 * q - 0.5 * ld - 0.5 * (double)n * std::log(2.0 * M_PI);
            if (logdet)
                *logdet = ld;
            if (quad)
                *quad = q;
            return st;
        }
        std::vector<int64_t> perm(n);
        if (o.presorted)
            for (int64_t i = 0; i < n; ++i)
                perm[i] = i;
        else
            order_points(x, n, dim, leaf, perm.data());
        Plan plan;
        plan_build(plan, n, dim, leaf, &o);
        plan_upload(plan);
        struct PlanGuard {
            Plan &p;
            ~PlanGuard() { plan_release(p); }
        } pg{plan};
        Layout lay = make_layout(plan, false);
        DevBuf ws(lay.total), dxb(sizeof(double) * n * dim), dyb(sizeof(double) * n);
        DevBuf dnz(o.noise ? sizeof(double) * n : 8);
        upload_noise(dnz, o.noise, perm);
        std::vector<double> xs = ordered_soa(x, n, dim, perm);
        std::vector<double> ys(n);
        for (int64_t i = 0; i < n; ++i)
            ys[i] = y[perm[i]];
        HIP_TRY(hipMemcpy(dxb.p, xs.data(), sizeof(double) * xs.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(dyb.p, ys.data(), sizeof(double) * n, hipMemcpyHostToDevice));
        Pipeline P;
        P.plan = &plan;
        P.lay = lay;
        P.ws = (char *)ws.p;
        P.stream = nullptr;
        P.x = (const double *)dxb.p;
        P.kp = make_kparams(k, dim, theta, sigma2);
        P.kp.noise = o.noise ? (const double *)dnz.p : nullptr;
        P.tol = tol;
        double *d_out = wsp<double>(P, lay.out);
        factor_pipeline(P, (const double *)dyb.p, d_out);
        double hout[8];
        HIP_TRY(hipMemcpyAsync(hout, d_out, sizeof(double) * 8, hipMemcpyDeviceToHost, P.stream));
        raise_status(read_status(P));
        *loglik = hout[0];
        if (logdet)
            *logdet = hout[1];
        if (quad)
            *quad = hout[2];
        return HODLR_OK;
    });
}

hodlr_status hodlr_info(hodlr_factor f, hodlr_info_t *out)
{
    if (!f || !out)
        return fail(HODLR_EINVAL, "NULL argument");
    hodlr_info_t I;
    std::memset(&I, 0, sizeof(I));
    I.n = f->plan.n;
    I.dim = f->plan.dim;
    I.levels = f->plan.L;
    I.leaf_max = f->plan.leafmax;
    I.capped_blocks = f->capped;
    I.precision = f->opts.precision;
    I.refine_steps = f->refine_steps;
    I.refine_residual = f->refine_residual;
    I.fp64_fallback = f->fp64_fallback;
    for (int d = 0; d < f->plan.L && d < HODLR_MAX_LEVELS; ++d) {
        int64_t h0 = f->plan.first_at(d), h1 = f->plan.first_at(d + 1);
        int mx = 0;
        double sum = 0;
        for (int64_t h = h0; h < h1; ++h) {
            mx = std::max(mx, f->ranks[h]);
            sum += f->ranks[h];
        }
        I.rank_max[d] = mx;
        I.rank_mean[d] = sum / (double)(h1 - h0);
        I.max_rank_used = std::max(I.max_rank_used, mx);
    }
    I.device_bytes = (int64_t)f->lay.total + (int64_t)f->plan.dev_tables_bytes +
                     (int64_t)sizeof(double) * f->plan.n * (f->plan.dim + (f->dnoise ? 1 : 0));
    *out = I;
    return HODLR_OK;
}

void hodlr_free(hodlr_factor f) { delete f; }

hodlr_status hodlr_plan_create(int64_t n, int32_t dim, int32_t leaf, const hodlr_opts *opts,
                               hodlr_plan *out)
{
    return guarded([&]() {
        hodlr_opts o = opts ? *opts : default_opts();
        check_sizes(n, dim, leaf);
        check_opts(o);
        no_noise(o);
        if (!out)
            throw Error{HODLR_EINVAL, "out is NULL"};
        auto p = std::make_unique<hodlr_plan_s>();
        p->opts = o;
        plan_build(p->plan, n, dim, leaf, &o);
        if (p->plan.leafmax > LEAF_MAX)
            throw Error{HODLR_EINVAL, "leaf size above 256 is not supported"};
        plan_upload(p->plan);
        p->lay = make_layout(p->plan, false);
        p->make_fp64_shadow();
        *out = p.release();
        return HODLR_OK;
    });
}

hodlr_status hodlr_plan_tuned_create(int64_t n, int32_t dim, const hodlr_opts *opts,
                                     const hodlr_tune_t *tune, hodlr_plan *out)
{
    return guarded([&]() {
        if (!tune)
            throw Error{HODLR_EINVAL, "tune is NULL"};
        hodlr_opts o = opts ? *opts : default_opts();
        check_sizes(n, dim, tune->leaf);
        check_opts(o);
        no_noise(o);
        if (!out)
            throw Error{HODLR_EINVAL, "out is NULL"};
        auto p = std::make_unique<hodlr_plan_s>();
        p->opts = o;
        plan_build(p->plan, n, dim, tune->leaf, &o, tune->level_rows, tune->reduce_cols,
                   tune->reduce_group);
        if (p->plan.leafmax > LEAF_MAX)
            throw Error{HODLR_EINVAL, "leaf size above 256 is not supported"};
        plan_upload(p->plan);
        p->lay = make_layout(p->plan, false);
        p->make_fp64_shadow();
        *out = p.release();
        return HODLR_OK;
    });
}

void hodlr_plan_destroy(hodlr_plan p)
{
    if (p) {
        plan_release(p->plan);
        delete p;
    }
}

hodlr_status hodlr_plan_workspace_size(hodlr_plan p, size_t *bytes)
{
    if (!p || !bytes)
        return fail(HODLR_EINVAL, "NULL argument");
    *bytes = p->single_bytes();
    return HODLR_OK;
}

hodlr_status gp_loglik_dev(hodlr_plan p, const double *d_x, hodlr_kernel k, const double theta[2],
                           double sigma2, const double *d_y, double tol, void *d_work,
                           size_t work_bytes, void *stream, double *d_out, double *d_z)
{
    return guarded([&]() {
        if (!p || !d_x || !d_y || !d_work || !d_out)
            throw Error{HODLR_EINVAL, "NULL argument"};
        check_params(k, theta, sigma2, tol);
        if (work_bytes < p->single_bytes())
            throw Error{HODLR_EINVAL, "workspace too small: need " +
                                          std::to_string(p->single_bytes()) + " bytes"};
        Pipeline P;
        P.plan = &p->plan;
        P.lay = p->lay;
        P.ws = (char *)d_work;
        P.stream = (hipStream_t)stream;
        P.x = d_x;
        P.kp = make_kparams(k, p->plan.dim, theta, sigma2);
        P.tol = tol;
        std::vector<int> spec;
        if (p->opts.speculate) {
            std::lock_guard<std::mutex> lk(p->last_mu);
            spec = p->spec_rmax;
        }
        if (!spec.empty())
            P.spec = &spec;
        factor_pipeline(P, d_y, d_out);
        if (d_z)
            run_widen(P.ws + P.lay.Xt, p->plan.f32(), d_z, p->plan.n, P.stream);
        // the status, with a mixed plan's log det and error estimate and (after
        // a speculative compression) the actual rank statistics and ranks
        double *hv = nullptr;
        int *hs = nullptr, *hr = nullptr;
        auto status = [&](bool spec_reads) {
            int *h8 = pinned_ints(16, 3);   // ints 0-3: the mixed values; int 8: status
            EndArgs E;
            E.status = wsp<int>(P, P.lay.status);
            E.h_status = device_alias(h8 + 8);
            if (p->plan.mixed_check) {
                hv = (double *)h8;
                E.ld = d_out + 1;
                E.est = wsp<double>(P, P.lay.misc + MISC_BOUND);
                E.h_vals = device_alias(hv);
            }
            if (spec_reads) {
                hs = pinned_ints(64, 2);
                hr = pinned_ints((size_t)p->plan.nint, 0);
                E.stats = wsp<int>(P, P.lay.misc + MISC_SPEC);
                E.h_stats = device_alias(hs);
                E.ranks = wsp<int>(P, P.lay.rank);
                E.nint = p->plan.nint;
                E.h_ranks = device_alias(hr);
            }
            end_read_kernel<<<1, 256, 0, P.stream>>>(E);
            HIP_TRY(hipGetLastError());
            host_wait(P.stream);
            prof_collect();
            return h8[8];
        };
        int st = 0;
        std::vector<int> actual;   // per depth index, of this call's compression
        if (P.spec_run) {
            st = status(true);
            if (st & DS_SPEC_MISS) {
                // the assumed widths or step count did not hold: the ordinary way
                P.spec = nullptr;
                factor_pipeline(P, d_y, d_out);
                if (d_z)
                    run_widen(P.ws + P.lay.Xt, p->plan.f32(), d_z, p->plan.n, P.stream);
                st = status(false);
                actual = P.rmax;
            } else {
                actual.assign(hs, hs + p->plan.L + 2);
                P.capped = hs[48];
                std::memcpy(P.ranks.data(), hr, sizeof(int) * p->plan.nint);
            }
        } else {
            st = status(false);
            actual = P.rmax;
        }
        raise_status(st);
        int fallback = 0;
        if (hv) {
            if (mixed_estimate_exceeds(hv[1], hv[0])) {
                // the same likelihood with FP64 panels on the same workspace
                P.plan = &p->plan64;
                P.lay = p->lay64;
                P.spec = nullptr;
                factor_pipeline(P, d_y, d_out);
                if (d_z)
                    run_widen(P.ws + P.lay.Xt, false, d_z, p->plan.n, P.stream);
                raise_status(read_status(P));
                fallback = 1;
            }
        }
        {
            std::lock_guard<std::mutex> lk(p->last_mu);
            if (fallback)
                actual = P.rmax;   // the FP64 redo's own compression
            p->last_rmax = actual;
            p->last_ranks = P.ranks;
            p->last_capped = P.capped;
            p->last_fallback = fallback;
            p->spec_rmax = actual;
            p->last_spec = P.spec_run && !(st & DS_SPEC_MISS) && !fallback ? 1 : 0;
            p->last_proj = P.proj_run ? 1 : 0;
        }
        return HODLR_OK;
    });
}

hodlr_status hodlr_plan_info(hodlr_plan p, hodlr_info_t *out)
{
    if (!p || !out)
        return fail(HODLR_EINVAL, "NULL argument");
    hodlr_info_t I;
    std::memset(&I, 0, sizeof(I));
    I.n = p->plan.n;
    I.dim = p->plan.dim;
    I.levels = p->plan.L;
    I.leaf_max = p->plan.leafmax;
    I.precision = p->opts.precision;
    I.device_bytes = (int64_t)p->single_bytes() + (int64_t)p->plan.dev_tables_bytes;
    std::lock_guard<std::mutex> lk(p->last_mu);
    I.capped_blocks = p->last_capped;
    I.fp64_fallback = p->last_fallback;
    I.speculated = p->last_spec;
    I.projected = p->last_proj;
    for (int d = 0; d < p->plan.L && d < HODLR_MAX_LEVELS && d + 1 < (int)p->last_rmax.size();
         ++d) {
        I.rank_max[d] = p->last_rmax[d + 1];
        I.max_rank_used = std::max(I.max_rank_used, I.rank_max[d]);
    }
    if (!p->last_ranks.empty())
        for (int d = 0; d < p->plan.L && d < HODLR_MAX_LEVELS; ++d) {
            const int64_t h0 = p->plan.first_at(d), h1 = p->plan.first_at(d + 1);
            int mx = 0;
            double sum = 0;
            for (int64_t h = h0; h < h1; ++h) {
                mx = std::max(mx, p->last_ranks[h]);
                sum += p->last_ranks[h];
            }
            I.rank_max[d] = mx;
            I.rank_mean[d] = sum / (double)(h1 - h0);
            I.max_rank_used = std::max(I.max_rank_used, mx);
        }
    *out = I;
    return HODLR_OK;
}

}  // extern "C"

extern "C" {

// bytes of a batched call's workspace: the items, and for a mixed plan room
// for one FP64 likelihood at its start (the redo of an item that misses the
// mixed log-det bar)
static size_t batch_bytes(hodlr_plan p, int32_t nitems)
{
    const size_t b = item_stride(p->lay) * (size_t)nitems;
    return p->plan.f32() ? std::max(b, p->lay64.total) : b;
}

// Mixed plans: after the batch, every item whose log-det error estimate misses
// the bar is computed again with FP64 panels on the workspace (in FP64
// batches when the observations are shared, else one at a time) and its row
// of d_out replaced (synchronizes the stream).
static void batch_fp64_redo(hodlr_plan p, const Pipeline &B, const double *d_params, int nitems,
                            const double *d_y, int64_t y_stride, double *d_out)
{
    if (!p->plan.mixed_check)
        return;
    std::vector<double> bound(nitems), out(3 * (size_t)nitems), par(3 * (size_t)nitems);
    HIP_TRY(hipStreamSynchronize(B.stream));
    HIP_TRY(hipMemcpy2D(bound.data(), sizeof(double), B.ws + B.lay.misc + MISC_BOUND,
                        (size_t)B.batch.istride, sizeof(double), nitems, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(out.data(), d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(par.data(), d_params, sizeof(double) * par.size(), hipMemcpyDeviceToHost));
    std::vector<int> flag;
    for (int i = 0; i < nitems; ++i) {
        const double ld = out[3 * (size_t)i + 1];
        if (std::isfinite(ld) && mixed_estimate_exceeds(bound[i], ld))
            flag.push_back(i);
    }
    const int redo = (int)flag.size();
    const size_t s64 = item_stride(p->lay64);
    const size_t room = batch_bytes(p, nitems);
    // shared observations: the flagged items as FP64 batches (as many as the
    // workspace holds, their parameters and results after them)
    size_t k = 0;
    if (y_stride == 0 && redo > 1)
        k = std::min<size_t>(redo, (room - 256) / (s64 + 6 * sizeof(double)));
    for (size_t c0 = 0; k > 1 && c0 < flag.size(); c0 += k) {
        const size_t kk = std::min(k, flag.size() - c0);
        double *dpar = (double *)(B.ws + ((kk * s64 + 255) & ~(size_t)255));
        double *dres = dpar + 3 * kk;
        std::vector<double> sub(3 * kk), res(3 * kk);
        for (size_t j = 0; j < kk; ++j)
            for (int q = 0; q < 3; ++q)
                sub[3 * j + q] = par[3 * (size_t)flag[c0 + j] + q];
        HIP_TRY(hipMemcpyAsync(dpar, sub.data(), sizeof(double) * sub.size(), hipMemcpyHostToDevice,
                               B.stream));
        Pipeline Q;
        Q.plan = &p->plan64;
        Q.lay = p->lay64;
        Q.ws = B.ws;
        Q.stream = B.stream;
        Q.x = B.x;
        Q.kp = B.kp;
        Q.tol = B.tol;
        Q.nitems = (int)kk;
        Q.batch.istride = (int64_t)s64;
        Q.batch.params = dpar;
        Q.batch.ystride = 0;
        zero_status_kernel<<<(unsigned)kk, 64, 0, Q.stream>>>(wsp<int>(Q, Q.lay.status), Q.batch);
        HIP_TRY(hipGetLastError());
        run_aca_batched(Q);
        make_columns(Q);
        run_leaf_factor(Q, d_y);
        run_levels_factor(Q);
        run_finish(Q, d_y, dres, 3);
        HIP_TRY(hipMemcpyAsync(res.data(), dres, sizeof(double) * res.size(), hipMemcpyDeviceToHost,
                               Q.stream));
        HIP_TRY(hipStreamSynchronize(Q.stream));
        for (size_t j = 0; j < kk; ++j)
            for (int q = 0; q < 3; ++q)
                out[3 * (size_t)flag[c0 + j] + q] = res[3 * j + q];
    }
    if (k > 1) {
        HIP_TRY(hipMemcpy(d_out, out.data(), sizeof(double) * out.size(), hipMemcpyHostToDevice));
        flag.clear();
    }
    for (int i : flag) {
        Pipeline Q;
        Q.plan = &p->plan64;
        Q.lay = p->lay64;
        Q.ws = B.ws;
        Q.stream = B.stream;
        Q.x = B.x;
        const double th[2] = {par[3 * (size_t)i], par[3 * (size_t)i + 1]};
        Q.kp = make_kparams(B.kp.kind, p->plan.dim, th, par[3 * (size_t)i + 2]);
        Q.tol = B.tol;
        double *o = wsp<double>(Q, Q.lay.out);
        factor_pipeline(Q, d_y + (size_t)i * y_stride, o);
        const int st = read_status(Q);
        const double nan3[3] = {NAN, NAN, NAN};
        if (st)
            HIP_TRY(hipMemcpy(d_out + 3 * (size_t)i, nan3, sizeof(nan3), hipMemcpyHostToDevice));
        else
            HIP_TRY(hipMemcpy(d_out + 3 * (size_t)i, o, sizeof(double) * 3,
                              hipMemcpyDeviceToDevice));
    }
    std::lock_guard<std::mutex> lk(p->last_mu);
    p->last_fallback = redo;
}

hodlr_status hodlr_plan_batch_workspace_size(hodlr_plan p, int32_t nitems, size_t *bytes)
{
    if (!p || !bytes || nitems < 1)
        return fail(HODLR_EINVAL, "bad argument");
    *bytes = batch_bytes(p, nitems);
    return HODLR_OK;
}

hodlr_status gp_loglik_batch_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                                 const double *d_params, int32_t nitems, const double *d_y,
                                 int64_t y_stride, double tol, void *d_work, size_t work_bytes,
                                 void *stream, double *d_out, int32_t use_graph)
{
    return guarded([&]() {
        if (!p || !d_x || !d_params || !d_y || !d_work || !d_out || nitems < 1)
            throw Error{HODLR_EINVAL, "bad argument"};
        if (k < HODLR_K_SE || k > HODLR_K_IMQ)
            throw Error{HODLR_EINVAL, "unknown kernel"};
        if (!(tol > 0.0) || !std::isfinite(tol))
            throw Error{HODLR_EINVAL, "tol must be positive and finite"};
        if (y_stride < 0)
            throw Error{HODLR_EINVAL, "y_stride must be >= 0"};
        const size_t istride = item_stride(p->lay);
        if (work_bytes < batch_bytes(p, nitems))
            throw Error{HODLR_EINVAL, "workspace too small: need " +
                                          std::to_string(batch_bytes(p, nitems)) + " bytes"};
        if (p->plan.leafmax > LEAF_MAX)
            throw Error{HODLR_EINVAL, "leaf size above 256 is not supported"};
        if (p->plan.compressor != HODLR_COMPRESS_ACA)
            throw Error{HODLR_EINVAL, "the batched form compresses by cross approximation only"};
        Pipeline P;
        P.plan = &p->plan;
        P.lay = p->lay;
        P.ws = (char *)d_work;
        P.stream = (hipStream_t)stream;
        P.x = d_x;
        const double one[2] = {1.0, 1.0};
        P.kp = make_kparams(k, p->plan.dim, one, 0.0);
        P.tol = tol;
        P.nitems = nitems;
        P.batch.istride = (int64_t)istride;
        P.batch.params = d_params;
        P.batch.ystride = y_stride;
        zero_status_kernel<<<nitems, 64, 0, P.stream>>>(wsp<int>(P, P.lay.status), P.batch);
        HIP_TRY(hipGetLastError());
        run_aca_batched(P);
        make_columns(P);
        {
            std::lock_guard<std::mutex> lk(p->last_mu);
            p->last_rmax = P.rmax;
            p->last_ranks.clear();
            p->last_capped = P.capped;
        }
        const bool graph = use_graph && stream != nullptr;
        if (!graph) {
            run_leaf_factor(P, d_y);
            run_levels_factor(P);
            run_finish(P, d_y, d_out, 3);
            batch_fp64_redo(p, P, d_params, nitems, d_y, y_stride, d_out);
            return HODLR_OK;
        }
        BatchGraph *hit = nullptr;
        for (auto &g : p->graphs)
            if (g.rmax == P.rmax && g.ws == d_work && g.x == d_x && g.y == d_y &&
                g.params == d_params && g.out == d_out && g.ystride == y_stride &&
                g.stream == stream && g.kind == (int)k && g.nitems == nitems) {
                hit = &g;
                break;
            }
        if (!hit) {
            prime_level_attributes();
            BatchGraph g;
            g.rmax = P.rmax;
            g.ws = d_work;
            g.x = d_x;
            g.y = d_y;
            g.params = d_params;
            g.out = d_out;
            g.ystride = y_stride;
            g.stream = stream;
            g.kind = (int)k;
            g.nitems = nitems;
            prof_suspend(true);
            hipError_t e = hipStreamBeginCapture(P.stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                try {
                    run_leaf_factor(P, d_y);
                    run_levels_factor(P);
                    run_finish(P, d_y, d_out, 3);
                } catch (...) {
                    hipGraph_t dead = nullptr;
                    (void)hipStreamEndCapture(P.stream, &dead);
                    if (dead)
                        (void)hipGraphDestroy(dead);
                    prof_suspend(false);
                    throw;
                }
                e = hipStreamEndCapture(P.stream, &g.graph);
            }
            prof_suspend(false);
            HIP_TRY(e);
            HIP_TRY(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
            if (p->graphs.size() >= 8) {   // small cache: drop the oldest
                (void)hipGraphExecDestroy(p->graphs.front().exec);
                (void)hipGraphDestroy(p->graphs.front().graph);
                p->graphs.erase(p->graphs.begin());
            }
            p->graphs.push_back(g);
            hit = &p->graphs.back();
        }
        HIP_TRY(hipGraphLaunch(hit->exec, P.stream));
        batch_fp64_redo(p, P, d_params, nitems, d_y, y_stride, d_out);
        return HODLR_OK;
    });
}

// ---------------------------------------------------------------- gradient
// Central differences of 7 likelihoods: item 0 at the point, items 2q+1 and
// 2q+2 with parameter q (a, l, sigma2) shifted up and down.  Each item runs
// the single-likelihood pipeline on the workspace (the batched form, one
// work-group per block, suits many small items, not the long top blocks of a
// large n); on FP64 plans the two sigma2 items reuse the point's compression
// (the off-diagonal blocks do not depend on sigma2) and redo only the
// leaves, levels and sums.  The divisor is the difference of the two
// parameter values as stored, so the step's own rounding does not enter.
constexpr int GRAD_ITEMS = 7;
constexpr int GRAD_OSTRIDE = 8;   // the finish stage's output row (it writes 5 values)

struct GradPar {
    double v[3 * GRAD_ITEMS];
};

__global__ void grad_combine_kernel(GradPar par, const double *res, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    out[0] = res[0];
    out[1] = res[1];
    out[2] = res[2];
    for (int q = 0; q < 3; ++q) {
        const double up = res[GRAD_OSTRIDE * (2 * q + 1)], dn = res[GRAD_OSTRIDE * (2 * q + 2)];
        out[3 + q] = (up - dn) / (par.v[3 * (2 * q + 1) + q] - par.v[3 * (2 * q + 2) + q]);
    }
}

__global__ void zero_one_status_kernel(int *status)
{
    if (threadIdx.x < 4)
        status[threadIdx.x] = 0;
}

// the single likelihood's workspace, then (256-byte aligned) the 7 result rows
static size_t grad_bytes(hodlr_plan p)
{
    return ((p->single_bytes() + 255) & ~(size_t)255) + GRAD_OSTRIDE * GRAD_ITEMS * sizeof(double);
}

hodlr_status hodlr_plan_grad_workspace_size(hodlr_plan p, size_t *bytes)
{
    if (!p || !bytes)
        return fail(HODLR_EINVAL, "bad argument");
    *bytes = grad_bytes(p);
    return HODLR_OK;
}

hodlr_status gp_loglik_grad_dev(hodlr_plan p, const double *d_x, hodlr_kernel k,
                                const double theta[2], double sigma2, const double *d_y,
                                double tol, double rel_step, void *d_work, size_t work_bytes,
                                void *stream, double *d_out)
{
    return guarded([&]() {
        if (!p || !d_x || !theta || !d_y || !d_work || !d_out)
            throw Error{HODLR_EINVAL, "bad argument"};
        check_params(k, theta, sigma2, tol);
        if (!(sigma2 > 0.0))
            throw Error{HODLR_EINVAL, "the gradient needs sigma2 > 0"};
        if (!(rel_step < 0.5) || std::isnan(rel_step))
            throw Error{HODLR_EINVAL, "rel_step must be below 0.5"};
        if (work_bytes < grad_bytes(p))
            throw Error{HODLR_EINVAL, "workspace too small: need " + std::to_string(grad_bytes(p)) +
                                          " bytes"};
        const double h = rel_step > 0.0 ? rel_step : (p->plan.f32() ? 1e-3 : 1e-4);
        const double base[3] = {theta[0], theta[1], sigma2};
        GradPar par;
        for (int i = 0; i < GRAD_ITEMS; ++i)
            for (int q = 0; q < 3; ++q)
                par.v[3 * i + q] = base[q];
        for (int q = 0; q < 3; ++q) {
            par.v[3 * (2 * q + 1) + q] = base[q] * (1.0 + h);
            par.v[3 * (2 * q + 2) + q] = base[q] * (1.0 - h);
        }
        double *d_res = (double *)((char *)d_work + ((p->single_bytes() + 255) & ~(size_t)255));
        hipStream_t s = (hipStream_t)stream;
        Pipeline P0;   // the point's pipeline (its compression serves the sigma2 items)
        int fallback = 0;
        // the sigma2 items right after the point, while its compression is
        // still the one in the workspace
        static const int order[GRAD_ITEMS] = {0, 5, 6, 1, 2, 3, 4};
        for (int i : order) {
            const double th[2] = {par.v[3 * i], par.v[3 * i + 1]};
            Pipeline P;
            P.plan = &p->plan;
            P.lay = p->lay;
            P.ws = (char *)d_work;
            P.stream = s;
            P.x = d_x;
            P.tol = tol;
            const bool reuse = i >= 5 && !p->plan.f32();
            if (reuse) {
                P = P0;
                zero_one_status_kernel<<<1, 64, 0, s>>>(wsp<int>(P, P.lay.status));
                HIP_TRY(hipGetLastError());
            }
            P.kp = make_kparams(k, p->plan.dim, th, par.v[3 * i + 2]);
            double *o = d_res + GRAD_OSTRIDE * i;
            if (reuse) {
                run_leaf_factor(P, d_y);
                run_levels_factor(P);
                run_finish(P, d_y, o, GRAD_OSTRIDE);
            } else {
                factor_pipeline(P, d_y, o);
            }
            const double *hv = p->plan.mixed_check ? queue_mixed_check(P, o) : nullptr;
            const int st = read_status(P);
            if (st)
                throw Error{HODLR_ENOTSPD,
                            "factorization " + std::to_string(i) + " of the gradient's 7 failed"};
            if (hv) {
                if (mixed_estimate_exceeds(hv[1], hv[0])) {
                    P.plan = &p->plan64;
                    P.lay = p->lay64;
                    factor_pipeline(P, d_y, o);
                    raise_status(read_status(P));
                    ++fallback;
                }
            }
            if (i == 0)
                P0 = P;
        }
        grad_combine_kernel<<<1, 64, 0, s>>>(par, d_res, d_out);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        {
            std::lock_guard<std::mutex> lk(p->last_mu);
            p->last_rmax = P0.rmax;
            p->last_ranks = P0.ranks;
            p->last_capped = P0.capped;
            p->last_fallback = fallback;
        }
        return HODLR_OK;
    });
}

hodlr_status hodlr_matvec_dev(int64_t n, int32_t dim, const double *d_x, hodlr_kernel k,
                              const double theta[2], double sigma2, const double *d_v,
                              double *d_out, void *stream)
{
    return guarded([&]() {
        check_sizes(n, dim, 1);
        check_params(k, theta, sigma2, 1.0);
        if (!d_x || !d_v || !d_out)
            throw Error{HODLR_EINVAL, "NULL argument"};
        run_matvec(n, make_kparams(k, dim, theta, sigma2), d_x, d_v, d_out, (hipStream_t)stream);
        return HODLR_OK;
    });
}

}  // extern "C"

namespace hodlr {
hodlr_status report(hodlr_status st, const std::string &msg) { return fail(st, msg); }
}  // namespace hodlr
