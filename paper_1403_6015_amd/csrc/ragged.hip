// Many independent Gaussian processes of uneven size: a pool of host worker
// threads, each driving its own HIP stream and a device arena sized once for
// the largest item.  Items are taken largest first from an atomic counter;
// per item the worker orders the points, uploads the tree tables, points and
// observations into its arena (asynchronously on its stream) and runs the
// full likelihood pipeline.  Small items overlap on the GPU through the
// concurrent streams.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>

#include "common.h"

using namespace hodlr;

extern "C" hodlr_status hodlr_tune_lookup(int64_t n, int32_t dim, hodlr_kernel k,
                                          int32_t precision, hodlr_tune_t *out);

namespace hodlr {
void prime_level_attributes();
hodlr_status report(hodlr_status st, const std::string &msg);   // sets hodlr_last_error
}  // namespace hodlr

namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct RaggedJob {
    int m;
    const int64_t *ns;
    const double *const *xs;
    const double *const *ys;
    int dim;
    int kernel;
    const double *params;
    int leaf;
    double tol;
    hodlr_opts opts;
    double *out;
    std::vector<int> order;
    std::atomic<int> next{0};
    size_t arena = 0;
    int device = 0;
    std::atomic<int> device_error{0};
    std::mutex mu;
    std::string msg;   // first device error seen by a worker

    void device_failed(const std::string &m)
    {
        std::lock_guard<std::mutex> g(mu);
        if (!device_error.exchange(1))
            msg = m;
    }
};

void nan_out(double *o)
{
    o[0] = o[1] = o[2] = __builtin_nan("");
}

bool item_valid(const RaggedJob &J, int i)
{
    const double a = J.params[3 * i], l = J.params[3 * i + 1], s2 = J.params[3 * i + 2];
    if (!(a > 0.0) || !(l > 0.0) || !(s2 >= 0.0) || !std::isfinite(a) || !std::isfinite(l) ||
        !std::isfinite(s2) || J.ns[i] < 1 || !J.xs[i] || !J.ys[i])
        return false;
    for (int64_t k = 0; k < J.ns[i] * J.dim; ++k)
        if (!std::isfinite(J.xs[i][k]))
            return false;
    for (int64_t k = 0; k < J.ns[i]; ++k)
        if (!std::isfinite(J.ys[i][k]))
            return false;
    return true;
}

void worker(RaggedJob *J)
{
    prof_suspend(true);   // event timing is per call, not per worker
    if (hipSetDevice(J->device) != hipSuccess) {
        J->device_failed("hipSetDevice failed in a worker");
        return;
    }
    hipStream_t s = nullptr;
    char *arena = nullptr;
    if (hipStreamCreate(&s) != hipSuccess || hipMalloc((void **)&arena, J->arena) != hipSuccess) {
        (void)hipGetLastError();
        J->device_failed("worker stream or arena allocation failed");
        if (s)
            (void)hipStreamDestroy(s);
        return;
    }
    std::vector<char> image;
    std::vector<int64_t> perm;
    std::vector<double> xsoa, yord;
    double host_out[8];
    for (;;) {
        const int t = J->next.fetch_add(1);
        if (t >= J->m || J->device_error)
            break;
        const int i = J->order[t];
        double *o = J->out + 3 * i;
        if (!item_valid(*J, i)) {
            nan_out(o);
            continue;
        }
        try {
            const int64_t n = J->ns[i];
            const int dim = J->dim;
            perm.resize(n);
            if (J->opts.presorted)
                std::iota(perm.begin(), perm.end(), 0);
            else
                order_points(J->xs[i], n, dim, J->leaf, perm.data());
            xsoa.resize((size_t)n * dim);
            yord.resize(n);
            for (int d = 0; d < dim; ++d)
                for (int64_t k = 0; k < n; ++k)
                    xsoa[(size_t)d * n + k] = J->xs[i][perm[k] * dim + d];
            for (int64_t k = 0; k < n; ++k)
                yord[k] = J->ys[i][perm[k]];
            // tiles from the autotuner's cache for this size class, if tuned
            // (the leaf size stays the caller's: it changes the approximation)
            hodlr_tune_t tt{J->leaf, LVL_ROWS, 4, 8};
            if (hodlr_tune_lookup(n, dim, (hodlr_kernel)J->kernel, J->opts.precision, &tt) !=
                HODLR_OK)
                tt = {J->leaf, LVL_ROWS, 4, 8};
            Plan plan;
            plan_build(plan, n, dim, J->leaf, &J->opts, tt.level_rows, tt.reduce_cols,
                       tt.reduce_group);
            if (plan.leafmax > LEAF_MAX)
                throw Error{HODLR_EINVAL, "leaf above 256"};
            Layout lay = make_layout(plan, false);
            Plan plan64;
            Layout lay64 = lay;
            if (plan.f32()) {   // the FP64 redo's layout shares the workspace
                Plan q = plan;
                q.precision = HODLR_FP64;
                lay64 = make_layout(q, false);
            }
            const size_t wsz = std::max(lay.total, lay64.total);
            size_t tb = plan_image(plan, image);
            // arena: [workspace | tables | x | y]
            if (a256(wsz) + a256(tb) + a256(sizeof(double) * n * dim) + sizeof(double) * n >
                J->arena)
                throw Error{HODLR_ENOMEM, "item layout exceeds the worker arena"};
            char *ws = arena;
            char *tables = arena + a256(wsz);
            double *dx = (double *)(tables + a256(tb));
            double *dy = dx + (size_t)n * dim;
            HIP_TRY(hipMemcpyAsync(tables, image.data(), tb, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(dx, xsoa.data(), sizeof(double) * xsoa.size(),
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(dy, yord.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
            plan_bind(plan, tables);
            Pipeline P;
            P.plan = &plan;
            P.lay = lay;
            P.ws = ws;
            P.stream = s;
            // the workers' own streams already overlap items; a second stream
            // per worker measured slower (4.7k vs 5.3k likelihoods/s)
            P.side_stream = false;
            P.x = dx;
            const double th[2] = {J->params[3 * i], J->params[3 * i + 1]};
            P.kp = make_kparams(J->kernel, dim, th, J->params[3 * i + 2]);
            P.tol = J->tol;
            double *d_out = wsp<double>(P, lay.out);
            factor_pipeline(P, dy, d_out);
            HIP_TRY(hipMemcpyAsync(host_out, d_out, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
            const double *hv = plan.mixed_check ? queue_mixed_check(P, d_out) : nullptr;
            int st = read_status(P);   // synchronizes: host buffers above are free again
            if (!st && hv && mixed_estimate_exceeds(hv[1], hv[0])) {
                plan64 = plan;   // bound to the uploaded tables
                plan64.precision = HODLR_FP64;
                P.plan = &plan64;
                P.lay = lay64;
                d_out = wsp<double>(P, lay64.out);
                factor_pipeline(P, dy, d_out);
                HIP_TRY(hipMemcpyAsync(host_out, d_out, sizeof(double) * 3, hipMemcpyDeviceToHost,
                                       s));
                st = read_status(P);
            }
            if (st)
                nan_out(o);
            else
                std::memcpy(o, host_out, sizeof(double) * 3);
        } catch (const Error &e) {
            if (e.st == HODLR_EDEVICE)
                J->device_failed(e.msg);
            nan_out(o);
        } catch (...) {
            nan_out(o);
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(arena);
    (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" hodlr_status gp_loglik_ragged(int32_t m, const int64_t *ns, const double *const *xs,
                                         const double *const *ys, int32_t dim, hodlr_kernel k,
                                         const double *params, int32_t leaf, double tol,
                                         const hodlr_opts *opts, int32_t nworkers, double *out)
{
    try {
        if (m < 1 || !ns || !xs || !ys || !params || !out || dim < 1 || dim > 3 || leaf < 1 ||
            k < HODLR_K_SE || k > HODLR_K_IMQ || !(tol > 0.0) || !std::isfinite(tol))
            return report(HODLR_EINVAL, "bad shared argument");
        if (opts && opts->noise)
            return report(HODLR_EINVAL, "per-point noise is taken by hodlr_build and gp_loglik only");
        if (opts && opts->compressor != HODLR_COMPRESS_ACA)
            return report(HODLR_EINVAL, "the uneven-size form compresses by cross approximation only");
        RaggedJob J;
        J.m = m;
        J.ns = ns;
        J.xs = xs;
        J.ys = ys;
        J.dim = dim;
        J.kernel = k;
        J.params = params;
        J.leaf = leaf;
        J.tol = tol;
        if (opts) {
            J.opts = *opts;
        } else {
            J.opts.max_rank = 64;
            J.opts.precision = HODLR_FP64;
            J.opts.refine_tol = 1e-10;
            J.opts.max_refine = 8;
            J.opts.presorted = 0;
            J.opts.noise = nullptr;
            J.opts.refine = 0;
            J.opts.mixed_unchecked = 0;
            J.opts.compressor = HODLR_COMPRESS_ACA;
            J.opts.speculate = 0;
            J.opts.level_form = 0;
        }
        if (J.opts.max_rank < 0 || J.opts.max_rank > RMAX_ABS ||
            (J.opts.precision != HODLR_FP64 && J.opts.precision != HODLR_MIXED) ||
            (J.opts.level_form != 0 && J.opts.level_form != 1))
            return report(HODLR_EINVAL, "unsupported options");
        J.out = out;
        J.order.resize(m);
        std::iota(J.order.begin(), J.order.end(), 0);
        std::stable_sort(J.order.begin(), J.order.end(),
                         [&](int a, int b) { return ns[a] > ns[b]; });
        // arena size from the largest item (layouts grow with n)
        int64_t nmax = 1;
        for (int i = 0; i < m; ++i)
            nmax = std::max(nmax, ns[i]);
        // the largest item with the smallest level chunks (256 rows: the most
        // partial-sum records) bounds every item's layout
        Plan big;
        plan_build(big, nmax, dim, leaf, &J.opts, 256, 4, 8);
        std::vector<char> img;
        size_t tb = plan_image(big, img);
        big.precision = HODLR_FP64;   // room for an FP64 redo of a mixed item
        Layout lay = make_layout(big, false);
        J.arena = a256(lay.total) + a256(tb) + 2 * a256(sizeof(double) * nmax * (dim + 1)) + 4096;
        if (hipGetDevice(&J.device) != hipSuccess)
            return report(HODLR_EDEVICE, "no current device");
        prime_level_attributes();   // before the workers launch anything
        int nw = nworkers > 0 ? nworkers : 8;
        nw = std::min(nw, m);
        std::vector<std::thread> pool;
        for (int w = 0; w < nw; ++w)
            pool.emplace_back(worker, &J);
        for (auto &t : pool)
            t.join();
        if (J.device_error)
            return report(HODLR_EDEVICE, J.msg);
        return HODLR_OK;
    } catch (const Error &e) {
        return report(e.st, e.msg);
    } catch (...) {
        return report(HODLR_EDEVICE, "unexpected exception");
    }
}
