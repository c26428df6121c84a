// Autotuner of the launch shape: leaf size (the block size of the finest
// level, which trades leaf work against tree depth) and the level stage's
// tiles (rows per chunk, columns per reduction step, columns per reduction
// work-group).  Candidates are timed on
// the caller's own problem (points, observations, hyperparameters), wall clock
// around the whole likelihood pipeline including its one synchronization, the
// best of `reps` runs after a warm-up.  Search: leaf sizes first with the
// default tiles, then the twelve tile shapes at the best leaf.  Results are
// cached per (ceil log2 n, dim, kernel, precision) for hodlr_tune_lookup.
#include <chrono>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>

#include "common.h"

using namespace hodlr;

namespace hodlr {
hodlr_status report(hodlr_status st, const std::string &msg);   // sets hodlr_last_error
void prime_level_attributes();
}  // namespace hodlr

namespace {

using Key = std::tuple<int, int, int, int>;
std::mutex g_mu;
std::map<Key, hodlr_tune_t> g_cache;

int ceil_log2(int64_t n)
{
    int l = 0;
    while (((int64_t)1 << l) < n)
        ++l;
    return l;
}

struct Dev {
    void *p = nullptr;
    explicit Dev(size_t b)
    {
        if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess)
            throw Error{HODLR_ENOMEM, "device allocation failed in the autotuner"};
    }
    ~Dev()
    {
        if (p)
            (void)hipFree(p);
    }
};

// best wall time (ms) of one likelihood for this configuration
double time_config(const double *x, int64_t n, int dim, int k, const double theta[2],
                   double sigma2, const double *y, double tol, const hodlr_opts &o, int leaf,
                   int rows, int cols, int grp, int reps, hipStream_t s)
{
    std::vector<int64_t> perm(n);
    if (o.presorted)
        std::iota(perm.begin(), perm.end(), 0);
    else
        order_points(x, n, dim, leaf, perm.data());
    Plan plan;
    plan_build(plan, n, dim, leaf, &o, rows, cols, grp);
    if (plan.leafmax > LEAF_MAX)
        throw Error{HODLR_EINVAL, "leaf candidate above 256"};
    plan_upload(plan);
    struct Guard {
        Plan &p;
        ~Guard() { plan_release(p); }
    } g{plan};
    Layout lay = make_layout(plan, false);
    Dev ws(lay.total), dx(sizeof(double) * n * dim), dy(sizeof(double) * n);
    std::vector<double> xs((size_t)n * dim), ys(n);
    for (int d = 0; d < dim; ++d)
        for (int64_t i = 0; i < n; ++i)
            xs[(size_t)d * n + i] = x[perm[i] * dim + d];
    for (int64_t i = 0; i < n; ++i)
        ys[i] = y[perm[i]];
    HIP_TRY(hipMemcpy(dx.p, xs.data(), sizeof(double) * xs.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dy.p, ys.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    Pipeline P;
    P.plan = &plan;
    P.lay = lay;
    P.ws = (char *)ws.p;
    P.stream = s;
    P.x = (const double *)dx.p;
    P.kp = make_kparams(k, dim, theta, sigma2);
    P.tol = tol;
    double *d_out = wsp<double>(P, lay.out);
    double best = 1e300;
    for (int r = -1; r < reps; ++r) {   // r = -1: warm-up
        HIP_TRY(hipStreamSynchronize(s));
        auto t0 = std::chrono::steady_clock::now();
        factor_pipeline(P, (const double *)dy.p, d_out);
        const int st = read_status(P);   // synchronizes
        auto t1 = std::chrono::steady_clock::now();
        if (st)
            throw Error{HODLR_ENOTSPD, "the tuning problem is not positive definite"};
        if (r >= 0)
            best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    return best;
}

}  // namespace

extern "C" {

hodlr_status hodlr_plan_tuned_create(int64_t n, int32_t dim, const hodlr_opts *opts,
                                     const hodlr_tune_t *tune, hodlr_plan *out);

hodlr_status hodlr_autotune(const double *x, int64_t n, int32_t dim, hodlr_kernel k,
                            const double theta[2], double sigma2, const double *y, double tol,
                            const hodlr_opts *opts, const int32_t *leaf_cands, int32_t nleaf,
                            int32_t reps, hodlr_tune_t *best, double *times_ms)
{
    try {
        if (!x || !y || !theta || !best || n < 1 || dim < 1 || dim > 3 ||
            k < HODLR_K_SE || k > HODLR_K_IMQ || !(tol > 0.0) || reps < 1 ||
            (nleaf > 0 && !leaf_cands) || nleaf < 0)
            return report(HODLR_EINVAL, "bad autotune argument");
        hodlr_opts o;
        if (opts) {
            o = *opts;
        } else {
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
        }
        if (o.compressor != HODLR_COMPRESS_ACA)
            return report(HODLR_EINVAL, "the autotuner times cross approximation only");
        if (o.max_rank < 0 || o.max_rank > RMAX_ABS ||
            (o.precision != HODLR_FP64 && o.precision != HODLR_MIXED))
            return report(HODLR_EINVAL, "unsupported options");
        if (o.noise)
            return report(HODLR_EINVAL, "per-point noise is taken by hodlr_build and gp_loglik only");
        std::vector<int> leaves;
        if (nleaf > 0)
            leaves.assign(leaf_cands, leaf_cands + nleaf);
        else
            leaves = {32, 64, 96, 128};
        for (int l : leaves)
            if (l < 1 || l > LEAF_MAX)
                return report(HODLR_EINVAL, "leaf candidates must be in [1, 256]");
        prime_level_attributes();
        hipStream_t s = nullptr;
        HIP_TRY(hipStreamCreate(&s));
        struct SGuard {
            hipStream_t s;
            ~SGuard() { (void)hipStreamDestroy(s); }
        } sg{s};
        int slot = 0;
        double bt = 1e300;
        hodlr_tune_t b{leaves[0], LVL_ROWS, 4, 8};
        for (int l : leaves) {
            const double t = time_config(x, n, dim, k, theta, sigma2, y, tol, o, l, LVL_ROWS, 4, 8,
                                         reps, s);
            if (times_ms)
                times_ms[slot] = t;
            ++slot;
            if (t < bt) {
                bt = t;
                b = {l, LVL_ROWS, 4, 8};
            }
        }
        const int rows_c[3] = {256, 512, 1024}, cols_c[2] = {4, 8}, grp_c[2] = {8, 64};
        const int leaf = b.leaf;
        for (int rr : rows_c)
            for (int cc : cols_c)
                for (int gg : grp_c) {
                    const double t = time_config(x, n, dim, k, theta, sigma2, y, tol, o, leaf, rr,
                                                 cc, gg, reps, s);
                    if (times_ms)
                        times_ms[slot] = t;
                    ++slot;
                    if (t < bt) {
                        bt = t;
                        b = {leaf, rr, cc, gg};
                    }
                }
        *best = b;
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[Key{ceil_log2(n), dim, (int)k, o.precision}] = b;
        return HODLR_OK;
    } catch (const Error &e) {
        return report(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return report(HODLR_ENOMEM, "host allocation failed");
    } catch (...) {
        return report(HODLR_EDEVICE, "unexpected exception");
    }
}

hodlr_status hodlr_tune_lookup(int64_t n, int32_t dim, hodlr_kernel k, int32_t precision,
                               hodlr_tune_t *out)
{
    if (!out || n < 1)
        return report(HODLR_EINVAL, "bad lookup argument");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(Key{ceil_log2(n), dim, (int)k, precision});
    if (it == g_cache.end())
        return report(HODLR_EINVAL, "no tuned configuration for this problem class");
    *out = it->second;
    return HODLR_OK;
}

}  // extern "C"
