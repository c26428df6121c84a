// The plan handle of the C ABI and the argument checks its entry points
// share.
#pragma once

#include <algorithm>
#include <mutex>

#include "common.h"

namespace hodlr {
void check_params(int k, const double theta[2], double sigma2, double tol);
hodlr_status report(hodlr_status st, const std::string &msg);
}  // namespace hodlr

// graph of the synchronization-free stages of a batched call, valid for one
// column layout and one set of buffers
struct BatchGraph {
    std::vector<int> rmax;
    const void *ws, *x, *y, *params, *out;
    int64_t ystride;
    void *stream;
    int kind, nitems;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct hodlr_plan_s {
    hodlr::Plan plan;
    hodlr::Layout lay;
    hodlr_opts opts;
    // mixed plans: the same tree with FP64 panels (sharing the device tables)
    // for likelihoods whose mixed log-det error bound misses the bar
    hodlr::Plan plan64;
    hodlr::Layout lay64;
    void make_fp64_shadow()
    {
        if (!plan.f32())
            return;
        plan64 = plan;
        plan64.precision = HODLR_FP64;
        lay64 = hodlr::make_layout(plan64, false);
    }
    // one likelihood (gp_loglik_dev): room for the FP64 redo of a mixed plan
    size_t single_bytes() const { return plan.f32() ? std::max(lay.total, lay64.total) : lay.total; }
    std::vector<BatchGraph> graphs;
    // ranks of the last gp_loglik_dev call that completed (per node and per
    // depth) or of the last batched call's compression (per depth, maxima over
    // its items) for hodlr_plan_info
    std::mutex last_mu;
    std::vector<int> last_ranks, last_rmax;
    int last_capped = 0;
    int last_fallback = 0;   // likelihoods of the last call redone with FP64 panels
    // panel widths per depth index of the last completed gp_loglik_dev (the
    // widths a speculative call assumes); empty before the first
    std::vector<int> spec_rmax;
    int last_proj = 0;       // 1: the last gp_loglik_dev ran the projected levels
    int last_spec = 0;       // 1: the last gp_loglik_dev ran speculatively without a redo
    ~hodlr_plan_s()
    {
        for (auto &g : graphs) {
            if (g.exec)
                (void)hipGraphExecDestroy(g.exec);
            if (g.graph)
                (void)hipGraphDestroy(g.graph);
        }
    }
};
