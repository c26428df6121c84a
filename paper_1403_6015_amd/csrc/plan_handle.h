// The plan handle of the C ABI (shared by the entry points of api.hip and
// noalloc.hip), and the argument checks they share.
#pragma once

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
    std::vector<BatchGraph> graphs;
    // host vectors of one pipeline, reserved at plan creation and lent to
    // gp_loglik_dev_noalloc so that its calls do no heap allocation
    std::vector<int> h_rmax, h_cols, h_cnt, h_ranks, h_ints;
    void reserve_host()
    {
        h_rmax.reserve(plan.L + 2);
        h_cols.reserve(plan.ncol + 1);
        h_cnt.reserve(plan.L + 1);
        h_ranks.reserve(std::max<int64_t>(plan.nint, 1));
        h_ints.assign(64, 0);
    }
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
