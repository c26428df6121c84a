// HIP-event timing of the library's launches, per kernel kind.  Events are
// recorded on the stream a kernel is launched on; elapsed times are read
// only after the call has synchronized that stream.
#include <atomic>
#include <cstring>
#include <mutex>

#include "common.h"

namespace hodlr {

namespace {
struct Rec {
    hipEvent_t a, b;
    int stage;
};
struct Prof {
    std::atomic<bool> on{false};
    std::atomic<uint32_t> mask{~0u};   // bit s: time stage s
    std::mutex mu;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[PS_COUNT] = {};
    int64_t cnt[PS_COUNT] = {};
};
Prof &P()
{
    static Prof *p = new Prof();   // never destroyed: outlives the HIP runtime teardown
    return *p;
}
const char *kNames[PS_COUNT] = {"aca_row_pass", "aca_col_pass", "aca_small", "aca_misc",
                                "leaf_factor",
                                "leaf_solve",   "level_reduce", "level_solve", "level_update",
                                "finish",       "matvec",      "predict",
                                "sketch",       "sketch_core"};

hipEvent_t take(Prof &p)
{
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}
}  // namespace

thread_local bool t_suspended = false;

bool prof_on(int stage)
{
    if (t_suspended)
        return false;
    Prof &p = P();
    return p.on.load(std::memory_order_relaxed) &&
           ((p.mask.load(std::memory_order_relaxed) >> stage) & 1u);
}

void prof_suspend(bool on) { t_suspended = on; }

int prof_begin(hipStream_t s)
{
    Prof &p = P();
    std::lock_guard<std::mutex> g(p.mu);
    Rec r{take(p), take(p), -1};
    if (!r.a || !r.b)
        return -1;
    if (hipEventRecord(r.a, s) != hipSuccess)
        return -1;
    p.pending.push_back(r);
    return (int)p.pending.size() - 1;
}

void prof_end(int slot, hipStream_t s, int stage)
{
    Prof &p = P();
    std::lock_guard<std::mutex> g(p.mu);
    if (slot < 0 || slot >= (int)p.pending.size())
        return;
    p.pending[slot].stage = stage;
    (void)hipEventRecord(p.pending[slot].b, s);
}

void prof_collect()
{
    if (t_suspended)
        return;   // records of other calls stay pending for their own collection
    Prof &p = P();
    std::lock_guard<std::mutex> g(p.mu);
    for (Rec &r : p.pending) {
        float ms = 0.f;
        if (r.stage >= 0 && hipEventSynchronize(r.b) == hipSuccess &&
            hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            p.ms[r.stage] += ms;
            p.cnt[r.stage] += 1;
        }
        p.pool.push_back(r.a);
        p.pool.push_back(r.b);
    }
    p.pending.clear();
}

}  // namespace hodlr

extern "C" {

hodlr_status hodlr_profile_enable(int32_t on)
{
    using namespace hodlr;
    Prof &p = P();
    {
        std::lock_guard<std::mutex> g(p.mu);
        if (on) {
            std::memset(p.ms, 0, sizeof(p.ms));
            std::memset(p.cnt, 0, sizeof(p.cnt));
        }
    }
    p.on.store(on != 0);
    return HODLR_OK;
}

hodlr_status hodlr_profile_select(uint32_t mask)
{
    hodlr::P().mask.store(mask);
    return HODLR_OK;
}

hodlr_status hodlr_profile_read(hodlr_profile_t *out)
{
    using namespace hodlr;
    if (!out)
        return HODLR_EINVAL;
    // calls that return without synchronizing (the batched form) leave their
    // records pending: wait for their events and add them first
    prof_collect();
    Prof &p = P();
    std::lock_guard<std::mutex> g(p.mu);
    std::memset(out, 0, sizeof(*out));
    out->nstages = PS_COUNT;
    for (int i = 0; i < PS_COUNT; ++i) {
        std::strncpy(out->name[i], kNames[i], 31);
        out->ms[i] = p.ms[i];
        out->launches[i] = p.cnt[i];
    }
    return HODLR_OK;
}

}  // extern "C"
