// Per-kernel event timing for awg_profile_*: each timed kernel's dispatch
// records a start and a stop event (hipExtLaunchKernel); one launch in
// `period` of each kernel is timed; totals are accumulated on read.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "awg_internal.h"

namespace awg {

// timed launches held between two reads; later launches go untimed until the
// next awg_profile_read folds the held ones into the totals
constexpr size_t kMaxPending = 65536;

// A fresh pair of events per timed launch, destroyed once read: an event that
// already took a launch's timestamps and is handed to hipExtLaunchKernel again
// stalls that dispatch (by up to a millisecond) and returns a wrong interval.
static hipEvent_t take_event()
{
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(awg_ctx *ctx, hipStream_t s, const char *name)
    : ctx_(ctx), s_(s), name_(name), start_(nullptr), stop_(nullptr), launched_(false)
{
    if (!ctx_) return;
    const int32_t period = ctx_->prof_period.load(std::memory_order_relaxed);
    if (period <= 0) return;
    std::lock_guard<std::mutex> g(ctx_->prof_mu);
    if (ctx_->prof_seen[name_]++ % (uint64_t)period != 0) return;
    if (ctx_->prof_pending.size() >= kMaxPending) return;
    start_ = take_event();
    stop_ = start_ ? take_event() : nullptr;
    if (!stop_ && start_) {
        (void)hipEventDestroy(start_);
        start_ = nullptr;
    }
}

ProfScope::~ProfScope()
{
    if (!stop_) return;
    std::lock_guard<std::mutex> g(ctx_->prof_mu);
    if (!launched_) {
        (void)hipEventDestroy(start_);
        (void)hipEventDestroy(stop_);
        return;
    }
    ctx_->prof_pending.push_back(ProfRecord{name_, start_, stop_, work_});
}

}  // namespace awg

using namespace awg;

extern "C" {

awg_status awg_profile_enable(awg_ctx *ctx, int32_t enable)
{
    if (!ctx) return AWG_E_INVALID;
    if (enable < 0) return AWG_E_INVALID;
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    ctx->prof_seen.clear();
    ctx->prof_period.store(enable, std::memory_order_relaxed);
    return AWG_OK;
}

awg_status awg_profile_read(awg_ctx *ctx, awg_kernel_stat *out, int32_t max_stats, int32_t *n_stats,
                            int32_t reset)
{
    if (!ctx || (max_stats > 0 && !out) || max_stats < 0) return AWG_E_INVALID;
    std::lock_guard<std::mutex> g(ctx->prof_mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return AWG_E_HIP;
    awg_status st = AWG_OK;
    for (auto &r : ctx->prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            st = AWG_E_HIP;
        ProfTotal &t = ctx->prof_totals[r.name];
        t.launches += 1;
        t.total_ms += ms;
        t.work += r.work;
        if (ms > t.max_ms) t.max_ms = ms;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    ctx->prof_pending.clear();
    int32_t i = 0;
    for (auto &kv : ctx->prof_totals) {
        if (i < max_stats) {
            std::memset(&out[i], 0, sizeof(awg_kernel_stat));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.launches;
            out[i].total_ms = kv.second.total_ms;
            out[i].max_ms = kv.second.max_ms;
            out[i].work = kv.second.work;
        }
        ++i;
    }
    if (n_stats) *n_stats = i;
    if (reset) ctx->prof_totals.clear();
    return st;
}

}  // extern "C"
