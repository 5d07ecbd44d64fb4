// extern "C" entry points of libawg: context, plan, synthesis, streaming.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "awg_internal.h"

using namespace awg;

namespace {

constexpr uint64_t kHybridMin = 1ull << 16;           // shortest request for the hybrid path
constexpr uint64_t kMaxSample = 1ull << 63;          // n0 + count must stay below
constexpr size_t kTablePtrCap = 1024;                 // distinct smooth tables per plan
constexpr size_t kSlots = 16;                         // retune staging slots
constexpr size_t kSlotRecords = 16384;                // events per call (records per slot)

awg_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    if (e == hipErrorOutOfMemory) return AWG_E_NOMEM;
    return AWG_E_HIP;
}

bool smooth(int32_t shape) { return shape == AWG_RAMP_COSINE || shape == AWG_RAMP_MINJERK; }

// Fill H_N[0..N] with up to 8 host threads.
void fill_table(int32_t shape, uint64_t n, uint64_t *out)
{
    unsigned nt = std::thread::hardware_concurrency();
    if (nt == 0) nt = 1;
    if (nt > 8) nt = 8;
    if (n < 65536) nt = 1;
    auto work = [=](unsigned id) {
        const uint64_t total = n + 1;
        const uint64_t b = total * id / nt, e = total * (id + 1) / nt;
        for (uint64_t d = b; d < e; ++d)
            out[d] = (uint64_t)(shape == AWG_RAMP_MINJERK ? minjerk_entry(n, d) : cosine_entry(n, d));
    };
    if (nt == 1) { work(0); return; }
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nt; ++i) th.emplace_back(work, i);
    for (auto &t : th) t.join();
}

// Words of one tone with one (optional) window, starting from the line (p, f).
awg_status tone_words(const awg_plan_params &pp, uint64_t p_line, uint64_t f_line, int32_t shape,
                      uint64_t a, uint64_t n, double f_end, ToneHost *t)
{
    t->p0 = p_line;
    t->f0 = f_line;
    t->shape = shape;
    if (shape == AWG_RAMP_NONE) {
        t->p1 = p_line; t->f1 = f_line; t->a = UINT64_MAX; t->n = 0; t->coef = 0;
        return AWG_OK;
    }
    if (!(shape == AWG_RAMP_LINEAR || smooth(shape))) return AWG_E_INVALID;
    if (n == 0 || n >= (1ull << 31)) return AWG_E_RANGE;
    if (a >= kMaxSample || n >= kMaxSample - a) return AWG_E_RANGE;
    uint64_t f1;
    awg_status st = freq_word(f_end, pp.fs_hz, pp.period_log2, &f1);
    if (st != AWG_OK) return st;
    const int64_t dF = (int64_t)(f1 - f_line);      // both < 2^63
    t->f1 = f1;
    t->a = a;
    t->n = n;
    t->coef = shape == AWG_RAMP_LINEAR ? rne_div(dF, n) : dF;
    const uint64_t end = a + n;
    const uint64_t phi_end = p_line + f_line * end + chirp_end_term(shape, t->coef, dF, n);
    t->p1 = phi_end - f1 * end;
    return AWG_OK;
}

awg_status table_slot(awg_plan *p, int32_t shape, uint64_t n, uint16_t *idx, bool *added)
{
    *added = false;
    auto key = std::make_pair(shape, n);
    auto it = p->table_index.find(key);
    if (it != p->table_index.end()) { *idx = it->second; return AWG_OK; }
    if (p->table_ptrs.size() >= kTablePtrCap) return AWG_E_UNSUPPORTED;
    const uint64_t *d = nullptr;
    if (p->ctx) {
        awg_status st = get_table(p->ctx, shape, n, &d);
        if (st != AWG_OK) return st;
    }
    *idx = (uint16_t)p->table_ptrs.size();
    p->table_ptrs.push_back(d);
    p->table_index[key] = *idx;
    *added = true;
    return AWG_OK;
}

void free_plan_device(awg_plan *p)
{
    hybrid_release(p);
    if (p->d_tones) (void)hipFree(p->d_tones);
    if (p->d_blocks) (void)hipFree(p->d_blocks);
    if (p->d_table_ptrs) (void)hipFree(p->d_table_ptrs);
    if (p->work_done) {
        (void)hipEventSynchronize(p->work_done);
        (void)hipEventDestroy(p->work_done);
        p->work_done = nullptr;
    }
    if (p->d_work) (void)hipFree(p->d_work);
    for (auto &s : p->slots) {
        // the device reads the slots in place: their last readers finish first
        if (s.done && s.used) (void)hipEventSynchronize(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    p->slots.clear();
}

awg_status check_range(uint64_t n0, uint64_t count)
{
    if (n0 >= kMaxSample || count > kMaxSample - n0) return AWG_E_RANGE;
    return AWG_OK;
}

// An output buffer must be device (or managed) memory of the plan's device, and
// [d, d + count * elem) must lie inside one allocation when the runtime can say
// which (a host pointer here would make the kernels fault). Runtime errors of
// the queries are cleared so that they do not surface at a later launch.
awg_status check_out(const awg_plan *p, const void *d, uint64_t count, size_t elem)
{
    if (!d) return AWG_E_INVALID;
    if (count > SIZE_MAX / elem) return AWG_E_INVALID;
    const size_t bytes = (size_t)count * elem;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, d) != hipSuccess) {
        (void)hipGetLastError();
        return AWG_E_INVALID;
    }
    const bool managed = a.type == hipMemoryTypeManaged || a.isManaged;
    if (!managed && (a.type != hipMemoryTypeDevice || a.device != p->ctx->device)) return AWG_E_INVALID;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)d) == hipSuccess) {
        const size_t off = (size_t)((const char *)d - (const char *)base);
        if ((const char *)d < (const char *)base || off > size || bytes > size - off) return AWG_E_INVALID;
    } else {
        (void)hipGetLastError();
    }
    return AWG_OK;
}

awg_status device_ready(awg_plan *p)
{
    if (!p) return AWG_E_INVALID;
    if (!p->ctx) return AWG_E_INVALID;
    hipError_t e = hipSetDevice(p->ctx->device);
    return hip_status(e);
}

// The block table's offset in a retune slot: after the records of one call
// (at most one per tone, at most kSlotRecords), 16-byte aligned.
size_t slot_block_offset(const awg_plan *p)
{
    const size_t recs = std::min(kSlotRecords, (size_t)p->n_tones);
    return (sizeof(ScatterRecord) * recs + 15) / 16 * 16;
}

// Starts the duplicate-tone check of one event list.
void begin_event_check(awg_plan *p)
{
    if (p->ev_stamp.size() != (size_t)p->n_tones) {
        p->ev_stamp.assign((size_t)p->n_tones, 0);
        p->ev_gen = 0;
    }
    if (++p->ev_gen == 0) {                      // wrapped: clear the stamps
        std::fill(p->ev_stamp.begin(), p->ev_stamp.end(), 0);
        p->ev_gen = 1;
    }
}

// True when tone t was already named since begin_event_check.
bool seen_tone(awg_plan *p, int32_t t)
{
    if (p->ev_stamp[t] == p->ev_gen) return true;
    p->ev_stamp[t] = p->ev_gen;
    return false;
}

}  // namespace

static awg_status flush_locked(awg_plan *p, hipStream_t s);

namespace awg {

awg_status flush_tones(awg_plan *p, hipStream_t s)
{
    std::lock_guard<std::mutex> g(p->pend_mu);
    return flush_locked(p, s);
}

void take_pending_tones(awg_plan *p, const void **mapped, int32_t *n, int32_t *slot)
{
    std::lock_guard<std::mutex> g(p->pend_mu);
    *slot = p->pend_slot;
    *n = p->pend_slot >= 0 ? p->pend_n : 0;
    *mapped = p->pend_slot >= 0 ? p->slots[(size_t)p->pend_slot].mapped : nullptr;
    p->pend_slot = -1;
    p->pend_n = 0;
}

awg_status pending_tones_applied(awg_plan *p, int32_t slot, hipStream_t s)
{
    std::lock_guard<std::mutex> g(p->pend_mu);
    auto &sl = p->slots[(size_t)slot];
    const hipError_t e = hipEventRecord(sl.done, s);
    sl.used = true;
    return hip_status(e);
}

// Device table of a smooth shape, shared through the context.
awg_status get_table(awg_ctx *ctx, int32_t shape, uint64_t n, const uint64_t **d_out)
{
    std::lock_guard<std::mutex> g(ctx->mu);
    auto key = std::make_pair(shape, n);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *d_out = (const uint64_t *)((uintptr_t)it->second.d_data | (it->second.monotone ? 1u : 0u));
        return AWG_OK;
    }
    std::vector<uint64_t> h;
    try { h.resize(n + 1); } catch (...) { return AWG_E_NOMEM; }
    fill_table(shape, n, h.data());
    Table t;
    t.shape = shape;
    t.n = n;
    // tag for the kernels: never decreasing, steps below 2^19, so that the
    // rise over a lane's 16 samples stays below 2^23 (the smooth shapes step by
    // at most 2^16 + 1)
    t.monotone = true;
    for (uint64_t d = 0; d < n && t.monotone; ++d)
        t.monotone = h[d + 1] >= h[d] && h[d + 1] - h[d] < (1ull << 19);
    hipError_t e = hipMalloc((void **)&t.d_data, (n + 1) * sizeof(uint64_t));
    if (e != hipSuccess) return hip_status(e);
    e = hipMemcpy(t.d_data, h.data(), (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(t.d_data); return hip_status(e); }
    ctx->tables[key] = t;
    *d_out = (const uint64_t *)((uintptr_t)t.d_data | (t.monotone ? 1u : 0u));
    return AWG_OK;
}

}  // namespace awg

extern "C" {

int32_t awg_version(void) { return 100; }

const char *awg_strerror(awg_status s)
{
    switch (s) {
    case AWG_OK: return "ok";
    case AWG_E_INVALID: return "invalid argument";
    case AWG_E_NOMEM: return "out of memory";
    case AWG_E_HIP: return "HIP runtime error";
    case AWG_E_RANGE: return "value out of range";
    case AWG_E_UNSUPPORTED: return "unsupported request";
    case AWG_E_BUSY: return "busy";
    }
    return "unknown status";
}

awg_status awg_ctx_create(int device, awg_ctx **out)
{
    if (!out) return AWG_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return AWG_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return AWG_E_HIP;
    awg_ctx *c = new (std::nothrow) awg_ctx();
    if (!c) return AWG_E_NOMEM;
    c->device = device;
    // once per device, with the device current: the address of its copy of the
    // allocation-free peak call's scratch array
    if (noalloc_scratch(device, &c->noalloc_scratch) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return AWG_E_HIP;
    }
    *out = c;
    return AWG_OK;
}

void awg_ctx_destroy(awg_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->tables) (void)hipFree(kv.second.d_data);
    for (auto &r : ctx->prof_pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    delete ctx;
}

awg_status awg_ramp_table(int32_t shape, uint64_t n, uint64_t *out)
{
    if (!out || !smooth(shape)) return AWG_E_INVALID;
    if (n == 0 || n >= (1ull << 31)) return AWG_E_RANGE;
    fill_table(shape, n, out);
    return AWG_OK;
}

awg_status awg_plan_tones(awg_ctx *ctx, const awg_plan_params *params, const awg_tone *tones,
                          int32_t n_tones, awg_plan **out, double *f_quantised_hz)
{
    if (!out) return AWG_E_INVALID;
    *out = nullptr;
    if (!params || !tones || n_tones <= 0) return AWG_E_INVALID;
    const awg_plan_params pp = *params;
    if (!std::isfinite(pp.fs_hz) || !(pp.fs_hz > 0.0)) return AWG_E_INVALID;
    if (!std::isfinite(pp.gain_lsb) || pp.gain_lsb < 0.0) return AWG_E_INVALID;
    if (pp.period_log2 == 1 || pp.period_log2 > 63) return AWG_E_INVALID;
    if ((pp.flags & ~AWG_F_METHOD_MASK) != 0 || (pp.flags & AWG_F_METHOD_MASK) == 3) return AWG_E_INVALID;
    double asum = 0.0;
    for (int32_t k = 0; k < n_tones; ++k) {
        const awg_tone &t = tones[k];
        if (!std::isfinite(t.f_start_hz) || !std::isfinite(t.amplitude) ||
            !std::isfinite(t.phase_turns) || !(t.amplitude >= 0.0) || t.reserved != 0)
            return AWG_E_INVALID;
        if (t.ramp < AWG_RAMP_NONE || t.ramp > AWG_RAMP_MINJERK) return AWG_E_INVALID;
        if (t.ramp != AWG_RAMP_NONE && !std::isfinite(t.f_end_hz)) return AWG_E_INVALID;
        asum += std::fabs(t.amplitude);
    }
    double gain = pp.gain_lsb;
    if (gain == 0.0) {
        if (!(asum > 0.0)) return AWG_E_INVALID;
        gain = 32767.0 / asum;
    }

    awg_plan *p = new (std::nothrow) awg_plan();
    if (!p) return AWG_E_NOMEM;
    p->ctx = ctx;
    p->params = pp;
    p->gain = gain;
    p->n_tones = n_tones;
    p->n_ramped = 0;
    p->d_tones = nullptr;
    p->d_table_ptrs = nullptr;
    p->d_table_ptrs_cap = 0;
    p->cursor = 0;
    p->device_bytes = 0;
    p->next_slot = 0;
    p->d_work = nullptr;
    p->hyb = nullptr;
    p->d_work_bytes = 0;
    p->mfma_b_key = 0;
    p->d_blocks = nullptr;
    std::vector<uint16_t> tidx;
    try {
        p->host.resize(n_tones);
        p->dev_mirror.resize(n_tones);
        p->perm.resize(n_tones);
        p->inv.resize(n_tones);
        tidx.resize(n_tones);
    } catch (...) { delete p; return AWG_E_NOMEM; }

    awg_status st = AWG_OK;
    if (ctx && hipSetDevice(ctx->device) != hipSuccess) st = AWG_E_HIP;
    for (int32_t k = 0; k < n_tones && st == AWG_OK; ++k) {
        const awg_tone &t = tones[k];
        uint64_t f0;
        st = freq_word(t.f_start_hz, pp.fs_hz, pp.period_log2, &f0);
        if (st != AWG_OK) break;
        ToneHost &h = p->host[k];
        st = tone_words(pp, phase_word(t.phase_turns), f0, t.ramp, t.ramp_start, t.ramp_len,
                        t.f_end_hz, &h);
        if (st != AWG_OK) break;
        h.amp = t.amplitude * gain;
        h.ashape = AWG_RAMP_NONE;
        h.b = UINT64_MAX;
        h.m = 0;
        h.amp1 = h.amp;
        uint16_t idx = 0;
        if (smooth(t.ramp)) {
            bool added;
            st = table_slot(p, t.ramp, t.ramp_len, &idx, &added);
            if (st != AWG_OK) break;
        }
        if (t.ramp != AWG_RAMP_NONE) p->n_ramped++;
        tidx[k] = idx;
        if (f_quantised_hz) f_quantised_hz[k] = (double)f0 * pp.fs_hz * 0x1p-64;
    }
    if (st == AWG_OK) {
        // device order: tones that share shape and window next to each other, so
        // the kernel's blocks mostly take one regime per tile (stable: the
        // caller's order within a group, identity for all-static plans)
        for (int32_t k = 0; k < n_tones; ++k) p->perm[k] = k;
        std::stable_sort(p->perm.begin(), p->perm.end(), [&](int32_t x, int32_t y) {
            const ToneHost &a = p->host[x], &b = p->host[y];
            if (a.shape != b.shape) return a.shape < b.shape;
            if (a.a != b.a) return a.a < b.a;
            if (a.n != b.n) return a.n < b.n;
            return tidx[x] < tidx[y];
        });
        for (int32_t i = 0; i < n_tones; ++i) {
            p->inv[p->perm[i]] = i;
            p->dev_mirror[i] = to_device(p->host[p->perm[i]], tidx[p->perm[i]]);
        }
        build_blocks(p->dev_mirror, -1, &p->blocks);
    }
    const size_t blocks_cap = sizeof(Block) * ((size_t)n_tones + 1);     // largest possible table
    if (st == AWG_OK && ctx) {
        hipError_t e = hipMalloc((void **)&p->d_tones, sizeof(ToneDev) * (size_t)n_tones);
        if (e == hipSuccess) e = hipMalloc((void **)&p->d_blocks, blocks_cap);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_blocks, p->blocks.data(), sizeof(Block) * p->blocks.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_tones, p->dev_mirror.data(), sizeof(ToneDev) * (size_t)n_tones,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc((void **)&p->d_table_ptrs, sizeof(uint64_t *) * kTablePtrCap);
        if (e == hipSuccess) {
            p->d_table_ptrs_cap = kTablePtrCap;
            std::vector<const uint64_t *> ptrs(kTablePtrCap, nullptr);
            for (size_t i = 0; i < p->table_ptrs.size(); ++i) ptrs[i] = p->table_ptrs[i];
            e = hipMemcpy(p->d_table_ptrs, ptrs.data(), sizeof(uint64_t *) * kTablePtrCap,
                          hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) st = hip_status(e);
        p->device_bytes = sizeof(ToneDev) * (size_t)n_tones + sizeof(uint64_t *) * kTablePtrCap + blocks_cap;
    }
    if (st != AWG_OK) {
        free_plan_device(p);
        delete p;
        return st;
    }
    *out = p;
    return AWG_OK;
}

void awg_plan_destroy(awg_plan *p)
{
    if (!p) return;
    if (p->ctx) {
        (void)hipSetDevice(p->ctx->device);
        (void)hipDeviceSynchronize();
    }
    free_plan_device(p);
    delete p;
}

awg_status awg_plan_info_get(const awg_plan *p, awg_plan_info *info)
{
    if (!p || !info) return AWG_E_INVALID;
    info->n_tones = p->n_tones;
    info->n_ramped = p->n_ramped;
    info->gain_lsb = p->gain;
    info->flags = p->params.flags;
    info->period_log2 = p->params.period_log2;
    info->cursor = p->cursor;
    info->device_bytes = p->device_bytes + p->d_work_bytes + hybrid_bytes(p);
    return AWG_OK;
}

awg_status awg_plan_words(const awg_plan *p, uint64_t *p0, uint64_t *f0, uint64_t *f1, int64_t *coef)
{
    if (!p) return AWG_E_INVALID;
    for (int32_t k = 0; k < p->n_tones; ++k) {
        const ToneHost &h = p->host[k];
        if (p0) p0[k] = h.p0;
        if (f0) f0[k] = h.f0;
        if (f1) f1[k] = h.f1;
        if (coef) coef[k] = h.coef;
    }
    return AWG_OK;
}

static awg_status push_tones(awg_plan *p, const int32_t *changed, int32_t n_ev, hipStream_t s);

static bool windowed(const ToneHost &h) { return h.shape != AWG_RAMP_NONE || h.ashape != AWG_RAMP_NONE; }

awg_status awg_plan_retune(awg_plan *p, const awg_retune *ev, int32_t n_ev, void *hip_stream)
{
    if (!p || (n_ev > 0 && !ev) || n_ev < 0) return AWG_E_INVALID;
    if (n_ev == 0) return AWG_OK;
    if ((size_t)n_ev > kSlotRecords) return AWG_E_UNSUPPORTED;
    // validate all events first so that a failing call changes nothing
    try { begin_event_check(p); } catch (...) { return AWG_E_NOMEM; }
    std::vector<ToneHost> next;
    std::vector<uint16_t> tidx;
    try { next.resize(n_ev); tidx.resize(n_ev); } catch (...) { return AWG_E_NOMEM; }
    for (int32_t i = 0; i < n_ev; ++i) {
        const awg_retune &r = ev[i];
        if (r.tone < 0 || r.tone >= p->n_tones) return AWG_E_INVALID;
        if (!(r.ramp == AWG_RAMP_LINEAR || smooth(r.ramp))) return AWG_E_INVALID;
        if (!std::isfinite(r.f_end_hz)) return AWG_E_INVALID;
        if (seen_tone(p, r.tone)) return AWG_E_UNSUPPORTED;    // one window per tone and call
        const ToneHost &cur = p->host[r.tone];
        const uint64_t free_from = cur.shape == AWG_RAMP_NONE ? 0 : cur.a + cur.n;
        if (r.ramp_start < free_from) return AWG_E_RANGE;
        ToneHost h;
        awg_status st = tone_words(p->params, cur.p1, cur.f1, r.ramp, r.ramp_start, r.ramp_len,
                                   r.f_end_hz, &h);
        if (st != AWG_OK) return st;
        h.amp = cur.amp;
        h.ashape = cur.ashape;
        h.b = cur.b;
        h.m = cur.m;
        h.amp1 = cur.amp1;
        next[i] = h;
    }
    awg_status st = AWG_OK;
    for (int32_t i = 0; i < n_ev && st == AWG_OK; ++i) {
        tidx[i] = 0;
        if (smooth(ev[i].ramp)) {
            bool added;
            st = table_slot(p, ev[i].ramp, ev[i].ramp_len, &tidx[i], &added);
            if (st == AWG_OK && added && p->ctx) {
                hipError_t e = hipSetDevice(p->ctx->device);
                if (e == hipSuccess)
                    e = hipMemcpy(p->d_table_ptrs + tidx[i], &p->table_ptrs[tidx[i]], sizeof(uint64_t *),
                                  hipMemcpyHostToDevice);
                st = hip_status(e);
            }
        }
    }
    if (st != AWG_OK) return st;
    p->mfma_b_key = 0;
    std::vector<int32_t> changed(n_ev);
    for (int32_t i = 0; i < n_ev; ++i) {
        const int32_t k = ev[i].tone;
        if (!windowed(p->host[k])) p->n_ramped++;
        p->host[k] = next[i];
        p->dev_mirror[p->inv[k]] = to_device(next[i], tidx[i]);
        changed[i] = k;
    }
    return push_tones(p, changed.data(), n_ev, (hipStream_t)hip_stream);
}

awg_status awg_plan_amplitude(awg_plan *p, const awg_amp_ramp *ev, int32_t n_ev, void *hip_stream)
{
    if (!p || (n_ev > 0 && !ev) || n_ev < 0) return AWG_E_INVALID;
    if (n_ev == 0) return AWG_OK;
    if ((size_t)n_ev > kSlotRecords) return AWG_E_UNSUPPORTED;
    try { begin_event_check(p); } catch (...) { return AWG_E_NOMEM; }
    std::vector<ToneHost> next;
    try { next.resize(n_ev); } catch (...) { return AWG_E_NOMEM; }
    for (int32_t i = 0; i < n_ev; ++i) {
        const awg_amp_ramp &r = ev[i];
        if (r.tone < 0 || r.tone >= p->n_tones) return AWG_E_INVALID;
        if (!(r.ramp == AWG_RAMP_LINEAR || smooth(r.ramp))) return AWG_E_INVALID;
        if (!std::isfinite(r.amplitude_end) || r.amplitude_end < 0.0) return AWG_E_INVALID;
        if (seen_tone(p, r.tone)) return AWG_E_UNSUPPORTED;    // one window per tone and call
        if (r.ramp_len == 0 || r.ramp_len >= (1ull << 31)) return AWG_E_RANGE;
        if (r.ramp_start >= kMaxSample || r.ramp_len >= kMaxSample - r.ramp_start) return AWG_E_RANGE;
        const ToneHost &cur = p->host[r.tone];
        const uint64_t free_from = cur.ashape == AWG_RAMP_NONE ? 0 : cur.b + cur.m;
        if (r.ramp_start < free_from) return AWG_E_RANGE;
        ToneHost h = cur;
        h.amp = cur.ashape == AWG_RAMP_NONE ? cur.amp : cur.amp1;     // the amplitude it holds now
        h.amp1 = r.amplitude_end * p->gain;
        h.ashape = r.ramp;
        h.b = r.ramp_start;
        h.m = r.ramp_len;
        next[i] = h;
    }
    std::vector<int32_t> changed(n_ev);
    for (int32_t i = 0; i < n_ev; ++i) {
        const int32_t k = ev[i].tone;
        if (!windowed(p->host[k])) p->n_ramped++;
        const uint16_t table = p->dev_mirror[p->inv[k]].table;
        p->host[k] = next[i];
        p->dev_mirror[p->inv[k]] = to_device(next[i], table);
        changed[i] = k;
    }
    return push_tones(p, changed.data(), n_ev, (hipStream_t)hip_stream);
}

// Device copy of the tones changed on the host (caller indices), in stream order:
// their records are written to a pinned slot that the scatter kernel reads in
// place (for a plan on the line buffer, later: see flush_tones), and the rebuilt
// block table is uploaded from a slot by a kernel (no DMA engine in the chain).
// The retune staging slots, all at once on first use (or awg_plan_reserve);
// when an allocation fails none are kept, so a later call starts over.
static awg_status ensure_retune_slots(awg_plan *p)
{
    if (!p->slots.empty()) return AWG_OK;
    std::vector<awg_plan::Slot> v;
    try { v.resize(kSlots); } catch (...) { return AWG_E_NOMEM; }
    for (auto &sl : v) {
        sl.host = nullptr; sl.mapped = nullptr; sl.done = nullptr; sl.used = false;
    }
    hipError_t e = hipSuccess;
    for (auto &sl : v) {
        e = alloc_upload_host(slot_block_offset(p) + sizeof(Block) * ((size_t)p->n_tones + 1), &sl.host, &sl.mapped);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) break;
    }
    if (e != hipSuccess) {
        for (auto &sl : v) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
        return hip_status(e);
    }
    p->slots.swap(v);
    return AWG_OK;
}

// The pending records applied on s (p->pend_mu held).
static awg_status flush_locked(awg_plan *p, hipStream_t s)
{
    if (p->pend_slot < 0) return AWG_OK;
    auto &slot = p->slots[(size_t)p->pend_slot];
    hipError_t e = launch_scatter_tones(p->d_tones, slot.mapped, p->pend_n, s);
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    if (e != hipSuccess) return hip_status(e);
    slot.used = true;
    p->pend_slot = -1;
    p->pend_n = 0;
    return AWG_OK;
}

static awg_status push_tones(awg_plan *p, const int32_t *changed, int32_t n_ev, hipStream_t s)
{
    if (p->plb) {
        int32_t pos[kSlotRecords];
        for (int32_t i = 0; i < n_ev; ++i) pos[i] = p->inv[changed[i]];
        plb_note_changed(p, pos, n_ev);
    }
    if (!p->ctx) {
        build_blocks(p->dev_mirror, -1, &p->blocks);
        return AWG_OK;
    }
    // the block table is rebuilt by the next call that reads it: the line-buffer
    // path (a stream of retunes and chunks) never does
    p->blocks_stale = true;
    // stage the new records; scatter them on the stream now, or (line-buffer
    // plans) leave them to the next call's first launch
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e != hipSuccess) return hip_status(e);
    awg_status st = ensure_retune_slots(p);
    if (st != AWG_OK) return st;
    std::unique_lock<std::mutex> pend(p->pend_mu, std::defer_lock);
    if (p->plb) {
        pend.lock();
        if ((st = flush_locked(p, s)) != AWG_OK) return st;       // one pending call at a time
    }
    const size_t si = p->next_slot;
    p->next_slot = (p->next_slot + 1) % kSlots;
    auto &slot = p->slots[si];
    if (slot.used) {
        e = hipEventSynchronize(slot.done);
        if (e != hipSuccess) return hip_status(e);
    }
    ScatterRecord *rec = (ScatterRecord *)slot.host;
    for (int32_t i = 0; i < n_ev; ++i) {
        rec[i].index = (uint32_t)p->inv[changed[i]];
        rec[i].pad = 0;
        rec[i].tone = p->dev_mirror[p->inv[changed[i]]];
    }
    if (p->plb) {
        slot.used = false;
        p->pend_slot = (int32_t)si;
        p->pend_n = n_ev;
        return AWG_OK;
    }
    e = launch_scatter_tones(p->d_tones, slot.mapped, n_ev, s);
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    slot.used = true;
    return hip_status(e);
}

// The plan's block table for its current tones, on the device in stream order
// before the caller's kernels (after retunes it is rebuilt here, staged in a
// retune slot and moved by the copy kernel).
static awg_status sync_blocks(awg_plan *p, hipStream_t s)
{
    if (!p->blocks_stale) return AWG_OK;
    build_blocks(p->dev_mirror, -1, &p->blocks);
    awg_status st = ensure_retune_slots(p);
    if (st != AWG_OK) return st;
    const size_t si = p->next_slot;
    p->next_slot = (p->next_slot + 1) % kSlots;
    auto &slot = p->slots[si];
    hipError_t e = slot.used ? hipEventSynchronize(slot.done) : hipSuccess;
    if (e != hipSuccess) return hip_status(e);
    Block *blk = (Block *)((char *)slot.host + slot_block_offset(p));
    const size_t blk_bytes = sizeof(Block) * p->blocks.size();
    std::memcpy(blk, p->blocks.data(), blk_bytes);
    e = launch_upload((const char *)slot.mapped + slot_block_offset(p), p->d_blocks, blk_bytes, s);
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    slot.used = true;
    if (e == hipSuccess) p->blocks_stale = false;
    return hip_status(e);
}

// Samples of any plan with the given method: the direct kernel; the matrix
// cores for static plans; the hybrid of both for ramped plans (short requests
// stay on the direct kernel, which gains nothing from the matrix cores there).
static awg_status synth_any(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16,
                            float *out_f32, hipStream_t s)
{
    // (the hybrid path applies pending retune records itself)
    if (method != AWG_F_METHOD_DIRECT && p->n_ramped > 0 && count >= kHybridMin)
        return hybrid_synth(p, method, n0, count, out_i16, out_f32, s);
    awg_status st = flush_tones(p, s);
    if (st != AWG_OK) return st;
    if (method != AWG_F_METHOD_DIRECT && p->n_ramped == 0) return mfma_static(p, method, n0, count, out_i16, out_f32, s);
    st = sync_blocks(p, s);
    if (st != AWG_OK) return st;
    return hip_status(out_f32 ? launch_direct_f32(p, n0, count, out_f32, s) : launch_direct_i16(p, n0, count, out_i16, s));
}

awg_status awg_plan_reserve(awg_plan *p, uint32_t method, uint64_t max_count)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (method > AWG_F_METHOD_MFMA_BF16X3) return AWG_E_INVALID;
    if ((st = ensure_retune_slots(p)) != AWG_OK) return st;
    if (method == AWG_F_METHOD_DIRECT || max_count < kHybridMin) return AWG_OK;
    // a static plan's matrix-core calls use the product workspace; a ramped
    // plan's take the hybrid path (and a plan retuned later may need both)
    if ((st = mfma_static_reserve(p, max_count)) != AWG_OK) return st;
    return p->n_ramped > 0 ? hybrid_reserve(p, method, max_count) : AWG_OK;
}

awg_status awg_synth_chirp(awg_plan *p, uint64_t n0, uint64_t count, int16_t *d_out, void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count == 0) return AWG_OK;
    if ((st = check_out(p, d_out, count, sizeof(int16_t))) != AWG_OK) return st;
    return synth_any(p, p->params.flags & AWG_F_METHOD_MASK, n0, count, d_out, nullptr, (hipStream_t)hip_stream);
}

awg_status awg_synth_static(awg_plan *p, uint64_t n0, uint64_t count, int16_t *d_out, void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (p->n_ramped > 0) return AWG_E_UNSUPPORTED;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count == 0) return AWG_OK;
    if ((st = check_out(p, d_out, count, sizeof(int16_t))) != AWG_OK) return st;
    if ((st = flush_tones(p, (hipStream_t)hip_stream)) != AWG_OK) return st;
    const uint32_t method = p->params.flags & AWG_F_METHOD_MASK;
    if (method == AWG_F_METHOD_DIRECT) {
        if ((st = sync_blocks(p, (hipStream_t)hip_stream)) != AWG_OK) return st;
        return hip_status(launch_direct_i16(p, n0, count, d_out, (hipStream_t)hip_stream));
    }
    return mfma_static(p, method, n0, count, d_out, nullptr, (hipStream_t)hip_stream);
}

awg_status awg_synth_f32(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, float *d_y,
                         void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (method > AWG_F_METHOD_MFMA_BF16X3) return AWG_E_INVALID;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count == 0) return AWG_OK;
    if ((st = check_out(p, d_y, count, sizeof(float))) != AWG_OK) return st;
    return synth_any(p, method, n0, count, nullptr, d_y, (hipStream_t)hip_stream);
}

awg_status awg_stream_next(awg_plan *p, uint64_t count, int16_t *d_out, void *hip_stream, uint64_t *n0_out)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    const uint64_t n0 = p->cursor;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count > 0) {
        if ((st = check_out(p, d_out, count, sizeof(int16_t))) != AWG_OK) return st;
        st = synth_any(p, p->params.flags & AWG_F_METHOD_MASK, n0, count, d_out, nullptr,
                       (hipStream_t)hip_stream);
        if (st != AWG_OK) return st;
    }
    p->cursor = n0 + count;
    if (n0_out) *n0_out = n0;
    return AWG_OK;
}

awg_status awg_stream_seek(awg_plan *p, uint64_t n0)
{
    if (!p) return AWG_E_INVALID;
    if (n0 >= kMaxSample) return AWG_E_RANGE;
    p->cursor = n0;
    return AWG_OK;
}

awg_status awg_stream_tell(const awg_plan *p, uint64_t *n0)
{
    if (!p || !n0) return AWG_E_INVALID;
    *n0 = p->cursor;
    return AWG_OK;
}

static awg_status mux_items(awg_plan *const *plans, int32_t n, uint64_t n0, uint64_t count, int16_t *d_out,
                            BatchItem *items)
{
    if (!plans || n < 1 || n > kMaxChannels) return AWG_E_INVALID;
    for (int32_t c = 0; c < n; ++c) {
        awg_plan *p = plans[c];
        if (!p || !p->ctx || p->ctx->device != plans[0]->ctx->device) return AWG_E_INVALID;
        BatchItem &b = items[c];
        b.tones = p->d_tones;
        b.tables = p->d_table_ptrs;
        b.out = d_out + c;
        b.n0 = n0;
        b.count = count;
        b.tile_begin = 0;
        b.n_tones = p->n_tones;
        b.out_stride = n;
        b.is_static = p->n_ramped == 0;
        b.blocks = p->d_blocks;
    }
    return device_ready(plans[0]);
}

awg_status awg_synth_multiplex(awg_plan *const *plans, int32_t n_channels, uint64_t n0, uint64_t count,
                               int16_t *d_out, void *hip_stream)
{
    BatchItem items[kMaxChannels];
    awg_status st = mux_items(plans, n_channels, n0, count, d_out, items);
    if (st != AWG_OK) return st;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count == 0) return AWG_OK;
    if (count > UINT64_MAX / (uint64_t)n_channels) return AWG_E_INVALID;
    if ((st = check_out(plans[0], d_out, count * (uint64_t)n_channels, sizeof(int16_t))) != AWG_OK) return st;
    for (int32_t c = 0; c < n_channels; ++c) {
        if ((st = flush_tones(plans[c], (hipStream_t)hip_stream)) != AWG_OK) return st;
        if ((st = sync_blocks(plans[c], (hipStream_t)hip_stream)) != AWG_OK) return st;
    }
    ProfScope prof(plans[0]->ctx, (hipStream_t)hip_stream, "mux_kernel");
    for (int32_t c = 0; c < n_channels; ++c) prof.add_work((double)plans[c]->n_tones * (double)count);
    return hip_status(launch_mux(items, n_channels, count, (hipStream_t)hip_stream, prof));
}

awg_status awg_stream_next_multiplex(awg_plan *const *plans, int32_t n_channels, uint64_t count, int16_t *d_out,
                                     void *hip_stream, uint64_t *n0_out)
{
    if (!plans || n_channels < 1 || n_channels > kMaxChannels || !plans[0]) return AWG_E_INVALID;
    const uint64_t n0 = plans[0]->cursor;
    for (int32_t c = 0; c < n_channels; ++c)
        if (!plans[c] || plans[c]->cursor != n0) return AWG_E_INVALID;
    awg_status st = awg_synth_multiplex(plans, n_channels, n0, count, d_out, hip_stream);
    if (st != AWG_OK) return st;
    for (int32_t c = 0; c < n_channels; ++c) plans[c]->cursor = n0 + count;   // repeated plans: same value
    if (n0_out) *n0_out = n0;
    return AWG_OK;
}

awg_status awg_peak(awg_plan *p, uint64_t n0, uint64_t count, float *d_scratch, float *d_peak, void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (!d_scratch || !d_peak || count == 0) return AWG_E_INVALID;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if ((st = check_out(p, d_scratch, count, sizeof(float))) != AWG_OK) return st;
    if ((st = check_out(p, d_peak, 1, sizeof(float))) != AWG_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;
    if ((st = flush_tones(p, s)) != AWG_OK) return st;
    if ((st = sync_blocks(p, s)) != AWG_OK) return st;
    hipError_t e = launch_direct_f32(p, n0, count, d_scratch, s);
    if (e == hipSuccess) e = launch_peak(d_scratch, count, d_peak, s);
    return hip_status(e);
}

awg_status awg_peak_noalloc(awg_plan *p, uint64_t n0, uint64_t count, float *d_peak, void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (!d_peak || count == 0) return AWG_E_INVALID;
    if (count > AWG_PEAK_NOALLOC_MAX) return AWG_E_UNSUPPORTED;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if ((st = check_out(p, d_peak, 1, sizeof(float))) != AWG_OK) return st;
    float *scr = p->ctx->noalloc_scratch;      // this device's copy, never the symbol itself
    if (!scr) return AWG_E_HIP;
    hipStream_t s = (hipStream_t)hip_stream;
    // after a retune (whose call set up the staging slots) its pending records
    // and the block table are staged in them: no allocation here either
    if ((st = flush_tones(p, s)) != AWG_OK) return st;
    if ((st = sync_blocks(p, s)) != AWG_OK) return st;
    hipError_t e = launch_direct_f32(p, n0, count, scr, s, false);
    if (e == hipSuccess) e = launch_peak(scr, count, d_peak, s);
    return hip_status(e);
}

awg_status awg_phase_dump(awg_plan *p, int32_t tone, uint64_t n0, uint64_t count, uint64_t *d_words,
                          void *hip_stream)
{
    awg_status st = device_ready(p);
    if (st != AWG_OK) return st;
    if (tone < 0 || tone >= p->n_tones) return AWG_E_INVALID;
    if ((st = check_range(n0, count)) != AWG_OK) return st;
    if (count == 0) return AWG_OK;
    if ((st = check_out(p, d_words, count, sizeof(uint64_t))) != AWG_OK) return st;
    if ((st = flush_tones(p, (hipStream_t)hip_stream)) != AWG_OK) return st;
    return hip_status(launch_phase_dump(p, p->inv[tone], n0, count, d_words, (hipStream_t)hip_stream));
}

}  // extern "C"
