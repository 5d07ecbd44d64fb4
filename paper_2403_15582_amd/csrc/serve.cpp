// Batched serving of synthesis jobs (continuous batching) on one device.
//
// A job is a tone set with its own sample rate and length (for example one
// tweezer rearrangement: every tone chirps over the whole job). submit() plans
// its exact words on the host and queues it. A scheduler thread
//   * admits queued jobs in arrival order while job slots and device memory
//     (a first-fit arena for the jobs' tone tables) allow;
//   * forms a step from one chunk of every admitted job that has samples left,
//     no chunk in flight and a free slot in the device output ring, so jobs that
//     arrive while others run join the next step;
//   * launches the step as a replay of a captured hipGraph (work-list copy +
//     one batched kernel over all chunks' tiles) on its own stream, two steps
//     in flight at most;
//   * turns completed steps into chunk events (ring slot, samples, timing).
// The consumer (standing in for the DAC) polls events, reads the ring slot and
// releases it. Each chunk is computed by exactly the code of awg_synth_chirp, so
// a job's samples do not depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "awg_internal.h"

using namespace awg;

namespace {

constexpr uint32_t kBatchGrid = 2048;   // workgroups of the batched kernel (8 per CU)
constexpr size_t kItemsOffset = 256;    // work-list items after the 2-word header
constexpr size_t kAlign = 256;
constexpr size_t kStageInit = 512 * 1024;   // admission staging buffer set up at creation (~5000 tones)
constexpr size_t kStatWindow = 1u << 20;    // chunks whose latencies the percentiles cover

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Pending {
    uint64_t id, tag;
    double t_submit;
    awg_plan *plan;              // host-only plan: words and table keys
    uint64_t n_samples;
    double fs;
};

struct Job {
    uint64_t id, tag;
    double t_submit, t_admit, fs;
    awg_plan *plan;
    size_t off, bytes;           // arena block
    ToneDev *d_tones;
    const uint64_t **d_tabs;
    Block *d_blocks;
    int32_t n_tones, is_static;
    uint64_t n_samples, next_n0;
    uint32_t chunks_total, chunks_done;
    bool in_flight;
    double t_first_ready;
};

struct StepItem { uint64_t job; int32_t slot; uint64_t n0, count; uint32_t chunk; };

struct Step {
    bool in_flight = false;
    std::vector<StepItem> items;
    double t_launch = 0;
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    // the step's work list: one pinned coherent blob (header at 0, items at
    // kItemsOffset) that the step graph uploads by a kernel into d_blob
    void *h_blob = nullptr, *m_blob = nullptr, *d_blob = nullptr;
    BatchItem *h_items = nullptr;
    uint32_t *h_hdr = nullptr;
    BatchItem *d_items = nullptr;
    uint32_t *d_hdr = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

awg_status hipst(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    return e == hipErrorOutOfMemory ? AWG_E_NOMEM : AWG_E_HIP;
}

double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double r = p / 100.0 * (double)(v.size() - 1);
    const size_t i = (size_t)r;
    const double f = r - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct awg_server {
    awg_ctx *ctx;
    awg_server_params prm;
    hipStream_t stream = nullptr;
    char *d_arena = nullptr;
    size_t ring_bytes = 0, pool_bytes = 0, pool_off = 0;
    std::map<size_t, size_t> free_blocks;      // offset -> size (pool, relative to pool_off)
    std::vector<int> slot_state;               // 0 free, 1 scheduled, 2 held by the consumer
    Step steps[2];
    std::deque<Pending> pending;
    std::map<uint64_t, Job> jobs;              // admitted, by id (id order = arrival order)
    std::deque<awg_chunk_event> done;
    uint64_t next_id = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::thread th;
    bool stop = false;
    awg_status error = AWG_OK;
    // statistics
    uint64_t n_submitted = 0, n_admitted = 0, n_jobs_done = 0, n_chunks = 0, n_steps = 0;
    uint64_t n_items_total = 0, max_batch = 0, deadline_misses = 0;
    double tone_samples = 0, busy_ms = 0, t_first_submit = -1, t_last_ready = 0, audio_s = 0;
    // device rate (tone-samples per ms) measured on completed steps, for the step work budget
    double rate_ts_per_ms = 2e9;
    // latency samples of the most recent kStatWindow chunks (rings, oldest overwritten)
    struct Ring {
        std::vector<double> v;
        size_t next = 0;
        void add(double x)
        {
            if (v.size() < kStatWindow) v.push_back(x);
            else { v[next] = x; next = (next + 1) % kStatWindow; }
        }
    };
    Ring lat_chunk, lat_first, lateness;
    // admission staging: pinned coherent buffers holding a job's tables in their
    // arena layout, uploaded by a kernel; a buffer is reused once its upload is done
    struct Stage { void *host = nullptr, *mapped = nullptr; size_t cap = 0; hipEvent_t done = nullptr; bool used = false; };
    Stage stage[8];
    int stage_next = 0;
};

namespace {

bool pool_alloc(awg_server *s, size_t bytes, size_t *off)
{
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t roff = it->first + bytes;
            s->free_blocks.erase(it);
            if (rest) s->free_blocks[roff] = rest;
            return true;
        }
    }
    return false;
}

void pool_free(awg_server *s, size_t off, size_t bytes)
{
    auto nx = s->free_blocks.lower_bound(off);
    if (nx != s->free_blocks.end() && off + bytes == nx->first) {   // merge with the next block
        bytes += nx->second;
        nx = s->free_blocks.erase(nx);
    }
    if (nx != s->free_blocks.begin()) {                               // merge with the previous block
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += bytes;
            return;
        }
    }
    s->free_blocks[off] = bytes;
}

size_t job_bytes(const awg_plan *p)
{
    return align_up(sizeof(ToneDev) * (size_t)p->n_tones) + align_up(sizeof(uint64_t *) * (p->table_ptrs.size() + 1)) +
           align_up(sizeof(Block) * p->blocks.size());
}

// Admit queued jobs in order while a job slot and arena space are available.
void admit(awg_server *s)
{
    while (!s->pending.empty() && (int32_t)s->jobs.size() < s->prm.max_jobs) {
        Pending &pd = s->pending.front();
        const size_t bytes = job_bytes(pd.plan);
        size_t off;
        if (!pool_alloc(s, bytes, &off)) break;                      // wait for memory
        Job j;
        j.id = pd.id; j.tag = pd.tag; j.t_submit = pd.t_submit; j.t_admit = now_ms(); j.fs = pd.fs;
        j.plan = pd.plan; j.off = off; j.bytes = bytes;
        char *base = s->d_arena + s->pool_off + off;
        j.d_tones = (ToneDev *)base;
        j.d_tabs = (const uint64_t **)(base + align_up(sizeof(ToneDev) * (size_t)pd.plan->n_tones));
        j.d_blocks = (Block *)((char *)j.d_tabs + align_up(sizeof(uint64_t *) * (pd.plan->table_ptrs.size() + 1)));
        j.n_tones = pd.plan->n_tones;
        j.is_static = pd.plan->n_ramped == 0;
        j.n_samples = pd.n_samples;
        j.next_n0 = 0;
        j.chunks_total = (uint32_t)((pd.n_samples + s->prm.chunk_len - 1) / s->prm.chunk_len);
        j.chunks_done = 0;
        j.in_flight = false;
        j.t_first_ready = -1;
        // words, table pointers and block table into the arena, in stream order
        // before any step using them: laid out in a staging buffer as in the
        // arena, then one upload kernel
        awg_server::Stage &sg = s->stage[s->stage_next];
        s->stage_next = (s->stage_next + 1) % (int)(sizeof(s->stage) / sizeof(s->stage[0]));
        hipError_t e = hipSuccess;
        if (!sg.done) e = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming);
        if (e == hipSuccess && sg.used) e = hipEventSynchronize(sg.done);
        if (e == hipSuccess && sg.cap < bytes) {
            if (sg.host) (void)hipHostFree(sg.host);
            sg.host = sg.mapped = nullptr;
            sg.cap = 0;
            e = alloc_upload_host(std::max<size_t>(bytes, 1 << 16), &sg.host, &sg.mapped);
            if (e == hipSuccess) sg.cap = std::max<size_t>(bytes, 1 << 16);
        }
        if (e == hipSuccess) {
            sg.used = false;
            char *h = (char *)sg.host;
            std::memcpy(h, pd.plan->dev_mirror.data(), sizeof(ToneDev) * (size_t)j.n_tones);
            const size_t nt = pd.plan->table_ptrs.size();
            if (nt > 0) std::memcpy(h + ((char *)j.d_tabs - base), pd.plan->table_ptrs.data(), sizeof(uint64_t *) * nt);
            std::memcpy(h + ((char *)j.d_blocks - base), pd.plan->blocks.data(), sizeof(Block) * pd.plan->blocks.size());
            e = launch_upload(sg.mapped, base, bytes, s->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(sg.done, s->stream);
        if (e == hipSuccess) sg.used = true;
        if (e != hipSuccess) { s->error = hipst(e); pool_free(s, off, bytes); break; }
        s->jobs[j.id] = j;
        s->pending.pop_front();
        s->n_admitted++;
    }
}

// Harvest completed steps into chunk events.
void harvest(awg_server *s)
{
    for (auto &st : s->steps) {
        if (!st.in_flight) continue;
        const hipError_t q = hipEventQuery(st.ev_done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) { s->error = hipst(q); st.in_flight = false; continue; }
        const double t = now_ms();
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, st.ev_start, st.ev_done) == hipSuccess) {
            s->busy_ms += ms;
            double work = 0;
            for (const StepItem &it : st.items) {
                auto jt = s->jobs.find(it.job);
                if (jt != s->jobs.end()) work += (double)jt->second.n_tones * (double)it.count;
            }
            if (ms > 0.05f && work > 0) s->rate_ts_per_ms = 0.8 * s->rate_ts_per_ms + 0.2 * (work / ms);
        }
        for (const StepItem &it : st.items) {
            auto jt = s->jobs.find(it.job);
            if (jt == s->jobs.end()) continue;
            Job &j = jt->second;
            j.in_flight = false;
            j.chunks_done++;
            s->slot_state[it.slot] = 2;
            awg_chunk_event ev;
            ev.job_id = j.id;
            ev.user_tag = j.tag;
            ev.chunk_index = it.chunk;
            ev.n0 = it.n0;
            ev.count = it.count;
            ev.slot = it.slot;
            ev.last = j.chunks_done == j.chunks_total ? 1 : 0;
            ev.t_submit_ms = j.t_submit;
            ev.t_ready_ms = t;
            s->done.push_back(ev);
            s->n_chunks++;
            s->tone_samples += (double)j.n_tones * (double)it.count;
            s->audio_s += (double)it.count / j.fs;
            s->lat_chunk.add(t - j.t_submit);
            if (it.chunk == 0) s->lat_first.add(t - j.t_submit);
            const double deadline = j.t_submit + s->prm.playout_delay_ms + 1e3 * (double)it.n0 / j.fs;
            if (t > deadline) s->deadline_misses++;
            s->lateness.add(t - deadline);
            s->t_last_ready = t;
            if (ev.last) {
                pool_free(s, j.off, j.bytes);
                awg_plan_destroy(j.plan);
                s->jobs.erase(jt);
                s->n_jobs_done++;
            }
        }
        st.items.clear();
        st.in_flight = false;
    }
}

// Form and launch one step if a step buffer is free and there is work. The
// admitted jobs with a chunk to do are taken earliest deadline first (the
// deadline of a job's next chunk: arrival + playout delay + chunk start / fs),
// and a step stops growing at about a quarter of the playout delay of device
// work (at least 0.5 ms, at the measured rate), so that a chunk that falls due
// soon does not wait behind a long step; a step always takes at least one chunk.
bool launch_step(awg_server *s)
{
    Step *st = nullptr;
    for (auto &c : s->steps)
        if (!c.in_flight) { st = &c; break; }
    if (!st) return false;
    st->items.clear();
    std::vector<std::pair<double, Job *>> cand;
    for (auto &kv : s->jobs) {
        Job &j = kv.second;
        if (j.in_flight || j.next_n0 >= j.n_samples) continue;
        cand.emplace_back(j.t_submit + s->prm.playout_delay_ms + 1e3 * (double)j.next_n0 / j.fs, &j);
    }
    std::stable_sort(cand.begin(), cand.end(),
                     [](const std::pair<double, Job *> &a, const std::pair<double, Job *> &b) { return a.first < b.first; });
    const double budget = s->rate_ts_per_ms * std::max(0.5, s->prm.playout_delay_ms / 4.0);
    double work = 0;
    uint32_t tiles = 0;
    int32_t slot = 0;
    const int32_t n_slots = (int32_t)s->slot_state.size();
    for (auto &c : cand) {
        Job &j = *c.second;
        if ((int32_t)st->items.size() >= s->prm.max_jobs) break;
        while (slot < n_slots && s->slot_state[slot] != 0) ++slot;
        if (slot >= n_slots) break;                                    // ring full: back-pressure
        const uint64_t count = std::min<uint64_t>(s->prm.chunk_len, j.n_samples - j.next_n0);
        const double w = (double)j.n_tones * (double)count;
        if (!st->items.empty() && work + w > budget) break;
        work += w;
        BatchItem &b = st->h_items[st->items.size()];
        b.tones = j.d_tones;
        b.tables = j.d_tabs;
        b.out = s->d_arena + (size_t)slot * s->prm.chunk_len * sizeof(int16_t);
        b.n0 = j.next_n0;
        b.count = count;
        b.tile_begin = tiles;
        b.n_tones = j.n_tones;
        b.out_stride = 1;
        b.is_static = j.is_static;
        b.blocks = j.d_blocks;
        tiles += (uint32_t)((count + kTileSamples - 1) / kTileSamples);
        st->items.push_back(StepItem{j.id, slot, j.next_n0, count, (uint32_t)(j.next_n0 / s->prm.chunk_len)});
        s->slot_state[slot] = 1;
        j.next_n0 += count;
        j.in_flight = true;
    }
    if (st->items.empty()) return false;
    st->h_hdr[0] = (uint32_t)st->items.size();
    st->h_hdr[1] = tiles;
    hipError_t e = hipEventRecord(st->ev_start, s->stream);
    if (e == hipSuccess) e = hipGraphLaunch(st->exec, s->stream);
    if (e == hipSuccess) e = hipEventRecord(st->ev_done, s->stream);
    if (e != hipSuccess) { s->error = hipst(e); return false; }
    st->in_flight = true;
    st->t_launch = now_ms();
    s->n_steps++;
    s->n_items_total += st->items.size();
    s->max_batch = std::max<uint64_t>(s->max_batch, st->items.size());
    return true;
}

void scheduler(awg_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        harvest(s);
        admit(s);
        bool launched = false;
        while (launch_step(s)) launched = true;
        const bool busy = s->steps[0].in_flight || s->steps[1].in_flight;
        if (!launched) {
            // sleep briefly while steps run (polling their events), longer when idle
            s->cv.wait_for(lk, std::chrono::microseconds(busy ? 20 : 200));
        }
    }
    lk.unlock();
    for (auto &st : s->steps)
        if (st.in_flight) (void)hipEventSynchronize(st.ev_done);
}

awg_status build_step(awg_server *s, Step &st)
{
    const size_t items_bytes = sizeof(BatchItem) * (size_t)s->prm.max_jobs;
    const size_t blob_bytes = kItemsOffset + items_bytes;
    hipError_t e = alloc_upload_host(blob_bytes, &st.h_blob, &st.m_blob);
    if (e == hipSuccess) e = hipMalloc(&st.d_blob, blob_bytes);
    if (e == hipSuccess) e = hipEventCreate(&st.ev_start);
    if (e == hipSuccess) e = hipEventCreate(&st.ev_done);
    if (e != hipSuccess) return hipst(e);
    st.h_hdr = (uint32_t *)st.h_blob;
    st.h_items = (BatchItem *)((char *)st.h_blob + kItemsOffset);
    st.d_hdr = (uint32_t *)st.d_blob;
    st.d_items = (BatchItem *)((char *)st.d_blob + kItemsOffset);
    std::memset(st.h_blob, 0, blob_bytes);
    // the step graph: upload the work list (a kernel reading the pinned blob, so
    // the step stays on the compute queue), then the batched kernel
    e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_upload(st.m_blob, st.d_blob, blob_bytes, s->stream);
    if (e == hipSuccess) e = launch_batch(st.d_items, st.d_hdr, kBatchGrid, s->stream);
    hipError_t e2 = hipStreamEndCapture(s->stream, &st.graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&st.exec, st.graph, nullptr, nullptr, 0);
    return hipst(e);
}

void free_server(awg_server *s)
{
    for (auto &st : s->steps) {
        if (st.exec) (void)hipGraphExecDestroy(st.exec);
        if (st.graph) (void)hipGraphDestroy(st.graph);
        if (st.ev_start) (void)hipEventDestroy(st.ev_start);
        if (st.ev_done) (void)hipEventDestroy(st.ev_done);
        if (st.h_blob) (void)hipHostFree(st.h_blob);
        if (st.d_blob) (void)hipFree(st.d_blob);
    }
    for (auto &p : s->pending) awg_plan_destroy(p.plan);
    for (auto &kv : s->jobs) awg_plan_destroy(kv.second.plan);
    for (auto &sg : s->stage) {
        if (sg.done && sg.used) (void)hipEventSynchronize(sg.done);
        if (sg.host) (void)hipHostFree(sg.host);
        if (sg.done) (void)hipEventDestroy(sg.done);
    }
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

extern "C" {

awg_status awg_server_create(awg_ctx *ctx, const awg_server_params *prm, awg_server **out)
{
    if (!out) return AWG_E_INVALID;
    *out = nullptr;
    if (!ctx || !prm) return AWG_E_INVALID;
    if (prm->max_jobs <= 0 || prm->max_jobs > 65536 || prm->ring_slots <= 0 || prm->chunk_len == 0 ||
        prm->chunk_len % kTileSamples != 0 || !(prm->playout_delay_ms >= 0.0) || prm->max_pending <= 0)
        return AWG_E_INVALID;
    const size_t ring = (size_t)prm->ring_slots * prm->chunk_len * sizeof(int16_t);
    if (prm->mem_budget_bytes < ring + kAlign) return AWG_E_RANGE;
    awg_server *s = new (std::nothrow) awg_server();
    if (!s) return AWG_E_NOMEM;
    s->ctx = ctx;
    s->prm = *prm;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void **)&s->d_arena, prm->mem_budget_bytes);
    if (e != hipSuccess) { free_server(s); return hipst(e); }
    s->ring_bytes = ring;
    s->pool_off = align_up(ring);
    s->pool_bytes = prm->mem_budget_bytes - s->pool_off;
    s->pool_bytes -= s->pool_bytes % kAlign;
    s->free_blocks[0] = s->pool_bytes;
    s->slot_state.assign(prm->ring_slots, 0);
    for (auto &st : s->steps) {
        awg_status rs = build_step(s, st);
        if (rs != AWG_OK) { free_server(s); return rs; }
    }
    // admission staging buffers up front: the scheduler then allocates pinned
    // memory only for a job larger than any before it
    for (auto &sg : s->stage) {
        e = alloc_upload_host(kStageInit, &sg.host, &sg.mapped);
        if (e == hipSuccess) sg.cap = kStageInit;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sg.done, hipEventDisableTiming);
        if (e != hipSuccess) { free_server(s); return hipst(e); }
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return AWG_OK;
}

awg_status awg_server_destroy(awg_server *s)
{
    if (!s) return AWG_E_INVALID;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(s->stream);
    free_server(s);
    return AWG_OK;
}

awg_status awg_server_submit(awg_server *s, const awg_job *job, uint64_t *job_id)
{
    if (!s || !job || !job->tones || job->n_tones <= 0 || job->n_samples == 0 || job->reserved != 0 ||
        job->reserved2 != 0)
        return AWG_E_INVALID;
    awg_plan_params pp;
    pp.fs_hz = job->fs_hz;
    pp.gain_lsb = job->gain_lsb;
    pp.period_log2 = job->period_log2;
    pp.flags = 0;
    if (job->n_samples >= (1ull << 62)) return AWG_E_RANGE;
    awg_plan *plan = nullptr;
    awg_status st = awg_plan_tones(nullptr, &pp, job->tones, job->n_tones, &plan, nullptr);
    if (st != AWG_OK) return st;
    // smooth ramps: resolve the shared device tables now
    for (auto &kv : plan->table_index) {
        const uint64_t *d = nullptr;
        awg_status ts = get_table(s->ctx, kv.first.first, kv.first.second, &d);
        if (ts != AWG_OK) { awg_plan_destroy(plan); return ts; }
        plan->table_ptrs[kv.second] = d;
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error != AWG_OK) { awg_plan_destroy(plan); return s->error; }
    if (job_bytes(plan) > s->pool_bytes) { awg_plan_destroy(plan); return AWG_E_NOMEM; }
    if ((int32_t)s->pending.size() >= s->prm.max_pending) { awg_plan_destroy(plan); return AWG_E_BUSY; }
    Pending p;
    p.id = s->next_id++;
    p.tag = job->user_tag;
    p.t_submit = now_ms();
    p.plan = plan;
    p.n_samples = job->n_samples;
    p.fs = job->fs_hz;
    s->pending.push_back(p);
    s->n_submitted++;
    if (s->t_first_submit < 0) s->t_first_submit = p.t_submit;
    if (job_id) *job_id = p.id;
    s->cv.notify_all();
    return AWG_OK;
}

awg_status awg_server_poll(awg_server *s, awg_chunk_event *out, int32_t max_events, int32_t *n_events)
{
    if (!s || !n_events || max_events < 0 || (max_events > 0 && !out)) return AWG_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    int32_t n = 0;
    while (n < max_events && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_events = n;
    return s->error;
}

awg_status awg_server_slot(awg_server *s, int32_t slot, int16_t **d_ptr)
{
    if (!s || !d_ptr || slot < 0 || slot >= s->prm.ring_slots) return AWG_E_INVALID;
    *d_ptr = (int16_t *)(s->d_arena + (size_t)slot * s->prm.chunk_len * sizeof(int16_t));
    return AWG_OK;
}

awg_status awg_server_read(awg_server *s, int32_t slot, uint64_t count, int16_t *dst)
{
    if (!s || !dst || slot < 0 || slot >= s->prm.ring_slots || count > s->prm.chunk_len) return AWG_E_INVALID;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->slot_state[slot] != 2) return AWG_E_INVALID;
    }
    const int16_t *src = (const int16_t *)(s->d_arena + (size_t)slot * s->prm.chunk_len * sizeof(int16_t));
    hipError_t e = hipSetDevice(s->ctx->device);
    if (e == hipSuccess) e = hipMemcpy(dst, src, count * sizeof(int16_t), hipMemcpyDefault);
    return hipst(e);
}

awg_status awg_server_release(awg_server *s, int32_t slot)
{
    if (!s || slot < 0 || slot >= s->prm.ring_slots) return AWG_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->slot_state[slot] != 2) return AWG_E_INVALID;
    s->slot_state[slot] = 0;
    s->cv.notify_all();
    return AWG_OK;
}

awg_status awg_server_stats_get(awg_server *s, awg_server_stats *o)
{
    if (!s || !o) return AWG_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(o, 0, sizeof(*o));
    o->jobs_submitted = s->n_submitted;
    o->jobs_admitted = s->n_admitted;
    o->jobs_done = s->n_jobs_done;
    o->jobs_pending = s->pending.size();
    o->jobs_active = s->jobs.size();
    o->chunks_done = s->n_chunks;
    o->steps = s->n_steps;
    o->max_batch = s->max_batch;
    o->mean_batch = s->n_steps ? (double)s->n_items_total / (double)s->n_steps : 0.0;
    o->tone_samples = s->tone_samples;
    o->audio_seconds = s->audio_s;
    o->device_busy_ms = s->busy_ms;
    o->wall_ms = s->t_first_submit >= 0 ? s->t_last_ready - s->t_first_submit : 0.0;
    o->chunk_latency_p50_ms = percentile(s->lat_chunk.v, 50);
    o->chunk_latency_p99_ms = percentile(s->lat_chunk.v, 99);
    o->first_chunk_latency_p50_ms = percentile(s->lat_first.v, 50);
    o->first_chunk_latency_p99_ms = percentile(s->lat_first.v, 99);
    o->deadline_misses = s->deadline_misses;
    o->lateness_p50_ms = percentile(s->lateness.v, 50);
    o->lateness_p99_ms = percentile(s->lateness.v, 99);
    o->pool_free_bytes = 0;
    for (auto &kv : s->free_blocks) o->pool_free_bytes += kv.second;
    return s->error;
}

}  // extern "C"
