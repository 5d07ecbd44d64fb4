// Hybrid synthesis of ramped plans: matrix cores for the tones on a line,
// the direct kernel for the tones that ramp.
//
// The additive sum of Eq. (3) splits by tone. Over a row of 1024 samples a tone
// whose window [a, a+N] misses the row is on one straight phase line, either
// p0 + F0 n before the window or p1 + F1 n after it (Eq. (8) cases 1 and 3).
// Such (tone, row) pairs are summed by angle addition on the matrix cores. Only
// the pairs whose row meets the window run on the direct kernel, with the exact
// chirp phase. The paper's split of a static buffer plus a dynamic part
// (Eqs. (5)-(7), the add/subtract of the weighted combination) is the same idea.
// Here it is taken per row, from the exact line words, so nothing accumulates
// across calls.
//
// Per call (in pieces of at most 2^22 samples) the host classifies every tone
// against the rows [n0 + 1024 c, n0 + 1024 c + 1023]:
//  * window outside all rows: one line entry for the whole range;
//  * window meets some rows, and the rows where the tone is on a line are at
//    least 1/8 of all rows: "split". Line entries cover the rows before and
//    after the window. The direct kernel takes the tone only on the other rows.
//  * otherwise the direct kernel takes the tone on every row.
// The product writes gz FP32 partial-sum planes. The direct kernel adds them in
// plane order to its own sum of the ramping tones, then rounds.
//
// Results depend on (n0, count) through the row grid. They are deterministic
// for equal calls, but differ by rounding from the direct method, and from
// calls over other ranges.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "awg_internal.h"

namespace awg {

namespace {

constexpr uint64_t kRow = kTileSamples;          // product row == direct-kernel tile
constexpr uint64_t kPiece = 1ull << 22;          // samples per pass (bounds the workspace)
constexpr int kHybSlots = 4;                     // pinned staging slots in flight

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

awg_status hst(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    return e == hipErrorOutOfMemory ? AWG_E_NOMEM : AWG_E_HIP;
}

}  // namespace

struct HybridState {
    std::mutex mu;
    struct Slot {
        void *host = nullptr;          // pinned, coherent (alloc_upload_host)
        void *mapped = nullptr;        // its device-mapped address
        size_t host_cap = 0;
        void *dev = nullptr;
        size_t dev_cap = 0;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    Slot slots[kHybSlots];
    int next = 0;
    void *d_work = nullptr;
    size_t work_cap = 0;
    hipEvent_t work_done = nullptr;              // last use of d_work, on whatever stream
    bool work_used = false;
    // B operand cache: the frequency word each entry slot had when its k-block
    // was last built, for the method b_method; invalid after a reallocation
    std::vector<uint64_t> b_word;
    uint32_t b_method = 0;
    bool b_valid = false;
    // host scratch kept between calls
    std::vector<uint32_t> entries, extras;
    std::vector<int32_t> split, only, dirty;
    int32_t n_line = 0;
    double line_work = 0.0, direct_work = 0.0;   // tone-samples of the product / the direct kernel
    std::vector<ToneDev> direct;
    std::vector<Block> blocks;
    std::vector<float> cost;
    std::vector<uint32_t> order;
};

void hybrid_release(awg_plan *p)
{
    plb_release(p);
    HybridState *h = p->hyb;
    if (!h) return;
    for (auto &s : h->slots) {
        if (s.done) (void)hipEventSynchronize(s.done);
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.done) (void)hipEventDestroy(s.done);
    }
    if (h->work_done) (void)hipEventSynchronize(h->work_done);
    if (h->d_work) (void)hipFree(h->d_work);
    if (h->work_done) (void)hipEventDestroy(h->work_done);
    delete h;
    p->hyb = nullptr;
}

size_t hybrid_bytes(const awg_plan *p)
{
    const HybridState *h = p->hyb;
    if (!h) return plb_bytes_of(p);
    size_t b = h->work_cap + plb_bytes_of(p);
    for (const auto &s : h->slots) b += s.dev_cap;
    return b;
}

// Sorts tone positions so that tones sharing shape, window and table sit together
// (uniform blocks for the direct kernel).
static void sort_group(const std::vector<ToneDev> &tones, std::vector<int32_t> *idx)
{
    std::stable_sort(idx->begin(), idx->end(), [&](int32_t x, int32_t y) {
        const ToneDev &a = tones[x], &b = tones[y];
        if (a.shape != b.shape) return a.shape < b.shape;
        if (a.a != b.a) return a.a < b.a;
        if (a.n != b.n) return a.n < b.n;
        if (a.table != b.table) return a.table < b.table;
        if (a.ashape != b.ashape) return a.ashape < b.ashape;
        if (a.b != b.b) return a.b < b.b;
        return a.m < b.m;
    });
}

// Line entries and the direct kernel's tone list for rows [0, rows) from n0.
// Entry slots are stable from call to call: slot k is tone k's first line (or
// kLineNone when the direct kernel takes the tone on every row), slots up to a
// multiple of 8 are padding, and the second lines of tones split on both sides
// follow. A tone's slot then keeps its frequency word, and with it its columns
// of the B operand, until its line changes.
static void classify(const awg_plan *p, HybridState *h, uint64_t n0, uint64_t rows, uint64_t count)
{
    const int32_t K = p->n_tones;
    h->entries.assign((size_t)(K + 7) / 8 * 8, kLineNone << kLineShift);
    h->extras.clear();
    h->split.clear();
    h->only.clear();
    h->n_line = 0;
    // line rows are whole rows, except that the last row holds count - (rows - 1) * kRow samples
    const double full = (double)count;
    const double tail_short = (double)(rows * kRow - count);
    h->line_work = 0.0;
    h->direct_work = 0.0;
    const uint64_t last = n0 + rows * kRow - 1;
    for (int32_t k = 0; k < K; ++k) {
        const ToneDev &t = p->dev_mirror[k];
        const uint32_t kk = (uint32_t)k;
        // the tone's windows (frequency and amplitude) span [lo, hi]
        if (t.lo > t.hi || last < t.lo) {
            h->entries[k] = kk | (kLinePre << kLineShift);
            h->n_line++;
            h->line_work += full;
            continue;
        }
        if (n0 > t.hi) {
            h->entries[k] = kk | (kLinePost << kLineShift);
            h->n_line++;
            h->line_work += full;
            continue;
        }
        // rows ending before lo (n0 + 1024c + 1023 < lo) and starting after hi
        const uint64_t pre_rows = t.lo > n0 ? std::min<uint64_t>(rows, (t.lo - n0) / kRow) : 0;
        const uint64_t q = (t.hi - n0) / kRow;
        const uint64_t post_rows = rows > q + 1 ? rows - (q + 1) : 0;
        const uint64_t line_rows = pre_rows + post_rows;
        if (line_rows > 0 && line_rows * 8 >= rows) {
            h->entries[k] = kk | ((pre_rows ? kLineSplitPre : kLineSplitPost) << kLineShift);
            h->n_line++;
            if (pre_rows && post_rows) h->extras.push_back(kk | (kLineSplitPost << kLineShift));
            h->split.push_back(k);
            const double line = (double)(line_rows * kRow) - (post_rows ? tail_short : 0.0);
            h->line_work += line;
            h->direct_work += full - line;
        } else {
            h->entries[k] = kk | (kLineNone << kLineShift);
            h->only.push_back(k);
            h->direct_work += full;
        }
    }
    h->entries.insert(h->entries.end(), h->extras.begin(), h->extras.end());
    sort_group(p->dev_mirror, &h->split);
    sort_group(p->dev_mirror, &h->only);
    h->direct.clear();
    for (int32_t k : h->split) h->direct.push_back(p->dev_mirror[k]);
    for (int32_t k : h->only) h->direct.push_back(p->dev_mirror[k]);
}

// Launch order of the direct kernel's tiles, costliest first (a stable sort
// on an estimate: a tile where a tone's window opens or closes weighs 3.5
// tiles inside the window, for its per-sample choice of increment; a
// direct-only tone on its line costs about 0.6; split tones on a line
// nothing). Weights of 1.3 to 3.5 for the edge tiles time the same on the
// 10,000-tone array stream.
static void tile_order(HybridState *h, uint64_t n0, uint64_t rows, int32_t n_split)
{
    h->cost.assign(rows + 1, 0.0f);
    std::vector<float> &c = h->cost;
    const uint64_t last = n0 + rows * kRow - 1;
    float base = 0.0f;                                  // cost on every tile
    for (size_t i = 0; i < h->direct.size(); ++i) {
        const ToneDev &t = h->direct[i];
        const bool split = (int32_t)i < n_split;
        const uint64_t a = t.lo, e = t.hi;
        // tiles meeting the window: [ca, ce]
        const uint64_t ca = a <= n0 ? 0 : (a - n0) / kRow;
        const uint64_t ce = e >= last ? rows - 1 : (e - n0) / kRow;
        if (!split) {
            base += 0.6f;
            c[ca] -= 0.6f;
            c[ce + 1] += 0.6f;
        }
        c[ca] += 1.0f;                                  // in-window cost over [ca, ce]
        c[ce + 1] -= 1.0f;
        // tiles where an edge falls inside (closed form per sample)
        if (a > n0 && (a - n0) % kRow != 0) { c[ca] += 2.5f; c[ca + 1] -= 2.5f; }
        if (e < last && (e - n0) % kRow != kRow - 1) { c[ce] += 2.5f; c[ce + 1] -= 2.5f; }
    }
    float run = base;
    for (uint64_t r = 0; r < rows; ++r) { run += c[r]; c[r] = run; }
    h->order.resize(rows);
    for (uint64_t r = 0; r < rows; ++r) h->order[r] = (uint32_t)r;
    std::stable_sort(h->order.begin(), h->order.end(), [&](uint32_t x, uint32_t y) { return c[x] > c[y]; });
}

// Frequency word of an entry's line (what the B operand of its slot holds).
static uint64_t entry_word(const awg_plan *p, uint32_t ent)
{
    const ToneDev &t = p->dev_mirror[ent & ((1u << kLineShift) - 1)];
    return ((ent >> kLineShift) & 1u) ? t.f1 : t.f0;
}

// k-blocks whose B operand must be rebuilt: those holding an entry with a line
// whose frequency word differs from the one built last; b_word is updated for
// them. All of them (dirty empty, return false) when nothing is cached.
static bool dirty_blocks(const awg_plan *p, HybridState *h, uint32_t method, int32_t kb_n)
{
    h->dirty.clear();
    const int32_t n = (int32_t)h->entries.size();
    if (!h->b_valid || h->b_method != method) {
        h->b_word.assign((size_t)kb_n * 8, 0);
        for (int32_t e = 0; e < n; ++e) h->b_word[e] = entry_word(p, h->entries[e]);
        h->b_method = method;
        h->b_valid = true;
        return false;
    }
    if (h->b_word.size() < (size_t)kb_n * 8) h->b_word.resize((size_t)kb_n * 8, 0);
    for (int32_t kb = 0; kb < kb_n; ++kb) {
        bool d = false;
        for (int32_t e = 8 * kb; e < std::min(n, 8 * kb + 8) && !d; ++e)
            d = (h->entries[e] >> kLineShift) != kLineNone && entry_word(p, h->entries[e]) != h->b_word[e];
        if (!d) continue;
        h->dirty.push_back(kb);
        for (int32_t e = 8 * kb; e < std::min(n, 8 * kb + 8); ++e) h->b_word[e] = entry_word(p, h->entries[e]);
    }
    return true;
}

// Staging blob capacity for the largest blob the plan can produce (every tone
// with two lines, every tone direct, a full piece of rows, every k-block dirty).
static size_t staging_cap(const awg_plan *p)
{
    const int32_t max_entries = (p->n_tones + 7) / 8 * 8 + p->n_tones;
    const size_t kb_max = ((size_t)max_entries + 7) / 8;
    return align_up(sizeof(uint32_t) * (size_t)max_entries, 256) + align_up(sizeof(ToneDev) * (size_t)p->n_tones, 256) +
           align_up(sizeof(Block) * ((size_t)p->n_tones + 1), 256) + align_up(sizeof(uint32_t) * (kPiece / kRow), 256) +
           sizeof(int32_t) * kb_max;
}

// Every staging slot with `bytes` of pinned host and device memory (slots that
// already have them are left alone).
static awg_status setup_slots(HybridState *h, size_t bytes)
{
    hipError_t e = hipSuccess;
    for (auto &sl : h->slots) {
        if (!sl.done) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess && !sl.host) {
            e = alloc_upload_host(bytes, &sl.host, &sl.mapped);
            if (e == hipSuccess) sl.host_cap = bytes;
        }
        if (e == hipSuccess && !sl.dev) {
            e = hipMalloc(&sl.dev, bytes);
            if (e == hipSuccess) sl.dev_cap = bytes;
        }
        if (e != hipSuccess) return hst(e);
    }
    return AWG_OK;
}

// The operand and plane workspace of at least `bytes` (a quarter more when it
// grows, since the rows of a call vary); growing it waits for its last user
// and drops the cached B operand.
static awg_status ensure_work(HybridState *h, size_t bytes)
{
    if (h->work_cap >= bytes) return AWG_OK;
    if (h->work_used) {
        const hipError_t e = hipEventSynchronize(h->work_done);
        if (e != hipSuccess) return hst(e);
    }
    if (h->d_work) (void)hipFree(h->d_work);
    h->d_work = nullptr;
    h->work_cap = 0;
    const size_t want = bytes + bytes / 4;
    const hipError_t e = hipMalloc(&h->d_work, want);
    if (e != hipSuccess) return hst(e);
    h->work_cap = want;
    h->b_valid = false;
    return AWG_OK;
}

static awg_status piece(awg_plan *p, HybridState *h, uint32_t method, uint64_t n0, uint64_t count,
                        int16_t *out_i16, float *out_f32, hipStream_t s)
{
    const uint64_t rows = (count + kRow - 1) / kRow;
    classify(p, h, n0, rows, count);
    const int32_t n_entries = (int32_t)h->entries.size();
    const int32_t max_entries = (p->n_tones + 7) / 8 * 8 + p->n_tones;
    const int32_t n_direct = (int32_t)h->direct.size();
    build_blocks(h->direct, (int32_t)h->split.size(), &h->blocks);
    tile_order(h, n0, rows, (int32_t)h->split.size());
    const LinesGeom g = lines_geometry(n_entries, max_entries, count);
    const bool gemm = h->n_line > 0 && g.gz > 0;

    // staging blob: entries | direct tone list | block table | tile order | dirty k-blocks
    const size_t off_t = align_up(sizeof(uint32_t) * (size_t)n_entries, 256);
    const size_t off_b = align_up(off_t + sizeof(ToneDev) * (size_t)n_direct, 256);
    const size_t off_o = align_up(off_b + sizeof(Block) * h->blocks.size(), 256);
    const size_t off_d = align_up(off_o + sizeof(uint32_t) * rows, 256);
    const size_t kb_max = ((size_t)max_entries + 7) / 8;
    const size_t total = off_d + sizeof(int32_t) * kb_max;
    // slots are sized for the largest blob this plan can produce, so they are allocated once
    const size_t cap = staging_cap(p);
    hipError_t e = hipSuccess;
    // the first call sets up every slot, so that the calls after it (the next
    // chunks of a stream) do not each pay for a pinned allocation
    if (!h->slots[0].host) {
        const awg_status st = setup_slots(h, std::max(cap, total));
        if (st != AWG_OK) return st;
    }
    HybridState::Slot &slot = h->slots[h->next];
    h->next = (h->next + 1) % kHybSlots;
    if (!slot.done) e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
    if (e == hipSuccess && slot.used) e = hipEventSynchronize(slot.done);
    if (e != hipSuccess) return hst(e);
    slot.used = false;
    if (slot.host_cap < total) {
        if (slot.host) (void)hipHostFree(slot.host);
        slot.host = nullptr;
        slot.mapped = nullptr;
        slot.host_cap = 0;
        e = alloc_upload_host(std::max(cap, total), &slot.host, &slot.mapped);
        if (e != hipSuccess) return hst(e);
        slot.host_cap = std::max(cap, total);
    }
    if (slot.dev_cap < total) {
        if (slot.dev) (void)hipFree(slot.dev);
        slot.dev = nullptr;
        slot.dev_cap = 0;
        e = hipMalloc(&slot.dev, std::max(cap, total));
        if (e != hipSuccess) return hst(e);
        slot.dev_cap = std::max(cap, total);
    }
    char *hb = (char *)slot.host;
    if (n_entries) std::memcpy(hb, h->entries.data(), sizeof(uint32_t) * (size_t)n_entries);
    if (n_direct) std::memcpy(hb + off_t, h->direct.data(), sizeof(ToneDev) * (size_t)n_direct);
    std::memcpy(hb + off_b, h->blocks.data(), sizeof(Block) * h->blocks.size());
    std::memcpy(hb + off_o, h->order.data(), sizeof(uint32_t) * rows);

    // workspace for the operands and the partial planes
    if (!h->work_done) {
        e = hipEventCreateWithFlags(&h->work_done, hipEventDisableTiming);
        if (e != hipSuccess) return hst(e);
    }
    if (gemm) {
        const awg_status st = ensure_work(h, g.work_bytes());
        if (st != AWG_OK) return st;
    }
    const bool partial = gemm && dirty_blocks(p, h, method, g.kb_n);
    if (partial && !h->dirty.empty())
        std::memcpy(hb + off_d, h->dirty.data(), sizeof(int32_t) * h->dirty.size());

    char *db = (char *)slot.dev;
    e = launch_upload(slot.mapped, db, total, s);
    if (e == hipSuccess && h->work_used) e = hipStreamWaitEvent(s, h->work_done, 0);
    if (e == hipSuccess && gemm)
        e = launch_lines(p, method, g, (const uint32_t *)db, n_entries, partial ? (const int32_t *)(db + off_d) : nullptr,
                         partial ? (int32_t)h->dirty.size() : 0, n0, count, h->d_work, s, h->line_work);
    const float *planes = gemm ? (const float *)((char *)h->d_work + 2 * (g.a_bytes + g.b_bytes)) : nullptr;
    if (e == hipSuccess)
        e = launch_direct_hybrid(p, (const ToneDev *)(db + off_t), (const Block *)(db + off_b),
                                 (const uint32_t *)(db + off_o), n0, count, planes, gemm ? g.gz : 0, g.plane,
                                 out_i16, out_f32, s, h->direct_work);
    if (e == hipSuccess) e = hipEventRecord(h->work_done, s);
    if (e == hipSuccess) h->work_used = true;
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    if (e == hipSuccess) slot.used = true;
    return hst(e);
}

awg_status hybrid_reserve(awg_plan *p, uint32_t method, uint64_t max_count)
{
    if (plb_eligible(p)) return plb_reserve(p, method);
    if (p->n_tones >= (int32_t)(1u << kLineShift)) return AWG_E_UNSUPPORTED;
    if (!p->hyb) {
        try { p->hyb = new HybridState(); } catch (...) { return AWG_E_NOMEM; }
    }
    HybridState *h = p->hyb;
    std::lock_guard<std::mutex> lock(h->mu);
    if (!h->work_done) {
        const hipError_t e = hipEventCreateWithFlags(&h->work_done, hipEventDisableTiming);
        if (e != hipSuccess) return hst(e);
    }
    awg_status st = setup_slots(h, staging_cap(p));
    if (st != AWG_OK) return st;
    // the workspace of a full piece with every tone on two lines
    const int32_t max_entries = (p->n_tones + 7) / 8 * 8 + p->n_tones;
    const LinesGeom g = lines_geometry(max_entries, max_entries, std::min<uint64_t>(max_count, kPiece));
    return g.gz > 0 ? ensure_work(h, g.work_bytes()) : AWG_OK;
}

awg_status hybrid_synth(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16,
                        float *out_f32, hipStream_t s)
{
    if (plb_eligible(p)) return plb_synth(p, method, n0, count, out_i16, out_f32, s);
    if (p->n_tones >= (int32_t)(1u << kLineShift)) return AWG_E_UNSUPPORTED;
    {
        const awg_status st = flush_tones(p, s);
        if (st != AWG_OK) return st;
    }
    if (!p->hyb) {
        try { p->hyb = new HybridState(); } catch (...) { return AWG_E_NOMEM; }
    }
    HybridState *h = p->hyb;
    std::lock_guard<std::mutex> lock(h->mu);
    while (count > 0) {
        const uint64_t now = count < kPiece ? count : kPiece;
        awg_status st = piece(p, h, method, n0, now, out_i16, out_f32, s);
        if (st != AWG_OK) return st;
        n0 += now;
        count -= now;
        if (out_i16) out_i16 += now;
        if (out_f32) out_f32 += now;
    }
    return AWG_OK;
}

}  // namespace awg
