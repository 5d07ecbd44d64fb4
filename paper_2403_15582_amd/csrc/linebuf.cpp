// Periodic line buffer: the hybrid path for ramped plans whose tones sit on the
// bins of a period L = 2^p (Eq. (4)).
//
// Eqs. (5)-(7) split the waveform into a static buffer (the tones on a line)
// and the dynamic tones, and the paper's combiner adds or subtracts wavetables
// as tones move between the two. With bin frequencies every line is periodic in
// L, so its contribution over one period can be kept on the device and read at
// m = n mod L by every later call, instead of being recomputed for each chunk.
//
// Tones are cut into fixed groups of kGroupTones consecutive tones (caller
// order). For a group and a choice of one line per tone (its "version": words
// P, F and amplitude per tone), Q(version) is the group's period sum
// sum_k A_k sin(2 pi (P_k + F_k m) / 2^64), m in [0, L), computed on the matrix
// cores by angle addition (FP32 accumulation) and cached by version. S, an
// int64 period buffer, holds sum over groups of fix(Q) with fix(x) = x 2^32
// rounded, for one version per group; folding a group from one version to
// another adds fix(Q_new) - fix(Q_old), so S is always exactly the sum of the
// fixed-point sums of the versions it holds, in any order of folds.
//
// Each call over [n0, n0 + count) in rows of 1024 samples is evaluated from
// the call alone (the plan's state and the range), so equal calls give equal
// samples whatever the plan computed before:
//  * a tone's "next" line is the one it is on at the call's last sample (none,
//    i.e. zero amplitude, if that sample is still inside its windows); each
//    group's version of next lines is folded into S before the call is summed;
//  * rows before a tone's windows, where it is still on its line before them
//    while its next line is the one after, hold a different version of the
//    group: for those rows the call adds Q(row version) - Q(next version)
//    ("segments");
//  * on the rows its windows meet, a tone runs on the direct kernel with its
//    exact chirp phase, together with a copy of its next line, if it has one,
//    at minus its amplitude (the line S and the segments count for it there).
// The direct kernel adds, per tile, S, the segments and its own sum, and rounds.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "awg_internal.h"

namespace awg {

namespace {

constexpr int32_t kGroupTones = 128;                 // tones per group (16 k-blocks)
constexpr uint64_t kRow = kTileSamples;
constexpr uint64_t kPiece = 1ull << 22;               // samples per pass
constexpr int32_t kMaxSegs = 64;                      // segments of one pass (more: the pass is halved)
constexpr int32_t kBuildBatch = 32;                   // groups per product launch
constexpr int kSlots = 4;                             // pinned staging slots in flight
constexpr size_t kMaxBytes = 16ull << 30;             // device memory of the buffer and its cache

awg_status hst(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    return e == hipErrorOutOfMemory ? AWG_E_NOMEM : AWG_E_HIP;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint32_t fbits(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, sizeof(u));
    return u;
}

// One line of a tone: exact words (no device bias) and the amplitude (A G, FP32).
struct Line {
    uint64_t p, f;
    float a;
    bool operator==(const Line &o) const { return p == o.p && f == o.f && fbits(a) == fbits(o.a); }
    bool operator!=(const Line &o) const { return !(*this == o); }
};

// A line with zero amplitude contributes nothing, whatever its words: all such
// lines are one line, kNoLine, so that versions differing only there are equal.
constexpr Line kNoLine{0, 0, 0.0f};

Line line_of(uint64_t p, uint64_t f, float a) { return a == 0.0f ? kNoLine : Line{p, f, a}; }

uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h * 0xff51afd7ed558ccdull;
}

}  // namespace

struct LineBuf {
    std::mutex mu;
    uint32_t method = 0;
    uint64_t L = 0;
    int32_t K = 0, n_groups = 0, n_slots = 0;
    int64_t *d_S = nullptr;
    float *d_Q = nullptr;                 // n_slots period sums
    void *d_bwork = nullptr;              // product operands of one batch of groups
    size_t bwork_bytes = 0;
    bool s_zeroed = false;
    hipEvent_t work_done = nullptr;
    bool work_used = false;
    // cache of group sums: per group, version hash -> slot; the slot's words
    struct Entry { int32_t group; uint64_t hash; uint64_t last_use; bool live; std::vector<Line> words; };
    std::vector<Entry> slot_entry;        // per slot
    std::vector<std::unordered_multimap<uint64_t, int32_t>> index;   // per group
    std::vector<int32_t> free_slots;
    std::vector<int32_t> s_slot;          // per group: the slot S holds (-1: none)
    uint64_t tick = 0;
    // staging
    struct Slot { void *host = nullptr, *mapped = nullptr, *dev = nullptr; size_t cap = 0; hipEvent_t done = nullptr; bool used = false; };
    Slot slots[kSlots];
    int next_slot = 0;
    // host scratch of one pass
    std::vector<Line> next, l1, l2;
    std::vector<uint32_t> sw;             // per tone: first window row when it switches lines there, else 0
    std::vector<int32_t> wr_lo, wr_hi;    // per tone: window rows of the pass (wr_lo > wr_hi: none)
    std::vector<ToneDev> build_list, direct;
    std::vector<int32_t> build_map;
    std::vector<PlbSeg> segs;
    std::vector<PlbFold> folds;
    std::vector<int32_t> seg_slot;        // slots of the segments (pointers filled at staging)
    std::vector<int32_t> seg_next;
    std::vector<std::pair<int32_t, int32_t>> fold_slots;
    std::vector<Block> blocks;
    std::vector<uint32_t> order;
    std::vector<float> cost;
    std::vector<int32_t> pinned;          // per slot: pass stamp
    std::vector<uint32_t> bps;
    std::vector<Line> ver;
};

namespace {

size_t plb_bytes(uint64_t L, int32_t n_groups, int32_t n_slots)
{
    return sizeof(int64_t) * L + sizeof(float) * L * (size_t)n_slots + group_work_bytes(kBuildBatch, kGroupTones, L);
}

int32_t groups_of(int32_t K) { return (K + kGroupTones - 1) / kGroupTones; }

// The largest staging blob of a pass: the build list (a next version of every
// group and a version per segment), its map, the direct list (every tone and
// its negative line), blocks, tile order, segments, folds.
size_t blob_cap(const LineBuf &b)
{
    const size_t ng = (size_t)b.n_groups, K = (size_t)b.K, nb = ng + kMaxSegs;
    return align_up(sizeof(ToneDev) * nb * kGroupTones, 256) + align_up(sizeof(int32_t) * nb, 256) +
           align_up(sizeof(ToneDev) * 2 * K, 256) + align_up(sizeof(Block) * (2 * K + 1), 256) +
           align_up(sizeof(uint32_t) * (kPiece / kRow), 256) + align_up(sizeof(PlbSeg) * kMaxSegs, 256) +
           align_up(sizeof(PlbFold) * ng, 256);
}

ToneDev line_record(const Line &l, float sign)
{
    ToneDev t;
    std::memset(&t, 0, sizeof(t));
    t.p0 = t.p1 = l.p + kPhaseBias;
    t.f0 = t.f1 = l.f;
    t.a = UINT64_MAX;
    t.n = 0;
    t.amp = t.amp1 = sign * l.a;
    t.shape = AWG_RAMP_NONE;
    t.ashape = AWG_RAMP_NONE;
    t.lo = 1;
    t.hi = 0;
    return t;
}

uint64_t version_hash(const Line *w, int32_t n)
{
    uint64_t h = 0x243f6a8885a308d3ull;
    for (int32_t i = 0; i < n; ++i) {
        h = mix(h, w[i].p);
        h = mix(h, w[i].f);
        h = mix(h, fbits(w[i].a));
    }
    return h;
}

// The slot holding group g's version w (nullptr-free), or -1.
int32_t find_version(LineBuf &b, int32_t g, const Line *w, int32_t n, uint64_t h)
{
    auto range = b.index[g].equal_range(h);
    for (auto it = range.first; it != range.second; ++it) {
        const LineBuf::Entry &e = b.slot_entry[it->second];
        if (e.live && std::equal(e.words.begin(), e.words.end(), w, w + n)) return it->second;
    }
    return -1;
}

// A slot for a new version: a free one, else the least recently used one that
// this pass does not need and S does not hold.
int32_t take_slot(LineBuf &b, int32_t stamp)
{
    if (!b.free_slots.empty()) {
        const int32_t s = b.free_slots.back();
        b.free_slots.pop_back();
        return s;
    }
    int32_t best = -1;
    for (int32_t s = 0; s < b.n_slots; ++s) {
        const LineBuf::Entry &e = b.slot_entry[s];
        if (!e.live || b.pinned[s] == stamp || b.s_slot[e.group] == s) continue;
        if (best < 0 || e.last_use < b.slot_entry[best].last_use) best = s;
    }
    if (best >= 0) {
        LineBuf::Entry &e = b.slot_entry[best];
        auto range = b.index[e.group].equal_range(e.hash);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second == best) {
                b.index[e.group].erase(it);
                break;
            }
        e.live = false;
    }
    return best;
}

// Slot of group g's version w for this pass (stamp): cached, or a new one added
// to the build list.
int32_t need(LineBuf &b, int32_t g, const Line *w, int32_t n, int32_t stamp)
{
    const uint64_t h = version_hash(w, n);
    int32_t s = find_version(b, g, w, n, h);
    if (s < 0) {
        s = take_slot(b, stamp);
        if (s < 0) return -1;
        LineBuf::Entry &e = b.slot_entry[s];
        e.group = g;
        e.hash = h;
        e.live = true;
        e.words.assign(w, w + n);
        b.index[g].emplace(h, s);
        for (int32_t i = 0; i < kGroupTones; ++i) {
            const int32_t k = g * kGroupTones + i;
            b.build_list.push_back(k < b.K && i < n ? line_record(w[i], 1.0f) : line_record(Line{0, 0, 0.0f}, 0.0f));
        }
        b.build_map.push_back(s);
    }
    b.slot_entry[s].last_use = b.tick;
    b.pinned[s] = stamp;
    return s;
}

awg_status setup(LineBuf &b, const awg_plan *p, uint32_t method)
{
    b.method = method;
    b.L = 1ull << p->params.period_log2;
    b.K = p->n_tones;
    b.n_groups = groups_of(b.K);
    b.n_slots = 2 * b.n_groups + kMaxSegs;
    b.bwork_bytes = group_work_bytes(kBuildBatch, kGroupTones, b.L);
    hipError_t e = hipMalloc(&b.d_S, sizeof(int64_t) * b.L);
    if (e == hipSuccess) e = hipMalloc(&b.d_Q, sizeof(float) * b.L * (size_t)b.n_slots);
    if (e == hipSuccess) e = hipMalloc(&b.d_bwork, b.bwork_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.work_done, hipEventDisableTiming);
    const size_t cap = blob_cap(b);
    for (auto &sl : b.slots) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = alloc_upload_host(cap, &sl.host, &sl.mapped);
        if (e == hipSuccess) e = hipMalloc(&sl.dev, cap);
        if (e == hipSuccess) sl.cap = cap;
    }
    if (e != hipSuccess) return hst(e);
    b.slot_entry.assign(b.n_slots, LineBuf::Entry{0, 0, 0, false, {}});
    b.index.assign(b.n_groups, {});
    b.free_slots.clear();
    for (int32_t s = b.n_slots - 1; s >= 0; --s) b.free_slots.push_back(s);
    b.s_slot.assign(b.n_groups, -1);
    b.pinned.assign(b.n_slots, -1);
    return AWG_OK;
}

// Launch order of the tiles, costliest first: a window tile costs 1 per tone
// (2 with its negative line), a tile where a window opens or closes 3.5 more.
void tile_order(LineBuf &b, uint64_t n0, uint64_t rows)
{
    b.cost.assign(rows + 1, 0.0f);
    for (int32_t k = 0; k < b.K; ++k) {
        if (b.wr_lo[k] > b.wr_hi[k]) continue;
        const float c = b.next[k] != kNoLine ? 2.0f : 1.0f;
        b.cost[b.wr_lo[k]] += c;
        b.cost[b.wr_hi[k] + 1] -= c;
    }
    float run = 0.0f;
    for (uint64_t r = 0; r < rows; ++r) {
        run += b.cost[r];
        b.cost[r] = run;
    }
    for (const ToneDev &t : b.direct) {
        if (t.shape == AWG_RAMP_NONE && t.ashape == AWG_RAMP_NONE) continue;
        const uint64_t ends[2] = {t.a, t.a + t.n};
        for (uint64_t x : ends)
            if (x >= n0 && (x - n0) / kRow < rows && (x - n0) % kRow != 0) b.cost[(x - n0) / kRow] += 3.5f;
    }
    b.order.resize(rows);
    for (uint64_t r = 0; r < rows; ++r) b.order[r] = (uint32_t)r;
    std::stable_sort(b.order.begin(), b.order.end(), [&](uint32_t x, uint32_t y) { return b.cost[x] > b.cost[y]; });
}

void sort_direct(std::vector<ToneDev> *v)
{
    std::stable_sort(v->begin(), v->end(), [](const ToneDev &a, const ToneDev &b) {
        // ramped tones first, in the plan's device order (shape, window, table),
        // so that a call whose tones all ramp sums them as the direct kernel
        // does; lines last
        const bool la = a.shape == AWG_RAMP_NONE, lb = b.shape == AWG_RAMP_NONE;
        if (la != lb) return lb;
        if (a.shape != b.shape) return a.shape < b.shape;
        if (a.a != b.a) return a.a < b.a;
        if (a.n != b.n) return a.n < b.n;
        if (a.table != b.table) return a.table < b.table;
        if (a.ashape != b.ashape) return a.ashape < b.ashape;
        if (a.b != b.b) return a.b < b.b;
        if (a.m != b.m) return a.m < b.m;
        return a.lo < b.lo;
    });
}

// One pass of at most kPiece samples. *split: the pass needs more than kMaxSegs
// segments and nothing was done (the caller halves it).
awg_status pass(awg_plan *p, LineBuf &b, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32, hipStream_t s,
                bool *split)
{
    *split = false;
    const uint64_t rows = (count + kRow - 1) / kRow;
    const uint64_t last = n0 + count - 1;
    const int32_t K = b.K;
    b.tick++;
    const int32_t stamp = (int32_t)(b.tick & 0x7fffffff);
    b.next.resize(K);
    b.l1.resize(K);
    b.l2.resize(K);
    b.sw.assign(K, 0);
    b.wr_lo.assign(K, 1);
    b.wr_hi.assign(K, 0);
    b.build_list.clear();
    b.build_map.clear();
    b.direct.clear();
    b.segs.clear();
    b.seg_slot.clear();
    b.seg_next.clear();
    b.fold_slots.clear();
    double direct_work = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        const ToneDev &t = p->dev_mirror[p->inv[k]];
        b.l1[k] = line_of(t.p0 - kPhaseBias, t.f0, t.amp);
        b.l2[k] = line_of(t.p1 - kPhaseBias, t.f1, t.amp1);
        const bool windowed = t.lo <= t.hi;
        // still inside its windows at the call's last sample: on no line (the
        // direct kernel takes it on every row its windows meet)
        b.next[k] = !windowed || last < t.lo ? b.l1[k] : (last > t.hi ? b.l2[k] : kNoLine);
        if (windowed && t.hi >= n0 && t.lo <= last) {
            const uint64_t lo = t.lo <= n0 ? 0 : (t.lo - n0) / kRow;
            const uint64_t hi = std::min<uint64_t>(rows - 1, (t.hi - n0) / kRow);
            b.wr_lo[k] = (int32_t)lo;
            b.wr_hi[k] = (int32_t)hi;
            if (lo > 0 && b.l1[k] != b.next[k]) b.sw[k] = (uint32_t)lo;
            // the tone on its window rows, and its next line (if any) with the
            // opposite sign
            ToneDev d = t;
            d.lo = n0 + lo * kRow;
            d.hi = n0 + hi * kRow + (kRow - 1);
            b.direct.push_back(d);
            const double n_samp = (double)(std::min(d.hi, last) - d.lo + 1);
            direct_work += n_samp;
            if (b.next[k] != kNoLine) {
                ToneDev neg = line_record(b.next[k], -1.0f);
                neg.lo = d.lo;
                neg.hi = d.hi;
                b.direct.push_back(neg);
                direct_work += n_samp;
            }
        }
    }
    // segments of the pass: one per distinct switch row of each group (counted
    // before the cache is touched)
    int64_t n_segs = 0;
    for (int32_t g = 0; g < b.n_groups; ++g) {
        const int32_t k0 = g * kGroupTones, n = std::min(kGroupTones, K - k0);
        b.bps.clear();
        for (int32_t i = 0; i < n; ++i)
            if (b.sw[k0 + i]) b.bps.push_back(b.sw[k0 + i]);
        std::sort(b.bps.begin(), b.bps.end());
        n_segs += std::unique(b.bps.begin(), b.bps.end()) - b.bps.begin();
    }
    if (n_segs > kMaxSegs) {
        *split = true;
        return AWG_OK;
    }
    // versions: each group's next version (held by S), and the versions of its
    // rows before the switch rows of its tones
    for (int32_t g = 0; g < b.n_groups; ++g) {
        const int32_t k0 = g * kGroupTones, n = std::min(kGroupTones, K - k0);
        const int32_t snext = need(b, g, &b.next[k0], n, stamp);
        if (snext < 0) return AWG_E_NOMEM;
        if (b.s_slot[g] != snext) b.fold_slots.emplace_back(snext, b.s_slot[g]);
        b.bps.clear();
        for (int32_t i = 0; i < n; ++i)
            if (b.sw[k0 + i]) b.bps.push_back(b.sw[k0 + i]);
        if (b.bps.empty()) continue;
        std::sort(b.bps.begin(), b.bps.end());
        b.bps.erase(std::unique(b.bps.begin(), b.bps.end()), b.bps.end());
        uint32_t begin = 0;
        for (uint32_t bp : b.bps) {
            // rows [begin, bp): tones that switch at bp or later are still on their first line
            b.ver.assign(&b.next[k0], &b.next[k0] + n);
            for (int32_t i = 0; i < n; ++i)
                if (b.sw[k0 + i] >= bp) b.ver[i] = b.l1[k0 + i];
            const int32_t sv = need(b, g, b.ver.data(), n, stamp);
            if (sv < 0) return AWG_E_NOMEM;
            b.segs.push_back(PlbSeg{begin, bp - 1, nullptr, nullptr});
            b.seg_slot.push_back(sv);
            b.seg_next.push_back(snext);
            begin = bp;
        }
    }
    sort_direct(&b.direct);
    build_blocks(b.direct, (int32_t)b.direct.size(), &b.blocks);
    tile_order(b, n0, rows);

    // staging blob: build list | build map | direct list | blocks | tile order | segments | folds
    const int32_t n_built = (int32_t)b.build_map.size();
    const int32_t n_direct = (int32_t)b.direct.size();
    const int32_t n_seg = (int32_t)b.segs.size();
    const int32_t n_fold = (int32_t)b.fold_slots.size();
    const size_t off_m = align_up(sizeof(ToneDev) * b.build_list.size(), 256);
    const size_t off_d = off_m + align_up(sizeof(int32_t) * (size_t)n_built, 256);
    const size_t off_b = off_d + align_up(sizeof(ToneDev) * (size_t)n_direct, 256);
    const size_t off_o = off_b + align_up(sizeof(Block) * b.blocks.size(), 256);
    const size_t off_s = off_o + align_up(sizeof(uint32_t) * rows, 256);
    const size_t off_f = off_s + align_up(sizeof(PlbSeg) * (size_t)n_seg, 256);
    const size_t total = off_f + sizeof(PlbFold) * (size_t)n_fold;
    LineBuf::Slot &slot = b.slots[b.next_slot];
    b.next_slot = (b.next_slot + 1) % kSlots;
    if (total > slot.cap) return AWG_E_UNSUPPORTED;
    hipError_t e = slot.used ? hipEventSynchronize(slot.done) : hipSuccess;
    if (e != hipSuccess) return hst(e);
    slot.used = false;
    char *hb = (char *)slot.host;
    char *db = (char *)slot.dev;
    if (!b.build_list.empty()) std::memcpy(hb, b.build_list.data(), sizeof(ToneDev) * b.build_list.size());
    if (n_built) std::memcpy(hb + off_m, b.build_map.data(), sizeof(int32_t) * (size_t)n_built);
    if (n_direct) std::memcpy(hb + off_d, b.direct.data(), sizeof(ToneDev) * (size_t)n_direct);
    std::memcpy(hb + off_b, b.blocks.data(), sizeof(Block) * b.blocks.size());
    std::memcpy(hb + off_o, b.order.data(), sizeof(uint32_t) * rows);
    PlbSeg *sg = (PlbSeg *)(hb + off_s);
    for (int32_t i = 0; i < n_seg; ++i) {
        sg[i] = b.segs[i];
        sg[i].q_row = b.d_Q + (size_t)b.seg_slot[i] * b.L;
        sg[i].q_next = b.d_Q + (size_t)b.seg_next[i] * b.L;
    }
    PlbFold *fd = (PlbFold *)(hb + off_f);
    for (int32_t i = 0; i < n_fold; ++i) {
        fd[i].q_new = b.d_Q + (size_t)b.fold_slots[i].first * b.L;
        fd[i].q_old = b.fold_slots[i].second >= 0 ? b.d_Q + (size_t)b.fold_slots[i].second * b.L : nullptr;
    }
    e = launch_upload(slot.mapped, db, total, s);
    if (e == hipSuccess && b.work_used) e = hipStreamWaitEvent(s, b.work_done, 0);
    if (e == hipSuccess && !b.s_zeroed) {
        e = launch_plb_zero(b.d_S, b.L, s);
        if (e == hipSuccess) b.s_zeroed = true;
    }
    // the new versions' period sums, in batches
    for (int32_t i = 0; e == hipSuccess && i < n_built; i += kBuildBatch) {
        const int32_t nb = std::min(kBuildBatch, n_built - i);
        double work = 0.0;
        for (int32_t z = i; z < i + nb; ++z)
            work += (double)std::min(kGroupTones, K - b.slot_entry[b.build_map[z]].group * kGroupTones) * (double)b.L;
        e = launch_group_sums(p, b.method, (const ToneDev *)db + (size_t)i * kGroupTones, nb, kGroupTones, b.L,
                              b.d_bwork, b.d_Q, (const int32_t *)(db + off_m) + i, s, work);
    }
    // S to the call's next versions, then the call
    if (e == hipSuccess) e = launch_plb_fold(p, b.d_S, b.L, (const PlbFold *)(db + off_f), n_fold, s);
    if (e == hipSuccess)
        e = launch_plb(p, (const ToneDev *)(db + off_d), (const Block *)(db + off_b), (const uint32_t *)(db + off_o),
                       n0, count, b.d_S, b.L, (const PlbSeg *)(db + off_s), n_seg, out_i16, out_f32, s, direct_work);
    if (e == hipSuccess) e = hipEventRecord(b.work_done, s);
    if (e == hipSuccess) b.work_used = true;
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    if (e == hipSuccess) slot.used = true;
    if (e != hipSuccess) {
        // the device state is unknown: start over on the next call
        for (int32_t sl = 0; sl < b.n_slots; ++sl) {
            if (b.slot_entry[sl].live) b.slot_entry[sl].live = false;
        }
        for (auto &ix : b.index) ix.clear();
        b.free_slots.clear();
        for (int32_t sl = b.n_slots - 1; sl >= 0; --sl) b.free_slots.push_back(sl);
        b.s_slot.assign(b.n_groups, -1);
        b.s_zeroed = false;
        return hst(e);
    }
    for (const auto &f : b.fold_slots) b.s_slot[b.slot_entry[f.first].group] = f.first;
    return AWG_OK;
}

}  // namespace

bool plb_eligible(const awg_plan *p)
{
    const uint32_t pl = p->params.period_log2;
    if (pl < 10 || pl > 24 || p->n_tones <= 0) return false;
    const int32_t ng = groups_of(p->n_tones);
    return plb_bytes(1ull << pl, ng, 2 * ng + kMaxSegs) <= kMaxBytes;
}

void plb_release(awg_plan *p)
{
    LineBuf *b = p->plb;
    if (!b) return;
    if (b->work_done) (void)hipEventSynchronize(b->work_done);
    for (auto &sl : b->slots) {
        if (sl.done) (void)hipEventSynchronize(sl.done);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (b->d_S) (void)hipFree(b->d_S);
    if (b->d_Q) (void)hipFree(b->d_Q);
    if (b->d_bwork) (void)hipFree(b->d_bwork);
    if (b->work_done) (void)hipEventDestroy(b->work_done);
    delete b;
    p->plb = nullptr;
}

size_t plb_bytes_of(const awg_plan *p)
{
    const LineBuf *b = p->plb;
    if (!b) return 0;
    size_t n = plb_bytes(b->L, b->n_groups, b->n_slots);
    for (const auto &sl : b->slots) n += sl.cap;
    return n;
}

// The buffer for `method` (a change of method, or of the tone count, starts over).
static awg_status plb_state(awg_plan *p, uint32_t method, LineBuf **out)
{
    if (p->plb && (p->plb->method != method || p->plb->K != p->n_tones)) plb_release(p);
    if (!p->plb) {
        try { p->plb = new LineBuf(); } catch (...) { return AWG_E_NOMEM; }
        const awg_status st = setup(*p->plb, p, method);
        if (st != AWG_OK) {
            plb_release(p);
            return st;
        }
    }
    *out = p->plb;
    return AWG_OK;
}

awg_status plb_reserve(awg_plan *p, uint32_t method)
{
    LineBuf *b = nullptr;
    return plb_state(p, method, &b);
}

// A range of at most kPiece samples as one pass, or halved (at a row boundary)
// while a pass would need too many segments; a pass of one row has none.
static awg_status run(awg_plan *p, LineBuf &b, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32,
                      hipStream_t s)
{
    bool split = false;
    awg_status st = pass(p, b, n0, count, out_i16, out_f32, s, &split);
    if (st != AWG_OK || !split) return st;
    const uint64_t rows = (count + kRow - 1) / kRow;
    const uint64_t half = rows / 2 * kRow;
    st = run(p, b, n0, half, out_i16, out_f32, s);
    if (st != AWG_OK) return st;
    return run(p, b, n0 + half, count - half, out_i16 ? out_i16 + half : nullptr, out_f32 ? out_f32 + half : nullptr, s);
}

awg_status plb_synth(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32,
                     hipStream_t s)
{
    LineBuf *b = nullptr;
    awg_status st = plb_state(p, method, &b);
    if (st != AWG_OK) return st;
    std::lock_guard<std::mutex> lock(b->mu);
    while (count > 0) {
        const uint64_t now = count < kPiece ? count : kPiece;
        st = run(p, *b, n0, now, out_i16, out_f32, s);
        if (st != AWG_OK) return st;
        n0 += now;
        count -= now;
        if (out_i16) out_i16 += now;
        if (out_f32) out_f32 += now;
    }
    return AWG_OK;
}

}  // namespace awg
