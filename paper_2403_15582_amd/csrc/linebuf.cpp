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
//  * a tone's "next" line is the one it is on at the call's last row: the
//    line before or after its windows, or none (zero amplitude) while they are
//    open there; each group's version of next lines is folded into S before
//    the call is summed;
//  * on the rows its windows meet, a tone runs on the direct kernel with its
//    exact phase and holds no line;
//  * on the call's rows where a group holds another version than its next one
//    (lines before a window, none on window rows, lines after), each run of
//    rows with one version adds Q(row version) - Q(next version)
//    ("segments").
// The direct kernel adds, per tile, S, the segments and its own sum, and rounds.
// Versions that only segments need are made on the tile rows of the period
// (2^18 samples each) their segments cover. A one-row pass that would need more
// segments than a pass takes runs with next lines of none for every tone whose
// windows meet it (no segments at all).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "awg_internal.h"

namespace awg {

namespace {

constexpr int32_t kGroupTones = 128;                 // tones per group (16 k-blocks)
constexpr int kTileLog2 = 18;                        // samples per tile row of the group product (256 rows)
constexpr uint64_t kRow = kTileSamples;
constexpr uint64_t kPiece = 1ull << 22;               // samples per pass
constexpr uint64_t kCntWords = kPiece / kTileSamples / 2;   // split-tile counters (int32, two per word)
constexpr int32_t kMaxSegs = 64;                      // segments of one pass (more: the pass is halved)
constexpr int32_t kBuildBatch = 32;                   // groups per product launch
constexpr int kSlots = 4;                             // pinned staging slots in flight
constexpr size_t kMaxBytes = 16ull << 30;             // device memory of the buffer and its cache
constexpr int32_t kMaxParts = 1024;                   // partial sums of split tiles per pass (4 MiB)
constexpr int32_t kPartPieces = 4;                    // pieces per part: one per wave
constexpr int32_t kPieceTones = 2;                    // tones per piece of a block with a window edge in the row
constexpr int32_t kMaxPieces = kMaxParts * kPartPieces;

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
    float *d_part = nullptr;              // kMaxParts partial tile sums
    int32_t *d_cnt = nullptr;             // per split tile of a launch: parts done (zero between launches)
    void *d_bwork = nullptr;              // product operands of one batch of groups
    size_t bwork_bytes = 0;
    bool s_zeroed = false;
    int last_slot = -1;                   // staging slot of the latest pass (its event ends that pass)
    hipStream_t last_stream = nullptr;
    // cache of group sums: per group, version hash -> slot; the slot's words
    // valid: the tile rows of the period (2^18 samples each) that the slot's
    // sum holds; a version that only segments need is made on their rows only
    struct Entry { int32_t group; uint64_t hash; uint64_t last_use; bool live; std::vector<Line> words; uint64_t valid = 0; };
    std::vector<Entry> slot_entry;        // per slot
    std::vector<std::unordered_multimap<uint64_t, int32_t>> index;   // per group
    std::vector<int32_t> free_slots;
    std::vector<int32_t> s_slot;          // per group: the slot S holds (-1: none)
    uint64_t tick = 0;
    // staging
    struct Slot {
        void *host = nullptr, *mapped = nullptr, *dev = nullptr;
        size_t cap_h = 0, cap_d = 0;
        hipEvent_t done = nullptr;
        bool used = false;
    };
    Slot slots[kSlots];
    int next_slot = 0;
    // host scratch of one pass
    std::vector<Line> next;               // per tone: the line at the last sample of the latest pass
    bool next_held = false;               // S holds exactly the versions of `next` (the latest pass completed)
    // a pass looks at every tone (full), or at the tones whose windows were
    // ahead or open at the previous pass (live) and those changed since
    bool full = true;
    uint64_t prev_n0 = 0;
    std::vector<int32_t> live, live2, changed, todo;   // device positions
    std::vector<uint32_t> seen;
    uint32_t seen_gen = 0;
    std::vector<uint8_t> dirty;           // per group: a tone's next line changed in this pass
    // per tone whose windows meet the pass (wlo >= 0): its window rows and its
    // lines before (l1) and after (l2) them
    std::vector<int32_t> wlo, whi;
    std::vector<Line> l1, l2;
    struct Win { int32_t k; int32_t lo, hi; };
    std::vector<Win> win;                 // tones whose windows meet the pass: their window rows
    std::vector<std::pair<int32_t, uint32_t>> gsw;   // distinct (group, row where a line starts or ends), sorted
    std::vector<uint32_t> didx;           // sort order of a part of the direct list
    std::vector<PlbDesc> dsorted;
    std::vector<PlbDesc> build_list;      // kGroupTones lines per version to build
    std::vector<PlbDesc> direct;          // the tones whose windows meet the pass
    std::vector<int32_t> key, cnt;        // tile order
    std::vector<int32_t> blo, bhi;        // per block: the rows its tones are summed on
    std::vector<int32_t> span;            // the same, interleaved (staged)
    std::vector<PlbItem> items;           // work items: parts of split tiles, then whole tiles
    std::vector<PlbPiece> pieces;
    std::vector<PlbSplit> splits;
    std::vector<uint8_t> is_split;        // per row
    std::vector<int32_t> build_map;
    std::vector<int32_t> build_rng;       // per build: first tile row, tile rows
    int32_t n_tiles = 1;                  // tile rows of the period
    uint64_t all_tiles = 1;
    std::vector<PlbSeg> segs;
    std::vector<PlbFold> folds;
    std::vector<int32_t> seg_slot;        // slots of the segments (pointers filled at staging)
    std::vector<int32_t> seg_next;
    std::vector<std::pair<int32_t, int32_t>> fold_slots;
    std::vector<Block> blocks;
    std::vector<uint32_t> order;
    std::vector<float> cost;
    std::vector<int32_t> pinned;          // per slot: pass stamp
    std::vector<Line> ver;
};

namespace {

size_t plb_bytes(uint64_t L, int32_t n_groups, int32_t n_slots)
{
    return sizeof(int64_t) * L + sizeof(float) * L * (size_t)n_slots + group_work_bytes(kBuildBatch, kGroupTones, L) +
           sizeof(float) * kRow * kMaxParts;
}

int32_t groups_of(int32_t K) { return (K + kGroupTones - 1) / kGroupTones; }

// Entries of the largest pass: a version of every group and one per segment
// (build list), every tone (direct list).
size_t max_entries(const LineBuf &b) { return (size_t)(b.n_groups + kMaxSegs) * kGroupTones + (size_t)b.K; }

// The part of a staging blob copied as it is: build map, blocks, work items,
// pieces, split tiles, segments, folds (at their largest).
size_t raw_cap(const LineBuf &b)
{
    const size_t ng = (size_t)b.n_groups, K = (size_t)b.K, nb = ng + kMaxSegs, rows = kPiece / kRow;
    return align_up(sizeof(ToneDev) * K, 256) + align_up(sizeof(int32_t) * nb, 256) +
           align_up(sizeof(int32_t) * 2 * nb, 256) +
           align_up(sizeof(Block) * (2 * K + 1), 256) +
           align_up(sizeof(PlbItem) * (rows + kMaxParts), 256) + align_up(sizeof(PlbPiece) * kMaxPieces, 256) +
           align_up(sizeof(int32_t) * 2 * (2 * K + 1), 256) +
           align_up(sizeof(PlbSplit) * rows, 256) + align_up(sizeof(PlbSeg) * kMaxSegs, 256) +
           align_up(sizeof(PlbFold) * ng, 256);
}

// Host blob: descriptors, then the raw part. Device blob: the build list's and
// the direct list's records, then the raw part.
size_t host_cap(const LineBuf &b) { return align_up(sizeof(PlbDesc) * max_entries(b), 256) + raw_cap(b); }
size_t dev_cap(const LineBuf &b) { return align_up(sizeof(ToneDev) * max_entries(b), 256) + 256 + raw_cap(b); }

// A line as a staged entry (no window), amplitude times sign.
PlbDesc line_desc(const Line &l, float sign, int32_t lo_row = -1, int32_t hi_row = -1)
{
    return PlbDesc{l.p, l.f, sign * l.a, -1, lo_row, hi_row};
}

// The fields that cut blocks, shared by every line record
ToneDev line_key()
{
    ToneDev t;
    std::memset(&t, 0, sizeof(t));
    t.a = UINT64_MAX;
    t.shape = AWG_RAMP_NONE;
    t.ashape = AWG_RAMP_NONE;
    return t;
}

// Three independent hash chains (words, frequencies, amplitudes) joined at the end.
uint64_t version_hash(const Line *w, int32_t n)
{
    uint64_t h0 = 0x243f6a8885a308d3ull, h1 = 0x13198a2e03707344ull, h2 = 0xa4093822299f31d0ull;
    for (int32_t i = 0; i < n; ++i) {
        h0 = mix(h0, w[i].p);
        h1 = mix(h1, w[i].f);
        h2 = mix(h2, fbits(w[i].a));
    }
    return mix(mix(h0, h1), h2);
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

// The tile rows of the period (2^18 samples each) that the call rows
// [begin, end) of a pass from n0 cover (m = n mod L; they may wrap round).
uint64_t tiles_of_rows(const LineBuf &b, uint64_t n0, uint32_t begin, uint32_t end)
{
    const uint64_t len = (uint64_t)(end - begin) * kRow;
    if (len >= b.L || b.n_tiles == 1) return b.all_tiles;
    const uint64_t m0 = (n0 + (uint64_t)begin * kRow) & (b.L - 1), m1 = m0 + len - 1;
    const int32_t t0 = (int32_t)(m0 >> kTileLog2);
    auto span = [](int32_t lo, int32_t hi) {
        return (hi == 63 ? ~0ull : (1ull << (hi + 1)) - 1) & ~((1ull << lo) - 1);
    };
    if (m1 < b.L) return span(t0, (int32_t)(m1 >> kTileLog2));
    return span(t0, b.n_tiles - 1) | span(0, (int32_t)((m1 - b.L) >> kTileLog2));
}

// Slot of group g's version w for this pass (stamp), with at least the tile
// rows `want`: cached, or a new one; the tile rows it lacks (their hull) are
// added to the build list.
int32_t need(LineBuf &b, int32_t g, const Line *w, int32_t n, int32_t stamp, uint64_t want)
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
        e.valid = 0;
        e.words.assign(w, w + n);
        b.index[g].emplace(h, s);
    }
    LineBuf::Entry &e = b.slot_entry[s];
    const uint64_t make = want & ~e.valid;
    if (make) {
        const int32_t lo = __builtin_ctzll(make), hi = 63 - __builtin_clzll(make);
        const uint64_t hull = (hi == 63 ? ~0ull : (1ull << (hi + 1)) - 1) & ~((1ull << lo) - 1);
        for (int32_t i = 0; i < kGroupTones; ++i)
            b.build_list.push_back(i < n ? line_desc(e.words[i], 1.0f) : line_desc(kNoLine, 0.0f));
        b.build_map.push_back(s);
        b.build_rng.push_back(lo);
        b.build_rng.push_back(hi - lo + 1);
        e.valid |= hull;
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
    b.n_tiles = (int32_t)std::max<uint64_t>(1, b.L >> kTileLog2);
    b.all_tiles = b.n_tiles >= 64 ? ~0ull : (1ull << b.n_tiles) - 1;
    hipError_t e = hipMalloc(&b.d_S, sizeof(int64_t) * b.L);
    if (e == hipSuccess) e = hipMalloc(&b.d_Q, sizeof(float) * b.L * (size_t)b.n_slots);
    if (e == hipSuccess) e = hipMalloc(&b.d_bwork, b.bwork_bytes);
    if (e == hipSuccess) e = hipMalloc(&b.d_part, sizeof(float) * kRow * kMaxParts);
    if (e == hipSuccess) e = hipMalloc(&b.d_cnt, sizeof(int64_t) * kCntWords);
    const size_t ch = host_cap(b), cd = dev_cap(b);
    for (auto &sl : b.slots) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = alloc_upload_host(ch, &sl.host, &sl.mapped);
        if (e == hipSuccess) e = hipMalloc(&sl.dev, cd);
        if (e == hipSuccess) {
            sl.cap_h = ch;
            sl.cap_d = cd;
        }
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

// Work items of a pass. A row's cost: 1 per window tone summed on it, 3.5 more
// per window that opens or closes inside it. All
// rows of a 2^20-sample call run at once (four workgroups per compute unit),
// so the costliest rows would set the launch time: rows above 1.5 times the
// mean are split into parts of kPartPieces pieces (one per wave), a piece
// being a block or, for a block with a window edge in the row, kPieceTones of
// its tones; the parts run first and write partial sums, which the part that
// finishes last adds in part order. Whole rows follow, costliest first: those that
// find no free slot start when the first parts end, so small parts keep the
// launch near the time of one whole row. Costs are
// multiples of 1/2, so the order is a counting sort on twice the cost, rows of
// equal cost in row order.
void plan_items(LineBuf &b, const awg_plan *p, uint64_t n0, uint64_t rows)
{
    const uint64_t last = n0 + rows * kRow - 1;
    auto edge_in = [&](uint64_t x) { return x >= n0 && x <= last && (x - n0) % kRow != 0; };
    b.cost.assign(rows + 1, 0.0f);
    for (const LineBuf::Win &w : b.win) {
        b.cost[w.lo] += 1.0f;
        b.cost[w.hi + 1] -= 1.0f;
    }
    float run = 0.0f;
    for (uint64_t r = 0; r < rows; ++r) {
        run += b.cost[r];
        b.cost[r] = run;
    }
    for (const PlbDesc &d : b.direct) {
        if (d.src < 0) continue;
        const ToneDev &t = p->dev_mirror[d.src];
        if (t.shape == AWG_RAMP_NONE && t.ashape == AWG_RAMP_NONE) continue;
        const uint64_t ends[2] = {t.a, t.a + t.n};
        for (uint64_t x : ends)
            if (edge_in(x)) b.cost[(x - n0) / kRow] += 3.5f;
    }
    b.key.resize(rows);
    int32_t top = 0;
    double total = 0.0;
    for (uint64_t r = 0; r < rows; ++r) {
        b.key[r] = (int32_t)(2.0f * b.cost[r] + 0.5f);
        top = std::max(top, b.key[r]);
        total += b.cost[r];
    }
    b.cnt.assign((size_t)top + 2, 0);
    for (uint64_t r = 0; r < rows; ++r) b.cnt[top - b.key[r] + 1]++;
    for (int32_t c = 1; c <= top + 1; ++c) b.cnt[c] += b.cnt[c - 1];
    b.order.resize(rows);
    for (uint64_t r = 0; r < rows; ++r) b.order[b.cnt[top - b.key[r]]++] = (uint32_t)r;

    // the rows each block's tones are summed on, and whether a window of its
    // (uniform) tones opens or closes inside a row of the pass
    const int32_t nbk = (int32_t)b.blocks.size() - 1;
    b.blo.assign(nbk, INT32_MAX);
    b.bhi.assign(nbk, -1);
    for (int32_t bi = 0; bi < nbk; ++bi) {
        const Block &bk = b.blocks[1 + bi];
        for (uint32_t k = bk.begin; k < bk.begin + bk.count; ++k) {
            b.blo[bi] = std::min(b.blo[bi], b.direct[k].lo_row);
            b.bhi[bi] = std::max(b.bhi[bi], b.direct[k].hi_row);
        }
    }
    b.span.resize(2 * (size_t)nbk);
    for (int32_t bi = 0; bi < nbk; ++bi) {
        b.span[2 * bi] = b.blo[bi];
        b.span[2 * bi + 1] = b.bhi[bi];
    }
    b.items.clear();
    b.pieces.clear();
    b.splits.clear();
    b.is_split.assign(rows, 0);
    const float thr = std::max(1.5f * (float)(total / (double)rows), 16.0f);
    int32_t slots = 0;
    for (uint64_t oi = 0; oi < rows; ++oi) {
        const uint32_t r = b.order[oi];
        if (b.cost[r] <= thr) break;
        const size_t first = b.pieces.size();
        for (int32_t bi = 0; bi < nbk; ++bi) {
            if (b.blo[bi] > (int32_t)r || b.bhi[bi] < (int32_t)r) continue;
            const Block &bk = b.blocks[1 + bi];
            bool cut = false;
            if (bk.flags & kBlockUniform) {
                const PlbDesc &d = b.direct[bk.begin];
                if (d.src >= 0) {
                    const ToneDev &t = p->dev_mirror[d.src];
                    const uint64_t x0 = t.a, x1 = t.a + t.n;
                    cut = t.shape != AWG_RAMP_NONE && ((edge_in(x0) && (x0 - n0) / kRow == r) ||
                                                       (edge_in(x1) && (x1 - n0) / kRow == r));
                }
            }
            if (!cut) {
                b.pieces.push_back(PlbPiece{(uint32_t)bi, 0, 0});
                continue;
            }
            for (uint32_t o = 0; o < bk.count; o += kPieceTones)
                b.pieces.push_back(PlbPiece{(uint32_t)bi, (uint16_t)o,
                                            (uint16_t)std::min<uint32_t>(kPieceTones, bk.count - o)});
        }
        const int32_t n_pc = (int32_t)(b.pieces.size() - first);
        const int32_t P = (n_pc + kPartPieces - 1) / kPartPieces;
        if (P < 2 || slots + P > kMaxParts) {
            b.pieces.resize(first);
            continue;
        }
        const int32_t si = (int32_t)b.splits.size();
        b.splits.push_back(PlbSplit{r, (uint32_t)slots, (uint32_t)P, 0});
        for (int32_t q = 0; q < P; ++q)
            b.items.push_back(PlbItem{r, slots + q, (uint32_t)(first + (size_t)q * kPartPieces),
                                      (uint32_t)std::min<int32_t>(kPartPieces, n_pc - q * kPartPieces), si});
        slots += P;
        b.is_split[r] = 1;
    }
    for (uint64_t oi = 0; oi < rows; ++oi)
        if (!b.is_split[b.order[oi]]) b.items.push_back(PlbItem{b.order[oi], -1, 0, 0, -1});
}

// Order of the direct list: plan tones (ramped ones first, then by window,
// table and amplitude window, then window rows) and after them the negative
// lines by window rows, ties in list order. The tones arrive in the plan's
// device order, which is the same for the first keys (so that a call whose
// tones all ramp sums them as the direct kernel does), and the lines in their
// tones' order; each part is sorted only if it is not in order already.
void sort_part(LineBuf &lb, const awg_plan *p, std::vector<PlbDesc> *v)
{
    const ToneDev lk = line_key();
    auto rec = [&](const PlbDesc &d) -> const ToneDev & { return d.src >= 0 ? p->dev_mirror[d.src] : lk; };
    auto less = [&](const PlbDesc &x, const PlbDesc &y) {
        const ToneDev &a = rec(x), &b = rec(y);
        const bool la = a.shape == AWG_RAMP_NONE, lb = b.shape == AWG_RAMP_NONE;
        if (la != lb) return lb;
        if (a.shape != b.shape) return a.shape < b.shape;
        if (a.a != b.a) return a.a < b.a;
        if (a.n != b.n) return a.n < b.n;
        if (a.table != b.table) return a.table < b.table;
        if (a.ashape != b.ashape) return a.ashape < b.ashape;
        if (a.b != b.b) return a.b < b.b;
        if (a.m != b.m) return a.m < b.m;
        return x.lo_row < y.lo_row;
    };
    bool sorted = true;
    for (size_t i = 1; sorted && i < v->size(); ++i) sorted = !less((*v)[i], (*v)[i - 1]);
    if (sorted) return;
    lb.didx.resize(v->size());
    for (size_t i = 0; i < v->size(); ++i) lb.didx[i] = (uint32_t)i;
    std::sort(lb.didx.begin(), lb.didx.end(), [&](uint32_t x, uint32_t y) {
        if (less((*v)[x], (*v)[y])) return true;
        if (less((*v)[y], (*v)[x])) return false;
        return x < y;
    });
    lb.dsorted.resize(v->size());
    for (size_t i = 0; i < v->size(); ++i) lb.dsorted[i] = (*v)[lb.didx[i]];
    v->swap(lb.dsorted);
}

// The synthesis record of an entry of the direct list, as the staging kernel
// makes it from the descriptor: a plan tone (the host mirror of the plan's
// device table) or a static line, with the window rows from n0.
ToneDev direct_record(const awg_plan *p, const PlbDesc &d, uint64_t n0)
{
    ToneDev t;
    if (d.src >= 0) {
        t = p->dev_mirror[d.src];
    } else {
        t.p0 = t.p1 = d.p + kPhaseBias;
        t.f0 = t.f1 = d.f;
        t.a = UINT64_MAX;
        t.coef = 0;
        t.n = 0;
        t.amp = t.amp1 = d.a;
        t.shape = AWG_RAMP_NONE;
        t.table = 0;
        t.ashape = AWG_RAMP_NONE;
        t.pad = 0;
        t.b = 0;
        t.m = 0;
    }
    if (d.lo_row >= 0) {
        t.lo = n0 + (uint64_t)d.lo_row * kTileSamples;
        t.hi = n0 + (uint64_t)d.hi_row * kTileSamples + (kTileSamples - 1);
    } else {
        t.lo = 1;
        t.hi = 0;
    }
    return t;
}

// One pass of at most kPiece samples. *split: the pass needs more than kMaxSegs
// segments and nothing was done (the caller halves it).
awg_status pass(awg_plan *p, LineBuf &b, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32, hipStream_t s,
                bool through, bool *split)
{
    *split = false;
    const uint64_t rows = (count + kRow - 1) / kRow;
    const uint64_t last = n0 + count - 1;
    const int32_t K = b.K;
    b.tick++;
    const int32_t stamp = (int32_t)(b.tick & 0x7fffffff);
    // the previous pass's next lines are what S holds only if it completed
    const bool held = b.next_held && (int32_t)b.next.size() == K;
    const bool incremental = held && !b.full && n0 >= b.prev_n0 && (int32_t)b.wlo.size() == K;
    b.next_held = false;
    b.full = true;                 // until this pass completes
    b.next.resize(K);
    b.dirty.assign(b.n_groups, held ? 0 : 1);
    if ((int32_t)b.wlo.size() != K) b.wlo.assign(K, -1);
    for (const LineBuf::Win &w : b.win) b.wlo[w.k] = -1;
    b.whi.resize(K);
    b.l1.resize(K);
    b.l2.resize(K);
    b.win.clear();
    // the tones to look at, in device order: on a forward call after a
    // completed pass, those whose windows were ahead or open then and those
    // changed since (every other tone is on the line it was on, before any
    // window or after its last one); else every tone
    b.todo.clear();
    if (incremental) {
        b.seen.resize(K);
        if (++b.seen_gen == 0) {
            std::fill(b.seen.begin(), b.seen.end(), 0u);
            b.seen_gen = 1;
        }
        for (const int32_t i : b.live) {
            b.seen[i] = b.seen_gen;
            b.todo.push_back(i);
        }
        for (const int32_t i : b.changed)
            if (b.seen[i] != b.seen_gen) {
                b.seen[i] = b.seen_gen;
                b.todo.push_back(i);
            }
        std::sort(b.todo.begin(), b.todo.end());
    } else {
        b.todo.resize(K);
        for (int32_t i = 0; i < K; ++i) b.todo[i] = i;
    }
    b.changed.clear();
    b.live2.clear();
    b.gsw.clear();
    b.build_list.clear();
    b.build_map.clear();
    b.build_rng.clear();
    b.direct.clear();
    b.segs.clear();
    b.seg_slot.clear();
    b.seg_next.clear();
    b.fold_slots.clear();
    double direct_work = 0.0;
    for (const int32_t i : b.todo) {               // device order
        const ToneDev &t = p->dev_mirror[i];
        const int32_t k = p->perm[i];
        const bool windowed = t.lo <= t.hi;
        if (windowed && t.hi >= n0) b.live2.push_back(i);
        const bool meets = windowed && t.hi >= n0 && t.lo <= last;
        // the line the tone is on at the call's last row: none while its
        // windows are open there (it runs on the direct kernel); without
        // `through`, none for every tone whose windows meet the call (its window
        // rows then need no segment)
        const Line nx = !windowed || last < t.lo    ? line_of(t.p0 - kPhaseBias, t.f0, t.amp)
                        : last > t.hi && (through || !meets) ? line_of(t.p1 - kPhaseBias, t.f1, t.amp1)
                                                     : kNoLine;
        if (nx != b.next[k]) {
            b.next[k] = nx;
            b.dirty[k / kGroupTones] = 1;
        }
        if (meets) {
            const uint64_t lo = t.lo <= n0 ? 0 : (t.lo - n0) / kRow;
            const uint64_t hi = std::min<uint64_t>(rows - 1, (t.hi - n0) / kRow);
            b.win.push_back(LineBuf::Win{k, (int32_t)lo, (int32_t)hi});
            b.wlo[k] = (int32_t)lo;
            b.whi[k] = (int32_t)hi;
            b.l1[k] = line_of(t.p0 - kPhaseBias, t.f0, t.amp);
            b.l2[k] = line_of(t.p1 - kPhaseBias, t.f1, t.amp1);
            // rows before and after the window rows that the call covers; a
            // tone whose next line is l2 also needs its window rows' run (its
            // group has a run even when those rows are all of the call's)
            if ((lo > 0 && b.l1[k] != kNoLine) || nx != kNoLine) b.gsw.emplace_back(k / kGroupTones, (uint32_t)lo);
            if (hi + 1 < rows && b.l2[k] != kNoLine) b.gsw.emplace_back(k / kGroupTones, (uint32_t)(hi + 1));
            // the tone on its window rows
            b.direct.push_back(PlbDesc{0, 0, 0.0f, i, (int32_t)lo, (int32_t)hi});
            direct_work += (double)(std::min(n0 + hi * kRow + (kRow - 1), last) - (n0 + lo * kRow) + 1);
        }
    }
    b.live.swap(b.live2);
    // segments of the pass: per group, the runs of rows between the rows where
    // a line starts or ends (at most one more than those rows; counted before
    // the cache is touched)
    std::sort(b.gsw.begin(), b.gsw.end());
    b.gsw.erase(std::unique(b.gsw.begin(), b.gsw.end()), b.gsw.end());
    {
        int64_t n_runs = 0;
        for (size_t x = 0; x < b.gsw.size(); ++x)
            n_runs += (x == 0 || b.gsw[x].first != b.gsw[x - 1].first) ? 2 : 1;
        if (n_runs > kMaxSegs) {
            *split = true;        // next[] is this range's, not what S holds
            return AWG_OK;
        }
    }
    // versions: each group's next version (held by S), and the versions of its
    // rows before the switch rows of its tones
    size_t gi = 0;
    for (int32_t g = 0; g < b.n_groups; ++g) {
        const int32_t k0 = g * kGroupTones, n = std::min(kGroupTones, K - k0);
        // most groups keep the version S already holds: no line of theirs
        // changed since a completed pass (or their words equal it), so no hash
        int32_t snext = b.s_slot[g];
        if (snext >= 0 && b.slot_entry[snext].live &&
            (!b.dirty[g] || std::equal(b.slot_entry[snext].words.begin(), b.slot_entry[snext].words.end(),
                                       &b.next[k0], &b.next[k0] + n))) {
            b.slot_entry[snext].last_use = b.tick;
            b.pinned[snext] = stamp;
        } else {
            snext = need(b, g, &b.next[k0], n, stamp, b.all_tiles);
        }
        if (snext < 0) return AWG_E_NOMEM;
        if (b.s_slot[g] != snext) b.fold_slots.emplace_back(snext, b.s_slot[g]);
        // runs [begin, end) between this group's line rows: each tone whose
        // windows meet the call is on l1 before its window rows, on l2 after
        // them, and on none (the direct kernel) on them
        const size_t g_end = [&] {
            size_t x = gi;
            while (x < b.gsw.size() && b.gsw[x].first == g) ++x;
            return x;
        }();
        if (gi == g_end) continue;
        uint32_t begin = 0;
        for (size_t x = gi; x <= g_end; ++x) {
            const uint32_t end = x < g_end ? b.gsw[x].second : (uint32_t)rows;
            if (end <= begin) continue;
            b.ver.assign(&b.next[k0], &b.next[k0] + n);
            bool differs = false;          // from the group's next version
            for (int32_t i = 0; i < n; ++i) {
                const int32_t k = k0 + i;
                if (b.wlo[k] < 0) continue;
                const Line l = (int32_t)begin < b.wlo[k] ? b.l1[k] : ((int32_t)begin > b.whi[k] ? b.l2[k] : kNoLine);
                b.ver[i] = l;
                differs = differs || l != b.next[k];
            }
            if (differs) {
                const int32_t sv = need(b, g, b.ver.data(), n, stamp, tiles_of_rows(b, n0, begin, end));
                if (sv < 0) return AWG_E_NOMEM;
                b.segs.push_back(PlbSeg{begin, end - 1, nullptr, nullptr});
                b.seg_slot.push_back(sv);
                b.seg_next.push_back(snext);
            }
            begin = end;
        }
        gi = g_end;
    }
    sort_part(b, p, &b.direct);
    {
        const ToneDev lk = line_key();
        build_blocks_by((int32_t)b.direct.size(), (int32_t)b.direct.size(),
                        [&](int32_t i) -> const ToneDev & {
                            return b.direct[i].src >= 0 ? p->dev_mirror[b.direct[i].src] : lk;
                        },
                        &b.blocks);
    }
    plan_items(b, p, n0, rows);

    // host blob: descriptors (build list, then direct list) | raw part
    // device blob: build records | direct records | raw part
    // raw part: build map | blocks | work items | pieces | split tiles | segments | folds
    // With the prep launch (below) the direct list goes as records made here,
    // at the head of the raw part, and no descriptor of it is staged.
    const int32_t n_built = (int32_t)b.build_map.size();
    const bool prep = n_built > 0 && n_built <= kBuildBatch;
    const int32_t n_be = (int32_t)b.build_list.size();
    const int32_t n_direct = (int32_t)b.direct.size();
    const int32_t n_seg = (int32_t)b.segs.size();
    const int32_t n_fold = (int32_t)b.fold_slots.size();
    const int32_t n_items = (int32_t)b.items.size();
    const int32_t n_split = (int32_t)b.splits.size();
    const size_t r_m = prep ? align_up(sizeof(ToneDev) * (size_t)n_direct, 256) : 0;
    const size_t r_g = r_m + align_up(sizeof(int32_t) * (size_t)n_built, 256);
    const size_t r_b = r_g + align_up(sizeof(int32_t) * 2 * (size_t)n_built, 256);
    const size_t r_o = r_b + align_up(sizeof(Block) * b.blocks.size(), 256);
    const size_t r_p = r_o + align_up(sizeof(PlbItem) * (size_t)n_items, 256);
    const size_t r_x = r_p + align_up(sizeof(PlbPiece) * b.pieces.size(), 256);
    const size_t r_y = r_x + align_up(sizeof(PlbSplit) * (size_t)n_split, 256);
    const size_t r_s = r_y + align_up(sizeof(int32_t) * b.span.size(), 256);
    const size_t r_f = r_s + align_up(sizeof(PlbSeg) * (size_t)n_seg, 256);
    const size_t raw = align_up(r_f + sizeof(PlbFold) * (size_t)n_fold, 16);
    const size_t h_raw = align_up(sizeof(PlbDesc) * (size_t)(n_be + (prep ? 0 : n_direct)), 256);
    const size_t d_dir = align_up(sizeof(ToneDev) * (size_t)n_be, 256);
    const size_t d_raw = align_up(d_dir + sizeof(ToneDev) * (size_t)n_direct, 256);
    LineBuf::Slot &slot = b.slots[b.next_slot];
    const int this_slot = b.next_slot;
    b.next_slot = (b.next_slot + 1) % kSlots;
    if (h_raw + raw > slot.cap_h || d_raw + raw > slot.cap_d) return AWG_E_UNSUPPORTED;
    hipError_t e = slot.used ? hipEventSynchronize(slot.done) : hipSuccess;
    if (e != hipSuccess) return hst(e);
    slot.used = false;
    char *hb = (char *)slot.host;
    char *db = (char *)slot.dev;
    PlbDesc *hd = (PlbDesc *)hb;
    if (n_be) std::memcpy(hd, b.build_list.data(), sizeof(PlbDesc) * (size_t)n_be);
    char *hr = hb + h_raw;
    if (prep) {
        ToneDev *dr_h = (ToneDev *)hr;
        for (int32_t i = 0; i < n_direct; ++i) dr_h[i] = direct_record(p, b.direct[i], n0);
    } else if (n_direct) {
        std::memcpy(hd + n_be, b.direct.data(), sizeof(PlbDesc) * (size_t)n_direct);
    }
    if (n_built) std::memcpy(hr + r_m, b.build_map.data(), sizeof(int32_t) * (size_t)n_built);
    if (n_built) std::memcpy(hr + r_g, b.build_rng.data(), sizeof(int32_t) * 2 * (size_t)n_built);
    std::memcpy(hr + r_b, b.blocks.data(), sizeof(Block) * b.blocks.size());
    std::memcpy(hr + r_o, b.items.data(), sizeof(PlbItem) * (size_t)n_items);
    if (!b.pieces.empty()) std::memcpy(hr + r_p, b.pieces.data(), sizeof(PlbPiece) * b.pieces.size());
    if (n_split) std::memcpy(hr + r_x, b.splits.data(), sizeof(PlbSplit) * (size_t)n_split);
    if (!b.span.empty()) std::memcpy(hr + r_y, b.span.data(), sizeof(int32_t) * b.span.size());
    PlbSeg *sg = (PlbSeg *)(hr + r_s);
    for (int32_t i = 0; i < n_seg; ++i) {
        sg[i] = b.segs[i];
        sg[i].q_row = b.d_Q + (size_t)b.seg_slot[i] * b.L;
        sg[i].q_next = b.d_Q + (size_t)b.seg_next[i] * b.L;
    }
    PlbFold *fd = (PlbFold *)(hr + r_f);
    for (int32_t i = 0; i < n_fold; ++i) {
        fd[i].q_new = b.d_Q + (size_t)b.fold_slots[i].first * b.L;
        fd[i].q_old = b.fold_slots[i].second >= 0 ? b.d_Q + (size_t)b.fold_slots[i].second * b.L : nullptr;
    }
    // the previous pass's work (S, the cache) precedes this one on s
    if (b.last_slot >= 0 && b.last_stream != s) e = hipStreamWaitEvent(s, b.slots[b.last_slot].done, 0);
    // one product launch's worth of versions: their operands are made from the
    // descriptors in place, in the launch that stages the rest and applies a
    // retune's pending records to the plan's device table (nothing in that
    // launch reads the table); else the pending records are applied first, the
    // build list is staged too and the operands made per product launch
    if (e == hipSuccess && prep) {
        const void *rec = nullptr;
        int32_t n_rec = 0, rec_slot = -1;
        take_pending_tones(p, &rec, &n_rec, &rec_slot);
        e = launch_plb_prep(p, b.method, (const PlbDesc *)slot.mapped, n_built, kGroupTones, b.L,
                            (const int2 *)((const char *)slot.mapped + h_raw + r_g), b.d_bwork,
                            (const char *)slot.mapped + h_raw, db + d_raw, raw, rec, n_rec, s);
        if (rec_slot >= 0) {
            const awg_status st = pending_tones_applied(p, rec_slot, s);
            if (e == hipSuccess && st != AWG_OK) return st;
        }
    } else if (e == hipSuccess) {
        const awg_status st = flush_tones(p, s);
        if (st != AWG_OK) return st;
        e = launch_plb_stage((const PlbDesc *)slot.mapped, n_be, n_be + n_direct, p->d_tones, n0, (ToneDev *)db,
                             (ToneDev *)(db + d_dir), (const char *)slot.mapped + h_raw, db + d_raw, raw, s);
    }
    if (e == hipSuccess && !b.s_zeroed) {
        e = launch_plb_zero(b.d_S, b.L, s);
        if (e == hipSuccess) e = launch_plb_zero((int64_t *)b.d_cnt, kCntWords, s);
        if (e == hipSuccess) b.s_zeroed = true;
    }
    char *dr = db + d_raw;
    // the new versions' period sums, in batches
    for (int32_t i = 0; e == hipSuccess && i < n_built; i += kBuildBatch) {
        const int32_t nb = std::min(kBuildBatch, n_built - i);
        double work = 0.0;
        int32_t max_tiles = 1;
        for (int32_t z = i; z < i + nb; ++z) {
            const int32_t cnt = b.build_rng[2 * z + 1];
            max_tiles = std::max(max_tiles, cnt);
            work += (double)std::min(kGroupTones, K - b.slot_entry[b.build_map[z]].group * kGroupTones) *
                    (double)std::min<uint64_t>(b.L, (uint64_t)cnt << kTileLog2);
        }
        e = launch_group_sums(p, b.method, (const ToneDev *)db + (size_t)i * kGroupTones, nb, kGroupTones, b.L,
                              b.d_bwork, b.d_Q, (const int32_t *)(dr + r_m) + i, (const int2 *)(dr + r_g) + i, max_tiles,
                              prep, s, work);
    }
    // S to the call's next versions, then the call; a call of exactly one
    // period folds in the kernels that read S (each m is read once)
    const bool fused = count == b.L;
    if (e == hipSuccess && !fused) e = launch_plb_fold(p, b.d_S, b.L, (const PlbFold *)(dr + r_f), n_fold, s);
    if (e == hipSuccess)
        e = launch_plb(p, prep ? (const ToneDev *)dr : (const ToneDev *)(db + d_dir), (const Block *)(dr + r_b),
                       (const PlbItem *)(dr + r_o), n_items,
                       (const PlbPiece *)(dr + r_p), (const int2 *)(dr + r_y), b.d_part, (const PlbSplit *)(dr + r_x),
                       b.d_cnt, n_split, n0, count, b.d_S, b.L, (const PlbSeg *)(dr + r_s), n_seg,
                       (const PlbFold *)(dr + r_f), fused ? n_fold : 0, out_i16, out_f32, s, direct_work);
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    if (e == hipSuccess) {
        slot.used = true;
        b.last_slot = this_slot;
        b.last_stream = s;
    }
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
    b.next_held = true;
    b.full = false;
    b.prev_n0 = n0;
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
    for (auto &sl : b->slots) {
        if (sl.done) (void)hipEventSynchronize(sl.done);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (b->d_S) (void)hipFree(b->d_S);
    if (b->d_Q) (void)hipFree(b->d_Q);
    if (b->d_bwork) (void)hipFree(b->d_bwork);
    if (b->d_part) (void)hipFree(b->d_part);
    if (b->d_cnt) (void)hipFree(b->d_cnt);
    delete b;
    p->plb = nullptr;
}

size_t plb_bytes_of(const awg_plan *p)
{
    const LineBuf *b = p->plb;
    if (!b) return 0;
    size_t n = plb_bytes(b->L, b->n_groups, b->n_slots);
    for (const auto &sl : b->slots) n += sl.cap_d;
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

void plb_note_changed(awg_plan *p, const int32_t *dev_pos, int32_t n)
{
    LineBuf *b = p->plb;
    if (!b || n <= 0) return;
    std::lock_guard<std::mutex> lock(b->mu);
    if (b->full) return;                          // the next pass looks at every tone anyway
    if (b->changed.size() + (size_t)n > (size_t)b->K) {
        b->full = true;
        b->changed.clear();
        return;
    }
    b->changed.insert(b->changed.end(), dev_pos, dev_pos + n);
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
    awg_status st = pass(p, b, n0, count, out_i16, out_f32, s, true, &split);
    if (st != AWG_OK || !split) return st;
    const uint64_t rows = (count + kRow - 1) / kRow;
    if (rows <= 1) {
        // one row cannot be halved: without the after-window lines it has no
        // segments at all
        st = pass(p, b, n0, count, out_i16, out_f32, s, false, &split);
        if (st == AWG_OK && split) st = AWG_E_UNSUPPORTED;
        return st;
    }
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
