// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "awg.h"

namespace awg {

// Device phase words carry this constant offset: half a step of the 23-bit turn
// fraction handed to v_sin_f32, so that truncating to 23 bits rounds to nearest.
constexpr uint64_t kPhaseBias = 1ull << 40;

// Ramp tables hold 2^16 * N * Psi(d / N).
constexpr int kTableShift = 16;

// Direct kernel geometry: a workgroup is 4 waves covering the same 64 * S
// samples; the tone list is cut into blocks (see Block), block i is summed by
// wave i % 4, and the 4 wave sums are added in a fixed order.
constexpr int kWaves = 4;
constexpr int kLanes = 64;
constexpr int kBlock = 32;          // largest block

// One tone as the kernels read it (96 bytes, read with scalar loads).
// Tones without a frequency ramp have a = UINT64_MAX, n = 0 (their window never
// opens) and p1, f1 = p0, f0; without an amplitude ramp ashape = AWG_RAMP_NONE
// and amp1 = amp.
struct ToneDev {
    uint64_t p0, f0;     // line before the window: phi = p0 + f0 * n (p0 includes kPhaseBias)
    uint64_t p1, f1;     // line after the window (p1 includes kPhaseBias)
    uint64_t a;          // frequency window [a, a + n]
    int64_t coef;        // linear: R; smooth: dF
    uint32_t n;          // window length, < 2^31
    float amp;           // A_k * G before the amplitude window
    uint16_t shape;      // awg_ramp of the frequency window
    uint16_t table;      // index into the plan's table pointer array (smooth shapes)
    uint16_t ashape;     // awg_ramp profile of the amplitude window (AWG_RAMP_NONE: none)
    uint16_t pad;
    uint64_t b;          // amplitude window [b, b + m]
    uint32_t m;          // its length, < 2^31
    float amp1;          // A_k * G after the amplitude window
    uint64_t lo, hi;     // samples outside [lo, hi] are on a line at a constant amplitude
                         // (lo > hi: no window at all)
};
static_assert(sizeof(ToneDev) == 96, "ToneDev must be 96 bytes");

// Host copy of a tone's state (exact words without the device bias).
struct ToneHost {
    uint64_t p0, f0, p1, f1, a, n;
    int64_t coef;
    int32_t shape;
    double amp;          // A_k * G in FP64 (before the amplitude window)
    int32_t ashape;      // amplitude window profile, AWG_RAMP_NONE if none
    uint64_t b, m;       // amplitude window [b, b + m]
    double amp1;         // A_k * G after it
};

// A block of contiguous tones [begin, begin + count) of a tone list, summed by
// one wave as one FMA chain per sample. A table of blocks starts with a header
// entry whose `begin` is the number of blocks that follow; block i (0-based,
// after the header) belongs to wave i % kWaves. Runs of tones sharing shape,
// window and table are cut into near-equal blocks in multiples of kWaves, so a
// run that ramps while the rest of the list is on a line still spreads over
// all four waves.
struct Block {
    uint32_t begin;
    uint16_t count;
    uint16_t flags;
};
static_assert(sizeof(Block) == 8, "Block must be 8 bytes");
constexpr uint16_t kBlockUniform = 1;   // every tone shares the first one's shape, window and table
constexpr uint16_t kBlockSplit = 2;     // hybrid path: on line tiles the tones are summed elsewhere
constexpr uint16_t kBlockAmp = 4;       // some tone has an amplitude window
constexpr uint16_t kBlockStep16 = 8;    // uniform smooth block: every tone's dF is a multiple of 2^16

// One chunk of one plan in a batched launch (64 bytes).
struct BatchItem {
    const ToneDev *tones;
    const uint64_t *const *tables;
    void *out;               // int16 output of this chunk
    uint64_t n0, count;      // absolute first sample, samples in the chunk
    uint32_t tile_begin;     // first tile of this item in the launch
    int32_t n_tones;
    int32_t out_stride;      // output elements between consecutive samples (1: contiguous)
    int32_t is_static;       // 1: no tone has a window
    const Block *blocks;     // the plan's block table
};
static_assert(sizeof(BatchItem) == 64, "BatchItem must be 64 bytes");

// Samples per direct-kernel tile (4 waves x 64 lanes x 16 samples per lane).
constexpr int kTileSamples = 1024;

// Geometry of the hybrid path's product over count samples in rows of
// kTileSamples (one row = one direct-kernel tile): row blocks padded to whole
// 256-row tiles, 8-entry k-blocks, gz split-K slices of kb_split k-blocks, and
// gz FP32 planes of `plane` elements. Workspace: B hi, B lo (each laid out for
// kb_cap k-blocks, so the B operand keeps its place from call to call), A hi,
// A lo, planes.
struct LinesGeom {
    int32_t kb_n, kb_cap, rb_pad, cb_n, gz, kb_split;
    uint64_t plane;
    size_t a_bytes, b_bytes, plane_bytes;       // b_bytes: one half at kb_cap k-blocks
    size_t work_bytes() const { return 2 * (a_bytes + b_bytes) + plane_bytes; }
};

struct HybridState;
struct LineBuf;

struct Table {
    int32_t shape;
    uint64_t n;
    uint64_t *d_data;    // device, n + 1 entries
    bool monotone;       // never decreasing with steps below 2^23 (pointers handed out carry it in bit 0)
};

}  // namespace awg

namespace awg {
struct ProfRecord { const char *name; hipEvent_t start, stop; double work; };
struct ProfTotal { uint64_t launches; double total_ms, max_ms, work; };
}  // namespace awg

struct awg_ctx {
    int device;
    std::mutex mu;
    // kernel timing (awg_profile_*): 0 = off, n = one launch in n of each kernel
    std::atomic<int32_t> prof_period{0};
    std::mutex prof_mu;
    std::map<std::string, uint64_t> prof_seen;   // launches per kernel since enable
    std::vector<awg::ProfRecord> prof_pending;
    std::map<std::string, awg::ProfTotal> prof_totals;
    // smooth-ramp tables shared by all plans of the context, keyed by (shape, N)
    std::map<std::pair<int32_t, uint64_t>, awg::Table> tables;
    // device address of this device's copy of the allocation-free peak call's
    // scratch array (looked up once per device when a context is created)
    float *noalloc_scratch = nullptr;
};

struct awg_plan {
    awg_ctx *ctx;                      // NULL for host-only plans
    awg_plan_params params;
    double gain;
    int32_t n_tones;
    int32_t n_ramped;
    std::vector<awg::ToneHost> host;   // authoritative tone state, caller's tone order
    std::vector<awg::ToneDev> dev_mirror;   // device order: sorted by (shape, window, table)
    std::vector<int32_t> perm;         // device position -> caller's tone index
    std::vector<int32_t> inv;          // caller's tone index -> device position
    std::vector<const uint64_t *> table_ptrs;   // device pointers, indexed by ToneDev::table
    std::map<std::pair<int32_t, uint64_t>, uint16_t> table_index;
    std::vector<awg::Block> blocks;    // block table of dev_mirror (header first)
    bool blocks_stale = false;         // a retune changed dev_mirror: blocks and d_blocks are rebuilt
                                       // by the next call that reads them (sync_blocks)
    awg::Block *d_blocks;              // device copy, room for n_tones + 1 entries
    awg::ToneDev *d_tones;             // device copy of dev_mirror
    const uint64_t **d_table_ptrs;     // device copy of table_ptrs
    size_t d_table_ptrs_cap;
    uint64_t cursor;
    uint64_t device_bytes;
    // retune staging: pinned coherent host slots (read by the device through
    // their mapped addresses) and their completion events
    struct Slot { void *host; void *mapped; hipEvent_t done; bool used; };
    std::vector<Slot> slots;
    size_t next_slot;
    // a line-buffer plan's retune records staged in slot pend_slot (pend_n of
    // them) and not yet applied to d_tones: the next line-buffer pass applies
    // them in its first launch, any other call that reads d_tones first
    int32_t pend_slot = -1;
    int32_t pend_n = 0;
    std::mutex pend_mu;
    // duplicate-tone check of one retune or amplitude call: ev_stamp[tone] ==
    // ev_gen marks a tone already named in the call being validated
    std::vector<uint32_t> ev_stamp;
    uint32_t ev_gen;
    // MFMA workspace (operands), grown on demand; B operand cached under mfma_b_key
    void *d_work;
    size_t d_work_bytes;
    uint64_t mfma_b_key;
    std::mutex work_mu;                // host-side use of d_work (calls may come from several threads)
    hipEvent_t work_done = nullptr;    // the last launch that used d_work, on whatever stream
    bool work_used = false;
    // hybrid path (matrix cores + direct kernel for ramped plans), created on first use
    awg::HybridState *hyb;
    // periodic line buffer (the hybrid path of plans on the bins of a period), created on first use
    awg::LineBuf *plb = nullptr;
};

namespace awg {

// Pending retune records of a plan (line-buffer plans defer them). flush_tones
// applies them on s (scatter kernel) if any; take_pending_tones hands them to
// a launch that applies them itself (*slot = -1: none), after which
// pending_tones_applied(p, slot, s) marks the slot in use until s passes it.
awg_status flush_tones(awg_plan *p, hipStream_t s);
void take_pending_tones(awg_plan *p, const void **mapped, int32_t *n, int32_t *slot);
awg_status pending_tones_applied(awg_plan *p, int32_t slot, hipStream_t s);

// Exact word arithmetic (plan.cpp)
bool rne_ratio_shift(double num, double den, int shift, uint64_t *out);
// Frequency word of f at fs: nint(f 2^64 / fs), or with p > 0 the bin
// nint(f 2^p / fs) (Eq. (4)) times 2^(64-p). AWG_E_INVALID unless 0 < f < fs/2,
// AWG_E_RANGE for the bins 0 and 2^(p-1).
awg_status freq_word(double f, double fs, uint32_t p, uint64_t *out);
uint64_t phase_word(double turns);
int64_t rne_div(int64_t num, uint64_t den);
int64_t minjerk_entry(uint64_t n, uint64_t d);
int64_t cosine_entry(uint64_t n, uint64_t d);
uint64_t chirp_end_term(int32_t shape, int64_t coef, int64_t dF, uint64_t n);
ToneDev to_device(const ToneHost &t, uint16_t table);
// Block table of a tone list (see Block). Tones [0, n_split) are marked split
// (hybrid path) and no block spans position n_split. At most n + 1 entries.
// build_blocks_by reads tone i of an n-tone list through tone(i), and cuts the
// run of like tones that starts at i into blocks of at most max_block(i) tones
// (at most kBlock).
template <class Get, class MaxBlock>
void build_blocks_by(int32_t n, int32_t n_split, Get &&tone, MaxBlock &&max_block, std::vector<Block> *out)
{
    constexpr int32_t kMinRun = 8;
    out->clear();
    out->push_back(Block{0, 0, 0});
    auto same = [&](int32_t x, int32_t y) {
        const ToneDev &a = tone(x), &b = tone(y);
        return a.shape == b.shape && a.a == b.a && a.n == b.n && a.table == b.table && a.ashape == b.ashape &&
               a.b == b.b && a.m == b.m && ((x < n_split) == (y < n_split));
    };
    int32_t mixed_begin = -1, mixed_count = 0;
    uint16_t mixed_flags = 0;
    auto flush = [&]() {
        if (mixed_count > 0) out->push_back(Block{(uint32_t)mixed_begin, (uint16_t)mixed_count, mixed_flags});
        mixed_begin = -1;
        mixed_count = 0;
    };
    for (int32_t i = 0; i < n;) {
        int32_t j = i + 1;
        while (j < n && same(i, j)) ++j;
        const int32_t L = j - i;
        const uint16_t flags = (i < n_split ? kBlockSplit : 0) | (tone(i).ashape != AWG_RAMP_NONE ? kBlockAmp : 0);
        if (L >= kMinRun) {
            flush();
            // at least kWaves tones per block: with runs of kMinRun or more, no block is empty
            const int32_t mb = std::max<int32_t>(kWaves, std::min<int32_t>(kBlock, max_block(i)));
            int32_t nb = (L + mb - 1) / mb;
            nb = (nb + kWaves - 1) / kWaves * kWaves;
            const int32_t base = L / nb, extra = L % nb;
            int32_t b = i;
            const bool smooth = tone(i).shape == AWG_RAMP_COSINE || tone(i).shape == AWG_RAMP_MINJERK;
            for (int32_t q = 0; q < nb; ++q) {
                const int32_t c = base + (q < extra ? 1 : 0);
                bool step16 = smooth;
                for (int32_t k = b; step16 && k < b + c; ++k) step16 = (tone(k).coef & 0xffff) == 0;
                out->push_back(Block{(uint32_t)b, (uint16_t)c,
                                     (uint16_t)(kBlockUniform | flags | (step16 ? kBlockStep16 : 0))});
                b += c;
            }
        } else {
            for (int32_t k = i; k < j; ++k) {
                if (mixed_count > 0 && (mixed_count == kBlock || mixed_flags != flags)) flush();
                if (mixed_count == 0) { mixed_begin = k; mixed_flags = flags; }
                ++mixed_count;
            }
        }
        i = j;
    }
    flush();
    (*out)[0].begin = (uint32_t)(out->size() - 1);
}
template <class Get>
void build_blocks_by(int32_t n, int32_t n_split, Get &&tone, std::vector<Block> *out)
{
    build_blocks_by(n, n_split, tone, [](int32_t) { return kBlock; }, out);
}
void build_blocks(const std::vector<ToneDev> &tones, int32_t n_split, std::vector<Block> *out);

// Device table H_N of a smooth shape, created once per context (capi.cpp).
awg_status get_table(awg_ctx *ctx, int32_t shape, uint64_t n, const uint64_t **d_out);

// Per-kernel timing when the context profiles: the scope's kernels are launched
// through launch() (defined in prof_launch.h, for the HIP sources), which hands
// the start event to the first launch and the stop event to every launch, so
// the dispatches themselves take the timestamps (no marker packets between
// kernels). A scope whose kernel never launched records nothing.
class ProfScope {
public:
    ProfScope(awg_ctx *ctx, hipStream_t s, const char *name);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;
    template <typename F, typename... Args>
    void launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, Args... args);
    // algorithmic work of the scope's launches (tone-samples), added up by
    // awg_profile_read for the launches that were timed
    void add_work(double tone_samples) { work_ += tone_samples; }
private:
    awg_ctx *ctx_;
    hipStream_t s_;
    const char *name_;
    hipEvent_t start_, stop_;
    bool launched_;
    double work_ = 0.0;
};

// Kernel launchers (direct.hip, mfma.hip). Return a HIP error code.
hipError_t launch_direct_i16(const awg_plan *p, uint64_t n0, uint64_t count, int16_t *out,
                             hipStream_t s);
hipError_t launch_direct_f32(const awg_plan *p, uint64_t n0, uint64_t count, float *out,
                             hipStream_t s, bool timed = true);
hipError_t launch_phase_dump(const awg_plan *p, int32_t tone, uint64_t n0, uint64_t count,
                             uint64_t *out, hipStream_t s);
// One changed tone for the scatter kernel: its device position and record.
struct ScatterRecord { uint32_t index; uint32_t pad; ToneDev tone; };
hipError_t launch_scatter_tones(ToneDev *d_tones, const void *d_records, int32_t n,
                                hipStream_t s);
hipError_t launch_peak(const float *d_y, uint64_t count, float *d_peak, hipStream_t s);
// Device address of the current device's copy of the allocation-free peak
// call's scratch array (AWG_PEAK_NOALLOC_MAX floats), looked up on the first
// call for a device (which must be current) and remembered per device.
hipError_t noalloc_scratch(int device, float **ptr);
// Copy `bytes` from pinned host memory (src: its device-mapped address, from a
// coherent hipHostMalloc allocation) to device memory dst, by a kernel on s: the
// copy stays on the compute queue in stream order, with no hand-off to a DMA
// engine. Used for the small per-call uploads (retune records, block tables,
// hybrid staging, serving work lists).
hipError_t launch_upload(const void *src, void *dst, size_t bytes, hipStream_t s);
// Pinned, coherent host memory for launch_upload: *host and its device-mapped
// address *mapped.
hipError_t alloc_upload_host(size_t bytes, void **host, void **mapped);
hipError_t launch_batch(const BatchItem *d_items, const uint32_t *d_header, uint32_t grid, hipStream_t s);

// Periodic line-buffer path (linebuf.cpp): a segment of rows [row_begin,
// row_end] of a call whose line tones of one group are q_row rather than the
// q_next that S holds (both period sums of L floats), and a fold of one group's
// sum into S (q_old: the sum S held for the group, or null).
struct PlbSeg {
    uint32_t row_begin, row_end;
    const float *q_row;
    const float *q_next;
};
static_assert(sizeof(PlbSeg) == 24, "PlbSeg must be 24 bytes");
struct PlbFold {
    const float *q_new;
    const float *q_old;
};
// An entry of the line-buffer path's staged tone lists, made into a ToneDev
// record on the device by launch_plb_stage: a plan tone's record (src >= 0:
// its device position) or a line (src < 0: words p, f without the device bias,
// signed amplitude a), summed on the rows [lo_row, hi_row] of the pass
// (lo_row < 0: no window, lo = 1 > hi = 0).
struct PlbDesc {
    uint64_t p, f;
    float a;
    int32_t src;
    int32_t lo_row, hi_row;
};
static_assert(sizeof(PlbDesc) == 32, "PlbDesc must be 32 bytes");
// One launch: the records of desc[0 .. n_first) to dst_first and of
// desc[n_first .. n_desc) to dst_rest (window rows start at n0), and a plain
// copy of raw_bytes (a multiple of 16) from raw_src (pinned, mapped) to raw_dst,
// both 16-byte aligned.
hipError_t launch_plb_stage(const PlbDesc *desc, int32_t n_first, int32_t n_desc, const ToneDev *plan_tones,
                            uint64_t n0, ToneDev *dst_first, ToneDev *dst_rest, const void *raw_src, void *raw_dst,
                            size_t raw_bytes, hipStream_t s);
// A piece of a split tile's work: tones off .. off + cnt - 1 of block `block`
// (cnt = 0: the whole block).
struct PlbPiece {
    uint32_t block;
    uint16_t off, cnt;
};
// A work item of the line-buffer kernel: a whole tile (part < 0: every block,
// then the line tones and the rounding) or one part of a split tile (the
// pieces [first, first + count), its sum into partial slot `part`).
struct PlbItem {
    uint32_t row;
    int32_t part;                // partial slot of a part of a split tile (-1: a whole tile)
    uint32_t first, count;       // a part's pieces
    int32_t split;               // a part's split tile (index into the split tiles)
};
// A split tile: its parts' sums sit in partial slots first .. first + n - 1.
struct PlbSplit {
    uint32_t row;
    uint32_t first, n;
    uint32_t pad;
};
// The line-buffer launch: n_items work items; the last part of a split tile to
// finish adds its parts (d_counts: one counter per split tile, zero before the
// launch and after it). d_partials holds 1024 floats per partial slot;
// d_span[i] = (first row, last row) the tones of block i are summed on.
// n_fold > 0 (only when count == L, so that each m = n mod L is one thread's):
// the folds d_folds[0 .. n_fold) are applied to S by the kernels that read it.
hipError_t launch_plb(const awg_plan *p, const ToneDev *d_tones, const Block *d_blocks, const PlbItem *d_items,
                      int32_t n_items, const PlbPiece *d_pieces, const int2 *d_span, float *d_partials,
                      const PlbSplit *d_splits, int32_t *d_counts,
                      int32_t n_split, uint64_t n0, uint64_t count, int64_t *d_S, uint64_t L,
                      const PlbSeg *d_segs, int32_t n_seg, const PlbFold *d_folds, int32_t n_fold,
                      int16_t *out_i16, float *out_f32, hipStream_t s, double work);
hipError_t launch_plb_fold(const awg_plan *p, int64_t *d_S, uint64_t L, const PlbFold *d_folds, int32_t n_fold,
                           hipStream_t s);
hipError_t launch_plb_zero(int64_t *d_S, uint64_t L, hipStream_t s);
// Period sums of groups of tones (mfma.hip): d_list holds n_built groups of
// group_tones static line records each (amplitude 0 for padding); the sum of
// group z over samples [0, L) goes to q_base + plane_map[z] * L (d_plane_map:
// device, n_built entries). d_work: at least group_work_bytes(...) bytes.
// d_ranges (device, n_built entries, or nullptr for whole sums): group z is
// made only on the samples [x * 2^18, (x + y) * 2^18) of (x, y) = d_ranges[z]
// (tile rows of 256 rows of 1024 samples), y >= 1, max_tiles the largest y.
size_t group_work_bytes(int32_t n_built, int32_t group_tones, uint64_t L);
// operands_ready: the operands are already in d_work (launch_plb_prep).
hipError_t launch_group_sums(const awg_plan *p, uint32_t method, const ToneDev *d_list, int32_t n_built,
                             int32_t group_tones, uint64_t L, void *d_work, float *q_base,
                             const int32_t *d_plane_map, const int2 *d_ranges, int32_t max_tiles,
                             bool operands_ready, hipStream_t s, double work);
// One launch for a line-buffer pass whose versions to build fit one product
// launch: the product operands of the n_built versions (bdesc: their line
// descriptors, group_tones per version, and ranges: their tile rows, both
// read in place from pinned memory) into d_work, the copy of raw_bytes (a
// multiple of 16) from raw_src to raw_dst, and the n_rec retune
// records at rec (ScatterRecord, pinned) applied to the plan's device table.
hipError_t launch_plb_prep(const awg_plan *p, uint32_t method, const PlbDesc *bdesc, int32_t n_built,
                           int32_t group_tones, uint64_t L, const int2 *ranges, void *d_work, const void *raw_src,
                           void *raw_dst, size_t raw_bytes, const void *rec, int32_t n_rec, hipStream_t s);
// Multiplexed channels: items[c] (c < n, n <= kMaxChannels) each cover the same
// count samples; one launch, items passed by value.
constexpr int kMaxChannels = 4;
hipError_t launch_mux(const BatchItem *items, int32_t n, uint64_t count, hipStream_t s, ProfScope &prof);
// MFMA static synthesis; out_i16 or out_f32 (exactly one non-null).
awg_status mfma_static(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count,
                       int16_t *out_i16, float *out_f32, hipStream_t s);

// Hybrid path (hybrid.cpp): a ramped plan's samples with the line tones on the
// matrix cores and the ramping ones on the direct kernel.
awg_status mfma_static_reserve(awg_plan *p, uint64_t max_count);
awg_status hybrid_reserve(awg_plan *p, uint32_t method, uint64_t max_count);
awg_status hybrid_synth(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16,
                        float *out_f32, hipStream_t s);
void hybrid_release(awg_plan *p);
size_t hybrid_bytes(const awg_plan *p);       // device memory held by the hybrid path
// Periodic line buffer (linebuf.cpp): the hybrid path of plans whose period
// L = 2^p is between 2^10 and 2^24 and whose buffer fits its memory bound.
bool plb_eligible(const awg_plan *p);
awg_status plb_reserve(awg_plan *p, uint32_t method);
awg_status plb_synth(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32,
                     hipStream_t s);
void plb_release(awg_plan *p);
// Tones changed on the host since the line buffer's last pass (device
// positions): retunes and amplitude ramps tell it, so that its passes need
// look only at those and at tones whose windows are still ahead or open.
void plb_note_changed(awg_plan *p, const int32_t *dev_pos, int32_t n);
size_t plb_bytes_of(const awg_plan *p);
// Its two launches (mfma.hip, direct.hip). Line entries: bits 0..28 the tone's
// device position, bits 29..31 the mode (kLine*; kLineNone: no rows, zero amplitude).
constexpr uint32_t kLineShift = 29;
enum : uint32_t { kLinePre = 0, kLinePost = 1, kLineSplitPre = 2, kLineSplitPost = 3, kLineNone = 4 };
LinesGeom lines_geometry(int32_t n_entries, int32_t max_entries, uint64_t count);
// d_blocks / n_blocks: the k-blocks whose B operand must be (re)built; all when d_blocks is null.
// work: the algorithmic tone-samples of the launch, for the profiler.
hipError_t launch_lines(const awg_plan *p, uint32_t method, const LinesGeom &g, const uint32_t *d_entries,
                        int32_t n_entries, const int32_t *d_blocks, int32_t n_blocks, uint64_t n0,
                        uint64_t count, void *d_work, hipStream_t s, double work);
hipError_t launch_direct_hybrid(const awg_plan *p, const ToneDev *d_tones, const Block *d_blocks,
                                const uint32_t *d_order, uint64_t n0, uint64_t count, const float *planes,
                                int32_t n_planes, uint64_t plane_stride, int16_t *out_i16, float *out_f32,
                                hipStream_t s, double work);

}  // namespace awg
