// Static synthesis on the matrix cores by angle addition.
//
// For static tones the sample n = n0 + c*M + m (row c, column m of an output
// matrix with M columns) has phase word theta_kc + w_km with
//   theta_kc = P_k + F_k (n0 + c M)   and   w_km = F_k m        (both exact words),
// so sin(theta + w) = sin(theta) cos(w) + cos(theta) sin(w) turns the sum over
// tones into a product
//   S[c][m] = sum_k [A_k sin theta_kc, A_k cos theta_kc] . [cos w_km ; sin w_km],
// a (C x 2K) by (2K x M) matrix multiply. The operands are generated from the
// exact words (one sincos per element), split into hi + lo halves in FP16 or
// BF16, and multiplied in three passes hi*hi + hi*lo + lo*hi accumulated in FP32
// by v_mfma_f32_32x32x16_{f16,bf16}; the epilogue rounds to int16.
//
// Operand layout ("fragment order"): for k-block kb (16 inner indices = 8 tones)
// and row block rb (32 rows), the 64 lanes' 8-element fragments are stored as
// 1 KB: A[kb][rb][lane][e] with row = rb*32 + lane%32 and inner index
// kb*16 + 8*(lane/32) + e; B likewise with columns. Inner index 2k is the sine
// (A) / cosine (B) of tone k, 2k+1 the cosine (A) / sine (B).
//
// Ramped plans (hybrid path): over a row of M samples a tone whose ramp window
// misses the row is on one of its two lines (before or after the window), so
// the same product serves it. The operands are then built from a list of line
// entries (tone, which line, and the rows the entry covers); a row outside an
// entry's rows gets a zero amplitude, and the direct kernel adds the tones
// that ramp inside the row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "awg_internal.h"
#include "plb_stage.h"
#include "prof_launch.h"

namespace awg {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int kTileRB = 8;            // row blocks per workgroup tile (256 rows)
constexpr int32_t kTargetGroups = 256; // workgroups a product should reach (one 8-wave workgroup per CU)
constexpr int kTileCB = 8;            // column blocks per workgroup tile (256 columns)
constexpr int kFragBytes = 64 * 16;   // one 32x16 fragment of 16-bit values

// sin and cos of an (unbiased) phase word to about one FP32 ulp: the turn
// t = hr * 2^-32, with hr the high word rounded to an FP32 value, goes through
// v_sin / v_cos (arguments in turns), and the residual word
// w - hr * 2^32 = (hi - hr) * 2^32 + lo (|hi - hr| <= 128, so under 2^40 and
// 1e-7 rad) is applied to first order. hr is kept below 2^31 so that it
// converts to an int32 exactly; the residual is then formed in 32-bit pieces
// and rounded once (to about 2^15 of 2^64 turn).
__device__ __forceinline__ void word_sincos(uint64_t w, float &s, float &c)
{
    const int32_t hi = (int32_t)(uint32_t)(w >> 32);
    const float hf = fminf((float)hi, 2147483520.0f);          // rounded to 24 bits, < 2^31
    const int32_t dh = hi - (int32_t)hf;                        // exact, |dh| <= 128
    const float t = hf * 0x1p-32f;
    const float res = __builtin_fmaf((float)dh, 0x1p32f, (float)(uint32_t)w);
    const float d = res * (6.283185307179586f * 0x1p-64f);
    const float s0 = __builtin_amdgcn_sinf(t), c0 = __builtin_amdgcn_cosf(t);
    s = __builtin_fmaf(d, c0, s0);
    c = __builtin_fmaf(-d, s0, c0);
}

template <typename T> struct Split;
template <> struct Split<_Float16> {
    typedef h8 vec;
    __device__ static void run(float x, _Float16 &h, _Float16 &l)
    {
        h = (_Float16)x;
        l = (_Float16)(x - (float)h);
    }
};
template <> struct Split<__bf16> {
    typedef b8 vec;
    __device__ static void run(float x, __bf16 &h, __bf16 &l)
    {
        h = (__bf16)x;
        l = (__bf16)(x - (float)h);
    }
};

// Line entry of the hybrid path (kLineShift, kLine*): pre / post: the line
// before / after the windows on every row; split-pre: the line before the
// windows on the rows that end before the first opens; split-post: the line
// after them on the rows that start after the last closes. A tone's windows
// (frequency and amplitude) span [lo, hi]; before it the tone is on
// p0 + f0 n at amplitude amp, after it on p1 + f1 n at amp1.

// Line (P, F) of entry e on the row [first, first + mcols - 1]; false when the
// entry does not cover the row. entries == nullptr: entry e is tone e's first line.
__device__ __forceinline__ bool entry_line(const ToneDev *__restrict__ tones, const uint32_t *__restrict__ entries,
                                           int32_t e, uint64_t first, uint64_t mcols, ToneDev &td)
{
    if (!entries) {
        td = tones[e];
        return true;
    }
    const uint32_t ent = entries[e];
    const uint32_t mode = ent >> kLineShift;
    td = tones[ent & ((1u << kLineShift) - 1)];
    if (mode & 1u) {                      // the line (and amplitude) after the windows
        td.p0 = td.p1;
        td.f0 = td.f1;
        td.amp = td.amp1;
    }
    if (mode == kLineSplitPre) return first + (mcols - 1) < td.lo;
    if (mode == kLineSplitPost) return first > td.hi;
    return mode != kLineNone;
}

// A operand: one thread per (row c, group g of 4 entries) -> 8 inner values.
// Entries are tones (ENTRIES false) or line entries. Grid: (rows / 256,
// groups from g_base on); the group is the workgroup's y index, so the
// entries' words are uniform (scalar loads). rows = 32 rb_pad is a multiple of 256.
template <typename T, bool ENTRIES>
__device__ __forceinline__ void gen_a_at(const ToneDev *__restrict__ tones, const uint32_t *__restrict__ entries,
                                         int32_t n_entries, int32_t g, int64_t c, uint64_t n0, uint64_t mcols,
                                         int32_t rb_pad, T *__restrict__ a_hi, T *__restrict__ a_lo)
{
    const uint64_t n = n0 + (uint64_t)c * mcols;
    typename Split<T>::vec hv, lv;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * g + t;
        float xs = 0.0f, xc = 0.0f;
        ToneDev td;
        if (k < n_entries && entry_line(tones, ENTRIES ? entries : nullptr, k, n, mcols, td)) {
            float s, co;
            word_sincos(td.p0 - kPhaseBias + td.f0 * n, s, co);
            xs = td.amp * s;
            xc = td.amp * co;
        }
        T h, l;
        Split<T>::run(xs, h, l); hv[2 * t] = h; lv[2 * t] = l;
        Split<T>::run(xc, h, l); hv[2 * t + 1] = h; lv[2 * t + 1] = l;
    }
    const int kb = g >> 1, rb = (int)(c >> 5);
    const int lane = (int)(c & 31) + 32 * (g & 1);
    const int64_t off = (((int64_t)kb * rb_pad + rb) * 64 + lane);
    ((typename Split<T>::vec *)a_hi)[off] = hv;
    ((typename Split<T>::vec *)a_lo)[off] = lv;
}

template <typename T, bool ENTRIES>
__global__ __launch_bounds__(256) void gen_a_kernel(const ToneDev *__restrict__ tones,
                                                    const uint32_t *__restrict__ entries, int32_t n_entries,
                                                    int32_t g_base, uint64_t n0, uint64_t mcols, int32_t rb_pad,
                                                    T *__restrict__ a_hi, T *__restrict__ a_lo)
{
    gen_a_at<T, ENTRIES>(tones, entries, n_entries, g_base + (int32_t)blockIdx.y,
                         (int64_t)blockIdx.x * blockDim.x + threadIdx.x, n0, mcols, rb_pad, a_hi, a_lo);
}

// B operand: one thread per (column m, group g of 4 entries); the frequency
// word of the entry's line (its rows do not matter here). With kb_list the
// groups are those of the listed k-blocks only (2 groups per k-block).
template <typename T>
__device__ __forceinline__ void gen_b_at(const ToneDev *__restrict__ tones, const uint32_t *__restrict__ entries,
                                         int32_t n_entries, int32_t n_groups, int32_t cb_n, T *__restrict__ b_hi,
                                         T *__restrict__ b_lo, const int32_t *__restrict__ kb_list, int64_t gid)
{
    const int64_t cols = (int64_t)cb_n * 32;
    if (gid >= cols * n_groups) return;
    const int32_t gi = (int32_t)(gid / cols);
    const int32_t g = kb_list ? 2 * kb_list[gi >> 1] + (gi & 1) : gi;
    const int64_t m = gid % cols;
    typename Split<T>::vec hv, lv;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * g + t;
        float xc = 0.0f, xs = 0.0f;
        if (k < n_entries) {
            uint64_t F;
            if (entries) {
                const uint32_t ent = entries[k];
                const ToneDev &td = tones[ent & ((1u << kLineShift) - 1)];
                F = ((ent >> kLineShift) & 1u) ? td.f1 : td.f0;
            } else {
                F = tones[k].f0;
            }
            word_sincos(F * (uint64_t)m, xs, xc);
        }
        T h, l;
        Split<T>::run(xc, h, l); hv[2 * t] = h; lv[2 * t] = l;
        Split<T>::run(xs, h, l); hv[2 * t + 1] = h; lv[2 * t + 1] = l;
    }
    const int kb = g >> 1, cb = (int)(m >> 5);
    const int lane = (int)(m & 31) + 32 * (g & 1);
    const int64_t off = (((int64_t)kb * cb_n + cb) * 64 + lane);
    ((typename Split<T>::vec *)b_hi)[off] = hv;
    ((typename Split<T>::vec *)b_lo)[off] = lv;
}

template <typename T>
__global__ __launch_bounds__(256) void gen_b_kernel(const ToneDev *__restrict__ tones,
                                                    const uint32_t *__restrict__ entries, int32_t n_entries,
                                                    int32_t n_groups, int32_t cb_n, T *__restrict__ b_hi,
                                                    T *__restrict__ b_lo, const int32_t *__restrict__ kb_list = nullptr)
{
    gen_b_at<T>(tones, entries, n_entries, n_groups, cb_n, b_hi, b_lo, kb_list,
                (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Both operands of the group sums in one launch: workgroups [0, a_blocks) make
// A (a_per_group of them per group of 4 tones, rows of mcols samples from 0),
// the rest make B. Each part runs the same code as gen_a_kernel / gen_b_kernel.
template <typename T>
__global__ __launch_bounds__(256) void gen_ab_kernel(const ToneDev *__restrict__ tones, int32_t n_entries,
                                                     uint32_t a_per_group, uint32_t a_blocks, uint64_t mcols,
                                                     int32_t rb_pad, T *__restrict__ a_hi, T *__restrict__ a_lo,
                                                     int32_t n_groups, int32_t cb_n, T *__restrict__ b_hi,
                                                     T *__restrict__ b_lo, const int2 *__restrict__ ty_range,
                                                     int32_t groups_per_slice)
{
    const uint32_t bx = blockIdx.x;
    if (bx < a_blocks) {
        // one workgroup = 256 rows = one tile row of the product: rows of tile
        // rows that the slice does not make are not needed
        if (ty_range) {
            const int2 rr = ty_range[(int32_t)(bx / a_per_group) / groups_per_slice];
            const int tr = (int)(bx % a_per_group);
            if (tr < rr.x || tr >= rr.x + rr.y) return;
        }
        gen_a_at<T, false>(tones, nullptr, n_entries, (int32_t)(bx / a_per_group),
                           (int64_t)(bx % a_per_group) * blockDim.x + threadIdx.x, 0, mcols, rb_pad, a_hi, a_lo);
    } else {
        gen_b_at<T>(tones, nullptr, n_entries, n_groups, cb_n, b_hi, b_lo, nullptr,
                    (int64_t)(bx - a_blocks) * blockDim.x + threadIdx.x);
    }
}

// A line-buffer pass's preparation in one launch. Workgroup g < n_gen takes
// the group g of 4 line descriptors of the versions to build (read once from
// pinned memory: p, f and amplitude of each line) and writes the A operand of
// its rows on the tile rows its version is made on, and the B operand of its
// columns, with the arithmetic of gen_ab_kernel on staged records (rows of
// 1024 samples from 0), so the operands are the same. The other workgroups
// copy the pass's staged blob (its records made on the host) and apply a
// retune's records to the plan's device table, which nothing else in the
// launch reads.
template <typename T>
__global__ __launch_bounds__(256) void plb_prep_kernel(const PlbDesc *__restrict__ bdesc, int32_t n_gen,
                                                       int32_t groups_per_slice, const int2 *__restrict__ ranges,
                                                       int32_t rb_pad, int32_t cb_n, T *__restrict__ a_hi,
                                                       T *__restrict__ a_lo, T *__restrict__ b_hi,
                                                       T *__restrict__ b_lo, const uint4 *__restrict__ raw_src,
                                                       uint4 *__restrict__ raw_dst, uint64_t n16,
                                                       const ScatterRecord *__restrict__ rec, int32_t n_rec,
                                                       ToneDev *__restrict__ plan_tones)
{
    typedef typename Split<T>::vec V;
    const int32_t bx = (int32_t)blockIdx.x;
    if (bx >= n_gen) {
        const uint64_t tid = (uint64_t)(bx - n_gen) * blockDim.x + threadIdx.x;
        const uint64_t stride = (uint64_t)(gridDim.x - (uint32_t)n_gen) * blockDim.x;
        plb_stage_range(nullptr, 0, 0, nullptr, 0, nullptr, nullptr, raw_src, raw_dst, n16, tid, stride);
        plb_scatter_range(plan_tones, rec, n_rec, tid, stride);
        return;
    }
    const int32_t g = bx;
    uint64_t P[4], Fw[4];
    float amp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const PlbDesc d = bdesc[4 * g + t];
        P[t] = d.p;
        Fw[t] = d.f;
        amp[t] = d.a;
    }
    const int2 rr = ranges[g / groups_per_slice];
    const int32_t kb = g >> 1, half = 32 * (g & 1);
    const int32_t r1 = min((rr.x + rr.y) * 256, rb_pad * 32);
    for (int32_t c = rr.x * 256 + (int32_t)threadIdx.x; c < r1; c += 256) {
        const uint64_t n = (uint64_t)c * kTileSamples;
        V hv, lv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float sn, co;
            word_sincos(P[t] + Fw[t] * n, sn, co);
            const float xs = amp[t] * sn, xc = amp[t] * co;
            T h, l;
            Split<T>::run(xs, h, l); hv[2 * t] = h; lv[2 * t] = l;
            Split<T>::run(xc, h, l); hv[2 * t + 1] = h; lv[2 * t + 1] = l;
        }
        const int64_t off = ((int64_t)kb * rb_pad + (c >> 5)) * 64 + (c & 31) + half;
        // the operands are read by the next launch only: stored non-temporal, so
        // that this launch's end has no L2 full of them to write back
        __builtin_nontemporal_store(hv, &((V *)a_hi)[off]);
        __builtin_nontemporal_store(lv, &((V *)a_lo)[off]);
    }
    for (int32_t m = (int32_t)threadIdx.x; m < cb_n * 32; m += 256) {
        V hv, lv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float xs, xc;
            word_sincos(Fw[t] * (uint64_t)m, xs, xc);
            T h, l;
            Split<T>::run(xc, h, l); hv[2 * t] = h; lv[2 * t] = l;
            Split<T>::run(xs, h, l); hv[2 * t + 1] = h; lv[2 * t + 1] = l;
        }
        const int64_t off = ((int64_t)kb * cb_n + (m >> 5)) * 64 + (m & 31) + half;
        __builtin_nontemporal_store(hv, &((V *)b_hi)[off]);
        __builtin_nontemporal_store(lv, &((V *)b_lo)[off]);
    }
}

template <typename T>
__device__ __forceinline__ f16v mfma(const typename Split<T>::vec &a, const typename Split<T>::vec &b, f16v c);
template <>
__device__ __forceinline__ f16v mfma<_Float16>(const h8 &a, const h8 &b, f16v c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f16v mfma<__bf16>(const b8 &a, const b8 &b, f16v c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int16_t to_i16(float y)
{
    float r = __builtin_rintf(y);
    r = fminf(fmaxf(r, -32768.0f), 32767.0f);
    return (int16_t)(int32_t)r;
}

typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediate that waits until at most v vector-memory operations are
// outstanding (expcnt and lgkmcnt left at their maxima).
constexpr int vmcnt_imm(int v) { return (v & 0xf) | ((v >> 4) << 14) | (0x7 << 4) | (0xf << 8); }

// One workgroup = WR x WC waves covering a 256 x 256 output tile; each wave owns
// (8/WR) x (8/WC) MFMA tiles of 32 x 32 (accumulators in AGPRs). Per k-block
// the tile needs 32 fragments (A hi/lo for 8 row blocks, B hi/lo for 8 column
// blocks, 1 KB each); every wave copies 32/(WR*WC) of them straight from global
// memory into LDS (global_load_lds_dwordx4, lane i -> bytes 16i..16i+15 of a
// fragment), into NST LDS stages, prefetch distance NST-1: block kb+NST-1 is in
// flight while block kb is multiplied. vmcnt counts the copies in issue order.
//
// Split K: the grid's z index z sums k-blocks [z*kb_split, (z+1)*kb_split) and
// writes its partial sums to plane z of the FP32 output (plane elements apart),
// or to plane plane_map[z] when a map is given (group products written straight
// into their slots of a cache). With ty_range, slice z covers only the tile rows
// ty_range[z].x .. + ty_range[z].y - 1, grid y being the largest such count.
template <typename T, bool F32OUT, int WR, int WC, int NST>
__global__ __launch_bounds__(64 * WR * WC, 1) void angle_gemm_kernel(
    const T *__restrict__ a_hi, const T *__restrict__ a_lo, const T *__restrict__ b_hi, const T *__restrict__ b_lo,
    int32_t kb_n, int32_t rb_pad, int32_t cb_n, int32_t kb_split, uint64_t plane, uint64_t mcols, uint64_t count,
    void *__restrict__ out, const int32_t *__restrict__ plane_map, const int2 *__restrict__ ty_range)
{
    typedef typename Split<T>::vec V;
    constexpr int W = WR * WC;
    constexpr int TI = kTileRB / WR, TJ = kTileCB / WC;         // MFMA tiles per wave
    constexpr int F = 32 / W;                                    // fragments copied per wave per block
    constexpr int kOperand = kTileRB * kFragBytes;               // 8 KB
    constexpr int kStage = 4 * kOperand;                         // A hi, A lo, B hi, B lo
    extern __shared__ __attribute__((aligned(1024))) char lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wr = wave / WC, wc = wave % WC;
    // Tile order: consecutive workgroups go to different XCDs (round robin), so
    // first make each XCD's share a contiguous range of tile indices, then walk
    // that range in groups of 4 tile rows, column by column: every XCD then
    // works on a compact block of tiles and re-reads fewer operand rows and
    // columns from HBM into its own L2.
    const uint32_t gx = gridDim.x, gy = gridDim.y, nt = gx * gy, nall = nt * gridDim.z;
    uint32_t b = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
    if (nall % 8 == 0) b = (b % 8) * (nall / 8) + b / 8;
    const uint32_t z = b / nt;                                  // split-K slice
    b %= nt;
    const int32_t kb_begin = (int32_t)z * kb_split;
    const int32_t kb_cnt = max(0, min(kb_n - kb_begin, kb_split));
    const uint32_t grp = gy < 4 ? gy : 4;
    const uint32_t full = (gy / grp) * grp;                     // rows covered by whole groups
    uint32_t ty, tx;
    if (b < full * gx) {
        const uint32_t g = b / (grp * gx), r = b % (grp * gx);
        ty = g * grp + r % grp;
        tx = r / grp;
    } else {
        const uint32_t r = b - full * gx, rows = gy - full;
        ty = full + r % rows;
        tx = r / rows;
    }
    if (ty_range) {                    // slice z makes tile rows [x, x + y) only (whole workgroup)
        const int2 rr = ty_range[z];
        if ((int)ty >= rr.y) return;
        ty += (uint32_t)rr.x;
    }
    const int rb0 = ty * kTileRB, cb0 = tx * kTileCB;

    // fragment f of a stage: operand f / 8 (A hi, A lo, B hi, B lo), block f % 8
    const int f0 = wave * F;
    const int opnd = f0 / 8;
    const T *gsrc = opnd == 0 ? a_hi : opnd == 1 ? a_lo : opnd == 2 ? b_hi : b_lo;
    const int64_t kb_stride = (int64_t)(opnd < 2 ? rb_pad : cb_n) * 512;
    gsrc += ((int64_t)(opnd < 2 ? rb0 : cb0) + (f0 % 8)) * 512 + lane * 8 + (int64_t)kb_begin * kb_stride;
    auto issue = [&](int kb) {
        const T *g = gsrc + (int64_t)kb * kb_stride;
        char *l = lds + (kb % NST) * kStage + f0 * kFragBytes;
#pragma unroll
        for (int i = 0; i < F; ++i)
            __builtin_amdgcn_global_load_lds((const void *)(g + i * 512), (lds_void *)(l + i * kFragBytes), 16, 0, 0);
    };

    f16v acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    // this wave's fragments of block kb: A hi (fa), B hi (fb), B lo (xb), A lo (xa)
    auto read = [&](int kb, V *fa, V *fb, V *xb, V *xa) {
        const char *st = lds + (kb % NST) * kStage;
        const V *ah = (const V *)(st + 0 * kOperand) + TI * wr * 64 + lane;
        const V *al = (const V *)(st + 1 * kOperand) + TI * wr * 64 + lane;
        const V *bh = (const V *)(st + 2 * kOperand) + TJ * wc * 64 + lane;
        const V *bl = (const V *)(st + 3 * kOperand) + TJ * wc * 64 + lane;
#pragma unroll
        for (int i = 0; i < TI; ++i) fa[i] = ah[i * 64];
#pragma unroll
        for (int j = 0; j < TJ; ++j) fb[j] = bh[j * 64];
#pragma unroll
        for (int j = 0; j < TJ; ++j) xb[j] = bl[j * 64];
#pragma unroll
        for (int i = 0; i < TI; ++i) xa[i] = al[i * 64];
    };
    // hi*hi, then hi*lo, then lo*hi
    auto multiply = [&](const V *fa, const V *fb, const V *xb, const V *xa) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = mfma<T>(fa[i], fb[j], acc[i][j]);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = mfma<T>(fa[i], xb[j], acc[i][j]);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = mfma<T>(xa[i], fb[j], acc[i][j]);
    };

#pragma unroll
    for (int s = 0; s < NST - 1; ++s)
        if (s < kb_cnt) issue(s);
    for (int kb = 0; kb < kb_cnt; ++kb) {
        // own copies of block kb landed, then a bare barrier (no fence: later
        // blocks stay in flight) makes every wave's copies visible
        if (kb + NST - 2 < kb_cnt) __builtin_amdgcn_s_waitcnt(vmcnt_imm(F * (NST - 2)));
        else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        asm volatile("s_barrier" ::: "memory");
        if (kb + NST - 1 < kb_cnt) issue(kb + NST - 1);
        V fa[TI], fb[TJ], xa[TI], xb[TJ];
        read(kb, fa, fb, xb, xa);
        multiply(fa, fb, xb, xa);
    }

    // epilogue: reg v of lane l in tile (i, j) is row 8(v/4) + 4(l/32) + v%4, column l%32
    const uint64_t pz = F32OUT && plane_map ? (uint64_t)plane_map[z] : (uint64_t)z;
#pragma unroll
    for (int i = 0; i < TI; ++i) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const uint64_t col = (uint64_t)(cb0 + TJ * wc + j) * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const uint64_t row = (uint64_t)(rb0 + TI * wr + i) * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const uint64_t rel = row * mcols + col;
                if (rel < count) {
                    if (F32OUT) ((float *)out)[pz * plane + rel] = acc[i][j][v];
                    else ((int16_t *)out)[rel] = to_i16(acc[i][j][v]);
                }
            }
        }
    }
}

// Launch one GEMM variant (waves WR x WC, NST LDS stages).
template <typename T, int WR, int WC, int NST>
static hipError_t launch_gemm(dim3 grid, ProfScope &prof, const T *a_hi, const T *a_lo, const T *b_hi,
                              const T *b_lo, int32_t kb_n, int32_t rb_pad, int32_t cb_n, int32_t kb_split,
                              uint64_t plane, uint64_t mcols, uint64_t count, int16_t *out_i16, float *out_f32,
                              const int32_t *plane_map, const int2 *ty_range)
{
    constexpr int kLds = NST * 4 * kTileRB * kFragBytes;
    // the dynamic LDS limit is raised once per device (calls may come from
    // several host threads and contexts on several devices)
    static std::mutex mu;
    static uint64_t set_mask = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lock(mu);
        const uint64_t bit = dev < 64 ? 1ull << dev : 0;
        if (!bit || !(set_mask & bit)) {
            e = hipFuncSetAttribute((const void *)angle_gemm_kernel<T, true, WR, WC, NST>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, kLds);
            if (e == hipSuccess)
                e = hipFuncSetAttribute((const void *)angle_gemm_kernel<T, false, WR, WC, NST>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, kLds);
            if (e != hipSuccess) return e;
            set_mask |= bit;
        }
    }
    if (out_f32)
        prof.launch(angle_gemm_kernel<T, true, WR, WC, NST>, grid, dim3(64 * WR * WC), (uint32_t)kLds, a_hi,
                    a_lo, b_hi, b_lo, kb_n, rb_pad, cb_n, kb_split, plane, mcols, count, (void *)out_f32, plane_map,
                    ty_range);
    else
        prof.launch(angle_gemm_kernel<T, false, WR, WC, NST>, grid, dim3(64 * WR * WC), (uint32_t)kLds, a_hi,
                    a_lo, b_hi, b_lo, kb_n, rb_pad, cb_n, kb_split, plane, mcols, count, (void *)out_i16,
                    (const int32_t *)nullptr, ty_range);
    return hipGetLastError();
}

// GEMM variant (waves, LDS stages): 0 = 4 / 2, 1 = 4 / 3, 2 = 8 / 2, 3 = 8 / 3,
// 4 = 8 / 4, 5 = 8 / 5 (160 KB of LDS). The default is the fastest measured on
// MI355X; the environment variable AWG_GEMM_VARIANT overrides it for tuning sweeps.
static int gemm_variant()
{
    static const int v = [] {
        const char *e = getenv("AWG_GEMM_VARIANT");
        return (e && e[0] >= '0' && e[0] <= '5') ? e[0] - '0' : 3;
    }();
    return v;
}

// A operand of groups [0, n_groups): launches of at most 65535 groups (grid y).
template <typename T>
static void launch_gen_a(ProfScope &prof, const ToneDev *tones, const uint32_t *entries, int32_t n_entries,
                         int32_t n_groups, uint64_t n0, uint64_t mcols, int32_t rb_pad, T *a_hi, T *a_lo)
{
    for (int32_t g0 = 0; g0 < n_groups; g0 += 65535) {
        const dim3 grid((uint32_t)(rb_pad * 32 / 256), (uint32_t)std::min(65535, n_groups - g0));
        if (entries)
            prof.launch(gen_a_kernel<T, true>, grid, dim3(256), 0, tones, entries, n_entries, g0, n0, mcols, rb_pad,
                        a_hi, a_lo);
        else
            prof.launch(gen_a_kernel<T, false>, grid, dim3(256), 0, tones, entries, n_entries, g0, n0, mcols, rb_pad,
                        a_hi, a_lo);
    }
}

template <typename T>
static hipError_t dispatch_gemm(dim3 grid, ProfScope &prof, const T *a_hi, const T *a_lo, const T *b_hi,
                                const T *b_lo, int32_t kb_n, int32_t rb_pad, int32_t cb_n, int32_t kb_split,
                                uint64_t plane, uint64_t mcols, uint64_t count, int16_t *out_i16, float *out_f32,
                                const int32_t *plane_map = nullptr, const int2 *ty_range = nullptr)
{
#define AWG_GEMM(WR, WC, NST)                                                                                  \
    return launch_gemm<T, WR, WC, NST>(grid, prof, a_hi, a_lo, b_hi, b_lo, kb_n, rb_pad, cb_n, kb_split, plane, \
                                       mcols, count, out_i16, out_f32, plane_map, ty_range)
    switch (gemm_variant()) {
    case 0: AWG_GEMM(2, 2, 2);
    case 1: AWG_GEMM(2, 2, 3);
    case 2: AWG_GEMM(2, 4, 2);
    case 4: AWG_GEMM(2, 4, 4);
    case 5: AWG_GEMM(2, 4, 5);
    default: AWG_GEMM(2, 4, 3);
    }
#undef AWG_GEMM
}

static awg_status hipst(hipError_t e)
{
    if (e == hipSuccess) return AWG_OK;
    return e == hipErrorOutOfMemory ? AWG_E_NOMEM : AWG_E_HIP;
}

// Split-K products of short requests: sample i is the sum of planes[z * plane
// + i] over the slices z in order, rounded to int16 (or kept in FP32).
__global__ __launch_bounds__(256) void plane_sum_kernel(const float *__restrict__ planes, int32_t gz,
                                                        uint64_t plane, uint64_t count, int16_t *__restrict__ out_i16,
                                                        float *__restrict__ out_f32)
{
    const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= count) return;
    float y[4];
    if (i0 + 4 <= count) {
        const float4 u = *(const float4 *)(planes + i0);
        y[0] = u.x; y[1] = u.y; y[2] = u.z; y[3] = u.w;
        for (int32_t z = 1; z < gz; ++z) {
            const float4 v = *(const float4 *)(planes + (uint64_t)z * plane + i0);
            y[0] += v.x; y[1] += v.y; y[2] += v.z; y[3] += v.w;
        }
    } else {
        for (int e = 0; e < 4; ++e) {
            y[e] = 0.0f;
            if (i0 + e < count) {
                y[e] = planes[i0 + e];
                for (int32_t z = 1; z < gz; ++z) y[e] += planes[(uint64_t)z * plane + i0 + e];
            }
        }
    }
    for (int e = 0; e < 4; ++e) {
        if (i0 + e >= count) break;
        if (out_f32) out_f32[i0 + e] = y[e];
        else out_i16[i0 + e] = to_i16(y[e]);
    }
}

// Geometry of a static product over count samples: columns per row (long
// requests take long rows, so that the per-call A operand (rows x 2K) stays
// small while B (2K x columns, cached in the plan) grows; 2^24 samples make 1024
// rows of 16384, 4 x 64 tiles of 256 x 256), operand sizes, split-K slices
// (short requests have few output tiles: the inner dimension is split over up
// to kTargetGroups workgroups, FP32 partial planes summed in slice order after)
// and the workspace the product needs.
struct StaticGeom {
    uint64_t mcols, rows, plane;
    int32_t rb_pad, cb_n, kb_n, gz, kb_split;
    size_t a_bytes, b_bytes, need;
};

static StaticGeom static_geometry(const awg_plan *p, uint64_t count)
{
    StaticGeom g;
    g.mcols = count >= (1ull << 24) ? 16384 : count >= (1ull << 20) ? 4096 : 1024;
    g.rows = (count + g.mcols - 1) / g.mcols;
    g.rb_pad = (int32_t)(((g.rows + 31) / 32 + kTileRB - 1) / kTileRB * kTileRB);
    g.cb_n = (int32_t)(g.mcols / 32);
    const int32_t n_groups = (p->n_tones + 3) / 4;
    g.kb_n = (n_groups + 1) / 2;                       // k-blocks of 8 tones (zero-padded)
    g.a_bytes = (size_t)g.kb_n * g.rb_pad * kFragBytes;
    g.b_bytes = (size_t)g.kb_n * g.cb_n * kFragBytes;
    const int32_t tiles = (g.rb_pad / kTileRB) * (g.cb_n / kTileCB);
    g.gz = 1;
    g.kb_split = g.kb_n;
    if (tiles < kTargetGroups && g.kb_n > 1) {
        g.gz = std::min(g.kb_n, (kTargetGroups + tiles - 1) / tiles);
        g.kb_split = (g.kb_n + g.gz - 1) / g.gz;
        g.gz = (g.kb_n + g.kb_split - 1) / g.kb_split;
    }
    g.plane = g.rows * g.mcols;
    const size_t plane_bytes = g.gz > 1 ? (size_t)g.gz * g.plane * sizeof(float) : 0;
    g.need = 2 * (g.a_bytes + g.b_bytes) + plane_bytes;
    return g;
}

// The plan's product workspace of at least `need` bytes (caller holds work_mu).
// Growing it waits for the last user of the old one and drops the cached B.
static awg_status ensure_static_work(awg_plan *p, size_t need)
{
    if (!p->work_done) {
        hipError_t e = hipEventCreateWithFlags(&p->work_done, hipEventDisableTiming);
        if (e != hipSuccess) return hipst(e);
    }
    if (p->d_work_bytes >= need) return AWG_OK;
    if (p->work_used) {
        hipError_t e = hipEventSynchronize(p->work_done);
        if (e != hipSuccess) return hipst(e);
    }
    if (p->d_work) (void)hipFree(p->d_work);
    p->d_work = nullptr;
    p->d_work_bytes = 0;
    p->mfma_b_key = 0;
    hipError_t e = hipMalloc(&p->d_work, need);
    if (e != hipSuccess) return hipst(e);
    p->d_work_bytes = need;
    return AWG_OK;
}

template <typename T>
static awg_status run(awg_plan *p, uint64_t n0, uint64_t count, int16_t *out_i16, float *out_f32, hipStream_t s)
{
    const StaticGeom g = static_geometry(p, count);
    const uint64_t mcols = g.mcols, rows = g.rows, plane = g.plane;
    const int32_t rb_pad = g.rb_pad, cb_n = g.cb_n, kb_n = g.kb_n, gz = g.gz, kb_split = g.kb_split;
    const size_t a_bytes = g.a_bytes, b_bytes = g.b_bytes;
    if (rows > (1ull << 26)) return AWG_E_UNSUPPORTED;
    // calls on one plan may come from several host threads and streams: one at a
    // time here, and each stream waits for the previous user of the workspace
    std::lock_guard<std::mutex> lock(p->work_mu);
    const awg_status ws = ensure_static_work(p, g.need);
    if (ws != AWG_OK) return ws;
    char *w = (char *)p->d_work;
    // B (depends on the tones and the column count only) is kept between calls
    T *b_hi = (T *)w, *b_lo = (T *)(w + b_bytes);
    T *a_hi = (T *)(w + 2 * b_bytes), *a_lo = (T *)(w + 2 * b_bytes + a_bytes);
    // zero the padding groups of the last k-block (odd group count)
    const int64_t b_threads = (int64_t)cb_n * 32 * (2 * kb_n);
    const bool f16 = sizeof(T) == 2 && std::is_same<T, _Float16>::value;
    hipError_t e = p->work_used ? hipStreamWaitEvent(s, p->work_done, 0) : hipSuccess;
    if (e != hipSuccess) return hipst(e);
    {
        ProfScope prof(p->ctx, s, f16 ? "gen_a_kernel_f16" : "gen_a_kernel_bf16");
        launch_gen_a<T>(prof, p->d_tones, nullptr, p->n_tones, 2 * kb_n, n0, mcols, rb_pad, a_hi, a_lo);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hipst(e);
    const uint64_t b_key = (mcols << 8) | (f16 ? 1u : 2u) | ((uint64_t)kb_n << 32);
    if (p->mfma_b_key != b_key) {
        ProfScope prof(p->ctx, s, f16 ? "gen_b_kernel_f16" : "gen_b_kernel_bf16");
        prof.launch(gen_b_kernel<T>, dim3((uint32_t)((b_threads + 255) / 256)), dim3(256), 0, p->d_tones,
                    (const uint32_t *)nullptr, p->n_tones, 2 * kb_n, cb_n, b_hi, b_lo, (const int32_t *)nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return hipst(e);
        p->mfma_b_key = b_key;
    }
    dim3 grid((uint32_t)(cb_n / kTileCB), (uint32_t)(rb_pad / kTileRB), (uint32_t)gz);
    float *planes = (float *)(w + 2 * (a_bytes + b_bytes));
    {
        ProfScope prof(p->ctx, s, f16 ? "angle_gemm_kernel_f16" : "angle_gemm_kernel_bf16");
        prof.add_work((double)p->n_tones * (double)count);
        if (gz == 1)
            e = dispatch_gemm<T>(grid, prof, a_hi, a_lo, b_hi, b_lo, kb_n, rb_pad, cb_n, kb_n, 0, mcols, count,
                                 out_i16, out_f32);
        else
            e = dispatch_gemm<T>(grid, prof, a_hi, a_lo, b_hi, b_lo, kb_n, rb_pad, cb_n, kb_split, plane, mcols,
                                 count, nullptr, planes);
    }
    if (e == hipSuccess && gz > 1) {
        ProfScope prof(p->ctx, s, "plane_sum_kernel");
        prof.launch(plane_sum_kernel, dim3((uint32_t)((count + 1023) / 1024)), dim3(256), 0, (const float *)planes,
                    gz, plane, count, out_i16, out_f32);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(p->work_done, s);
    if (e == hipSuccess) p->work_used = true;
    return hipst(e);
}

LinesGeom lines_geometry(int32_t n_entries, int32_t max_entries, uint64_t count)
{
    const uint64_t mcols = kTileSamples;
    const uint64_t rows = (count + mcols - 1) / mcols;
    LinesGeom g;
    g.rb_pad = (int32_t)(((rows + 31) / 32 + kTileRB - 1) / kTileRB * kTileRB);
    g.cb_n = (int32_t)(mcols / 32);
    g.kb_n = (n_entries + 7) / 8;
    g.kb_cap = std::max(g.kb_n, (max_entries + 7) / 8);
    const int32_t tiles = (g.rb_pad / kTileRB) * (g.cb_n / kTileCB);
    int32_t gz = (kTargetGroups + tiles - 1) / tiles;
    gz = std::max(1, std::min(gz, g.kb_n));
    g.kb_split = (g.kb_n + gz - 1) / gz;
    g.gz = g.kb_split > 0 ? (g.kb_n + g.kb_split - 1) / g.kb_split : 0;
    g.plane = rows * mcols;
    g.a_bytes = (size_t)g.kb_n * g.rb_pad * kFragBytes;
    g.b_bytes = (size_t)g.kb_cap * g.cb_n * kFragBytes;
    g.plane_bytes = (size_t)g.gz * g.plane * sizeof(float);
    return g;
}

template <typename T>
static hipError_t lines_run(const awg_plan *p, const LinesGeom &g, const uint32_t *d_entries, int32_t n_entries,
                            const int32_t *d_blocks, int32_t n_blocks, uint64_t n0, uint64_t count, char *w,
                            hipStream_t s, double work)
{
    const bool f16 = std::is_same<T, _Float16>::value;
    T *b_hi = (T *)w, *b_lo = (T *)(w + g.b_bytes);
    T *a_hi = (T *)(w + 2 * g.b_bytes), *a_lo = (T *)(w + 2 * g.b_bytes + g.a_bytes);
    float *planes = (float *)(w + 2 * (g.a_bytes + g.b_bytes));
    const uint64_t mcols = kTileSamples;
    const int64_t b_threads = (int64_t)g.cb_n * 32 * (2 * (d_blocks ? n_blocks : g.kb_n));
    hipError_t e;
    {
        ProfScope prof(p->ctx, s, f16 ? "hyb_gen_a_f16" : "hyb_gen_a_bf16");
        launch_gen_a<T>(prof, p->d_tones, d_entries, n_entries, 2 * g.kb_n, n0, mcols, g.rb_pad, a_hi, a_lo);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (b_threads > 0) {
        ProfScope prof(p->ctx, s, f16 ? "hyb_gen_b_f16" : "hyb_gen_b_bf16");
        prof.launch(gen_b_kernel<T>, dim3((uint32_t)((b_threads + 255) / 256)), dim3(256), 0, p->d_tones,
                    d_entries, n_entries, 2 * (d_blocks ? n_blocks : g.kb_n), g.cb_n, b_hi, b_lo, d_blocks);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    dim3 grid((uint32_t)(g.cb_n / kTileCB), (uint32_t)(g.rb_pad / kTileRB), (uint32_t)g.gz);
    ProfScope prof(p->ctx, s, f16 ? "hyb_gemm_f16" : "hyb_gemm_bf16");
    prof.add_work(work);
    return dispatch_gemm<T>(grid, prof, a_hi, a_lo, b_hi, b_lo, g.kb_n, g.rb_pad, g.cb_n, g.kb_split, g.plane,
                            mcols, count, nullptr, planes);
}

hipError_t launch_lines(const awg_plan *p, uint32_t method, const LinesGeom &g, const uint32_t *d_entries,
                        int32_t n_entries, const int32_t *d_blocks, int32_t n_blocks, uint64_t n0,
                        uint64_t count, void *d_work, hipStream_t s, double work)
{
    if (g.gz <= 0 || n_entries <= 0) return hipSuccess;
    if (method == AWG_F_METHOD_MFMA_F16X3)
        return lines_run<_Float16>(p, g, d_entries, n_entries, d_blocks, n_blocks, n0, count, (char *)d_work, s,
                                   work);
    if (method == AWG_F_METHOD_MFMA_BF16X3)
        return lines_run<__bf16>(p, g, d_entries, n_entries, d_blocks, n_blocks, n0, count, (char *)d_work, s,
                                 work);
    return hipErrorInvalidValue;
}

// Period sums of tone groups (the periodic line-buffer path): rows of 1024
// samples from 0 over one period L, k-blocks of 8 tones, group z = k-blocks
// [z * kpg, (z + 1) * kpg) summed by split-K slice z into plane plane_map[z].
struct GroupGeom {
    int32_t rb_pad, cb_n, kb_n, kpg;
    size_t a_bytes, b_bytes;
};

static GroupGeom group_geometry(int32_t n_built, int32_t group_tones, uint64_t L)
{
    GroupGeom g;
    const uint64_t rows = L / kTileSamples;
    g.rb_pad = (int32_t)(((rows + 31) / 32 + kTileRB - 1) / kTileRB * kTileRB);
    g.cb_n = (int32_t)(kTileSamples / 32);
    g.kpg = group_tones / 8;
    g.kb_n = n_built * g.kpg;
    g.a_bytes = (size_t)g.kb_n * g.rb_pad * kFragBytes;
    g.b_bytes = (size_t)g.kb_n * g.cb_n * kFragBytes;
    return g;
}

size_t group_work_bytes(int32_t n_built, int32_t group_tones, uint64_t L)
{
    const GroupGeom g = group_geometry(n_built, group_tones, L);
    return 2 * (g.a_bytes + g.b_bytes);
}

template <typename T>
static hipError_t group_run(const awg_plan *p, const ToneDev *d_list, int32_t n_built, int32_t group_tones,
                            uint64_t L, char *w, float *q_base, const int32_t *d_plane_map, const int2 *d_ranges,
                            int32_t max_tiles, bool operands_ready, hipStream_t s, double work)
{
    static_assert(kTileRB * 32 == 256, "a workgroup of gen_ab makes one tile row of A");
    const bool f16 = std::is_same<T, _Float16>::value;
    const GroupGeom g = group_geometry(n_built, group_tones, L);
    T *b_hi = (T *)w, *b_lo = (T *)(w + g.b_bytes);
    T *a_hi = (T *)(w + 2 * g.b_bytes), *a_lo = (T *)(w + 2 * g.b_bytes + g.a_bytes);
    const int32_t n_entries = n_built * group_tones;
    hipError_t e = hipSuccess;
    if (!operands_ready) {
        // A: 2 kb_n groups of 4 tones x rb_pad * 32 rows; B: the same groups x cb_n * 32 columns
        const int64_t a_per_group = (int64_t)g.rb_pad * 32 / 256;
        const int64_t a_blocks = a_per_group * (2 * g.kb_n);
        const int64_t b_blocks = ((int64_t)g.cb_n * 32 * (2 * g.kb_n) + 255) / 256;
        if (a_blocks + b_blocks > INT32_MAX) return hipErrorInvalidValue;
        ProfScope prof(p->ctx, s, f16 ? "plb_gen_f16" : "plb_gen_bf16");
        prof.launch(gen_ab_kernel<T>, dim3((uint32_t)(a_blocks + b_blocks)), dim3(256), 0, d_list, n_entries,
                    (uint32_t)a_per_group, (uint32_t)a_blocks, (uint64_t)kTileSamples, g.rb_pad, a_hi, a_lo,
                    2 * g.kb_n, g.cb_n, b_hi, b_lo, d_ranges, group_tones / 4);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const int32_t ty_n = d_ranges ? max_tiles : g.rb_pad / kTileRB;
    if (ty_n <= 0 || ty_n > g.rb_pad / kTileRB) return hipErrorInvalidValue;
    dim3 grid((uint32_t)(g.cb_n / kTileCB), (uint32_t)ty_n, (uint32_t)n_built);
    ProfScope prof(p->ctx, s, f16 ? "plb_gemm_f16" : "plb_gemm_bf16");
    prof.add_work(work);
    return dispatch_gemm<T>(grid, prof, a_hi, a_lo, b_hi, b_lo, g.kb_n, g.rb_pad, g.cb_n, g.kpg, L, kTileSamples, L,
                            nullptr, q_base, d_plane_map, d_ranges);
}

hipError_t launch_group_sums(const awg_plan *p, uint32_t method, const ToneDev *d_list, int32_t n_built,
                             int32_t group_tones, uint64_t L, void *d_work, float *q_base,
                             const int32_t *d_plane_map, const int2 *d_ranges, int32_t max_tiles,
                             bool operands_ready, hipStream_t s, double work)
{
    if (n_built <= 0) return hipSuccess;
    if (group_tones % 8 != 0 || L < kTileSamples || L % kTileSamples != 0 || n_built > 65535)
        return hipErrorInvalidValue;
    if (method == AWG_F_METHOD_MFMA_F16X3)
        return group_run<_Float16>(p, d_list, n_built, group_tones, L, (char *)d_work, q_base, d_plane_map, d_ranges,
                                   max_tiles, operands_ready, s, work);
    if (method == AWG_F_METHOD_MFMA_BF16X3)
        return group_run<__bf16>(p, d_list, n_built, group_tones, L, (char *)d_work, q_base, d_plane_map, d_ranges,
                                 max_tiles, operands_ready, s, work);
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t plb_prep_run(const awg_plan *p, const PlbDesc *bdesc, int32_t n_built, int32_t group_tones,
                               uint64_t L, const int2 *ranges, char *w, const void *raw_src, void *raw_dst,
                               uint64_t n16, const void *rec, int32_t n_rec, hipStream_t s)
{
    const bool f16 = std::is_same<T, _Float16>::value;
    const GroupGeom g = group_geometry(n_built, group_tones, L);
    T *b_hi = (T *)w, *b_lo = (T *)(w + g.b_bytes);
    T *a_hi = (T *)(w + 2 * g.b_bytes), *a_lo = (T *)(w + 2 * g.b_bytes + g.a_bytes);
    const int32_t n_gen = n_built * (group_tones / 4);
    const uint64_t stage = std::max<uint64_t>((uint64_t)n_rec, n16);
    const uint64_t n_stage = std::min<uint64_t>(std::max<uint64_t>((stage + 255) / 256, 1), 1024);
    ProfScope prof(p->ctx, s, f16 ? "plb_prep_f16" : "plb_prep_bf16");
    prof.launch(plb_prep_kernel<T>, dim3((uint32_t)(n_gen + (int64_t)n_stage)), dim3(256), 0, bdesc, n_gen,
                group_tones / 4, ranges, g.rb_pad, g.cb_n, a_hi, a_lo, b_hi, b_lo, (const uint4 *)raw_src,
                (uint4 *)raw_dst, n16, (const ScatterRecord *)rec, n_rec, p->d_tones);
    return hipGetLastError();
}

hipError_t launch_plb_prep(const awg_plan *p, uint32_t method, const PlbDesc *bdesc, int32_t n_built,
                           int32_t group_tones, uint64_t L, const int2 *ranges, void *d_work, const void *raw_src,
                           void *raw_dst, size_t raw_bytes, const void *rec, int32_t n_rec, hipStream_t s)
{
    if (n_built <= 0 || group_tones % 8 != 0 || L < kTileSamples || L % kTileSamples != 0 || n_rec < 0 ||
        (n_rec > 0 && !rec))
        return hipErrorInvalidValue;
    if (((uintptr_t)raw_src | (uintptr_t)raw_dst | raw_bytes) & 15) return hipErrorInvalidValue;
    if ((int64_t)n_built * (group_tones / 4) + 1024 > INT32_MAX) return hipErrorInvalidValue;
    const uint64_t n16 = raw_bytes / 16;
    if (method == AWG_F_METHOD_MFMA_F16X3)
        return plb_prep_run<_Float16>(p, bdesc, n_built, group_tones, L, ranges, (char *)d_work, raw_src, raw_dst,
                                      n16, rec, n_rec, s);
    if (method == AWG_F_METHOD_MFMA_BF16X3)
        return plb_prep_run<__bf16>(p, bdesc, n_built, group_tones, L, ranges, (char *)d_work, raw_src, raw_dst,
                                    n16, rec, n_rec, s);
    return hipErrorInvalidValue;
}

awg_status mfma_static_reserve(awg_plan *p, uint64_t max_count)
{
    // the workspace of the largest product among requests of up to max_count
    // samples (pieces of at most 2^28; short requests add split-K planes)
    size_t need = 0;
    const uint64_t top = std::min<uint64_t>(max_count, 1ull << 28);
    const uint64_t counts[] = {top, (1ull << 24) - 1, 1ull << 22, (1ull << 20) - 1, 1ull << 18, 1ull << 16};
    for (const uint64_t c : counts)
        if (c >= (1ull << 16) && c <= top) need = std::max(need, static_geometry(p, c).need);
    if (need == 0) return AWG_OK;
    std::lock_guard<std::mutex> lock(p->work_mu);
    return ensure_static_work(p, need);
}

awg_status mfma_static(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16,
                       float *out_f32, hipStream_t s)
{
    // short requests gain nothing from the matrix cores: the direct kernel serves them
    if (count < (1ull << 16)) {
        hipError_t e = out_f32 ? launch_direct_f32(p, n0, count, out_f32, s)
                               : launch_direct_i16(p, n0, count, out_i16, s);
        return hipst(e);
    }
    if (method != AWG_F_METHOD_MFMA_F16X3 && method != AWG_F_METHOD_MFMA_BF16X3) return AWG_E_INVALID;
    // pieces of at most 2^28 samples bound the per-call operand (16384 rows)
    constexpr uint64_t kPiece = 1ull << 28;
    while (count > 0) {
        const uint64_t now = count < kPiece ? count : kPiece;
        const awg_status st = method == AWG_F_METHOD_MFMA_F16X3 ? run<_Float16>(p, n0, now, out_i16, out_f32, s)
                                                                : run<__bf16>(p, n0, now, out_i16, out_f32, s);
        if (st != AWG_OK) return st;
        n0 += now;
        count -= now;
        if (out_i16) out_i16 += now;
        if (out_f32) out_f32 += now;
    }
    return AWG_OK;
}

}  // namespace awg
