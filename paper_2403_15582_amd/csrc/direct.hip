// Direct VALU synthesis on gfx950: exact 64-bit phase words, v_sin_f32, FP32 sum.
//
// y[n] = sum_k amp_k * sin(2 pi phi_k(n) / 2^64) for a tile of 64*S contiguous
// samples per workgroup. The 4 waves of a workgroup cover the same samples;
// lane l of a wave owns samples [tile0 + l*S, tile0 + (l+1)*S). The tone list
// comes with a block table (contiguous runs of at most 32 tones): wave w sums
// blocks w, w+4, w+8, ... (FMA chain per block, block sums added to the wave
// sum in block order), and the 4 wave sums meet in LDS and are added in the
// order ((s0 + s1) + s2) + s3. Tone parameters are wave-uniform and come in
// through scalar loads. The summation order therefore depends only on the tone
// list and its table, never on the sample range, the tile position or the
// batch, so chunked, one-shot and batched results are bit-identical.
//
// Phase words (the piecewise law of Eq. (8)) are computed per tone and tile in
// one of four uniform regimes: before the window (line p0 + f0 n), after it
// (line p1 + f1 n), entirely inside it (incremental exact updates), or
// straddling an edge (closed form per sample).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "awg_internal.h"
#include "plb_stage.h"
#include "prof_launch.h"

namespace awg {

// floor(R d^2 / 2) mod 2^64 for d < 2^31: R*floor(d^2/2) + (d odd) * floor(R/2).
__device__ __forceinline__ uint64_t lin_term(int64_t R, uint64_t d)
{
    const uint64_t dd = d * d;
    return (uint64_t)R * (dd >> 1) + ((d & 1) ? (uint64_t)(R >> 1) : 0ull);
}

// floor(dF * H / 2^16) mod 2^64 for H < 2^47: dF*(H>>16) + floor(dF*(H&0xffff) / 2^16).
__device__ __forceinline__ uint64_t smooth_term(int64_t dF, uint64_t H)
{
    const uint64_t hh = H >> 16;
    const uint32_t hl = (uint32_t)H & 0xffffu;
    const uint64_t t1 = (uint64_t)dF * hh;
    const uint64_t lo = (uint64_t)(uint32_t)dF * hl;                 // < 2^48
    const int64_t hi = (int64_t)(int32_t)(dF >> 32) * (int64_t)hl;   // |.| < 2^47
    return t1 + ((uint64_t)hi << 16) + (lo >> 16);
}

// Table pointers carry a tag in bit 0: set when the table never decreases and
// its steps are below 2^19 (a lane's rise over 16 samples below 2^23), which
// the incremental smooth paths rely on.
__device__ __forceinline__ const uint64_t *table_of(const uint64_t *const *tables, uint32_t i)
{
    return (const uint64_t *)((uintptr_t)tables[i] & ~(uintptr_t)1);
}

__device__ __forceinline__ bool table_monotone(const uint64_t *const *tables, uint32_t i)
{
    return ((uintptr_t)tables[i] & 1) != 0;
}

__device__ __forceinline__ uint64_t phase_general(const ToneDev &t, const uint64_t *const *tables,
                                                  uint64_t n)
{
    if (n < t.a) return t.p0 + t.f0 * n;
    const uint64_t d = n - t.a;
    if (d <= t.n) {
        const uint64_t base = t.p0 + t.f0 * n;
        if (t.shape == AWG_RAMP_LINEAR) return base + lin_term(t.coef, d);
        return base + smooth_term(t.coef, table_of(tables, t.table)[d]);
    }
    return t.p1 + t.f1 * n;
}

// sin(2 pi phi / 2^64): the top 23 fraction bits of the (biased) word become the
// mantissa of a float in [1, 2); v_sin_f32 takes its argument in turns.
__device__ __forceinline__ float word_sin(uint64_t w)
{
    const uint32_t hi = (uint32_t)(w >> 32);
    return __builtin_amdgcn_sinf(__uint_as_float(__builtin_amdgcn_alignbit(0x7fu, hi, 9u)));
}

// A tile in which an edge of the window falls (some samples before or after it,
// some inside): the lane's first word in closed form, then exact increments
// phi(n+1) - phi(n) picked per sample: f0 before the window, f1 after it, and
// inside a linear window f0 + T(d+1) - T(d) with T(d) = floor(R d^2 / 2), i.e.
// R d + floor(R/2) for even d and R (d+1) - floor(R/2) for odd d. A smooth
// window adds its table term to the line p0 + f0 min(n, a+N) + f1 max(d-N, 0)
// (the table starts at 0, so before the window the term vanishes).
template <int S, typename F>
__device__ __forceinline__ void edge_run(const ToneDev &t, const uint64_t *const *tables, uint64_t n, F &&f)
{
    int64_t d = (int64_t)(n - t.a);                    // |d| < 2^62 for valid inputs
    const int64_t N = (int64_t)t.n;
    if (t.shape == AWG_RAMP_LINEAR) {
        // sample s lies before the window for s < s_lo and inside it for
        // s_lo <= s < s_hi (32-bit thresholds: the per-sample tests compare
        // against the unrolled constant s)
        const int32_t s_lo = (int32_t)(d >= 0 ? 0 : (-d >= S ? S : -d));
        const int32_t s_hi = (int32_t)(d >= N ? 0 : (N - d >= S ? S : N - d));
        const uint64_t R = (uint64_t)t.coef, h = (uint64_t)(t.coef >> 1), r = R & 1u;
        // in-window increment f0 + R d + floor(R/2) (d even) or f0 + R d + R - floor(R/2)
        // (d odd), carried along for every d (it is only taken inside the window);
        // it moves by R + r from an even d and by R - r from an odd one
        uint64_t inc = t.f0 + R * (uint64_t)d + ((d & 1) ? R - h : h);
        const uint64_t De = R + r, Do = R - r;
        const uint64_t D0 = (d & 1) ? Do : De, D1 = (d & 1) ? De : Do;   // steps after even / odd s
        uint64_t ph = phase_general(t, tables, n);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            f(s, ph);
            if (s + 1 < S) {
                ph += s < s_lo ? t.f0 : (s < s_hi ? inc : t.f1);
                inc += (s & 1) ? D1 : D0;
            }
        }
    } else {
        const uint64_t *H = table_of(tables, t.table);
        uint64_t line = d < N ? t.p0 + t.f0 * n : t.p0 + t.f0 * (t.a + t.n) + t.f1 * (uint64_t)(d - N);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t e = d < 0 ? 0 : (d < N ? d : N);
            f(s, line + smooth_term(t.coef, H[e]));
            line += d < N ? t.f0 : t.f1;
            ++d;
        }
    }
}

// Calls f(s, phi) for the S samples tile0 + lane*S + s of tone t.
template <int S, typename F>
__device__ __forceinline__ void gen_phases(const ToneDev &t, const uint64_t *const *tables,
                                           uint64_t tile0, uint32_t lane, F &&f)
{
    const uint64_t tile_last = tile0 + (uint64_t)(kLanes * S - 1);
    const uint32_t j = lane * S;                                   // even offset in the tile
    if (tile_last < t.a || tile0 > t.a + t.n) {                     // static line
        const bool pre = tile_last < t.a;
        const uint64_t P = pre ? t.p0 : t.p1, Fw = pre ? t.f0 : t.f1;
        uint64_t ph = P + Fw * tile0 + Fw * (uint64_t)j;
#pragma unroll
        for (int s = 0; s < S; ++s) { f(s, ph); ph += Fw; }
    } else if (tile0 >= t.a && tile_last <= t.a + t.n) {           // inside the window
        const uint64_t dt = tile0 - t.a;
        if (t.shape == AWG_RAMP_LINEAR) {
            const int64_t R = t.coef;
            const uint64_t h = (uint64_t)(R >> 1), r = (uint64_t)(R & 1);
            const uint64_t W = t.p0 + t.f0 * tile0 + lin_term(R, dt);
            const uint64_t V = t.f0 + (uint64_t)R * dt;
            const uint64_t I = V + h + ((dt & 1) ? r : 0ull);
            const uint64_t Dp = (uint64_t)R + ((dt & 1) ? (0ull - r) : r);   // step when d has dt's parity
            const uint64_t Dq = (uint64_t)R + ((dt & 1) ? r : (0ull - r));   // the other parity
            uint64_t ph = W + V * (uint64_t)j + (uint64_t)R * (uint64_t)(j * j / 2);
            uint64_t inc = I + (uint64_t)R * (uint64_t)j;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                f(s, ph);
                ph += inc;
                inc += (s & 1) ? Dq : Dp;
            }
        } else {
            const uint64_t *H = table_of(tables, t.table) + dt + j;
            uint64_t ph = t.p0 + t.f0 * tile0 + t.f0 * (uint64_t)j;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                f(s, ph + smooth_term(t.coef, H[s]));
                ph += t.f0;
            }
        }
    } else {                                                        // straddles an edge
        edge_run<S>(t, tables, tile0 + j, f);
    }
}

// Regime loops for a block of tones that share one window and shape (one
// regime per tile for the whole block); same arithmetic as gen_phases.
template <int S, typename F>
__device__ __forceinline__ void static_run(uint64_t P, uint64_t Fw, uint64_t tile0, uint32_t j, F &&f)
{
    uint64_t ph = P + Fw * tile0 + Fw * (uint64_t)j;
#pragma unroll
    for (int s = 0; s < S; ++s) { f(s, ph); ph += Fw; }
}

template <int S, typename F>
__device__ __forceinline__ void linear_run(const ToneDev &t, uint64_t tile0, uint64_t dt, uint32_t j, F &&f)
{
    const int64_t R = t.coef;
    const uint64_t h = (uint64_t)(R >> 1), r = (uint64_t)(R & 1);
    const uint64_t W = t.p0 + t.f0 * tile0 + lin_term(R, dt);
    const uint64_t V = t.f0 + (uint64_t)R * dt;
    const uint64_t I = V + h + ((dt & 1) ? r : 0ull);
    const uint64_t Dp = (uint64_t)R + ((dt & 1) ? (0ull - r) : r);
    const uint64_t Dq = (uint64_t)R + ((dt & 1) ? r : (0ull - r));
    uint64_t ph = W + V * (uint64_t)j + (uint64_t)R * (uint64_t)(j * j / 2);
    uint64_t inc = I + (uint64_t)R * (uint64_t)j;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        f(s, ph);
        ph += inc;
        inc += (s & 1) ? Dq : Dp;
    }
}

// Amplitude of tone t at the lane's samples tile0 + j + s (the a_j[i] of
// Eq. (5)): amp before the amplitude window [b, b+m], amp1 after it, and
// inside amp (1 - w) + amp1 w with w the window's profile at (n - b) / m
// (linear, raised cosine, minimum jerk), exact at both ends.
template <int S>
__device__ __forceinline__ void amp_values(const ToneDev &t, uint64_t tile0, uint64_t tile_last, uint32_t j,
                                           float (&av)[S])
{
    if (t.ashape == AWG_RAMP_NONE || tile_last < t.b || tile0 > t.b + t.m) {
        const float c = (t.ashape == AWG_RAMP_NONE || tile_last < t.b) ? t.amp : t.amp1;
#pragma unroll
        for (int s = 0; s < S; ++s) av[s] = c;
        return;
    }
    const int64_t m = (int64_t)t.m;
    const float fm = (float)t.m;
    const int64_t d0 = (int64_t)(tile0 + j - t.b);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        int64_t d = d0 + s;
        d = d < 0 ? 0 : (d > m ? m : d);
        const float tau = (float)(int32_t)d / fm;               // correctly rounded: 0 and 1 exact
        float w;
        if (t.ashape == AWG_RAMP_LINEAR) w = tau;
        else if (t.ashape == AWG_RAMP_COSINE) w = 0.5f - 0.5f * __builtin_amdgcn_cosf(0.5f * tau);
        else w = tau * tau * tau * __builtin_fmaf(tau, __builtin_fmaf(6.0f, tau, -15.0f), 10.0f);
        av[s] = __builtin_fmaf(t.amp1, w, t.amp * (1.0f - w));
    }
}

__device__ __forceinline__ int16_t quantise(float y)
{
    float r = __builtin_rintf(y);
    r = fminf(fmaxf(r, -32768.0f), 32767.0f);
    return (int16_t)(int32_t)r;
}

// Extra input of the hybrid path: the tones of blocks flagged kBlockSplit are
// summed elsewhere (the matrix cores) on the tiles where they are on a line, so
// the tile skips them there; add[z * add_stride + i], z < n_add, are partial
// sums of sample i of the tile, added in z order before the tile's own sum.
struct HybridIn {
    int32_t n_add;
    const float *add;
    uint64_t add_stride;
};

// Extra input of the periodic line-buffer path (plans whose tones sit on bins of
// a period L): the line tones come from S, an exact fixed-point period sum
// (S[m] * 2^-32 at m = n mod L), plus for each segment whose rows hold this
// tile the difference q_row[m] - q_next[m] of two cached group sums; every
// tone of a split-flagged block is summed only on the tiles in [t.lo, t.hi]
// (window tiles and lines alike). Segments are applied in list order.
struct PlbIn {
    int64_t *S;                  // nullptr: not the line-buffer path
    uint64_t mask;               // L - 1
    const PlbSeg *segs;
    int32_t n_seg;
    uint32_t row;                // this tile's row in the call
    // one part of a split tile: only the pieces pieces[0 .. n_pieces) (piece j
    // on wave j mod 4), and the tile's sum goes to partial[0 .. 64 S) without
    // the line tones and the rounding (added by the part that finishes last)
    const PlbPiece *pieces;      // nullptr: every block, then the full epilogue
    uint32_t n_pieces;
    float *partial;
    // per block: the first and last row its tones are summed on (blocks whose
    // span misses this row are skipped whole)
    const int2 *span;
    // folds applied here, when the launch covers each m = n mod L exactly once:
    // the thread that reads S[m] first adds them and writes S[m] back
    const PlbFold *folds;
    int32_t n_fold;
};

typedef long long s64x2 __attribute__((ext_vector_type(2)));

// fix(x) = x * 2^32 rounded to an integer (the fixed point of S)
__device__ __forceinline__ int64_t plb_fix(float x) { return (int64_t)__builtin_rint((double)x * 0x1p32); }

// sum over the folds f of fix(q_new_f[m]) - fix(q_old_f[m]) at four consecutive m
// (loads of up to four folds in flight together; integer sums, so the order of
// the terms does not matter)
__device__ __forceinline__ void plb_fold4(const PlbFold *folds, int32_t n_fold, uint64_t m0, int64_t (&acc)[4])
{
    constexpr int32_t kBatch = 4;
    for (int32_t f0 = 0; f0 < n_fold; f0 += kBatch) {
        float4 a[kBatch], b[kBatch];
#pragma unroll
        for (int32_t j = 0; j < kBatch; ++j) {
            a[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            b[j] = a[j];
            if (f0 + j < n_fold) {
                const PlbFold fd = folds[f0 + j];
                a[j] = *(const float4 *)(fd.q_new + m0);
                if (fd.q_old) b[j] = *(const float4 *)(fd.q_old + m0);
            }
        }
#pragma unroll
        for (int32_t j = 0; j < kBatch; ++j) {
            acc[0] += plb_fix(a[j].x) - plb_fix(b[j].x);
            acc[1] += plb_fix(a[j].y) - plb_fix(b[j].y);
            acc[2] += plb_fix(a[j].z) - plb_fix(b[j].z);
            acc[3] += plb_fix(a[j].w) - plb_fix(b[j].w);
        }
    }
}

// A split tile's parts hand their partial sums to the part that finishes last,
// which may run on another XCD, whose L2 is not coherent with this one's. The
// sums travel as agent-scope relaxed atomic stores and loads, which are
// coherent at device scope on their own, so no agent-scope fence (on this chip
// a writeback or an invalidation of a whole L2, which stalls every workgroup
// on it) is needed: a part's stores have completed before its workgroup counts
// itself done, and the last part loads the sums after it has read that count.
__device__ __forceinline__ void plb_put_partial(float *dst, const float (&y)[4])
{
    uint64_t *d = (uint64_t *)dst;
    const uint64_t lo = (uint64_t)__float_as_uint(y[0]) | ((uint64_t)__float_as_uint(y[1]) << 32);
    const uint64_t hi = (uint64_t)__float_as_uint(y[2]) | ((uint64_t)__float_as_uint(y[3]) << 32);
    __hip_atomic_store(d, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(d + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float4 plb_get_partial(const float *src)
{
    uint64_t *s = (uint64_t *)src;
    const uint64_t lo = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t hi = __hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float4(__uint_as_float((uint32_t)lo), __uint_as_float((uint32_t)(lo >> 32)),
                       __uint_as_float((uint32_t)hi), __uint_as_float((uint32_t)(hi >> 32)));
}

// The line tones of samples tile0 + i0 .. i0 + PER - 1: S and the segments'
// group differences at m = n mod L, in list order.
template <int PER>
__device__ __forceinline__ void plb_lines(const PlbIn &plb, uint64_t tile0, uint32_t i0, uint32_t valid,
                                          float (&g)[PER])
{
    const uint64_t m0 = (tile0 + i0) & plb.mask;
    if (PER == 4 && i0 + PER <= valid && (m0 & 3) == 0 && m0 + 3 <= plb.mask) {
        longlong2 sa = *(const longlong2 *)(plb.S + m0), sb = *(const longlong2 *)(plb.S + m0 + 2);
        if (plb.n_fold > 0) {
            int64_t acc[4] = {0, 0, 0, 0};
            plb_fold4(plb.folds, plb.n_fold, m0, acc);
            sa.x += acc[0]; sa.y += acc[1]; sb.x += acc[2]; sb.y += acc[3];
            // S is read again a whole pass later: stored non-temporal, so that
            // the launch's end has no L2 full of it to write back
            __builtin_nontemporal_store((s64x2){sa.x, sa.y}, (s64x2 *)(plb.S + m0));
            __builtin_nontemporal_store((s64x2){sb.x, sb.y}, (s64x2 *)(plb.S + m0 + 2));
        }
        g[0] = (float)((double)sa.x * 0x1p-32);
        g[1] = (float)((double)sa.y * 0x1p-32);
        g[2] = (float)((double)sb.x * 0x1p-32);
        g[3] = (float)((double)sb.y * 0x1p-32);
        for (int32_t q = 0; q < plb.n_seg; ++q) {
            const PlbSeg sg = plb.segs[q];
            if (plb.row < sg.row_begin || plb.row > sg.row_end) continue;
            const float4 u = *(const float4 *)(sg.q_row + m0), v = *(const float4 *)(sg.q_next + m0);
            g[0] += u.x - v.x; g[1] += u.y - v.y; g[2] += u.z - v.z; g[3] += u.w - v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint64_t m = (m0 + (uint64_t)e) & plb.mask;
            int64_t v = plb.S[m];
            if (plb.n_fold > 0 && i0 + e < valid) {       // samples past the call: another thread's m
                for (int32_t f = 0; f < plb.n_fold; ++f) {
                    const PlbFold fd = plb.folds[f];
                    v += plb_fix(fd.q_new[m]);
                    if (fd.q_old) v -= plb_fix(fd.q_old[m]);
                }
                plb.S[m] = v;
            }
            g[e] = (float)((double)v * 0x1p-32);
        }
        for (int32_t q = 0; q < plb.n_seg; ++q) {
            const PlbSeg sg = plb.segs[q];
            if (plb.row < sg.row_begin || plb.row > sg.row_end) continue;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const uint64_t m = (m0 + (uint64_t)e) & plb.mask;
                g[e] += sg.q_row[m] - sg.q_next[m];
            }
        }
    }
}

// One tile: the 64*S samples tile0 .. tile0 + 64*S - 1 of a tone list, summed
// by the 4 waves of the workgroup and written to out[0 .. valid). STATIC: every
// tone is a static line (no windows), so the regime logic is compiled out; the
// arithmetic per sample is the same as the static regime of gen_phases, so both
// instantiations give identical sums. HYB: see HybridIn. Ends with a barrier so
// `part` can be reused by the next tile of the same workgroup.
template <int S, bool F32OUT, bool STATIC, bool HYB = false, bool PLB = false>
__device__ __forceinline__ void synth_tile(const ToneDev *__restrict__ tones, const Block *__restrict__ blocks,
                                           const uint64_t *const *__restrict__ tables, uint64_t tile0,
                                           uint32_t valid, void *__restrict__ out, float (*part)[kLanes * S],
                                           const HybridIn &hyb = HybridIn{0, nullptr, 0}, uint32_t ostride = 1,
                                           const PlbIn &plb = PlbIn{nullptr, 0, nullptr, 0, 0, nullptr, 0, nullptr, nullptr, nullptr, 0})
{
    constexpr int T = kLanes * S;                 // samples per tile
    const uint32_t lane = threadIdx.x & 63u;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    float acc[S];
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = 0.0f;

    const int n_blocks = (int)blocks[0].begin;
    const uint64_t tile_last = tile0 + (uint64_t)(T - 1);
    const uint32_t j = lane * S;
    const bool listed = PLB && plb.pieces != nullptr;
    const int n_iter = listed ? (int)plb.n_pieces : n_blocks;
    for (int it = wave; it < n_iter; it += kWaves) {
        PlbPiece pc{(uint32_t)it, 0, 0};
        if (listed) pc = plb.pieces[it];
        if (PLB && !listed) {
            const int2 sp = plb.span[pc.block];
            if ((int)plb.row < sp.x || (int)plb.row > sp.y) continue;
        }
        const Block bk = blocks[1 + pc.block];
        // a piece may take a sub-range of a block's tones (a uniform block's
        // tones share its regime, so any of them stands for the block)
        const int k0 = (int)bk.begin + (int)pc.off;
        const int k1 = pc.cnt ? k0 + (int)pc.cnt : (int)bk.begin + (int)bk.count;
        const bool split = HYB && (bk.flags & kBlockSplit);
        float blk[S];
#pragma unroll
        for (int s = 0; s < S; ++s) blk[s] = 0.0f;
        if (!STATIC && (bk.flags & kBlockAmp)) {
            // tones with an amplitude window: per-tone regimes, per-sample amplitude
            for (int k = k0; k < k1; ++k) {
                const ToneDev t = tones[k];
                if (split && (tile_last < t.lo || tile0 > t.hi)) continue;
                float av[S];
                amp_values<S>(t, tile0, tile_last, j, av);
                gen_phases<S>(t, tables, tile0, lane, [&](int s, uint64_t ph) {
                    blk[s] = __builtin_fmaf(av[s], word_sin(ph), blk[s]);
                });
            }
        } else if (!STATIC && (bk.flags & kBlockUniform)) {
            // every tone of the block has the window and shape of tones[k0]
            const ToneDev r = tones[k0];
            const bool pre = tile_last < r.a, post = tile0 > r.a + r.n;
            if (pre || post) {
                // (a block of split tones on a line is summed elsewhere, except on
                // the line-buffer path, where each tone is summed on its own tiles)
                for (int k = k0; k < (split && !PLB ? k0 : k1); ++k) {
                    if (PLB && split && (tile_last < tones[k].lo || tile0 > tones[k].hi)) continue;
                    const uint64_t P = pre ? tones[k].p0 : tones[k].p1, Fw = pre ? tones[k].f0 : tones[k].f1;
                    const float amp = tones[k].amp;
                    static_run<S>(P, Fw, tile0, j, [&](int s, uint64_t ph) {
                        blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                    });
                }
            } else if (tile0 >= r.a && tile_last <= r.a + r.n) {
                const uint64_t dt = tile0 - r.a;
                if (r.shape == AWG_RAMP_LINEAR) {
                    // two tones per iteration (unrolled; interleaving them sample by
                    // sample by hand measured 2% slower)
#pragma unroll 2
                    for (int k = k0; k < k1; ++k) {
                        const ToneDev t = tones[k];
                        const float amp = t.amp;
                        linear_run<S>(t, tile0, dt, j, [&](int s, uint64_t ph) {
                            blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                        });
                    }
                } else {
                    // the table values of this lane's samples serve every tone of the block
                    const uint64_t *H = table_of(tables, r.table) + dt + j;
                    // A tagged table: incremental steps below (dF a multiple of 2^16 for
                    // every tone of the block, always so for bin frequencies, or any dF);
                    // else the full product per sample. One loop per block, so the loops
                    // never hold registers at the same time.
                    const bool tagged = table_monotone(tables, r.table);
                    const bool step16 = (bk.flags & kBlockStep16) && tagged;
                    // the lane's first table value and the successive differences
                    // (non-negative, below 2^19 when tagged)
                    const uint64_t hv0 = H[0];
                    uint32_t dh[S];
                    if (step16) {
                        uint64_t prev = hv0;
#pragma unroll
                        for (int s = 0; s + 1 < S; ++s) {
                            const uint64_t cur = H[s + 1];
                            dh[s] = (uint32_t)(cur - prev);
                            prev = cur;
                        }
                    }
                    if (step16) {
                        // the chirp term is exactly m*H with m = dF/2^16, and moves by m*dh
                        // per sample. With |m| < 2^47 and dh < 2^23 the product's high word
                        // gains only the low 32 bits of (m >> 32) * dh, whose factors fit
                        // the 24-bit multiplier: one 32x32+64 and one 24x24+32 multiply-add
                        // per sample instead of a full 64x32 product.
                        // two tones at a time, interleaved sample by sample (each
                        // sample still adds tone k, then tone k + 1)
                        int k = k0;
                        for (; k + 1 < k1; k += 2) {
                            const uint64_t f0a = tones[k].f0, f0b = tones[k + 1].f0;
                            const uint64_t ma = (uint64_t)(tones[k].coef >> 16), mb = (uint64_t)(tones[k + 1].coef >> 16);
                            const uint32_t ma_lo = (uint32_t)ma, mb_lo = (uint32_t)mb;
                            const int32_t ma_hi = (int32_t)(ma >> 32), mb_hi = (int32_t)(mb >> 32);   // |.| <= 2^15
                            const float aa = tones[k].amp, ab = tones[k + 1].amp;
                            uint64_t pa = tones[k].p0 + f0a * tile0 + f0a * (uint64_t)j + ma * hv0;
                            uint64_t pb = tones[k + 1].p0 + f0b * tile0 + f0b * (uint64_t)j + mb * hv0;
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                const float sa = word_sin(pa), sb = word_sin(pb);
                                blk[s] = __builtin_fmaf(aa, sa, blk[s]);
                                blk[s] = __builtin_fmaf(ab, sb, blk[s]);
                                if (s + 1 < S) {
                                    const uint64_t la = (uint64_t)ma_lo * dh[s] + f0a;
                                    const uint64_t lb = (uint64_t)mb_lo * dh[s] + f0b;
                                    const uint32_t ha = (uint32_t)(la >> 32) + (uint32_t)__mul24(ma_hi, (int32_t)dh[s]);
                                    const uint32_t hb = (uint32_t)(lb >> 32) + (uint32_t)__mul24(mb_hi, (int32_t)dh[s]);
                                    pa += ((uint64_t)ha << 32) | (uint32_t)la;
                                    pb += ((uint64_t)hb << 32) | (uint32_t)lb;
                                }
                            }
                        }
                        if (k < k1) {
                            const uint64_t p0 = tones[k].p0, f0 = tones[k].f0;
                            const int64_t dF = tones[k].coef;
                            const float amp = tones[k].amp;
                            const uint64_t m = (uint64_t)(dF >> 16);
                            const uint32_t m_lo = (uint32_t)m;
                            const int32_t m_hi = (int32_t)(m >> 32);            // |m_hi| <= 2^15
                            uint64_t ph = p0 + f0 * tile0 + f0 * (uint64_t)j + m * hv0;
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                                if (s + 1 < S) {
                                    const uint64_t lo = (uint64_t)m_lo * dh[s] + f0;
                                    const uint32_t hi = (uint32_t)(lo >> 32) + (uint32_t)__mul24(m_hi, (int32_t)dh[s]);
                                    ph += ((uint64_t)hi << 32) | (uint32_t)lo;
                                }
                            }
                        }
                    } else if (tagged) {
                        // any dF = m 2^16 + r (m = floor(dF / 2^16), 0 <= r < 2^16): the chirp
                        // term floor(dF H / 2^16) is m H + floor(r H / 2^16). With the lane's
                        // rise dH_s = H[s] - H[0] (below 2^23 for a tagged table) and
                        // r H[0] = A_hi 2^16 + A_lo, the word of sample s is
                        //   P + f0 s + m dH_s + floor((A_lo + r dH_s) / 2^16),
                        //   P = p0 + f0 n + m H[0] + A_hi   (n the lane's first sample),
                        // every term exact mod 2^64 and no chain from sample to sample.
                        uint32_t dH[S];
                        dH[0] = 0;
#pragma unroll
                        for (int s = 1; s < S; ++s) dH[s] = (uint32_t)(H[s] - hv0);
                        for (int k = k0; k < k1; ++k) {
                            const uint64_t f0 = tones[k].f0;
                            const int64_t dF = tones[k].coef;
                            const float amp = tones[k].amp;
                            const uint64_t m = (uint64_t)(dF >> 16);
                            const uint32_t rr = (uint32_t)dF & 0xffffu;
                            const uint32_t m_lo = (uint32_t)m;
                            const int32_t m_hi = (int32_t)(m >> 32);            // |m_hi| <= 2^15
                            const uint64_t A = (uint64_t)rr * hv0;              // < 2^63
                            // the line part P + f0 s, advanced by f0 per sample
                            uint64_t ps = tones[k].p0 + f0 * tile0 + f0 * (uint64_t)j + m * hv0 + (A >> 16);
                            const uint32_t a_lo = (uint32_t)A & 0xffffu;
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                const uint64_t lo = (uint64_t)m_lo * dH[s] + ps;
                                const uint64_t t = (uint64_t)rr * dH[s] + a_lo;                 // < 2^40
                                const uint32_t c = __builtin_amdgcn_alignbit((uint32_t)(t >> 32), (uint32_t)t, 16u);
                                // only the word's high half feeds the sine: the low half
                                // gives its carry
                                unsigned int cy0, cy1;
                                (void)__builtin_addc((uint32_t)lo, c, 0u, &cy0);
                                const uint32_t whi = __builtin_addc((uint32_t)(lo >> 32),
                                                                    (uint32_t)__mul24(m_hi, (int32_t)dH[s]), cy0, &cy1);
                                blk[s] = __builtin_fmaf(amp, word_sin((uint64_t)whi << 32), blk[s]);
                                ps += f0;
                            }
                        }
                    } else {
                        for (int k = k0; k < k1; ++k) {
                            const uint64_t p0 = tones[k].p0, f0 = tones[k].f0;
                            const int64_t dF = tones[k].coef;
                            const float amp = tones[k].amp;
                            uint64_t ph = p0 + f0 * tile0 + f0 * (uint64_t)j;
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                blk[s] = __builtin_fmaf(amp, word_sin(ph + smooth_term(dF, H[s])), blk[s]);
                                ph += f0;
                            }
                        }
                    }
                }
            } else if (r.shape != AWG_RAMP_LINEAR && (bk.flags & kBlockStep16) && table_monotone(tables, r.table)) {
                // a smooth window's edge inside the tile, every dF a multiple of 2^16:
                // the word is line(d) + m H[clamp(d, 0, N)] with the line p0 + f0 n up
                // to the window's end and the post-window line after it, so it moves
                // by f0 (d < N) or f1, plus m times the step of the clamped table
                // (zero outside the window). The clamped table values of the lane's
                // samples serve every tone of the block.
                const uint64_t n = tile0 + j;
                const int64_t d0 = (int64_t)(n - r.a), N = (int64_t)r.n;
                const int32_t s_hi = (int32_t)(d0 >= N ? 0 : (N - d0 >= S ? S : N - d0));
                const uint64_t *H = table_of(tables, r.table);
                auto at = [&](int64_t d) { return H[d < 0 ? 0 : (d < N ? d : N)]; };
                const uint64_t hv0 = at(d0);
                uint32_t dh[S];
                uint64_t prev = hv0;
#pragma unroll
                for (int s = 0; s + 1 < S; ++s) {
                    const uint64_t cur = at(d0 + s + 1);
                    dh[s] = (uint32_t)(cur - prev);
                    prev = cur;
                }
                // two tones at a time: the edge tiles finish last
#pragma unroll 2
                for (int k = k0; k < k1; ++k) {
                    const uint64_t p0 = tones[k].p0, f0 = tones[k].f0, f1 = tones[k].f1;
                    const int64_t dF = tones[k].coef;
                    const float amp = tones[k].amp;
                    const uint64_t m = (uint64_t)(dF >> 16);
                    const uint32_t m_lo = (uint32_t)m;
                    const int32_t m_hi = (int32_t)(m >> 32);            // |m_hi| <= 2^15
                    uint64_t ph = (d0 < N ? p0 + f0 * n : p0 + f0 * (r.a + r.n) + f1 * (uint64_t)(d0 - N)) + m * hv0;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                        if (s + 1 < S) {
                            const uint64_t lo = (uint64_t)m_lo * dh[s] + (s < s_hi ? f0 : f1);
                            const uint32_t hi = (uint32_t)(lo >> 32) + (uint32_t)__mul24(m_hi, (int32_t)dh[s]);
                            ph += ((uint64_t)hi << 32) | (uint32_t)lo;
                        }
                    }
                }
            } else if (r.shape != AWG_RAMP_LINEAR && table_monotone(tables, r.table)) {
                // a smooth window's edge inside the tile, any dF: the in-window
                // closed form with the clamped table, H_c(d) = H[clamp(d, 0, N)]:
                // word = L_s + floor(dF H_c / 2^16), where the line part L_s moves by
                // f0 (d < N) or f1, the lane's rise dH_s = H_c(d0 + s) - H_c(d0) is
                // below 2^23, and dF = m 2^16 + r as in the in-window loop
                const uint64_t n = tile0 + j;
                const int64_t d0 = (int64_t)(n - r.a), N = (int64_t)r.n;
                const int32_t s_hi = (int32_t)(d0 >= N ? 0 : (N - d0 >= S ? S : N - d0));
                const uint64_t *H = table_of(tables, r.table);
                auto at = [&](int64_t d) { return H[d < 0 ? 0 : (d < N ? d : N)]; };
                const uint64_t hv0 = at(d0);
                uint32_t dH[S];
                dH[0] = 0;
#pragma unroll
                for (int s = 1; s < S; ++s) dH[s] = (uint32_t)(at(d0 + s) - hv0);
                for (int k = k0; k < k1; ++k) {
                    const uint64_t p0 = tones[k].p0, f0 = tones[k].f0, f1 = tones[k].f1;
                    const int64_t dF = tones[k].coef;
                    const float amp = tones[k].amp;
                    const uint64_t m = (uint64_t)(dF >> 16);
                    const uint32_t rr = (uint32_t)dF & 0xffffu;
                    const uint32_t m_lo = (uint32_t)m;
                    const int32_t m_hi = (int32_t)(m >> 32);            // |m_hi| <= 2^15
                    const uint64_t A = (uint64_t)rr * hv0;              // < 2^63
                    uint64_t ps = (d0 < N ? p0 + f0 * n : p0 + f0 * (r.a + r.n) + f1 * (uint64_t)(d0 - N)) + m * hv0 +
                                  (A >> 16);
                    const uint32_t a_lo = (uint32_t)A & 0xffffu;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const uint64_t lo = (uint64_t)m_lo * dH[s] + ps;
                        const uint64_t t = (uint64_t)rr * dH[s] + a_lo;                 // < 2^40
                        const uint32_t c = __builtin_amdgcn_alignbit((uint32_t)(t >> 32), (uint32_t)t, 16u);
                        unsigned int cy0, cy1;
                        (void)__builtin_addc((uint32_t)lo, c, 0u, &cy0);
                        const uint32_t whi = __builtin_addc((uint32_t)(lo >> 32), (uint32_t)__mul24(m_hi, (int32_t)dH[s]),
                                                            cy0, &cy1);
                        blk[s] = __builtin_fmaf(amp, word_sin((uint64_t)whi << 32), blk[s]);
                        ps += s < s_hi ? f0 : f1;
                    }
                }
            } else {
                // a window edge inside the tile: the slowest tiles of a launch, so
                // two tones at a time for two independent chains per lane
#pragma unroll 2
                for (int k = k0; k < k1; ++k) {
                    const ToneDev t = tones[k];
                    const float amp = t.amp;
                    edge_run<S>(t, tables, tile0 + j, [&](int s, uint64_t ph) {
                        blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                    });
                }
            }
        } else if (STATIC) {
#pragma unroll 2
            for (int k = k0; k < k1; ++k) {
                const uint64_t P = tones[k].p0, Fw = tones[k].f0;
                const float amp = tones[k].amp;
                uint64_t ph = (P + Fw * tile0) + Fw * (uint64_t)(lane * S);
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                    ph += Fw;
                }
            }
        } else {
            for (int k = k0; k < k1; ++k) {
                const ToneDev t = tones[k];
                if (split && (tile_last < t.lo || tile0 > t.hi)) continue;
                const float amp = t.amp;
                gen_phases<S>(t, tables, tile0, lane, [&](int s, uint64_t ph) {
                    blk[s] = __builtin_fmaf(amp, word_sin(ph), blk[s]);
                });
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += blk[s];
    }

#pragma unroll
    for (int s = 0; s < S; ++s) part[wave][lane * S + s] = acc[s];
    __syncthreads();

    constexpr int PER = T / 256;                  // samples per thread in the epilogue
    static_assert(PER == 4, "epilogue reads float4");
    const uint32_t i0 = threadIdx.x * PER;
    float g[PER];
    if (HYB && hyb.n_add > 0) {
        if (i0 + PER <= valid) {
            // loads of up to 8 planes in flight together, added in plane order
            constexpr int kBatch = 8;
            for (int z0 = 0; z0 < hyb.n_add; z0 += kBatch) {
                float4 u[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q)
                    if (z0 + q < hyb.n_add) u[q] = *(const float4 *)(hyb.add + (uint64_t)(z0 + q) * hyb.add_stride + i0);
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    if (z0 + q >= hyb.n_add) break;
                    if (z0 + q == 0) {
                        g[0] = u[q].x; g[1] = u[q].y; g[2] = u[q].z; g[3] = u[q].w;
                    } else {
                        g[0] += u[q].x; g[1] += u[q].y; g[2] += u[q].z; g[3] += u[q].w;
                    }
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                g[e] = 0.0f;
                if (i0 + e < valid) {
                    g[e] = hyb.add[i0 + e];
                    for (int z = 1; z < hyb.n_add; ++z) g[e] += hyb.add[(uint64_t)z * hyb.add_stride + i0 + e];
                }
            }
        }
    }
    if (PLB && plb.partial) {
        // one part of a split tile: its four wave sums, every sample of the tile
        float y[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint32_t i = i0 + e;
            y[e] = ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i];
        }
        plb_put_partial(plb.partial + i0, y);
        __syncthreads();
        return;
    }
    if (PLB) plb_lines<PER>(plb, tile0, i0, valid, g);
    int16_t *const o16 = (int16_t *)out + i0;
    if (PLB && !F32OUT && ostride == 1 && i0 + PER <= valid && ((uintptr_t)o16 & 7) == 0) {
        // a line-buffer thread's four codes in one 8-byte store, non-temporal:
        // nothing in the pass reads the chunk back
        uint64_t w = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint32_t i = i0 + e;
            const float y = g[e] + (((part[0][i] + part[1][i]) + part[2][i]) + part[3][i]);
            w |= (uint64_t)(uint16_t)quantise(y) << (16 * e);
        }
        __builtin_nontemporal_store(w, (uint64_t *)o16);
    } else {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint32_t i = i0 + e;
            float y = ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i];
            if (HYB && hyb.n_add > 0) y = g[e] + y;
            if (PLB) y = g[e] + y;
            if (i < valid) {
                if (F32OUT) ((float *)out)[(size_t)i * ostride] = y;
                else ((int16_t *)out)[(size_t)i * ostride] = quantise(y);
            }
        }
    }
    __syncthreads();
}

template <int S, bool F32OUT, bool STATIC>
__global__ __launch_bounds__(256) void direct_kernel(const ToneDev *__restrict__ tones,
                                                     const Block *__restrict__ blocks,
                                                     const uint64_t *const *__restrict__ tables, uint64_t n0,
                                                     uint64_t count, void *__restrict__ out)
{
    constexpr int T = kLanes * S;
    __shared__ float part[kWaves][T];
    const uint64_t rel = (uint64_t)blockIdx.x * T;
    const uint64_t left = count - rel;
    const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
    void *o = F32OUT ? (void *)((float *)out + rel) : (void *)((int16_t *)out + rel);
    synth_tile<S, F32OUT, STATIC>(tones, blocks, tables, n0 + rel, valid, o, part);
}

// Hybrid path: the tiles of a ramped plan's range with the line tones summed by
// the matrix cores into n_planes partial planes (see HybridIn). Workgroup b
// takes tile order[b]: the host puts the costliest tiles (window edges) first,
// so they do not start last and hold up the end of the launch.
template <int S, bool F32OUT>
__global__ __launch_bounds__(256) void direct_hybrid_kernel(const ToneDev *__restrict__ tones,
                                                            const Block *__restrict__ blocks,
                                                            const uint32_t *__restrict__ order,
                                                            const uint64_t *const *__restrict__ tables,
                                                            uint64_t n0, uint64_t count, void *__restrict__ out,
                                                            const float *__restrict__ planes, int32_t n_planes,
                                                            uint64_t plane_stride)
{
    constexpr int T = kLanes * S;
    __shared__ float part[kWaves][T];
    const uint64_t rel = (uint64_t)order[blockIdx.x] * T;
    const uint64_t left = count - rel;
    const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
    void *o = F32OUT ? (void *)((float *)out + rel) : (void *)((int16_t *)out + rel);
    const HybridIn hyb{n_planes, planes + rel, plane_stride};
    synth_tile<S, F32OUT, false, true>(tones, blocks, tables, n0 + rel, valid, o, part, hyb);
}

// A split tile of a line-buffer launch, by the workgroup of its last part: the
// parts' sums added in part order, then the line tones and the rounding, as
// the tile epilogue does for a whole tile (y = lines + sum).
template <bool F32OUT>
__device__ __forceinline__ void plb_finish(const PlbSplit sp, const float *__restrict__ partials, uint64_t n0,
                                           uint64_t count, void *__restrict__ out, int64_t *__restrict__ S_sum,
                                           uint64_t mask, const PlbSeg *__restrict__ segs, int32_t n_seg,
                                           const PlbFold *__restrict__ folds, int32_t n_fold)
{
    constexpr int T = kTileSamples;
    constexpr int PER = T / 256;
    const uint64_t rel = (uint64_t)sp.row * T;
    const uint64_t left = count - rel;
    const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
    const uint32_t i0 = threadIdx.x * PER;
    const float *pp = partials + (size_t)sp.first * T + i0;
    float y[PER] = {0.0f, 0.0f, 0.0f, 0.0f};
    // loads of up to 8 parts in flight together, added in part order
    constexpr uint32_t kBatch = 8;
    for (uint32_t q0 = 0; q0 < sp.n; q0 += kBatch) {
        float4 u[kBatch];
#pragma unroll
        for (uint32_t q = 0; q < kBatch; ++q)
            if (q0 + q < sp.n) u[q] = plb_get_partial(pp + (size_t)(q0 + q) * T);
#pragma unroll
        for (uint32_t q = 0; q < kBatch; ++q) {
            if (q0 + q >= sp.n) break;
            if (q0 + q == 0) {
                y[0] = u[q].x; y[1] = u[q].y; y[2] = u[q].z; y[3] = u[q].w;
            } else {
                y[0] += u[q].x; y[1] += u[q].y; y[2] += u[q].z; y[3] += u[q].w;
            }
        }
    }
    const PlbIn plb{S_sum, mask, segs, n_seg, sp.row, nullptr, 0, nullptr, nullptr, folds, n_fold};
    float g[PER];
    plb_lines<PER>(plb, n0 + rel, i0, valid, g);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const uint32_t i = i0 + e;
        const float z = g[e] + y[e];
        if (i < valid) {
            if (F32OUT) ((float *)out)[rel + i] = z;
            else ((int16_t *)out)[rel + i] = quantise(z);
        }
    }
}

// Periodic line-buffer path: tile order[b] of the range, the direct list's
// tones on their own tiles, the line tones from S and the segments (PlbIn).
template <int S, bool F32OUT>
__global__ __launch_bounds__(256) void plb_kernel(const ToneDev *__restrict__ tones, const Block *__restrict__ blocks,
                                                  const PlbItem *__restrict__ items,
                                                  const uint64_t *const *__restrict__ tables, uint64_t n0,
                                                  uint64_t count, void *__restrict__ out, int64_t *__restrict__ S_sum,
                                                  uint64_t mask, const PlbSeg *__restrict__ segs, int32_t n_seg,
                                                  const PlbPiece *__restrict__ pieces, float *__restrict__ partials,
                                                  const int2 *__restrict__ span, const PlbFold *__restrict__ folds,
                                                  int32_t n_fold, const PlbSplit *__restrict__ splits,
                                                  int32_t *__restrict__ counts)
{
    constexpr int T = kLanes * S;
    __shared__ float part[kWaves][T];
    __shared__ int32_t last;
    const PlbItem item = items[blockIdx.x];
    const uint32_t row = item.row;
    const uint64_t rel = (uint64_t)row * T;
    const uint64_t left = count - rel;
    const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
    void *o = F32OUT ? (void *)((float *)out + rel) : (void *)((int16_t *)out + rel);
    const bool is_part = item.part >= 0;
    const PlbIn plb{S_sum, mask, segs, n_seg, row, is_part ? pieces + item.first : nullptr, item.count,
                    is_part ? partials + (size_t)item.part * T : nullptr, span, folds, n_fold};
    synth_tile<S, F32OUT, false, true, true>(tones, blocks, tables, n0 + rel, valid, o, part,
                                             HybridIn{0, nullptr, 0}, 1, plb);
    if (!is_part) return;
    // count the part done once every thread's partial stores have completed;
    // the part that completes its tile loads the others' sums and adds them
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        last = __hip_atomic_fetch_add(&counts[item.split], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               (int32_t)splits[item.split].n - 1;
    __syncthreads();
    if (!last) return;
    plb_finish<F32OUT>(splits[item.split], partials, n0, count, out, S_sum, mask, segs, n_seg, folds, n_fold);
    if (threadIdx.x == 0) counts[item.split] = 0;        // ready for the next launch
}

// S[m] += sum over the folds f of fix(q_new_f[m]) - fix(q_old_f[m]) (q_old_f may
// be null), fix(x) = x * 2^32 rounded to an integer: S stays the exact sum of
// the fixed-point group sums it holds, whatever order groups come and go in.
// Four samples per thread; L a multiple of 1024.
__global__ __launch_bounds__(256) void plb_fold_kernel(int64_t *__restrict__ S_sum, uint64_t L,
                                                       const PlbFold *__restrict__ folds, int32_t n_fold)
{
    const uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= L) return;
    int64_t acc[4] = {0, 0, 0, 0};
    plb_fold4(folds, n_fold, i0, acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) S_sum[i0 + e] += acc[e];
}

// S[0 .. L) = 0 (a kernel, so the path records no memset).
__global__ __launch_bounds__(256) void plb_zero_kernel(int64_t *__restrict__ S_sum, uint64_t L)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L) S_sum[i] = 0;
}

// Batched synthesis of many plans' chunks in one launch (continuous batching).
// items[0 .. n_items) are sorted by tile_begin and cover tiles [0, total_tiles)
// without gaps; a fixed grid walks the tiles with a stride of gridDim.x, so one
// launch shape serves every batch (hipGraph replay). Each tile runs exactly the
// same code as direct_kernel, so a plan's output does not depend on the batch.
template <int S>
__global__ __launch_bounds__(256) void batch_kernel(const BatchItem *__restrict__ items,
                                                    const uint32_t *__restrict__ header)
{
    constexpr int T = kLanes * S;
    __shared__ float part[kWaves][T];
    const uint32_t n_items = header[0], total = header[1];
    for (uint32_t t = blockIdx.x; t < total; t += gridDim.x) {
        uint32_t lo = 0, hi = n_items;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (items[mid].tile_begin <= t) lo = mid; else hi = mid;
        }
        const BatchItem &it = items[lo];
        const uint64_t rel = (uint64_t)(t - it.tile_begin) * T;
        const uint64_t left = it.count - rel;
        const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
        const uint32_t st = (uint32_t)it.out_stride;
        int16_t *o = (int16_t *)it.out + rel * st;
        if (it.is_static)
            synth_tile<S, false, true>(it.tones, it.blocks, it.tables, it.n0 + rel, valid, o, part, HybridIn{0, nullptr, 0}, st);
        else
            synth_tile<S, false, false>(it.tones, it.blocks, it.tables, it.n0 + rel, valid, o, part, HybridIn{0, nullptr, 0}, st);
    }
}

// Multiplexed output (the paper's wavetable multiplexer fused into synthesis):
// channel c = blockIdx.y writes sample i of its range to out_c[i * out_stride],
// with out_c = base + c and out_stride = the channel count, so one buffer holds
// groups of one sample per channel. Same tile code as the direct kernel.
struct MuxArgs {
    BatchItem items[kMaxChannels];
};

template <int S>
__global__ __launch_bounds__(256) void mux_kernel(MuxArgs args)
{
    constexpr int T = kLanes * S;
    __shared__ float part[kWaves][T];
    const BatchItem &it = args.items[blockIdx.y];
    const uint64_t rel = (uint64_t)blockIdx.x * T;
    const uint64_t left = it.count - rel;
    const uint32_t valid = left < (uint64_t)T ? (uint32_t)left : (uint32_t)T;
    const uint32_t st = (uint32_t)it.out_stride;
    int16_t *o = (int16_t *)it.out + rel * st;
    if (it.is_static)
        synth_tile<S, false, true>(it.tones, it.blocks, it.tables, it.n0 + rel, valid, o, part, HybridIn{0, nullptr, 0}, st);
    else
        synth_tile<S, false, false>(it.tones, it.blocks, it.tables, it.n0 + rel, valid, o, part, HybridIn{0, nullptr, 0}, st);
}

template <int S>
__global__ __launch_bounds__(64) void phase_dump_kernel(const ToneDev *__restrict__ tones, int32_t tone,
                                                        const uint64_t *const *__restrict__ tables,
                                                        uint64_t n0, uint64_t count, uint64_t *__restrict__ out)
{
    constexpr int T = kLanes * S;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t tile0 = n0 + (uint64_t)blockIdx.x * T;
    const ToneDev t = tones[tone];
    gen_phases<S>(t, tables, tile0, lane, [&](int s, uint64_t ph) {
        const uint64_t rel = (uint64_t)blockIdx.x * T + lane * S + s;
        if (rel < count) out[rel] = ph - kPhaseBias;
    });
}

__global__ void scatter_tones_kernel(ToneDev *__restrict__ tones, const ScatterRecord *__restrict__ rec,
                                     int32_t n)
{
    plb_scatter_range(tones, rec, n, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                      (uint64_t)gridDim.x * blockDim.x);
}

constexpr int kS = 16;                             // samples per lane
constexpr uint64_t kMaxTilesPerLaunch = 1u << 30;

static_assert(kLanes * kS == kTileSamples, "tile size");

template <bool F32OUT>
static hipError_t launch_direct(const awg_plan *p, uint64_t n0, uint64_t count, void *out, hipStream_t s,
                                bool timed = true)
{
    constexpr uint64_t T = kLanes * kS;
    const uint64_t esz = F32OUT ? 4 : 2;
    while (count > 0) {
        const uint64_t tiles = (count + T - 1) / T;
        const uint64_t now_tiles = tiles < kMaxTilesPerLaunch ? tiles : kMaxTilesPerLaunch;
        const uint64_t now = now_tiles * T < count ? now_tiles * T : count;
        hipError_t e;
        {
            // untimed launches take no profiler events (the allocation-free call)
            ProfScope prof(timed ? p->ctx : nullptr, s, F32OUT ? "direct_kernel_f32" : "direct_kernel");
            prof.add_work((double)p->n_tones * (double)now);
            if (p->n_ramped == 0)
                prof.launch(direct_kernel<kS, F32OUT, true>, dim3((uint32_t)now_tiles), dim3(256), 0, p->d_tones,
                            p->d_blocks, p->d_table_ptrs, n0, now, out);
            else
                prof.launch(direct_kernel<kS, F32OUT, false>, dim3((uint32_t)now_tiles), dim3(256), 0, p->d_tones,
                            p->d_blocks, p->d_table_ptrs, n0, now, out);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        n0 += now;
        count -= now;
        out = (char *)out + now * esz;
    }
    return hipSuccess;
}

hipError_t launch_direct_i16(const awg_plan *p, uint64_t n0, uint64_t count, int16_t *out, hipStream_t s)
{
    return launch_direct<false>(p, n0, count, out, s);
}

hipError_t launch_direct_f32(const awg_plan *p, uint64_t n0, uint64_t count, float *out, hipStream_t s, bool timed)
{
    return launch_direct<true>(p, n0, count, out, s, timed);
}

hipError_t launch_phase_dump(const awg_plan *p, int32_t tone, uint64_t n0, uint64_t count,
                             uint64_t *out, hipStream_t s)
{
    constexpr uint64_t T = kLanes * kS;
    while (count > 0) {
        const uint64_t tiles = (count + T - 1) / T;
        const uint64_t now_tiles = tiles < kMaxTilesPerLaunch ? tiles : kMaxTilesPerLaunch;
        const uint64_t now = now_tiles * T < count ? now_tiles * T : count;
        hipError_t e;
        {
            ProfScope prof(p->ctx, s, "phase_dump_kernel");
            prof.launch(phase_dump_kernel<kS>, dim3((uint32_t)now_tiles), dim3(64), 0, p->d_tones, tone,
                        p->d_table_ptrs, n0, now, out);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
        n0 += now;
        count -= now;
        out += now;
    }
    return hipSuccess;
}

hipError_t launch_direct_hybrid(const awg_plan *p, const ToneDev *d_tones, const Block *d_blocks,
                                const uint32_t *d_order, uint64_t n0, uint64_t count, const float *planes,
                                int32_t n_planes, uint64_t plane_stride, int16_t *out_i16, float *out_f32,
                                hipStream_t s, double work)
{
    constexpr uint64_t T = kLanes * kS;
    const uint64_t tiles = (count + T - 1) / T;
    if (tiles == 0) return hipSuccess;
    if (tiles > kMaxTilesPerLaunch) return hipErrorInvalidValue;
    ProfScope prof(p->ctx, s, out_f32 ? "direct_hybrid_kernel_f32" : "direct_hybrid_kernel");
    prof.add_work(work);
    if (out_f32)
        prof.launch(direct_hybrid_kernel<kS, true>, dim3((uint32_t)tiles), dim3(256), 0, d_tones, d_blocks, d_order,
                    p->d_table_ptrs, n0, count, (void *)out_f32, planes, n_planes, plane_stride);
    else
        prof.launch(direct_hybrid_kernel<kS, false>, dim3((uint32_t)tiles), dim3(256), 0, d_tones, d_blocks,
                    d_order, p->d_table_ptrs, n0, count, (void *)out_i16, planes, n_planes, plane_stride);
    return hipGetLastError();
}

hipError_t launch_plb(const awg_plan *p, const ToneDev *d_tones, const Block *d_blocks, const PlbItem *d_items,
                      int32_t n_items, const PlbPiece *d_pieces, const int2 *d_span, float *d_partials,
                      const PlbSplit *d_splits, int32_t *d_counts,
                      int32_t n_split, uint64_t n0, uint64_t count, int64_t *d_S, uint64_t L,
                      const PlbSeg *d_segs, int32_t n_seg, const PlbFold *d_folds, int32_t n_fold,
                      int16_t *out_i16, float *out_f32, hipStream_t s, double work)
{
    constexpr uint64_t T = kLanes * kS;
    static_assert(T == kTileSamples, "line-buffer rows are direct-kernel tiles");
    const uint64_t tiles = (count + T - 1) / T;
    if (tiles == 0) return hipSuccess;
    if (tiles > kMaxTilesPerLaunch || L < T || (L & (L - 1)) != 0 || n_items <= 0 || n_split < 0)
        return hipErrorInvalidValue;
    if (n_fold > 0 && count != L) return hipErrorInvalidValue;      // each m once: see PlbIn
    {
        ProfScope prof(p->ctx, s, out_f32 ? "plb_kernel_f32" : "plb_kernel");
        prof.add_work(work);
        if (out_f32)
            prof.launch(plb_kernel<kS, true>, dim3((uint32_t)n_items), dim3(256), 0, d_tones, d_blocks, d_items,
                        p->d_table_ptrs, n0, count, (void *)out_f32, d_S, L - 1, d_segs, n_seg, d_pieces, d_partials,
                        d_span, d_folds, n_fold, d_splits, d_counts);
        else
            prof.launch(plb_kernel<kS, false>, dim3((uint32_t)n_items), dim3(256), 0, d_tones, d_blocks, d_items,
                        p->d_table_ptrs, n0, count, (void *)out_i16, d_S, L - 1, d_segs, n_seg, d_pieces, d_partials,
                        d_span, d_folds, n_fold, d_splits, d_counts);
    }
    return hipGetLastError();
}

hipError_t launch_plb_fold(const awg_plan *p, int64_t *d_S, uint64_t L, const PlbFold *d_folds, int32_t n_fold,
                           hipStream_t s)
{
    if (n_fold <= 0) return hipSuccess;
    if (L < 1024 || (L & (L - 1)) != 0) return hipErrorInvalidValue;
    ProfScope prof(p->ctx, s, "plb_fold_kernel");
    prof.launch(plb_fold_kernel, dim3((uint32_t)(L / 1024)), dim3(256), 0, d_S, L, d_folds, n_fold);
    return hipGetLastError();
}

hipError_t launch_plb_zero(int64_t *d_S, uint64_t L, hipStream_t s)
{
    hipLaunchKernelGGL(plb_zero_kernel, dim3((uint32_t)((L + 255) / 256)), dim3(256), 0, s, d_S, L);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchItem *d_items, const uint32_t *d_header, uint32_t grid, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel<kS>, dim3(grid), dim3(256), 0, s, d_items, d_header);
    return hipGetLastError();
}

// max |y| over y[0 .. count): per-thread grid-stride max, a wave max with
// cross-lane shuffles, then one atomic max per wave on the float's bit pattern
// (for non-negative floats the unsigned order is the numeric order).
__global__ __launch_bounds__(256) void peak_kernel(const float *__restrict__ y, uint64_t count,
                                                   unsigned int *__restrict__ peak_bits)
{
    float m = 0.0f;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(y[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(peak_bits, __float_as_uint(m));
}

__global__ void zero_word_kernel(unsigned int *w) { *w = 0u; }

// Scratch of awg_peak_noalloc: the FP32 samples of one request. A file-scope
// device array, so that the call allocates nothing; every device the library
// runs on holds its own copy until the process ends. Host code never passes
// the array's name to a kernel (on the host it only stands for the symbol):
// it uses the device address noalloc_scratch looked up for the device.
static __device__ __align__(256) float scratch[AWG_PEAK_NOALLOC_MAX];

hipError_t noalloc_scratch(int device, float **ptr)
{
    static std::mutex mu;
    static std::map<int, float *> addr;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void *a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!a) return hipErrorInvalidSymbol;
    addr[device] = (float *)a;
    *ptr = (float *)a;
    return hipSuccess;
}

hipError_t launch_peak(const float *d_y, uint64_t count, float *d_peak, hipStream_t s)
{
    hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(1), 0, s, (unsigned int *)d_peak);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(peak_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, d_y, count, (unsigned int *)d_peak);
    return hipGetLastError();
}

hipError_t launch_mux(const BatchItem *items, int32_t n, uint64_t count, hipStream_t s, ProfScope &prof)
{
    constexpr uint64_t T = kLanes * kS;
    if (n < 1 || n > kMaxChannels) return hipErrorInvalidValue;
    MuxArgs args;
    for (int c = 0; c < n; ++c) args.items[c] = items[c];
    while (count > 0) {
        const uint64_t tiles = (count + T - 1) / T;
        const uint64_t now_tiles = tiles < kMaxTilesPerLaunch ? tiles : kMaxTilesPerLaunch;
        const uint64_t now = now_tiles * T < count ? now_tiles * T : count;
        for (int c = 0; c < n; ++c) args.items[c].count = now;
        (void)s;
        prof.launch(mux_kernel<kS>, dim3((uint32_t)now_tiles, (uint32_t)n), dim3(256), 0, args);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        count -= now;
        for (int c = 0; c < n; ++c) {
            args.items[c].n0 += now;
            args.items[c].out = (int16_t *)args.items[c].out + now * (uint64_t)args.items[c].out_stride;
        }
    }
    return hipSuccess;
}

// Host-to-device copy by a kernel (see launch_upload): 16-byte words with a grid
// stride, then the tail bytes.
__global__ __launch_bounds__(256) void upload_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     uint64_t n16, const uint8_t *__restrict__ src_tail,
                                                     uint8_t *__restrict__ dst_tail, uint32_t tail)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0 && threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

hipError_t launch_upload(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return hipErrorInvalidValue;
    const uint64_t n16 = bytes / 16;
    const uint32_t tail = (uint32_t)(bytes % 16);
    const uint64_t blocks = std::min<uint64_t>(std::max<uint64_t>((n16 + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(upload_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n16,
                       (const uint8_t *)src + n16 * 16, (uint8_t *)dst + n16 * 16, tail);
    return hipGetLastError();
}

// The line-buffer path's staged lists: compact descriptors from pinned memory
// become ToneDev records in device memory (plan tones gathered from the plan's
// device table), and the rest of the staging blob is copied as it is.
__global__ __launch_bounds__(256) void plb_stage_kernel(const PlbDesc *__restrict__ desc, int32_t n_first,
                                                        int32_t n_desc, const ToneDev *__restrict__ plan_tones,
                                                        uint64_t n0, ToneDev *__restrict__ dst_first,
                                                        ToneDev *__restrict__ dst_rest,
                                                        const uint4 *__restrict__ raw_src, uint4 *__restrict__ raw_dst,
                                                        uint64_t n16)
{
    plb_stage_range(desc, n_first, n_desc, plan_tones, n0, dst_first, dst_rest, raw_src, raw_dst, n16,
                    (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x);
}

hipError_t launch_plb_stage(const PlbDesc *desc, int32_t n_first, int32_t n_desc, const ToneDev *plan_tones,
                            uint64_t n0, ToneDev *dst_first, ToneDev *dst_rest, const void *raw_src, void *raw_dst,
                            size_t raw_bytes, hipStream_t s)
{
    if (n_first < 0 || n_first > n_desc) return hipErrorInvalidValue;
    if (((uintptr_t)raw_src | (uintptr_t)raw_dst | raw_bytes) & 15) return hipErrorInvalidValue;
    const uint64_t n16 = raw_bytes / 16;
    const uint64_t work = std::max<uint64_t>((uint64_t)n_desc, n16);
    const uint64_t blocks = std::min<uint64_t>(std::max<uint64_t>((work + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(plb_stage_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, desc, n_first, n_desc, plan_tones,
                       n0, dst_first, dst_rest, (const uint4 *)raw_src, (uint4 *)raw_dst, n16);
    return hipGetLastError();
}

hipError_t alloc_upload_host(size_t bytes, void **host, void **mapped)
{
    *host = nullptr;
    *mapped = nullptr;
    hipError_t e = hipHostMalloc(host, bytes, hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(mapped, *host, 0);
    if (e != hipSuccess && *host) {
        (void)hipHostFree(*host);
        *host = nullptr;
        *mapped = nullptr;
    }
    return e;
}

hipError_t launch_scatter_tones(ToneDev *d_tones, const void *d_records, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_tones_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_tones,
                       (const ScatterRecord *)d_records, n);
    return hipGetLastError();
}

}  // namespace awg
