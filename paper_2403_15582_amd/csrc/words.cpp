// Exact word arithmetic of the plan step: frequency and phase words, chirp
// coefficients and the smooth-ramp tables. Integer-exact throughout: every
// rounding is half-to-even on an exactly computed rational.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <cstring>

#include "awg_internal.h"

namespace awg {

typedef unsigned __int128 u128;
typedef __int128 i128;

// x = m * 2^e with m < 2^53 an integer (x > 0, finite).
static void decompose(double x, uint64_t *m, int *e)
{
    uint64_t bits;
    std::memcpy(&bits, &x, sizeof bits);
    const int be = (int)((bits >> 52) & 0x7ff);
    if (be != 0 && be != 0x7ff) {                  // normal: the stored fields
        *m = (bits & ((1ull << 52) - 1)) | (1ull << 52);
        *e = be - 1075;
        return;
    }
    int ex;
    double fr = std::frexp(x, &ex);
    *m = (uint64_t)std::ldexp(fr, 53);
    *e = ex - 53;
}

// nint(num * 2^shift / den) for finite num, den > 0. False if it is >= 2^64.
bool rne_ratio_shift(double num, double den, int shift, uint64_t *out)
{
    uint64_t mn, md;
    int en, ed;
    decompose(num, &mn, &en);
    decompose(den, &md, &ed);
    const int e = en - ed + shift;           // value = mn * 2^e / md
    // usual case: the FP64 quotient as a first guess, settled exactly: q is
    // nint(value) iff (2q - 1) md <= 2 mn 2^e <= (2q + 1) md (ties to even);
    // products, no 128-bit division
    if (e >= 0 && e <= 70) {
        double scale = 0.0;                        // 2^shift
        if (shift >= -1022 && shift <= 1023) {
            const uint64_t sb = (uint64_t)(shift + 1023) << 52;
            std::memcpy(&scale, &sb, sizeof scale);
        }
        const double v = (num / den) * scale;
        if (scale > 0.0 && v >= 0.0 && v < 0x1p63) {
            const u128 A = (u128)mn << (e + 1), D = md;
            uint64_t q = (uint64_t)(v + 0.5);
            for (int it = 0; it < 4; ++it) {
                const u128 hi = ((u128)q * 2 + 1) * D;
                if (A > hi || (A == hi && (q & 1))) { ++q; continue; }
                if (q > 0) {
                    const u128 lo = ((u128)q * 2 - 1) * D;
                    if (A < lo || (A == lo && (q & 1))) { --q; continue; }
                }
                *out = q;
                return true;
            }
        }
    }
    u128 n, d;
    if (e >= 0) {
        if (e > 74) return false;            // value >= 2^73
        n = (u128)mn << e;
        d = md;
    } else {
        if (-e > 74) { *out = 0; return true; }   // value < 2^-73
        n = mn;
        d = (u128)md << (-e);
    }
    u128 q = n / d, r = n % d;
    u128 r2 = r << 1;                        // r < d < 2^127
    if (r2 > d || (r2 == d && (q & 1))) q += 1;
    if (q >> 64) return false;
    *out = (uint64_t)q;
    return true;
}

// Frequency word of f at fs (Eq. (4) when period_log2 > 0).
awg_status freq_word(double f, double fs, uint32_t p, uint64_t *out)
{
    if (!std::isfinite(f) || !(f > 0.0) || !(f < fs * 0.5)) return AWG_E_INVALID;
    uint64_t w;
    if (p > 0) {
        if (!rne_ratio_shift(f, fs, (int)p, &w)) return AWG_E_RANGE;
        if (w < 1 || w >= (1ull << (p - 1))) return AWG_E_RANGE;
        *out = w << (64 - p);
        return AWG_OK;
    }
    if (!rne_ratio_shift(f, fs, 64, &w)) return AWG_E_RANGE;
    if (w < 1 || w >= (1ull << 63)) return AWG_E_RANGE;
    *out = w;
    return AWG_OK;
}

// nint(turns * 2^64) mod 2^64 for any finite double.
uint64_t phase_word(double turns)
{
    if (turns == 0.0) return 0;
    int ex;
    double fr = std::frexp(turns, &ex);
    const int64_t m = (int64_t)std::ldexp(fr, 53);   // |m| < 2^53, exact
    const int e = ex - 53 + 64;                      // turns * 2^64 = m * 2^e
    if (e >= 64) return 0;
    if (e >= 0) return (uint64_t)m << e;
    const int sh = -e;
    if (sh >= 60) return 0;                          // |value| < 2^-7
    int64_t q = m >> sh;                             // floor
    const uint64_t r = (uint64_t)m - ((uint64_t)q << sh);
    const uint64_t half = 1ull << (sh - 1);
    if (r > half || (r == half && (q & 1))) q += 1;
    return (uint64_t)q;
}

// nint(num / den), ties to even, den >= 1.
int64_t rne_div(int64_t num, uint64_t den)
{
    if (den <= (uint64_t)INT64_MAX) {               // the same in 64-bit arithmetic
        const int64_t d = (int64_t)den;
        int64_t q = num / d, r = num % d;
        if (r < 0) { q -= 1; r += d; }               // floor division, r in [0, d)
        const uint64_t r2 = (uint64_t)r * 2;         // < 2^64
        if (r2 > den || (r2 == den && (q & 1))) q += 1;
        return q;
    }
    const i128 d = (i128)den;
    i128 q = (i128)num / d, r = (i128)num % d;
    if (r < 0) { q -= 1; r += d; }                   // floor division, r in [0, d)
    const i128 r2 = r * 2;
    if (r2 > d || (r2 == d && (q & 1))) q += 1;
    return (int64_t)q;
}

// ------------------------------------------------------------ 256-bit helpers

struct U256 { uint64_t w[4]; };

static U256 u256(u128 x)
{
    U256 r = {{(uint64_t)x, (uint64_t)(x >> 64), 0, 0}};
    return r;
}

static U256 mul_u64(const U256 &a, uint64_t b)
{
    U256 r = {{0, 0, 0, 0}};
    u128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        u128 t = (u128)a.w[i] * b + carry;
        r.w[i] = (uint64_t)t;
        carry = t >> 64;
    }
    return r;
}

static U256 add(const U256 &a, const U256 &b)
{
    U256 r;
    u128 carry = 0;
    for (int i = 0; i < 4; ++i) {
        u128 t = (u128)a.w[i] + b.w[i] + carry;
        r.w[i] = (uint64_t)t;
        carry = t >> 64;
    }
    return r;
}

static U256 mul_u128(const U256 &a, u128 b)
{
    U256 lo = mul_u64(a, (uint64_t)b);
    U256 hi = mul_u64(a, (uint64_t)(b >> 64));
    U256 sh = {{0, hi.w[0], hi.w[1], hi.w[2]}};
    return add(lo, sh);
}

static U256 shl(const U256 &a, int s)   // 0 < s < 64
{
    U256 r;
    for (int i = 3; i > 0; --i) r.w[i] = (a.w[i] << s) | (a.w[i - 1] >> (64 - s));
    r.w[0] = a.w[0] << s;
    return r;
}

static int cmp(const U256 &a, const U256 &b)
{
    for (int i = 3; i >= 0; --i) {
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    }
    return 0;
}

// Minimum-jerk table entry, exactly nint(2^15 d^4 (5N^2 - 6dN + 2d^2) / N^5),
// i.e. 2^16 N Psi(d/N) with Psi(t) = 5/2 t^4 - 3 t^5 + t^6 (the integral of the
// minimum-jerk frequency profile, Eq. (8) case 1). N < 2^31, 0 <= d <= N.
int64_t minjerk_entry(uint64_t n, uint64_t d)
{
    if (d == 0) return 0;
    if (d == n) return (int64_t)(n << 15);
    // estimate in long double, then settle the exact nearest integer
    const long double t = (long double)d / (long double)n;
    const long double v = 32768.0L * (long double)n * t * t * t * t * (5.0L - 6.0L * t + 2.0L * t * t);
    int64_t q = (int64_t)std::llround(v);
    const u128 d2 = (u128)d * d;
    const u128 u = (u128)5 * n * n - (u128)6 * d * n + (u128)2 * d * d;   // in [N^2, 5N^2]
    const U256 x = shl(mul_u128(u256(d2 * d2), u), 16);                    // 2 * num
    const U256 den = mul_u64(u256((u128)n * n * n * n), n);                // N^5
    for (int it = 0; it < 4; ++it) {
        // q is nint(x / 2den) iff (2q-1) den <= x <= (2q+1) den, ties to even
        const U256 hi = mul_u64(den, (uint64_t)(2 * q + 1));
        const int c_hi = cmp(x, hi);
        if (c_hi > 0 || (c_hi == 0 && (q & 1))) { q += 1; continue; }
        if (q > 0) {
            const U256 lo = mul_u64(den, (uint64_t)(2 * q - 1));
            const int c_lo = cmp(x, lo);
            if (c_lo < 0 || (c_lo == 0 && (q & 1))) { q -= 1; continue; }
        }
        return q;
    }
    return q;   // not reached for valid inputs: the estimate is within 2^-13
}

// Raised-cosine table entry: 2^15 d - nint(((32768 N) / pi) * sin((pi d) / N)),
// evaluated in FP64 in exactly this order with the C library's sin.
int64_t cosine_entry(uint64_t n, uint64_t d)
{
    const double s = std::sin((M_PI * (double)d) / (double)n);
    const double x = ((32768.0 * (double)n) / M_PI) * s;
    return (int64_t)(d << 15) - (int64_t)std::nearbyint(x);
}

// Chirp term at the end of the window, floor(R N^2 / 2) or floor(dF H_N[N] / 2^16).
uint64_t chirp_end_term(int32_t shape, int64_t coef, int64_t dF, uint64_t n)
{
    (void)dF;
    if (shape == AWG_RAMP_LINEAR) {
        const i128 p = (i128)coef * (i128)(n * n);
        return (uint64_t)(p >> 1);
    }
    const int64_t h = shape == AWG_RAMP_MINJERK ? minjerk_entry(n, n) : cosine_entry(n, n);
    const i128 p = (i128)coef * (i128)h;
    return (uint64_t)(p >> kTableShift);
}

ToneDev to_device(const ToneHost &t, uint16_t table)
{
    ToneDev d;
    d.p0 = t.p0 + kPhaseBias;
    d.f0 = t.f0;
    d.p1 = t.p1 + kPhaseBias;
    d.f1 = t.f1;
    d.a = t.a;
    d.n = (uint32_t)t.n;
    d.coef = t.coef;
    d.amp = (float)t.amp;
    d.shape = (uint16_t)t.shape;
    d.table = table;
    d.ashape = (uint16_t)t.ashape;
    d.pad = 0;
    d.b = t.ashape == AWG_RAMP_NONE ? UINT64_MAX : t.b;
    d.m = t.ashape == AWG_RAMP_NONE ? 0u : (uint32_t)t.m;
    d.amp1 = t.ashape == AWG_RAMP_NONE ? d.amp : (float)t.amp1;
    d.lo = UINT64_MAX;
    d.hi = 0;
    if (t.shape != AWG_RAMP_NONE) { d.lo = t.a; d.hi = t.a + t.n; }
    if (t.ashape != AWG_RAMP_NONE) { d.lo = std::min(d.lo, t.b); d.hi = std::max(d.hi, t.b + t.m); }
    return d;
}

// Block table (see Block): maximal runs of tones with equal shape, window,
// table and amplitude window (not crossing n_split) of at least kMinRun tones
// become uniform blocks, ceil(L / kBlock) of them rounded up to a multiple of
// kWaves and sized within one tone of each other; shorter runs are packed into
// mixed blocks of up to kBlock tones that share their flags (split, amplitude).
void build_blocks(const std::vector<ToneDev> &tones, int32_t n_split, std::vector<Block> *out)
{
    build_blocks_by((int32_t)tones.size(), n_split, [&](int32_t i) -> const ToneDev & { return tones[i]; }, out);
}

}  // namespace awg
