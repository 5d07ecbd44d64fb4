/*
 * FP64 direct sum of a multi-tone waveform: the oracle's bulk evaluator.
 *
 * TEST INFRASTRUCTURE. Plain C99 + OpenMP, built with gcc and
 * -ffp-contract=off. It receives the exact words computed by oracle/words.py and
 * evaluates, for every sample n and every tone k in ascending order,
 *
 *     y[n] = sum_k a_k(n) * sin(2*pi * phi_k(n) / 2^64)         (Eqs. (2), (5))
 *     q[n] = saturate_int16(round_half_even(y[n]))               (Q of Eq. (2))
 *
 * where phi_k(n) is the piecewise phase law of Eq. (8), evaluated from its
 * closed form at every sample (no recurrences, no blocking): before a ramp
 * window the tone is the line p + f*n; inside [a, a+N] the line plus the chirp
 * term; after it the line p_after + f_after*n. a_k(n) is the tone's amplitude
 * A_k G, or, inside an amplitude ramp [b, b+M], a_from (1 - s) + a_to s with
 * s the ramp's profile at (n - b) / M, and a_to after it (the a_j[i] of Eq. (5)).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

#define RAMP_LINEAR 1
#define RAMP_COSINE 2
#define RAMP_MINJERK 3

typedef struct {
    uint64_t a, n;               /* window [a, a+n] */
    uint64_t p_line, f_line;     /* line before the window */
    uint64_t p_after, f_after;   /* line after the window */
    int64_t coef;                /* linear: R; smooth: dF */
    const uint64_t *table;       /* smooth: H_N[0..n], entries < 2^47 */
    int32_t shape;
    int32_t pad;
} oracle_ramp;

typedef struct {
    uint64_t b, m;               /* amplitude window [b, b+m] */
    double a_from, a_to;         /* amplitude (x G) at its start and end */
    int32_t shape;
    int32_t pad;
} oracle_amp;

typedef struct {
    uint64_t p0, f0;
    double amp;                  /* A_k * G */
    int32_t first_ramp, n_ramps; /* ramps[first_ramp .. first_ramp+n_ramps), time order */
    int32_t first_amp, n_amps;   /* amps[first_amp .. first_amp+n_amps), time order */
} oracle_tone;

/* Amplitude profile s(tau), s(0) = 0, s(1) = 1: linear, raised cosine, minimum jerk. */
static double amp_shape(int32_t shape, double tau)
{
    const double pi = 3.14159265358979323846;
    if (shape == RAMP_LINEAR) return tau;
    if (shape == RAMP_COSINE) return (1.0 - cos(pi * tau)) / 2.0;
    return tau * tau * tau * (10.0 - 15.0 * tau + 6.0 * tau * tau);
}

double oracle_amp_at(const oracle_tone *t, const oracle_amp *amps, uint64_t n)
{
    const oracle_amp *r = 0;
    for (int32_t i = 0; i < t->n_amps; ++i) {
        const oracle_amp *c = &amps[t->first_amp + i];
        if (c->b <= n) r = c; else break;
    }
    if (!r) return t->amp;
    uint64_t d = n - r->b;
    if (d > r->m) return r->a_to;
    double s = amp_shape(r->shape, (double)d / (double)r->m);
    return r->a_from * (1.0 - s) + r->a_to * s;
}

/* Chirp term d samples into the window. Linear: floor(R d^2 / 2); smooth:
 * floor(dF * H[d] / 2^16). Both products fit a signed 128-bit integer
 * (|R|, |dF| < 2^63, d < 2^31, H < 2^47); >> on a negative signed value is
 * an arithmetic (flooring) shift with gcc. */
static uint64_t chirp_term(const oracle_ramp *r, uint64_t d)
{
    __int128 prod;
    if (r->shape == RAMP_LINEAR) {
        prod = (__int128)r->coef * (__int128)(d * d);   /* d < 2^31 */
        return (uint64_t)(prod >> 1);
    }
    prod = (__int128)r->coef * (__int128)r->table[d];
    return (uint64_t)(prod >> 16);
}

uint64_t oracle_phase_at(const oracle_tone *t, const oracle_ramp *ramps, uint64_t n)
{
    const oracle_ramp *r = 0;
    for (int32_t i = 0; i < t->n_ramps; ++i) {
        const oracle_ramp *c = &ramps[t->first_ramp + i];
        if (c->a <= n) r = c; else break;
    }
    if (!r) return t->p0 + t->f0 * n;
    uint64_t d = n - r->a;
    if (d <= r->n) return r->p_line + r->f_line * n + chirp_term(r, d);
    return r->p_after + r->f_after * n;
}

/* Fills q[0..count) and y[0..count) for samples n0 .. n0+count-1. */
void oracle_synth(const oracle_tone *tones, int32_t n_tones, const oracle_ramp *ramps, const oracle_amp *amps,
                  uint64_t n0, int64_t count, int16_t *q, double *y, int32_t threads)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t n = n0 + (uint64_t)i;
        double acc = 0.0;
        for (int32_t k = 0; k < n_tones; ++k) {
            uint64_t w = oracle_phase_at(&tones[k], ramps, n);
            double turns = (double)(int64_t)w * 0x1p-64;
            acc += oracle_amp_at(&tones[k], amps, n) * sin(two_pi * turns);
        }
        double r = nearbyint(acc);
        if (r > 32767.0) r = 32767.0;
        if (r < -32768.0) r = -32768.0;
        y[i] = acc;
        q[i] = (int16_t)r;
    }
}

/* Phase words of one tone over a range (for exact word comparisons). */
void oracle_phases(const oracle_tone *t, const oracle_ramp *ramps, uint64_t n0, int64_t count,
                   uint64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) out[i] = oracle_phase_at(t, ramps, n0 + (uint64_t)i);
}

/* Same as oracle_synth at an arbitrary list of absolute sample indices. */
void oracle_synth_at(const oracle_tone *tones, int32_t n_tones, const oracle_ramp *ramps, const oracle_amp *amps,
                     const uint64_t *ns, int64_t count, int16_t *q, double *y, int32_t threads)
{
    const double two_pi = 2.0 * 3.14159265358979323846;
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        const uint64_t n = ns[i];
        double acc = 0.0;
        for (int32_t k = 0; k < n_tones; ++k) {
            uint64_t w = oracle_phase_at(&tones[k], ramps, n);
            double turns = (double)(int64_t)w * 0x1p-64;
            acc += oracle_amp_at(&tones[k], amps, n) * sin(two_pi * turns);
        }
        double r = nearbyint(acc);
        if (r > 32767.0) r = 32767.0;
        if (r < -32768.0) r = -32768.0;
        y[i] = acc;
        q[i] = (int16_t)r;
    }
}
