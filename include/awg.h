/*
 * awg.h -- C ABI of the MI355X multi-tone additive-synthesis library.
 *
 * The library computes the discretised multi-tone waveform of the paper's
 * Theory section,
 *
 *     V[n] = Q( sum_k A_k sin(phi_k(n)) ),                     Eqs. (2), (5)-(7)
 *
 * for static tones (phi_k(n) = theta_k + 2 pi f_k n / fs, frequencies snapped to
 * the bins of a period L when one is given, Eq. (4)) and for chirped tones whose
 * frequency follows a linear, raised-cosine or minimum-jerk trajectory inside a
 * ramp window and is constant outside it (Eq. (8)). Q scales by a gain G (LSB
 * per unit amplitude), rounds half-to-even and saturates to int16 DAC codes.
 *
 * Phases are exact 64-bit fixed-point words (one turn = 2^64); the sinusoid and
 * the sum over tones run in FP32 on the GPU, or on the matrix cores by angle
 * addition with FP16 or BF16 hi/lo split operands and FP32 accumulation (static
 * tones, and the tones of a ramped plan that are on a line over a row).
 *
 * Conventions for every call:
 *  - All functions return an awg_status; none aborts and no C++ exception
 *    crosses this boundary.
 *  - "d_" pointers are device pointers on the context's device, owned by the
 *    caller; all other pointers are host pointers, owned by the caller. The
 *    synthesis calls check their output buffers first: AWG_E_INVALID for host
 *    memory, memory of another device, or a range that runs past the end of
 *    the allocation it starts in (when the runtime reports that allocation).
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream). Synthesis
 *    calls only enqueue work; results are valid once the stream has synchronised.
 *  - A plan may be used from several threads for awg_synth_* calls (they only
 *    read it); awg_stream_* and awg_plan_retune need one caller at a time.
 *  - awg_synth_static and awg_synth_chirp with the direct method, and
 *    awg_synth_static with a matrix-core method once the same call has run
 *    outside capture (which sets up the plan's workspace), may be captured into
 *    a HIP graph: they enqueue kernels and event records/waits only (no memset,
 *    no allocation). A replay uses the plan's workspace as the captured call
 *    did, so it must not overlap other matrix-core calls on the same plan.
 */
#ifndef AWG_H
#define AWG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct awg_ctx awg_ctx;     /* one HIP device */
typedef struct awg_plan awg_plan;   /* one tone set with its device tables */

typedef enum {
    AWG_OK = 0,
    AWG_E_INVALID = -1,      /* bad argument (null pointer, NaN, f outside (0, fs/2), ...) */
    AWG_E_NOMEM = -2,        /* host or device allocation failed */
    AWG_E_HIP = -3,          /* a HIP runtime call failed (also: no device) */
    AWG_E_RANGE = -4,        /* sample range overflow, bin on 0 or L/2, ramp too long */
    AWG_E_UNSUPPORTED = -5,  /* valid request the chosen call does not handle */
    AWG_E_BUSY = -6          /* resource temporarily exhausted (server admission) */
} awg_status;

/* Frequency trajectory inside a ramp window of N samples, tau = d / N in [0, 1]:
 *   LINEAR  f = f0 + df * tau
 *   COSINE  f = f0 + df * (1 - cos(pi tau)) / 2
 *   MINJERK f = f0 + df * (10 tau^3 - 15 tau^4 + 6 tau^5)          (Eq. (8)) */
typedef enum {
    AWG_RAMP_NONE = 0,
    AWG_RAMP_LINEAR = 1,
    AWG_RAMP_COSINE = 2,
    AWG_RAMP_MINJERK = 3
} awg_ramp;

/* One tone (56 bytes). Static tones use f_start_hz only. A ramped tone is static
 * at f_start_hz before sample ramp_start, sweeps to f_end_hz over the window
 * [ramp_start, ramp_start + ramp_len], and holds f_end_hz afterwards with the
 * phase it reached (Eq. (8) cases 1-3). phase_turns is theta in turns. */
typedef struct {
    double f_start_hz;
    double f_end_hz;
    double amplitude;        /* A_k >= 0, in units of the gain */
    double phase_turns;      /* theta_k / (2 pi) */
    uint64_t ramp_start;     /* absolute sample index a */
    uint64_t ramp_len;       /* N, 1 <= N < 2^31 for ramped tones */
    int32_t ramp;            /* awg_ramp */
    int32_t reserved;        /* must be 0 */
} awg_tone;

/* Static-synthesis method, flags bits 0-1. */
#define AWG_F_METHOD_DIRECT      0u   /* VALU: exact phase word, v_sin, FP32 FMA sum */
#define AWG_F_METHOD_MFMA_F16X3  1u   /* matrix cores: angle addition, FP16 hi/lo x3 */
#define AWG_F_METHOD_MFMA_BF16X3 2u   /* matrix cores: angle addition, BF16 hi/lo x3 */
#define AWG_F_METHOD_MASK        3u

typedef struct {
    double fs_hz;            /* sample rate, > 0 */
    double gain_lsb;         /* G in LSB per unit amplitude; 0 = 32767 / sum A_k (never clips) */
    uint32_t period_log2;    /* p > 0: snap every frequency to a bin of L = 2^p (Eq. (4)); 0: none */
    uint32_t flags;          /* AWG_F_METHOD_* */
} awg_plan_params;

typedef struct {
    int32_t n_tones;
    int32_t n_ramped;        /* tones with a ramp window */
    double gain_lsb;         /* the gain in use */
    uint32_t flags;
    uint32_t period_log2;
    uint64_t cursor;         /* next sample of awg_stream_next */
    uint64_t device_bytes;   /* device memory held by the plan (tables, workspaces) */
} awg_plan_info;

/* A new chirp appended to one tone of a plan (retuning a running stream). The
 * tone leaves the line it is on at sample ramp_start (which must not precede
 * the end of its previous window) and sweeps to f_end_hz over ramp_len samples. */
typedef struct {
    int32_t tone;
    int32_t ramp;            /* AWG_RAMP_LINEAR / COSINE / MINJERK */
    uint64_t ramp_start;
    uint64_t ramp_len;
    double f_end_hz;
} awg_retune;

/* ---------------------------------------------------------------- context */

/* Binds HIP device `device`. Fails with AWG_E_HIP when there is no such device.
 * The context owns the smooth ramp tables H_N of its plans and server jobs: one
 * device table per distinct (shape, N), (N + 1) x 8 bytes, shared by every plan
 * that uses it and kept until awg_ctx_destroy (a long-lived context that sees
 * many distinct smooth ramp lengths holds all of their tables). */
awg_status awg_ctx_create(int device, awg_ctx **out);
void awg_ctx_destroy(awg_ctx *ctx);

/* ------------------------------------------------------------------- plan */

/* Plan a tone set (initialisation state of the Software section: all
 * parameters are converted and uploaded once, no per-call host traffic).
 *
 * Per tone: frequency words F = nint(f 2^64 / fs), or with period_log2 = p the
 * bin j = nint(f L / fs) (Eq. (4)) and F = j 2^(64-p); phase word
 * P = nint(theta 2^64) mod 2^64; for ramps the chirp coefficient (linear:
 * R = nint((F1-F0)/N); smooth: dF = F1-F0 and the shared table
 * H_N[d] = nint(2^16 N Psi(d/N))) and the line after the window. All rounding
 * is half-to-even and exact (no floating-point shortcuts).
 *
 * ctx may be NULL: the plan is then host-only (words and tables only, for
 * inspection with awg_plan_words); synthesis calls on it return AWG_E_INVALID.
 * f_quantised_hz (nullable, n_tones entries) receives F * fs / 2^64 per tone.
 * Errors: AWG_E_INVALID for null tones/out/params, n_tones <= 0, fs not finite
 * and > 0, gain < 0 or not finite, non-finite tone fields, amplitude < 0,
 * unknown ramp, reserved != 0, period_log2 == 1 or > 63, f not in (0, fs/2),
 * all amplitudes 0 with gain 0; AWG_E_RANGE for a bin on 0 or L/2, ramp_len 0 or
 * >= 2^31, ramp_start + ramp_len >= 2^63; AWG_E_UNSUPPORTED when the smooth
 * ramps need more than 1024 distinct tables (shape, length) in one plan;
 * AWG_E_NOMEM / AWG_E_HIP on upload. */
awg_status awg_plan_tones(awg_ctx *ctx, const awg_plan_params *params, const awg_tone *tones,
                          int32_t n_tones, awg_plan **out, double *f_quantised_hz);
void awg_plan_destroy(awg_plan *plan);
awg_status awg_plan_info_get(const awg_plan *plan, awg_plan_info *info);

/* Words of every tone (host arrays of n_tones entries, each nullable): initial
 * phase P0, start and end frequency words F0, F1, and the chirp coefficient (R
 * for linear ramps, dF for smooth ones, 0 for static tones). After retuning
 * these describe the most recent ramp of each tone (P0 = line before it). */
awg_status awg_plan_words(const awg_plan *plan, uint64_t *p0, uint64_t *f0, uint64_t *f1,
                          int64_t *coef);

/* H_N[0..N] of a smooth ramp shape into out (host, N+1 entries): minimum jerk
 * exactly nint(2^15 d^4 (5N^2 - 6dN + 2d^2) / N^5); raised cosine
 * 2^15 d - nint(((32768 N) / pi) * sin((pi d) / N)) in FP64 in that order.
 * AWG_E_INVALID for other shapes, AWG_E_RANGE for N = 0 or N >= 2^31. */
awg_status awg_ramp_table(int32_t shape, uint64_t n, uint64_t *out);

/* Append chirps to tones of a planned stream (Streaming pathway with groups of
 * tones chirped in turn). The device tables are updated in stream order on
 * hip_stream: synthesis enqueued earlier on that stream sees the old tones,
 * synthesis enqueued later the new ones. (A plan that has run on the periodic
 * line buffer, a ramped plan on bins with a matrix-core method, stages the
 * update and leaves it to the next call that reads its tones, which applies it
 * first on that call's stream.) A tone keeps one window on the device,
 * so after a retune its samples are exact from the end of its previous window
 * on (the new window must not start earlier); samples before that end are no
 * longer reproducible from this plan. At most one event per tone per call.
 * AWG_E_INVALID for a bad tone index or shape, AWG_E_RANGE for a window that
 * starts before the tone's previous window ends or is too long,
 * AWG_E_UNSUPPORTED for two events on one tone, more than 16384 events, or a
 * plan that would need more than 1024 distinct smooth tables. */
awg_status awg_plan_retune(awg_plan *plan, const awg_retune *events, int32_t n_events,
                           void *hip_stream);

/* An amplitude ramp of one tone (the time-dependent amplitude a_j[i] of Eq. (5);
 * switching a tone off is a ramp to 0, switching one on a ramp up from a tone
 * planned with amplitude 0). Over the window [ramp_start, ramp_start + ramp_len]
 * the tone's amplitude moves from the value it holds (its planned amplitude, or
 * the end of its previous amplitude ramp) to amplitude_end:
 *   a(n) = a0 (1 - s) + a1 s,   s = profile((n - ramp_start) / ramp_len),
 * with profile linear t, raised cosine (1 - cos(pi t)) / 2 or minimum jerk
 * 10 t^3 - 15 t^4 + 6 t^5; a0 before the window, a1 after it. */
typedef struct {
    int32_t tone;
    int32_t ramp;            /* AWG_RAMP_LINEAR / COSINE / MINJERK: the profile */
    uint64_t ramp_start;
    uint64_t ramp_len;       /* 1 <= ramp_len < 2^31 */
    double amplitude_end;    /* >= 0, in the units of awg_tone.amplitude (scaled by the plan's gain) */
} awg_amp_ramp;

/* Append amplitude ramps to tones of a plan, in stream order on hip_stream like
 * awg_plan_retune (frequency windows and amplitude windows of a tone are
 * independent). A tone keeps one amplitude window on the device; a new one must
 * not start before the previous one ends. At most one event per tone per call.
 * The caller keeps the sum within int16 (the gain is fixed at planning).
 * AWG_E_INVALID for a bad tone, profile or amplitude, AWG_E_RANGE for a window
 * that starts too early or is too long, AWG_E_UNSUPPORTED for two events on one
 * tone or more than 16384 events. */
awg_status awg_plan_amplitude(awg_plan *plan, const awg_amp_ramp *events, int32_t n_events,
                              void *hip_stream);

/* -------------------------------------------------------------- synthesis */

/* Static pathway: samples n0 .. n0+count-1 of a plan without ramp windows into
 * d_out (int16, count entries). The method comes from the plan's flags.
 * The direct method gives each sample independently of the range. The MFMA
 * methods cut the range into rows from n0 and, for requests with few output
 * tiles, split the tone sum into slices added in a fixed order afterwards: the
 * codes depend on (n0, count) within the same error bar, and equal calls give
 * equal samples. They take a long range in pieces of 2^28 samples, which bounds
 * their per-call workspace.
 * AWG_E_UNSUPPORTED if the plan has ramps; AWG_E_RANGE if n0 + count >= 2^63. */
awg_status awg_synth_static(awg_plan *plan, uint64_t n0, uint64_t count, int16_t *d_out,
                            void *hip_stream);

/* Playback pathway: any sample range of any plan (static or chirped) with the
 * plan's method. count = 0 is a no-op.
 *  - AWG_F_METHOD_DIRECT: the direct kernel.
 *  - An MFMA method on a static plan: as awg_synth_static.
 *  - An MFMA method on a ramped plan, count >= 65536: the hybrid path.
 *    The range is cut into rows of 1024 samples from n0. On each row, the tones
 *    whose window [a, a+N] misses the row are on a straight phase line before or
 *    after the window. Those (tone, row) pairs are summed by angle addition on the
 *    matrix cores; the ramping pairs go to the direct kernel, which adds the two
 *    sums and rounds. This is the static-buffer plus dynamic-part split of
 *    Eqs. (5)-(7), taken per row from exact words. Same error bar as the
 *    static MFMA method. The result depends on (n0, count) through the row grid:
 *    equal calls give equal samples.
 *  - An MFMA method on a ramped plan, count < 65536: the direct kernel.
 * Retune and synthesise on one stream: the hybrid path reads the tones'
 * windows on the host when the call is made. */
awg_status awg_synth_chirp(awg_plan *plan, uint64_t n0, uint64_t count, int16_t *d_out,
                           void *hip_stream);

/* Set-up ahead of a stream (for real-time callers): allocates now what the
 * calls below would otherwise allocate on first use, so that the first chunk
 * does not pay for it: the retune and amplitude staging slots (16 pinned
 * buffers), and for an MFMA method and requests of up to max_count samples the
 * plan's product workspace and, on a plan with ramps, the hybrid path's
 * workspace and staging slots. Later calls reuse them (a plan retuned from
 * static to ramped after this call sets up the hybrid path on its first call).
 * AWG_E_INVALID for a host-only plan or an unknown method; AWG_E_NOMEM /
 * AWG_E_HIP when an allocation fails. */
awg_status awg_plan_reserve(awg_plan *plan, uint32_t method, uint64_t max_count);

/* Streaming pathway: the next count samples after the plan's cursor into d_out,
 * then advance the cursor. *n0_out (nullable) receives the first sample index.
 * Results are bit-identical to awg_synth_chirp over the same range: the phase is
 * a closed form in the absolute sample index and the sum order depends on the
 * plan only. With the direct method, any split of a range into consecutive
 * calls also gives bit-identical samples; with the hybrid path, only the same
 * (n0, count) does. */
awg_status awg_stream_next(awg_plan *plan, uint64_t count, int16_t *d_out, void *hip_stream,
                           uint64_t *n0_out);
/* Cursor access for checkpoint / resume: (plan inputs, cursor) restore a stream. */
awg_status awg_stream_seek(awg_plan *plan, uint64_t n0);
awg_status awg_stream_tell(const awg_plan *plan, uint64_t *n0);

/* Unquantised sum y[n] (FP32, LSB units) for error reporting: the same kernels
 * as the int16 calls with the rounding left out. method: AWG_F_METHOD_*,
 * overriding the plan's (an MFMA method on a ramped plan takes the hybrid path,
 * as in awg_synth_chirp). */
awg_status awg_synth_f32(awg_plan *plan, uint32_t method, uint64_t n0, uint64_t count,
                         float *d_y, void *hip_stream);

/* Multiplexed output for a multi-channel DAC (the paper's wavetable
 * multiplexer, fused into synthesis as in its Streaming pathway): samples
 * n0 .. n0+count-1 of plans[0 .. n_channels-1] (1 <= n_channels <= 4) written
 * interleaved into d_out, channel c's sample n0 + i at d_out[n_channels * i + c]
 * (d_out holds n_channels * count int16). Every channel runs the direct kernel,
 * so its codes are bit-identical to awg_synth_chirp of that plan with the direct
 * method; one launch covers all channels. A plan may appear more than once.
 * AWG_E_INVALID for a bad channel count, a NULL or host-only plan, or plans of
 * different devices; AWG_E_RANGE as awg_synth_chirp. */
awg_status awg_synth_multiplex(awg_plan *const *plans, int32_t n_channels, uint64_t n0, uint64_t count,
                               int16_t *d_out, void *hip_stream);
/* Streaming form: the next count samples of every channel after their common
 * cursor (all plans' cursors must be equal, else AWG_E_INVALID), multiplexed as
 * above; then every plan's cursor advances by count. */
awg_status awg_stream_next_multiplex(awg_plan *const *plans, int32_t n_channels, uint64_t count,
                                     int16_t *d_out, void *hip_stream, uint64_t *n0_out);

/* ----------------------------------------------------- crest-factor control */

/* Tone phases set the peak (crest) factor of the static waveform (Theory
 * section: large crest factors mean rf power spikes that can damage the AOD;
 * the paper cites Schroeder 1970 without a formula). awg_phase_plan returns
 * closed-form phases, tones ranked by frequency k = 1..K (equal frequencies in
 * input order), in turns in [0, 1), ready for awg_tone.phase_turns:
 *   AWG_PHASES_SCHROEDER  theta_k = -2 pi sum_{l<k} (k - l) p_l,
 *                         p_l = A_l^2 / sum A^2 (equal amplitudes: -pi k (k-1) / K)
 *   AWG_PHASES_NEWMAN     theta_k = pi (k - 1)^2 / K (amplitude may be NULL)
 * Host only. AWG_E_INVALID for n <= 0, NULL arrays, non-finite values, negative
 * or all-zero amplitudes (Schroeder). */
#define AWG_PHASES_SCHROEDER 1
#define AWG_PHASES_NEWMAN    2
#define AWG_PHASES_SEARCH    3   /* awg_phase_search only: phases found by the device search */
awg_status awg_phase_plan(int32_t method, const double *f_hz, const double *amplitude, int32_t n_tones,
                          double *phase_turns_out);

/* Crest-factor-aware phase planning on ctx's device, for tones on bins of the
 * period L = 2^period_log2 (14 <= period_log2 <= 26; f as in awg_plan_tones
 * with that period). Measures both closed forms above over one period, then
 * (max_evals > 0) lowers the crest factor further by minimising the l_p norm
 * of the period's samples, p = 8, 16, ..., 256, each stage by L-BFGS from the
 * previous one (Guillaume et al. 1991, a Chebyshev approximation of the peak;
 * max_evals bounds the evaluations, each one synthesis of the period plus one
 * gradient correlation of every tone over it). Returns the phases (turns in
 * [0, 1), input order) with the lowest crest factor found, which is
 * max|y| / sqrt(sum A^2 / 2) over one period of y = sum A_k sin(2 pi b_k n / L
 * + 2 pi phase_k) measured on the device for the phase words a plan makes of
 * the returned turns (*crest_out, nullable), and which method gave them
 * (*method_out, nullable: AWG_PHASES_*). Distinct bins are the caller's
 * business (the crest factor assumes them). Allocates device memory for the
 * period (4 L bytes) and partial sums (n_tones L / 4096 bytes), freed before
 * returning. AWG_E_INVALID for null pointers, n_tones <= 0, max_evals < 0,
 * bad fs, negative or all-zero amplitudes, f outside (0, fs/2);
 * AWG_E_RANGE for a bin on 0 or L/2; AWG_E_UNSUPPORTED for a period outside
 * [2^14, 2^26] or more than 2^20 tones (or partial sums above 1 GiB). */
awg_status awg_phase_search(awg_ctx *ctx, double fs_hz, uint32_t period_log2, const double *f_hz,
                            const double *amplitude, int32_t n_tones, int32_t max_evals, double *phase_turns_out,
                            double *crest_out, int32_t *method_out);

/* Peak |y| of a plan's unquantised sum over samples n0 .. n0+count-1, in LSB:
 * the direct kernel writes y (FP32) into d_scratch (device, count floats,
 * caller-owned), then a device max reduction writes the peak to *d_peak
 * (device, one float), both on hip_stream. With one full period of a plan whose
 * tones sit on distinct bins, peak / (G sqrt(sum A^2 / 2)) is its crest factor.
 * AWG_E_INVALID for NULL pointers or count = 0; AWG_E_RANGE as awg_synth_chirp. */
awg_status awg_peak(awg_plan *plan, uint64_t n0, uint64_t count, float *d_scratch, float *d_peak,
                    void *hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): awg_peak without the caller's
 * scratch. The FP32 samples go to a scratch array the library keeps in device
 * memory, one per device (AWG_PEAK_NOALLOC_MAX floats = 16 MiB, held until the
 * process ends; its address is looked up when a context is created). The call
 * enqueues the same kernels as awg_peak, so *d_peak is bit-identical to it, and
 * it calls no allocating routine: no hipMalloc/hipFree, no profiler events
 * (its launches are never timed by awg_profile_*). Calls on one device share
 * that array and each overwrites it, so calls that may overlap on one device
 * (two streams, two threads) race: serialise them. AWG_E_UNSUPPORTED for
 * count > AWG_PEAK_NOALLOC_MAX; otherwise errors as awg_peak. */
#define AWG_PEAK_NOALLOC_MAX (1u << 22)
awg_status awg_peak_noalloc(awg_plan *plan, uint64_t n0, uint64_t count, float *d_peak, void *hip_stream);


/* Phase words of one tone as the direct kernel generates them (same code path,
 * same sample-to-lane mapping), for exact comparison: d_words[i] = phi(n0 + i). */
awg_status awg_phase_dump(awg_plan *plan, int32_t tone, uint64_t n0, uint64_t count,
                          uint64_t *d_words, void *hip_stream);

/* ---------------------------------------------------------------- serving */

/* Continuous batching of synthesis jobs on one device. A job is one tone set
 * with its own sample rate and length (e.g. a tweezer rearrangement: every tone
 * chirps across the job). Jobs are admitted in arrival order as job slots and
 * device memory free up; every step takes one chunk from each admitted job that
 * has samples left and a free slot in the device output ring, and runs all of
 * them in one launch (a replayed hipGraph of the batched kernel). A job's
 * samples are bit-identical to awg_synth_chirp of the same tones, whatever it
 * is batched with. The consumer (the DAC's stand-in) polls chunk events, reads
 * the ring slot and releases it. */
typedef struct awg_server awg_server;

typedef struct {
    uint64_t mem_budget_bytes;   /* device memory for the ring and the jobs' tone tables */
    int32_t max_jobs;            /* jobs admitted at once (also the largest batch) */
    int32_t ring_slots;          /* output chunk slots in the device ring */
    uint32_t chunk_len;          /* samples per chunk, a multiple of 1024 */
    int32_t max_pending;         /* submitted jobs waiting for admission */
    double playout_delay_ms;     /* chunk c of a job is due at submit + delay + c * chunk_len / fs */
} awg_server_params;

typedef struct {
    double fs_hz;
    double gain_lsb;             /* as in awg_plan_params */
    uint32_t period_log2;
    uint32_t reserved;           /* must be 0 */
    const awg_tone *tones;       /* host, n_tones entries, read during the call */
    int32_t n_tones;
    int32_t reserved2;           /* must be 0 */
    uint64_t n_samples;          /* job length: samples 0 .. n_samples-1 */
    uint64_t user_tag;
} awg_job;

typedef struct {
    uint64_t job_id, user_tag;
    uint64_t chunk_index;
    uint64_t n0, count;          /* samples n0 .. n0+count-1 of the job */
    int32_t slot;                /* ring slot holding them (awg_server_slot) */
    int32_t last;                /* 1 on the job's final chunk */
    double t_submit_ms, t_ready_ms;   /* host steady clock */
} awg_chunk_event;

typedef struct {
    uint64_t jobs_submitted, jobs_admitted, jobs_done, jobs_pending, jobs_active;
    uint64_t chunks_done, steps, max_batch;
    double mean_batch;
    double tone_samples;             /* synthesised tone-samples */
    double audio_seconds;            /* synthesised output duration, sum over jobs */
    double device_busy_ms;           /* device time of all steps */
    double wall_ms;                  /* first submit to last chunk ready */
    /* percentiles cover the most recent 1,048,576 chunks */
    double chunk_latency_p50_ms, chunk_latency_p99_ms;            /* chunk ready - job submit */
    double first_chunk_latency_p50_ms, first_chunk_latency_p99_ms;
    uint64_t deadline_misses;        /* chunks ready after submit + delay + n0 / fs */
    uint64_t pool_free_bytes;
    double lateness_p50_ms, lateness_p99_ms;  /* chunk ready - (submit + delay + n0 / fs);
                                                 negative: ready before it is due */
} awg_server_stats;

/* Start a server (and its scheduler thread) on ctx's device. AWG_E_INVALID for
 * bad parameters, AWG_E_RANGE if the budget cannot hold the ring. */
awg_status awg_server_create(awg_ctx *ctx, const awg_server_params *params, awg_server **out);
/* Stop the scheduler, wait for running steps and free everything. */
awg_status awg_server_destroy(awg_server *srv);
/* Queue a job. The words are planned here (errors as awg_plan_tones);
 * AWG_E_BUSY when max_pending jobs already wait, AWG_E_NOMEM when the job's
 * tables can never fit the budget. */
awg_status awg_server_submit(awg_server *srv, const awg_job *job, uint64_t *job_id);
/* Completed chunks, oldest first (up to max_events into out, count in *n_events). */
awg_status awg_server_poll(awg_server *srv, awg_chunk_event *out, int32_t max_events, int32_t *n_events);
/* Device address of ring slot `slot` (chunk_len int16 samples). */
awg_status awg_server_slot(awg_server *srv, int32_t slot, int16_t **d_ptr);
/* Copy the first count samples of a ready slot (one the consumer holds) to dst,
 * host or device memory; returns when the copy is done. */
awg_status awg_server_read(awg_server *srv, int32_t slot, uint64_t count, int16_t *dst);
/* Hand a slot back after its chunk has been consumed. */
awg_status awg_server_release(awg_server *srv, int32_t slot);
awg_status awg_server_stats_get(awg_server *srv, awg_server_stats *stats);

/* -------------------------------------------------------------- profiling */

/* Per-kernel device time, measured with HIP events recorded on the launch
 * stream immediately before and after each kernel of the context's calls. */
typedef struct {
    char name[48];           /* kernel name */
    uint64_t launches;
    double total_ms;
    double max_ms;
    double work;             /* algorithmic tone-samples of the timed launches: tones x samples
                                summed (direct kernels), line tones x the samples of the rows
                                they cover (angle-addition products); 0 for helper kernels */
} awg_kernel_stat;

/* Event timing of the kernels of all calls on plans of ctx (off by default):
 * enable = 0 switches it off; enable = n >= 1 times one launch in n of each
 * kernel (the 1st, n+1-th, ... since this call; 1 = every launch). A timed
 * launch costs the stream some microseconds (the dispatch records its start
 * and stop events), so sampling keeps the overhead of a long run small. At
 * most 65,536 timed launches are held until the next awg_profile_read; later
 * ones run untimed. AWG_E_INVALID for enable < 0. */
awg_status awg_profile_enable(awg_ctx *ctx, int32_t enable);
/* Synchronise the recorded events and return up to max_stats per-kernel totals
 * in out (host array); *n_stats receives the number of distinct kernels. With
 * reset != 0 the totals start over. */
awg_status awg_profile_read(awg_ctx *ctx, awg_kernel_stat *out, int32_t max_stats, int32_t *n_stats,
                            int32_t reset);

/* ------------------------------------------------------------------- misc */

const char *awg_strerror(awg_status status);
/* Library version, major * 10000 + minor * 100 + patch. */
int32_t awg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AWG_H */
