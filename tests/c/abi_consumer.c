/* A plain C99 consumer of libawg: it uses only include/awg.h and the HIP
 * runtime's C API (device memory, copies), no Python and no C++.
 *
 *   abi_consumer OUT_FILE
 *
 * Plans 64 static tones on bins of L = 2^16 at 280 MS/s, then
 *  - synthesises samples n0 .. n0+count-1 in one call (direct method);
 *  - streams the same range in three calls and requires the same codes;
 *  - synthesises it again with BF16 hi/lo x3 on the matrix cores and
 *    requires codes within 2 of the direct ones (each is within 1 of the
 *    exact sum);
 *  - checks two error returns.
 * OUT_FILE receives the tone parameters and the direct codes, which the
 * calling test compares with the oracle. Exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "awg.h"

#define N_TONES 64
#define N0 5u
#define COUNT 70000u

static int fail(const char *what, int code)
{
    fprintf(stderr, "abi_consumer: %s failed (%d)\n", what, code);
    return 1;
}

static int plan(awg_ctx *ctx, const awg_tone *tones, uint32_t method, awg_plan **out)
{
    awg_plan_params pp;
    memset(&pp, 0, sizeof pp);
    pp.fs_hz = 280e6;
    pp.gain_lsb = 0.0;
    pp.period_log2 = 16;
    pp.flags = method;
    return awg_plan_tones(ctx, &pp, tones, N_TONES, out, NULL);
}

int main(int argc, char **argv)
{
    if (argc != 2) {
        fprintf(stderr, "usage: abi_consumer OUT_FILE\n");
        return 2;
    }
    awg_tone tones[N_TONES];
    memset(tones, 0, sizeof tones);
    for (int k = 0; k < N_TONES; ++k) {
        const double bin = 1000.0 + 373.0 * k;               /* distinct bins below L/2 */
        tones[k].f_start_hz = bin * 280e6 / 65536.0;
        tones[k].f_end_hz = tones[k].f_start_hz;
        tones[k].amplitude = 0.5 + (double)(k % 7) / 14.0;
        tones[k].phase_turns = (double)k / N_TONES;
        tones[k].ramp = AWG_RAMP_NONE;
    }
    awg_ctx *ctx = NULL;
    awg_plan *pd = NULL, *pm = NULL;
    int st = awg_ctx_create(0, &ctx);
    if (st != AWG_OK) return fail("awg_ctx_create", st);
    if ((st = plan(ctx, tones, AWG_F_METHOD_DIRECT, &pd)) != AWG_OK) return fail("awg_plan_tones direct", st);
    if ((st = plan(ctx, tones, AWG_F_METHOD_MFMA_BF16X3, &pm)) != AWG_OK) return fail("awg_plan_tones bf16", st);

    const size_t bytes = COUNT * sizeof(int16_t);
    int16_t *d_one = NULL, *d_str = NULL, *d_mat = NULL;
    if (hipMalloc((void **)&d_one, bytes) != hipSuccess || hipMalloc((void **)&d_str, bytes) != hipSuccess ||
        hipMalloc((void **)&d_mat, bytes) != hipSuccess)
        return fail("hipMalloc", -1);

    if ((st = awg_synth_static(pd, N0, COUNT, d_one, NULL)) != AWG_OK) return fail("awg_synth_static", st);
    if ((st = awg_stream_seek(pd, N0)) != AWG_OK) return fail("awg_stream_seek", st);
    const uint64_t parts[3] = {30000u, 25000u, COUNT - 55000u};
    uint64_t at = 0;
    for (int i = 0; i < 3; ++i) {
        uint64_t n0 = 0;
        if ((st = awg_stream_next(pd, parts[i], d_str + at, NULL, &n0)) != AWG_OK) return fail("awg_stream_next", st);
        if (n0 != N0 + at) return fail("awg_stream_next first sample", (int)n0);
        at += parts[i];
    }
    if ((st = awg_synth_static(pm, N0, COUNT, d_mat, NULL)) != AWG_OK) return fail("awg_synth_static bf16", st);
    if (hipDeviceSynchronize() != hipSuccess) return fail("hipDeviceSynchronize", -1);

    int16_t *one = malloc(bytes), *str = malloc(bytes), *mat = malloc(bytes);
    if (!one || !str || !mat) return fail("malloc", -1);
    if (hipMemcpy(one, d_one, bytes, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(str, d_str, bytes, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(mat, d_mat, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return fail("hipMemcpy", -1);
    if (memcmp(one, str, bytes) != 0) return fail("streamed == one-shot", -1);
    int dmax = 0;
    for (uint32_t i = 0; i < COUNT; ++i) {
        const int d = abs((int)one[i] - (int)mat[i]);
        if (d > dmax) dmax = d;
    }
    if (dmax > 2) return fail("matrix-core codes within 2 of direct", dmax);

    /* error returns: a range past the last sample, a NULL output */
    if ((st = awg_synth_static(pd, UINT64_MAX - 10, 100, d_one, NULL)) != AWG_E_RANGE) return fail("range error", st);
    if ((st = awg_synth_static(pd, 0, 100, NULL, NULL)) != AWG_E_INVALID) return fail("null output", st);

    FILE *f = fopen(argv[1], "wb");
    if (!f) return fail("fopen", -1);
    const uint32_t hdr[3] = {N_TONES, N0, COUNT};
    int ok = fwrite(hdr, sizeof hdr, 1, f) == 1 && fwrite(tones, sizeof tones, 1, f) == 1 &&
             fwrite(one, bytes, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail("write", -1);

    (void)hipFree(d_one);
    (void)hipFree(d_str);
    (void)hipFree(d_mat);
    free(one);
    free(str);
    free(mat);
    awg_plan_destroy(pm);
    awg_plan_destroy(pd);
    awg_ctx_destroy(ctx);
    printf("abi_consumer: %d tones x %u samples; streamed == one-shot; max |bf16 - direct| = %d\n", N_TONES,
           COUNT, dmax);
    return 0;
}
