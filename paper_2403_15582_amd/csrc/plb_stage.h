// Staging of a line-buffer pass on the device (HIP sources only): descriptor
// records to synthesis records, the plain copy of the pass's raw part, and a
// retune's records to the plan's table, as grid-stride loops over threads
// tid .. of stride.
#pragma once
#include <hip/hip_runtime.h>

#include "awg_internal.h"

namespace awg {

// desc[i] for i in [0, n_desc) to dst_first[i] (i < n_first) or
// dst_rest[i - n_first]: a plan tone (src >= 0) or a static line, with the
// window rows [lo_row, hi_row] from n0 (lo_row < 0: none); then raw_dst[0 ..
// n16) = raw_src[0 .. n16).
__device__ __forceinline__ void plb_stage_range(const PlbDesc *__restrict__ desc, int32_t n_first, int32_t n_desc,
                                                const ToneDev *__restrict__ plan_tones, uint64_t n0,
                                                ToneDev *__restrict__ dst_first, ToneDev *__restrict__ dst_rest,
                                                const uint4 *__restrict__ raw_src, uint4 *__restrict__ raw_dst,
                                                uint64_t n16, uint64_t tid, uint64_t stride)
{
    for (uint64_t i = tid; i < (uint64_t)n_desc; i += stride) {
        const PlbDesc d = desc[i];
        ToneDev t;
        if (d.src >= 0) {
            t = plan_tones[d.src];
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
        if (i < (uint64_t)n_first) dst_first[i] = t;
        else dst_rest[i - (uint64_t)n_first] = t;
    }
    for (uint64_t i = tid; i < n16; i += stride) raw_dst[i] = raw_src[i];
}

// A retune's records to the plan's device table: tones[rec[i].index] = rec[i].tone.
__device__ __forceinline__ void plb_scatter_range(ToneDev *__restrict__ tones, const ScatterRecord *__restrict__ rec,
                                                  int32_t n, uint64_t tid, uint64_t stride)
{
    for (uint64_t i = tid; i < (uint64_t)n; i += stride) tones[rec[i].index] = rec[i].tone;
}

}  // namespace awg
