// Matrix-core (MFMA) static synthesis by angle addition. Placeholder until the
// kernels land: the direct method serves every request.
#include <hip/hip_runtime.h>

#include "awg_internal.h"

namespace awg {

awg_status mfma_static(awg_plan *p, uint32_t method, uint64_t n0, uint64_t count, int16_t *out_i16,
                       float *out_f32, hipStream_t s)
{
    (void)p; (void)method; (void)n0; (void)count; (void)out_i16; (void)out_f32; (void)s;
    return AWG_E_UNSUPPORTED;
}

}  // namespace awg
