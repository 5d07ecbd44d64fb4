// ProfScope::launch for the HIP sources (needs the HIP language for the kernels).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "awg_internal.h"

namespace awg {

template <typename F, typename... Args>
void ProfScope::launch(F kernel, dim3 grid, dim3 block, uint32_t shmem, Args... args)
{
    if (stop_) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s_, launched_ ? nullptr : start_, stop_, 0, args...);
        launched_ = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s_, args...);
    }
}

}  // namespace awg
