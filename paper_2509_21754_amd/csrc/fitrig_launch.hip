// Host launchers of the kernels templated on the storage type. This file is
// compiled once per storage type (FITRIG_STORAGE = 0 FP32, 1 FP16, 2 BF16),
// so the instantiations of the three types build in parallel.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "fitrig_device.h"

#ifndef FITRIG_STORAGE
#error "FITRIG_STORAGE must be 0 (FP32), 1 (FP16) or 2 (BF16)"
#endif

namespace fitrig {

#if FITRIG_STORAGE == 0
using T = float;
#define SFX(name) name##_f32
#elif FITRIG_STORAGE == 1
using T = __half;
#define SFX(name) name##_f16
#else
using T = bf16_t;
#define SFX(name) name##_bf16
#endif

bool SFX(launch_stream)(int halo, bool rs, dim3 grid, hipStream_t st, const StreamArgs& A) {
  switch (halo) {
#define CASE(h)                                                                                  \
  case h:                                                                                        \
    if (rs)                                                                                      \
      hipLaunchKernelGGL((k_stream<T, h, true>), grid, dim3(kLanes), 0, st, A);                  \
    else                                                                                         \
      hipLaunchKernelGGL((k_stream<T, h, false>), grid, dim3(kLanes), 0, st, A);                 \
    return true;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return false;
  }
}

bool SFX(launch_tile_stream)(int tile, bool rs, dim3 grid, hipStream_t st, const TileStreamArgs& A) {
  switch (tile) {
#define CASE(t)                                                                                  \
  case t:                                                                                        \
    if (rs)                                                                                      \
      hipLaunchKernelGGL((k_tile_stream<T, t, true>), grid, dim3(kLanes), 0, st, A);             \
    else                                                                                         \
      hipLaunchKernelGGL((k_tile_stream<T, t, false>), grid, dim3(kLanes), 0, st, A);            \
    return true;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return false;
  }
}

bool SFX(launch_tile)(bool rs, dim3 grid, hipStream_t st, const TileArgs& A) {
  if (rs)
    hipLaunchKernelGGL((k_tile<T, true>), grid, dim3(kLanes), 0, st, A);
  else
    hipLaunchKernelGGL((k_tile<T, false>), grid, dim3(kLanes), 0, st, A);
  return true;
}

bool SFX(launch_recompute)(int halo, bool rs, dim3 grid, hipStream_t st, const RecomputeArgs& R) {
  switch (halo) {
#define CASE(h)                                                                                  \
  case h:                                                                                        \
    if (rs)                                                                                      \
      hipLaunchKernelGGL((k_recompute<T, h, true>), grid, dim3(64), 0, st, R);                   \
    else                                                                                         \
      hipLaunchKernelGGL((k_recompute<T, h, false>), grid, dim3(64), 0, st, R);                  \
    return true;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return false;
  }
}

bool SFX(launch_stack_max)(dim3 grid, hipStream_t st, const CallDev* cd, int64_t n, uint32_t* max_key) {
  hipLaunchKernelGGL((k_stack_max<T>), grid, dim3(256), 0, st, cd, n, max_key);
  return true;
}

}  // namespace fitrig
