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

// Each returns the kernel for the given template parameters (the host
// handle that hipLaunchKernel and graph kernel nodes take), or null when no
// instantiation covers them. Every kernel takes its argument struct by value.
const void* SFX(kernel_stream)(int halo, bool rs, bool q) {
  switch (halo) {
#define CASE(h)                                                                                     \
  case h:                                                                                           \
    return q ? (rs ? (const void*)&k_stream<T, h, true, true> : (const void*)&k_stream<T, h, false, true>) \
             : (rs ? (const void*)&k_stream<T, h, true, false> : (const void*)&k_stream<T, h, false, false>);
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return nullptr;
  }
}

const void* SFX(kernel_tile_stream)(int tile, bool rs) {
  switch (tile) {
#define CASE(t) \
  case t: return rs ? (const void*)&k_tile_stream<T, t, true> : (const void*)&k_tile_stream<T, t, false>;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return nullptr;
  }
}

const void* SFX(kernel_tile)(bool rs) { return rs ? (const void*)&k_tile<T, true> : (const void*)&k_tile<T, false>; }

const void* SFX(kernel_recompute)(int halo, bool rs) {
  switch (halo) {
#define CASE(h) \
  case h: return rs ? (const void*)&k_recompute<T, h, true> : (const void*)&k_recompute<T, h, false>;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return nullptr;
  }
}

// k_stack_max(const CallDev* cd, int64_t n, uint32_t* max_key)
const void* SFX(kernel_stack_max)() { return (const void*)&k_stack_max<T>; }

}  // namespace fitrig
