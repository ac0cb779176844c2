// Snapshot accumulation for short sampling periods.
//
// When the sampling period is very short, adjacent snapshots are nearly the
// same and the method is applied to sums of adjacent snapshots instead,
// combined until adjacent sums differ enough (Li, Adamek & Armour, arXiv
// 2509.21754, Sec. 3.3.2; the combination is a plain sum). The paper gives no
// criterion for "enough"; this library reads it as one factor K for the
// whole stack (the accumulated series stays uniformly sampled for the
// frequency branch) chosen by the contrast of adjacent sums:
//   Y_j  = sum_{k = jK}^{jK+K-1} X_k, j = 0 .. P-1, P = floor(n / K)  (FP32, frame order)
//   c_j  = sum_p |Y_{j+1}(p) - Y_j(p)| / sum_p |Y_j(p)|              (FP64 reductions)
//   C(K) = median_j c_j;  K = min{K <= k_max : P >= 3, C(K) >= gamma},
//          else the largest K <= k_max with P >= 3.
// Both steps stream the stack from HBM (no reuse): accumulation reads it
// once and writes 1/K of it; each contrast C(K) reads it about twice.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "fitrig.h"
#include "fitrig_device.h"

namespace fitrig {
namespace {

template <typename T>
__device__ __forceinline__ float accum_at(const T* X, int64_t plane, int K, int j, int64_t p) {
  const T* x = X + (int64_t)j * K * plane + p;
  float y = to_f<T>(x[0]);
  for (int k = 1; k < K; ++k) y += to_f<T>(x[(int64_t)k * plane]);
  return y;
}

// Y[j][p] for every accumulated snapshot j and pixel p (grid-stride).
template <typename T>
__global__ __launch_bounds__(256) void k_accum(const T* X, int64_t plane, int K, int P, float* Y) {
  const int64_t total = (int64_t)P * plane;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i / plane);
    const int64_t p = i - (int64_t)j * plane;
    Y[i] = accum_at<T>(X, plane, K, j, p);
  }
}

__device__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per adjacent pair j and workgroup b: sum |Y_{j+1} - Y_j| and sum |Y_j|
// over the workgroup's pixels (fixed order) -> part[(j * G + b) * 2].
template <typename T>
__global__ __launch_bounds__(256) void k_accum_pairs(const T* X, int64_t plane, int K, int P, double* part) {
  __shared__ double sh[256];
  const int G = gridDim.x, b = blockIdx.x;
  for (int j = 0; j + 1 < P; ++j) {
    double d = 0.0, a = 0.0;
    for (int64_t p = (int64_t)b * blockDim.x + threadIdx.x; p < plane; p += (int64_t)G * blockDim.x) {
      const float y0 = accum_at<T>(X, plane, K, j, p);
      const float y1 = accum_at<T>(X, plane, K, j + 1, p);
      d += (double)fabsf(y1 - y0);
      a += (double)fabsf(y0);
    }
    d = block_sum(d, sh);
    a = block_sum(a, sh);
    if (threadIdx.x == 0) {
      part[((int64_t)j * G + b) * 2 + 0] = d;
      part[((int64_t)j * G + b) * 2 + 1] = a;
    }
  }
}

// c_j from the workgroup partials (summed over workgroups in order).
__global__ __launch_bounds__(256) void k_accum_ratio(const double* part, int G, int npairs, double* c) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < npairs; j += gridDim.x * blockDim.x) {
    double d = 0.0, a = 0.0;
    for (int b = 0; b < G; ++b) {
      d += part[((int64_t)j * G + b) * 2 + 0];
      a += part[((int64_t)j * G + b) * 2 + 1];
    }
    c[j] = (d == 0.0 && a == 0.0) ? 0.0 : (a > 0.0 ? d / a : INFINITY);
  }
}

// Median of c[0 .. m) by ranks (ties broken by index, so ranks are unique):
// the values of ranks (m - 1) / 2 and m / 2 go to mid[0], mid[1].
__global__ __launch_bounds__(256) void k_accum_rank(const double* c, int m, double* mid) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const double v = c[i];
    int r = 0;
    for (int j = 0; j < m; ++j) r += (c[j] < v || (c[j] == v && j < i)) ? 1 : 0;
    if (r == (m - 1) / 2) mid[0] = v;
    if (r == m / 2) mid[1] = v;
  }
}

// C(K) from the middle values (NaN when there is no pair).
__global__ void k_accum_median(const double* mid, int m, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = m < 1 ? NAN : (m % 2) ? mid[0] : 0.5 * (mid[0] + mid[1]);
}

// The factor from the contrasts C(1 .. k_max) (NaN where P < 2).
__global__ void k_accum_pick(const double* C, int n, int k_max, double gamma, int32_t* K_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int pick = 0, last = 0;
  for (int K = 1; K <= k_max; ++K) {
    if (n / K < 3) continue;
    last = K;
    if (!pick && C[K - 1] >= gamma) pick = K;
  }
  K_out[0] = pick ? pick : last;
}

template <typename T>
void launch_accum(const void* X, int64_t plane, int K, int P, float* Y, hipStream_t st) {
  const int64_t total = (int64_t)P * plane;
  const int g = (int)std::min<int64_t>(std::max<int64_t>(1, (total + 255) / 256), 16384);
  hipLaunchKernelGGL((k_accum<T>), dim3(g), dim3(256), 0, st, (const T*)X, plane, K, P, Y);
}

template <typename T>
void launch_pairs(const void* X, int64_t plane, int K, int P, int G, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_accum_pairs<T>), dim3(G), dim3(256), 0, st, (const T*)X, plane, K, P, part);
}

fitrig_status check(const void* stack, fitrig_dtype dtype, int32_t n, int32_t H, int32_t W) {
  if (!stack || n < 1 || H < 1 || W < 1 || (uint64_t)H * (uint64_t)W >= (1ull << 32)) return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  return FITRIG_OK;
}

}  // namespace
}  // namespace fitrig

using namespace fitrig;

extern "C" {

fitrig_status fitrig_accumulate(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H, int32_t W,
                                int32_t K, float* out, void* hip_stream) {
  fitrig_status rc = check(stack, dtype, n_snap, H, W);
  if (rc != FITRIG_OK) return rc;
  if (!out || K < 1 || n_snap / K < 1) return FITRIG_E_INVAL;
  const int64_t plane = (int64_t)H * W;
  const int P = n_snap / K;
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == FITRIG_F32)
    launch_accum<float>(stack, plane, K, P, out, st);
  else if (dtype == FITRIG_F16)
    launch_accum<__half>(stack, plane, K, P, out, st);
  else
    launch_accum<bf16_t>(stack, plane, K, P, out, st);
  return hipGetLastError() == hipSuccess ? FITRIG_OK : FITRIG_E_HIP;
}

fitrig_status fitrig_accum_factor(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H, int32_t W,
                                  double gamma, int32_t k_max, int32_t* K_out, double* contrast, void* hip_stream) {
  fitrig_status rc = check(stack, dtype, n_snap, H, W);
  if (rc != FITRIG_OK) return rc;
  if (!K_out || k_max < 1 || !(gamma >= 0.0) || !isfinite(gamma) || n_snap < 3 || n_snap > 65536)
    return FITRIG_E_INVAL;
  const int64_t plane = (int64_t)H * W;
  const int G = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (plane + 4095) / 4096));
  hipStream_t st = (hipStream_t)hip_stream;
  const int pmax = n_snap;  // pairs of K = 1 bound every K's
  double* dev = nullptr;
  int32_t* dK = nullptr;
  const size_t part_b = (size_t)pmax * G * 2 * 8, c_b = (size_t)pmax * 8;
  if (hipMalloc((void**)&dev, part_b + c_b + 2 * 8 + (size_t)k_max * 8) != hipSuccess) return FITRIG_E_NOMEM;
  if (hipMalloc((void**)&dK, 4) != hipSuccess) {
    (void)hipFree(dev);
    return FITRIG_E_NOMEM;
  }
  double* part = dev;
  double* c = dev + (size_t)pmax * G * 2;
  double* mid = c + pmax;
  double* C = mid + 2;
  bool ok = true;
  for (int K = 1; K <= k_max && ok; ++K) {
    const int P = n_snap / K;
    if (P < 2) {
      hipLaunchKernelGGL(k_accum_median, dim3(1), dim3(64), 0, st, (const double*)mid, 0, C + (K - 1));
      ok = hipGetLastError() == hipSuccess;
      continue;
    }
    if (dtype == FITRIG_F32)
      launch_pairs<float>(stack, plane, K, P, G, part, st);
    else if (dtype == FITRIG_F16)
      launch_pairs<__half>(stack, plane, K, P, G, part, st);
    else
      launch_pairs<bf16_t>(stack, plane, K, P, G, part, st);
    const int m = P - 1;
    const int g = std::max(1, std::min(64, (m + 255) / 256));
    hipLaunchKernelGGL(k_accum_ratio, dim3(g), dim3(256), 0, st, (const double*)part, G, m, c);
    hipLaunchKernelGGL(k_accum_rank, dim3(g), dim3(256), 0, st, (const double*)c, m, mid);
    hipLaunchKernelGGL(k_accum_median, dim3(1), dim3(64), 0, st, (const double*)mid, m, C + (K - 1));
    ok = hipGetLastError() == hipSuccess;
  }
  if (ok) {
    hipLaunchKernelGGL(k_accum_pick, dim3(1), dim3(64), 0, st, (const double*)C, n_snap, k_max, gamma, dK);
    ok = hipGetLastError() == hipSuccess && hipMemcpyAsync(K_out, dK, 4, hipMemcpyDeviceToHost, st) == hipSuccess &&
         (!contrast ||
          hipMemcpyAsync(contrast, C, (size_t)k_max * 8, hipMemcpyDeviceToHost, st) == hipSuccess) &&
         hipStreamSynchronize(st) == hipSuccess;
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(dev);
  (void)hipFree(dK);
  return ok ? FITRIG_OK : FITRIG_E_HIP;
}

}  // extern "C"
