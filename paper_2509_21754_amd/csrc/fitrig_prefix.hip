// Index maps from full-image prefix sums: a comparison variant of the window
// sums, kept off the detection path.
//
// The sliding-window sums of Delta and r (Li, Adamek & Armour, arXiv
// 2509.21754, Sec. 2.3, Eq. (6)) are read from integral images
//   I(y, x) = sum_{y' < y, x' < x} a(y', x')      ((H + 1) x (W + 1), zero first row / column)
// as S = I(y2+1, x2+1) - I(y1, x2+1) - I(y2+1, x1) + I(y1, x1) over the clipped
// window [y1, y2] x [x1, x2]. The integral image's entries grow with the image
// (about H W mean(a)), so in FP32 the four-corner difference loses the window
// sum beyond a few thousand pixels on a side, while FP64 keeps it; the
// streaming kernel's direct sums (8-aligned blocks, at most 17 terms) have
// neither problem. The window maximum, which has no prefix form, is taken by
// a separable exact maximum. Per triple: pointwise terms (FP32, as the
// streaming kernel), column prefix (one thread per column, rows in order),
// row prefix (one workgroup per row, blocked scan), window sums and q.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "fitrig.h"
#include "fitrig_device.h"

namespace fitrig {
namespace {

// Delta and r of triple s for every pixel (FP32, Eqs. (3)-(5)).
template <typename T, bool RS>
__global__ __launch_bounds__(256) void k_pf_terms(const T* X, int64_t plane, int s, float Cf, float* dl, float* rl) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (int64_t)gridDim.x * blockDim.x) {
    const float a = to_f<T>(X[(int64_t)s * plane + p]);
    const float b = to_f<T>(X[(int64_t)(s + 1) * plane + p]);
    const float c = to_f<T>(X[(int64_t)(s + 2) * plane + p]);
    float d, r;
    pix3<RS>(a, b, c, Cf, d, r);
    dl[p] = fabsf(d);
    rl[p] = r;
  }
}

// Column prefix into rows 1.. of the integral images: I(y+1, x+1) = sum of
// a(0..y, x) (row pass still to come); row 0 and column 0 are zero.
template <typename P>
__global__ __launch_bounds__(256) void k_pf_cols(const float* dl, const float* rl, int H, int W, P* IA, P* IB) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t W1 = (int64_t)W + 1;
  if (x > W) return;
  IA[x] = (P)0;
  IB[x] = (P)0;
  if (x == W) {
    for (int y = 1; y <= H; ++y) {
      IA[(int64_t)y * W1] = (P)0;
      IB[(int64_t)y * W1] = (P)0;
    }
    return;
  }
  P sa = (P)0, sb = (P)0;
  for (int y = 0; y < H; ++y) {
    sa += (P)dl[(int64_t)y * W + x];
    sb += (P)rl[(int64_t)y * W + x];
    IA[(int64_t)(y + 1) * W1 + x + 1] = sa;
    IB[(int64_t)(y + 1) * W1 + x + 1] = sb;
  }
}

// Row prefix, in place, of rows 1 .. H (columns 1 .. W): one workgroup per
// row, chunks of 256 with a running carry; within a chunk a Hillis-Steele
// scan in LDS (fixed order).
template <typename P>
__global__ __launch_bounds__(256) void k_pf_rows(int W, P* IA, P* IB) {
  __shared__ P sa[256], sb[256];
  const int64_t W1 = (int64_t)W + 1;
  P* ra = IA + (int64_t)(blockIdx.x + 1) * W1 + 1;
  P* rb = IB + (int64_t)(blockIdx.x + 1) * W1 + 1;
  P ca = (P)0, cb = (P)0;
  const int t = threadIdx.x;
  for (int base = 0; base < W; base += 256) {
    const int x = base + t;
    sa[t] = x < W ? ra[x] : (P)0;
    sb[t] = x < W ? rb[x] : (P)0;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const P va = t >= off ? sa[t - off] : (P)0;
      const P vb = t >= off ? sb[t - off] : (P)0;
      __syncthreads();
      sa[t] += va;
      sb[t] += vb;
      __syncthreads();
    }
    if (x < W) {
      ra[x] = ca + sa[t];
      rb[x] = cb + sb[t];
    }
    const P ta = sa[255], tb = sb[255];
    __syncthreads();
    ca += ta;
    cb += tb;
  }
}

// Vertical window maximum of Delta (exact).
__global__ __launch_bounds__(256) void k_pf_vmax(const float* dl, int H, int W, int h, float* vm) {
  const int64_t plane = (int64_t)H * W;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    float m = 0.0f;
    for (int yy = max(y - h, 0); yy <= min(y + h, H - 1); ++yy) m = fmaxf(m, dl[(int64_t)yy * W + x]);
    vm[p] = m;
  }
}

// q per pixel from the integral images and the separable maximum.
template <typename P>
__global__ __launch_bounds__(256) void k_pf_q(const P* IA, const P* IB, const float* vm, int H, int W, int h,
                                              float* q) {
  const int64_t plane = (int64_t)H * W;
  const int64_t W1 = (int64_t)W + 1;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    const int y1 = max(y - h, 0), y2 = min(y + h, H - 1), x1 = max(x - h, 0), x2 = min(x + h, W - 1);
    const P sA = IA[(int64_t)(y2 + 1) * W1 + x2 + 1] - IA[(int64_t)y1 * W1 + x2 + 1] - IA[(int64_t)(y2 + 1) * W1 + x1] +
                 IA[(int64_t)y1 * W1 + x1];
    const P sB = IB[(int64_t)(y2 + 1) * W1 + x2 + 1] - IB[(int64_t)y1 * W1 + x2 + 1] - IB[(int64_t)(y2 + 1) * W1 + x1] +
                 IB[(int64_t)y1 * W1 + x1];
    float m = 0.0f;
    for (int xx = x1; xx <= x2; ++xx) m = fmaxf(m, vm[(int64_t)y * W + xx]);
    const P nc = (P)((y2 - y1 + 1) * (x2 - x1 + 1));
    q[p] = (float)((sA / nc) * (P)m * (sB / nc));
  }
}

template <typename T, typename P>
fitrig_status run(const void* stack, int n, int H, int W, int h, bool rs, float Cf, float* qmap, hipStream_t st,
                  char* scr) {
  const int64_t plane = (int64_t)H * W;
  const int64_t isz = ((int64_t)H + 1) * ((int64_t)W + 1);
  P* IA = (P*)scr;
  P* IB = IA + isz;
  float* dl = (float*)(IB + isz);
  float* rl = dl + plane;
  float* vm = rl + plane;
  const int g = (int)std::min<int64_t>(std::max<int64_t>(1, (plane + 255) / 256), 16384);
  for (int s = 0; s + 2 < n; ++s) {
    if (rs)
      hipLaunchKernelGGL((k_pf_terms<T, true>), dim3(g), dim3(256), 0, st, (const T*)stack, plane, s, Cf, dl, rl);
    else
      hipLaunchKernelGGL((k_pf_terms<T, false>), dim3(g), dim3(256), 0, st, (const T*)stack, plane, s, Cf, dl, rl);
    hipLaunchKernelGGL((k_pf_cols<P>), dim3((W + 1 + 255) / 256), dim3(256), 0, st, (const float*)dl,
                       (const float*)rl, H, W, IA, IB);
    hipLaunchKernelGGL((k_pf_rows<P>), dim3(H), dim3(256), 0, st, W, IA, IB);
    hipLaunchKernelGGL(k_pf_vmax, dim3(g), dim3(256), 0, st, (const float*)dl, H, W, h, vm);
    hipLaunchKernelGGL((k_pf_q<P>), dim3(g), dim3(256), 0, st, (const P*)IA, (const P*)IB, (const float*)vm, H, W, h,
                       qmap + (int64_t)s * plane);
    if (hipGetLastError() != hipSuccess) return FITRIG_E_HIP;
  }
  return FITRIG_OK;
}

}  // namespace
}  // namespace fitrig

using namespace fitrig;

extern "C" fitrig_status fitrig_index_prefix(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H,
                                             int32_t W, int32_t window, int32_t prefix_bits, int32_t r_signed,
                                             double C, float* index_map, void* hip_stream) {
  if (!stack || !index_map || n_snap < 3 || H < 1 || W < 1 || (uint64_t)H * (uint64_t)W >= (1ull << 32))
    return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  if (window < 1 || window % 2 == 0 || (prefix_bits != 32 && prefix_bits != 64) || (r_signed != 0 && r_signed != 1) ||
      !(C > 0.0) || !isfinite(C))
    return FITRIG_E_INVAL;
  const int64_t plane = (int64_t)H * W;
  const int64_t isz = ((int64_t)H + 1) * ((int64_t)W + 1);
  const size_t bytes = (size_t)isz * 2 * (prefix_bits / 8) + (size_t)plane * 3 * 4;
  char* scr = nullptr;
  if (hipMalloc((void**)&scr, bytes) != hipSuccess) return FITRIG_E_NOMEM;
  hipStream_t st = (hipStream_t)hip_stream;
  const int h = window / 2;
  const bool rs = r_signed != 0;
  const float Cf = (float)C;
  fitrig_status rc;
  if (prefix_bits == 64)
    rc = dtype == FITRIG_F32   ? run<float, double>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr)
         : dtype == FITRIG_F16 ? run<__half, double>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr)
                               : run<bf16_t, double>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr);
  else
    rc = dtype == FITRIG_F32   ? run<float, float>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr)
         : dtype == FITRIG_F16 ? run<__half, float>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr)
                               : run<bf16_t, float>(stack, n_snap, H, W, h, rs, Cf, index_map, st, scr);
  const hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(scr);
  if (rc == FITRIG_OK && e != hipSuccess) rc = FITRIG_E_HIP;
  return rc;
}
