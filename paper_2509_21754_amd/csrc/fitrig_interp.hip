// Sub-cell peak localisation: the paper interpolates the values of the
// selected tiles (the spectrum matrix eta) with a bilinear, spline, bicubic
// or Makima cubic interpolant and takes the interpolated maximum as the
// source position (Sec. 2.4.2; a spline on eta in Sec. 3.1).
//
// One workgroup per peak: the 5 x 5 cells around the peak (indices clamped
// into the map) are interpolated along x for each row at the 2 sub + 1
// offsets (LDS), then along y at every grid point; a workgroup reduction
// picks the largest value (ties to the lowest grid index: smallest y offset,
// then smallest x offset). Arithmetic in FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include <climits>

#include "fitrig.h"

namespace {

constexpr int kRad = 2;
constexpr int kNodes = 2 * kRad + 1;
constexpr int kMaxSub = 64;
constexpr int kThreads = 256;

// Inverse of the not-a-knot system for the second derivatives of a cubic
// spline through 5 unit-spaced nodes (row-major).
struct SplineInv {
  double a[kNodes * kNodes];
};

__device__ __forceinline__ double keys_w(double s) {
  // Keys' cubic convolution kernel, a = -1/2
  s = fabs(s);
  if (s <= 1.0) return (1.5 * s - 2.5) * s * s + 1.0;
  if (s < 2.0) return ((-0.5 * s + 2.5) * s - 4.0) * s + 2.0;
  return 0.0;
}

// Value at t in [0, 4] of the interpolant through f[0..4] (unit spacing).
__device__ double interp1(int method, const double* f, double t, const SplineInv& S) {
  int i = (int)floor(t);
  i = i < 0 ? 0 : (i > kNodes - 2 ? kNodes - 2 : i);
  const double u = t - i;
  if (method == FITRIG_INTERP_BILINEAR) return (1.0 - u) * f[i] + u * f[i + 1];
  if (method == FITRIG_INTERP_BICUBIC) {
    double s = 0.0;
    for (int k = i - 1; k <= i + 2; ++k) {
      const int kk = k < 0 ? 0 : (k > kNodes - 1 ? kNodes - 1 : k);
      s += keys_w(t - k) * f[kk];
    }
    return s;
  }
  if (method == FITRIG_INTERP_SPLINE) {
    double r[kNodes] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 1; k < kNodes - 1; ++k) r[k] = 6.0 * (f[k - 1] - 2.0 * f[k] + f[k + 1]);
    double M0 = 0.0, M1 = 0.0;
    for (int k = 0; k < kNodes; ++k) {
      M0 += S.a[i * kNodes + k] * r[k];
      M1 += S.a[(i + 1) * kNodes + k] * r[k];
    }
    const double v = 1.0 - u;
    return M0 * v * v * v / 6.0 + M1 * u * u * u / 6.0 + (f[i] - M0 / 6.0) * v + (f[i + 1] - M1 / 6.0) * u;
  }
  // modified Akima: interval slopes extended by two on each side
  double m[kNodes + 3];
  for (int k = 0; k < kNodes - 1; ++k) m[k + 2] = f[k + 1] - f[k];
  m[1] = 2.0 * m[2] - m[3];
  m[0] = 2.0 * m[1] - m[2];
  m[kNodes + 1] = 2.0 * m[kNodes] - m[kNodes - 1];
  m[kNodes + 2] = 2.0 * m[kNodes + 1] - m[kNodes];
  double d[2];
  for (int j = 0; j < 2; ++j) {
    const int n = i + j;  // node
    const double dm2 = m[n], dm1 = m[n + 1], d0 = m[n + 2], dp1 = m[n + 3];
    const double w1 = fabs(dp1 - d0) + fabs(dp1 + d0) / 2.0;
    const double w2 = fabs(dm1 - dm2) + fabs(dm1 + dm2) / 2.0;
    d[j] = (w1 + w2 == 0.0) ? 0.0 : (w1 * dm1 + w2 * d0) / (w1 + w2);
  }
  const double h00 = 2 * u * u * u - 3 * u * u + 1, h10 = u * u * u - 2 * u * u + u;
  const double h01 = -2 * u * u * u + 3 * u * u, h11 = u * u * u - u * u;
  return h00 * f[i] + h10 * d[0] + h01 * f[i + 1] + h11 * d[1];
}

__global__ __launch_bounds__(kThreads) void k_interp_peaks(const float* map, int H, int W, const int32_t* py,
                                                           const int32_t* px, int method, int sub, SplineInv S,
                                                           double* out) {
  __shared__ double F[kNodes * kNodes];
  __shared__ double G[kNodes][2 * kMaxSub + 1];
  __shared__ double bv[kThreads];
  __shared__ int bi[kThreads];
  const int c = blockIdx.x, t = threadIdx.x;
  const int y0 = py[c], x0 = px[c];
  if (t < kNodes * kNodes) {
    int y = y0 - kRad + t / kNodes, x = x0 - kRad + t % kNodes;
    y = y < 0 ? 0 : (y >= H ? H - 1 : y);
    x = x < 0 ? 0 : (x >= W ? W - 1 : x);
    F[t] = (double)map[(int64_t)y * W + x];
  }
  __syncthreads();
  const int ng = 2 * sub + 1;
  for (int j = t; j < kNodes * ng; j += kThreads) {
    const int r = j / ng, b = j - r * ng;
    G[r][b] = interp1(method, &F[r * kNodes], kRad + (double)(b - sub) / (double)sub, S);
  }
  __syncthreads();
  double best = -INFINITY;
  int idx = INT_MAX;
  for (int j = t; j < ng * ng; j += kThreads) {
    const int a = j / ng, b = j - a * ng;
    double col[kNodes];
    for (int r = 0; r < kNodes; ++r) col[r] = G[r][b];
    const double v = interp1(method, col, kRad + (double)(a - sub) / (double)sub, S);
    if (v > best) {  // j increases: the first of equal values is kept
      best = v;
      idx = j;
    }
  }
  bv[t] = best;
  bi[t] = idx;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if (t < w) {
      const double ov = bv[t + w];
      const int oi = bi[t + w];
      if (ov > bv[t] || (ov == bv[t] && oi < bi[t])) {
        bv[t] = ov;
        bi[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const int j = bi[0] == INT_MAX ? 0 : bi[0];
    const int a = j / ng, b = j - a * ng;
    out[3 * c + 0] = y0 + (double)(a - sub) / (double)sub;
    out[3 * c + 1] = x0 + (double)(b - sub) / (double)sub;
    out[3 * c + 2] = bv[0];
  }
}

// Gauss-Jordan inverse of the not-a-knot system (host, once per call).
SplineInv spline_inverse() {
  double A[kNodes][2 * kNodes] = {};
  A[0][0] = 1.0, A[0][1] = -2.0, A[0][2] = 1.0;
  for (int i = 1; i < kNodes - 1; ++i) A[i][i - 1] = 1.0, A[i][i] = 4.0, A[i][i + 1] = 1.0;
  A[kNodes - 1][kNodes - 3] = 1.0, A[kNodes - 1][kNodes - 2] = -2.0, A[kNodes - 1][kNodes - 1] = 1.0;
  for (int i = 0; i < kNodes; ++i) A[i][kNodes + i] = 1.0;
  for (int col = 0; col < kNodes; ++col) {
    int piv = col;
    for (int r = col + 1; r < kNodes; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    for (int k = 0; k < 2 * kNodes; ++k) {
      const double tmp = A[col][k];
      A[col][k] = A[piv][k];
      A[piv][k] = tmp;
    }
    const double p = A[col][col];
    for (int k = 0; k < 2 * kNodes; ++k) A[col][k] /= p;
    for (int r = 0; r < kNodes; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int k = 0; k < 2 * kNodes; ++k) A[r][k] -= f * A[col][k];
    }
  }
  SplineInv S;
  for (int i = 0; i < kNodes; ++i)
    for (int k = 0; k < kNodes; ++k) S.a[i * kNodes + k] = A[i][kNodes + k];
  return S;
}

}  // namespace

extern "C" fitrig_status fitrig_interp_peaks(const float* map, int32_t H, int32_t W, const int32_t* py,
                                             const int32_t* px, int32_t n, int32_t method, int32_t sub,
                                             double* out, void* hip_stream) {
  if (n < 0 || H < 1 || W < 1 || sub < 1 || sub > kMaxSub) return FITRIG_E_INVAL;
  if (method < FITRIG_INTERP_BILINEAR || method > FITRIG_INTERP_MAKIMA) return FITRIG_E_INVAL;
  if (n == 0) return FITRIG_OK;
  if (!map || !py || !px || !out) return FITRIG_E_INVAL;
  for (int32_t i = 0; i < n; ++i)
    if (py[i] < 0 || py[i] >= H || px[i] < 0 || px[i] >= W) return FITRIG_E_INVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  int32_t* dpk = nullptr;
  double* dout = nullptr;
  if (hipMalloc((void**)&dpk, (size_t)n * 8) != hipSuccess) return FITRIG_E_NOMEM;
  if (hipMalloc((void**)&dout, (size_t)n * 24) != hipSuccess) {
    (void)hipFree(dpk);
    return FITRIG_E_NOMEM;
  }
  hipError_t e = hipMemcpyAsync(dpk, py, (size_t)n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dpk + n, px, (size_t)n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_interp_peaks, dim3((unsigned)n), dim3(kThreads), 0, st, map, (int)H, (int)W,
                       (const int32_t*)dpk, (const int32_t*)(dpk + n), (int)method, (int)sub, spline_inverse(),
                       dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, (size_t)n * 24, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dpk);
  (void)hipFree(dout);
  return e == hipSuccess ? FITRIG_OK : FITRIG_E_HIP;
}
