// FITrig device code templated on the storage type (FP32 / FP16 / BF16):
// shared device helpers, the streaming index kernel, the tile-mode kernels and
// the exact recompute of selected segments. Included by the per-type launch
// translation units and by the rest of the device code.
//
// Method (Li, Adamek & Armour, arXiv 2509.21754):
//   Delta = ||x(s+2)-x(s+1)| - |x(s+1)-x(s)||, reference x(s+1)  Sec. 2.2.4, Eqs. (3)-(5)
//   r = min(Delta / |x_hat|, 1), x_hat = C where x(s+1) == 0       Eqs. (4)-(5)
//   q = mean(Delta) max(Delta) mean(r) over the window / tile       Eq. (2), Eq. (6)
//
// Window sums use 8-row / 8-column blocks aligned to absolute multiples of
// 8: a window [L, R] is suffix(block of L) + totals of whole blocks +
// prefix(block of R), with prefix / suffix defined by fixed left-to-right /
// right-to-left recurrences. The value of a cell therefore depends only on
// its absolute position, so the exact selection kernel recomputes it to the
// same bits as the streaming kernel.
#pragma once

#include <hip/hip_fp16.h>
#include <math.h>
#include <stdint.h>
#include <type_traits>

#include "fitrig.h"
#include "fitrig_internal.h"

namespace fitrig {

struct bf16_t {
  uint16_t v;
};

template <typename T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ float to_f<__half>(__half v) {
  return __half2float(v);
}
template <>
__device__ __forceinline__ float to_f<bf16_t>(bf16_t v) {
  return __uint_as_float(((uint32_t)v.v) << 16);
}

// p[o] widened to FP32, read through a global-address pointer (vector
// memory only, no LDS counter)
template <typename T>
__device__ __forceinline__ float ldg_f(const T* p, int64_t o);
template <>
__device__ __forceinline__ float ldg_f<float>(const float* p, int64_t o) {
  return ((__attribute__((address_space(1))) const float*)p)[o];
}
template <>
__device__ __forceinline__ float ldg_f<__half>(const __half* p, int64_t o) {
  return __half2float(__ushort_as_half(((__attribute__((address_space(1))) const unsigned short*)p)[o]));
}
template <>
__device__ __forceinline__ float ldg_f<bf16_t>(const bf16_t* p, int64_t o) {
  return __uint_as_float(((uint32_t)((__attribute__((address_space(1))) const uint16_t*)p)[o]) << 16);
}

template <typename T>
__device__ __forceinline__ const T* frame_ptr(const void* base, const void* c0, const void* c1,
                                              int ncarry, int64_t plane, int k) {
  if (k < ncarry) return (const T*)(k == 0 ? c0 : c1);
  return (const T*)base + (int64_t)(k - ncarry) * plane;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of logical tiles so neighbours share halo lines in its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// Order of the streaming kernel's (band, group) tiles along one XCD's run of
// workgroups: blocks of bb bands, group by group. With bb = 8 the workgroups
// resident on an XCD at a time cover about 8 bands x 8 groups, so the halo
// rows they share are fetched once into its L2; bb = 1 is row order.
__device__ __forceinline__ void tile_of(int t, int nbands, int ncol, int bb_size, int& band, int& grp) {
  const int per = bb_size * ncol;
  const int bb = t / per;
  const int rem = nbands - bb * bb_size;
  const int hb = rem < bb_size ? rem : bb_size;
  const int u = t - bb * per;
  grp = u / hb;
  band = bb * bb_size + (u - grp * hb);
}

typedef float fitrig_v4f __attribute__((ext_vector_type(4)));

// Order-preserving map of a float to uint32 (and back).
__device__ __forceinline__ uint32_t ord_key(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_val(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

constexpr int fdiv8(int a) { return a >= 0 ? a / 8 : -((-a + 7) / 8); }

// Window reduction over a register array.
//   a[i] holds the value at relative position P = i - H (P in [-H, NOUT+H-1]),
//   the base position (P = 0) being a multiple of 8 in absolute coordinates.
//   o[c] = op over positions [c-H, c+H]; tot[j] = prefix of block j at 7
//   (sum / max of the 8 positions [8j, 8j+7]). ABS: the values are |a[i]|
//   (the absolute value is a source modifier of the first operation).
template <int H, int NOUT, bool MAXOP, bool ABS = false>
struct Win {
  static constexpr int NIN = NOUT + 2 * H;
  static constexpr int MLO = -1;
  static constexpr int MHI = fdiv8(NOUT - 1 + H);
  static constexpr int NB = MHI - MLO + 1;
  __device__ static __forceinline__ float op(float x, float y) { return MAXOP ? fmaxf(x, y) : x + y; }
  __device__ static __forceinline__ float ld(const float* a, int i) { return ABS ? fabsf(a[i]) : a[i]; }

  __device__ static __forceinline__ void run(const float* a, float* o, float* tot) {
    if constexpr (H <= 2) {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        float s = ld(a, c);
#pragma unroll
        for (int j = 1; j <= 2 * H; ++j) s = op(s, ld(a, c + j));
        o[c] = s;
      }
      if (tot) {
#pragma unroll
        for (int j = 0; j < NOUT / 8; ++j) {
          float s = ld(a, H + 8 * j);
#pragma unroll
          for (int p = 1; p < 8; ++p) s = op(s, ld(a, H + 8 * j + p));
          tot[j] = s;
        }
      }
    } else {
      // Outputs are produced block by block (8 per block); a block's prefix
      // and suffix recurrences are evaluated just before their first use, so
      // only the blocks around the current outputs are live. The arithmetic
      // (each recurrence, each combination) does not depend on this order.
      float pre[NB][8] = {};
      float suf[NB][8] = {};
      bool have_pre[NB] = {}, have_suf[NB] = {};
      auto make_pre = [&](int mi) {
        const int st = H + 8 * (mi + MLO);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int idx = st + p;
          if (st >= 0 && idx < NIN) pre[mi][p] = (p == 0) ? ld(a, idx) : op(pre[mi][p - 1], ld(a, idx));
        }
      };
      auto make_suf = [&](int mi) {
        const int st = H + 8 * (mi + MLO);
#pragma unroll
        for (int p = 7; p >= 0; --p) {
          const int idx = st + p;
          if (st + 7 < NIN && idx >= 0) suf[mi][p] = (p == 7) ? ld(a, idx) : op(ld(a, idx), suf[mi][p + 1]);
        }
      };
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        const int L = c - H, R = c + H;
        const int bs = fdiv8(L), be = fdiv8(R);
        const int ps = L - 8 * bs, pe = R - 8 * be;
        if (bs == be) {
          if (ps == 0) {
            if (!have_pre[bs - MLO]) { make_pre(bs - MLO); have_pre[bs - MLO] = true; }
            o[c] = pre[bs - MLO][pe];
          } else {
            if (!have_suf[bs - MLO]) { make_suf(bs - MLO); have_suf[bs - MLO] = true; }
            o[c] = suf[bs - MLO][ps];
          }
        } else {
          if (!have_suf[bs - MLO]) { make_suf(bs - MLO); have_suf[bs - MLO] = true; }
          float s = suf[bs - MLO][ps];
#pragma unroll
          for (int m = bs + 1; m < be; ++m) {
            if (!have_pre[m - MLO]) { make_pre(m - MLO); have_pre[m - MLO] = true; }
            s = op(s, pre[m - MLO][7]);
          }
          if (!have_pre[be - MLO]) { make_pre(be - MLO); have_pre[be - MLO] = true; }
          o[c] = op(s, pre[be - MLO][pe]);
        }
      }
      if (tot) {
#pragma unroll
        for (int j = 0; j < NOUT / 8; ++j) {
          if (!have_pre[j - MLO]) { make_pre(j - MLO); have_pre[j - MLO] = true; }
          tot[j] = pre[j - MLO][7];
        }
      }
    }
  }
};

// Sum over the 64 lanes of a wave with DPP (quad swaps, half-row and row
// mirrors, row broadcasts); the total ends in lane 63. Fixed order.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __double_as_longlong(v);
  int lo, hi;
  if constexpr (ROWMASK == 0xF) {
    lo = __builtin_amdgcn_mov_dpp((int)(u & 0xFFFFFFFFu), CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xFFFFFFFFu), CTRL, ROWMASK, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROWMASK, 0xF, false);
  }
  return __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Sum over each row of 16 lanes (every lane of the row ends with it).
__device__ __forceinline__ double row_sum_f64(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  return v;
}
// Pointwise terms of one pixel: Delta from the two frame differences, r from
// the reference pixel (Eqs. (3)-(5)). RS selects the literal signed reading
// of Eq. (4); otherwise the ratio uses |x_hat| and is clamped to [0, 1].
template <bool RS>
__device__ __forceinline__ void pix_ratio(float dl, float ref, float Cf, float& rl) {
  const float den = (ref == 0.0f) ? Cf : ref;
  if constexpr (RS) {
    rl = fminf(dl * __builtin_amdgcn_rcpf(den), 1.0f);
  } else {
    // dl >= 0 and den != 0, so the product is finite and >= 0 and min(., 1)
    // is the [0, 1] clamp, which folds into the multiply
    rl = __builtin_amdgcn_fmed3f(dl * __builtin_amdgcn_rcpf(fabsf(den)), 0.0f, 1.0f);
  }
}

// Pointwise terms of one pixel from its three frames x0, x1, x2 (x1 the
// reference). The frame differences x2 - x1 and x1 - x0 are exact in FP64
// (24-bit significands), so Delta = ||x2 - x1| - |x1 - x0|| (Eq. (3)) is
// rounded once, to FP32, and its error stays within half an ulp of Delta.
// (Differences rounded to FP32 first leave an error of the order of
// ulp(x2 - x1) in Delta, which r = Delta / |x1| magnifies without bound as the
// reference approaches zero.) dd is returned signed, Delta = |dd| (the
// absolute value is applied where it is consumed).
template <bool RS>
__device__ __forceinline__ void pix3(float x0, float x1, float x2, float Cf, float& dd, float& rl) {
  const double a = (double)x2 - (double)x1;
  const double b = (double)x1 - (double)x0;
  dd = (float)(fabs(a) - fabs(b));
  pix_ratio<RS>(fabsf(dd), x1, Cf, rl);
}

// 1 / n^2 for a window of n in-image cells (n = rows * cols).
__device__ __forceinline__ float inv_count2(int y, int x, int H, int Hh, int Wh) {
  const int cy = min(y + H, Hh - 1) - max(y - H, 0) + 1;
  const int cx = min(x + H, Wh - 1) - max(x - H, 0) + 1;
  const int nn = cy * cx;
  return 1.0f / (float)(nn * nn);
}

// Window maximum by max3 tripling: t3[j] = max(a[j..j+2]), then each window
// of 2H+1 values is the max3 of at most three t3 terms (plus singles). The
// inputs are non-negative finite floats (Delta and its window maxima), whose
// bit patterns order like unsigned integers, so the maxima run on the bits
// (exact, no NaN canonicalisation) and agree with every other evaluation.
__device__ __forceinline__ uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) {
  // one v_max3_u32 (common-subexpression elimination would otherwise split
  // overlapping triples back into two-operand maxima)
  uint32_t r;
  asm("v_max3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

template <int H, int NOUT>
struct WinMax {
  static constexpr int L = 2 * H + 1;
  static constexpr int NIN = NOUT + 2 * H;
  __device__ static __forceinline__ void run(const float* af, float* o) {
    if constexpr (L == 1) {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) o[c] = af[c];
    } else {
      uint32_t a[NIN];
#pragma unroll
      for (int j = 0; j < NIN; ++j) a[j] = __float_as_uint(af[j]);
      uint32_t t3[NIN > 2 ? NIN - 2 : 1];
      int made = 0;  // t3[0 .. made) evaluated
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        // terms: t3 at c, c+3, ... while they fit, then singles
        uint32_t acc[8];
        int nt = 0, p = c;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (p + 2 <= c + L - 1) {
#pragma unroll
            for (; made <= p; ++made) t3[made] = umax3(a[made], a[made + 1], a[made + 2]);
            acc[nt++] = t3[p];
            p += 3;
          }
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (p <= c + L - 1) acc[nt++] = a[p++];
        uint32_t m = acc[0];
        int i = 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (i + 1 < nt) {
            m = umax3(m, acc[i], acc[i + 1]);
            i += 2;
          } else if (i < nt) {
            m = max(m, acc[i]);
            i += 1;
          }
        }
        o[c] = __uint_as_float(m);
      }
    }
  }
};

// Window maximum of |a| for register values produced by arithmetic (so no
// NaN canonicalisation is needed); the absolute value folds into the max3
// source modifiers. Same tripling as WinMax; max is exact in any order.
template <int H, int NOUT>
struct WinMaxAbs {
  static constexpr int L = 2 * H + 1;
  static constexpr int NIN = NOUT + 2 * H;
  __device__ static __forceinline__ float m3(float a, float b, float c) { return fmaxf(a, fmaxf(b, c)); }
  __device__ static __forceinline__ void run(const float* a, float* o) {
    if constexpr (L == 1) {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) o[c] = fabsf(a[c]);
    } else {
      float t3[NIN > 2 ? NIN - 2 : 1];
      int made = 0;  // t3[0 .. made) evaluated
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        float acc[8];
        int nt = 0, p = c;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (p + 2 <= c + L - 1) {
#pragma unroll
            for (; made <= p; ++made) t3[made] = m3(fabsf(a[made]), fabsf(a[made + 1]), fabsf(a[made + 2]));
            acc[nt++] = t3[p];
            p += 3;
          }
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (p <= c + L - 1) acc[nt++] = fabsf(a[p++]);
        float m = acc[0];
        int i = 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (i + 1 < nt) {
            m = m3(m, acc[i], acc[i + 1]);
            i += 2;
          } else if (i < nt) {
            m = fmaxf(m, acc[i]);
            i += 1;
          }
        }
        o[c] = m;
      }
    }
  }
};

template <typename T>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_ld<__half>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
}
template <>
__device__ __forceinline__ float buf_ld<bf16_t>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)) << 16);
}

// Buffer descriptor word 3 for gfx9 raw buffers; a lane offset at or beyond
// the record count reads 0, which masks columns outside the image.
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kRecords = 0x40000000;
constexpr int kOffMasked = 0x40000000;

// ---------------------------------------------------------------------------
// Streaming index kernel (sliding window). One workgroup owns 16 output rows
// x out_w output columns and walks every frame once, keeping the previous
// two frames of its (16 + 2H) x 256 input pixels in registers; the next
// frame is loaded while the current one is reduced.
// Per triple it writes FP64 moment partials (one per wave), the maximum q
// of every 64-cell row segment, optional q map rows, and (tile == 32) the
// per-column sums of the 32-row tiles for the frequency branch.
// ---------------------------------------------------------------------------
// Q: the call writes the q map (a compile-time switch: the map's stores and
// pointer would otherwise hold scalar registers the loop needs)
template <typename T, int H, bool RS, bool Q>
struct Stream {
  static constexpr int NR = kBand + 2 * H;
  static constexpr int NT = 16;            // outputs per horizontal task
  static constexpr int NH = NT + 2 * H;
  // LDS row layout for 32 banks (a half wave per cycle): column c at
  // c + ((c >> 5) & 7), row stride 264 = 8 (mod 16). A half wave writes 32
  // consecutive columns of one row (one 32-column run: 32 distinct banks); the
  // horizontal tasks of a half wave (2 rows x 16 chunks of 16 columns) read
  // 16 ch + i: run offsets 0..7 plus 8 per row and 16 per odd chunk give 32
  // distinct banks for every i.
  static constexpr int LDW = kLanes + 8;
  __device__ static __forceinline__ int lcol(int c) { return c + ((c >> 5) & 7); }

  // per-column tile sums of the group's columns, with 32 zero words on each
  // side so a 32-column tile piece is always 32 in-range reads
  static constexpr int CPAD = 32;
  struct Shared {
    float V[3][kBand][LDW];
    float col[3][kLanes + 2 * CPAD];  // also the per-wave maxima at the end
  };

  const StreamArgs& A;
  Shared& sh;
  const void *fbase, *fc0, *fc1;  // frame pointers of the call
  int lane, wave, bid, band, grp, y0, x0, nseg_row, voff;
  int64_t wg_off;
  // output offsets of the lane within one triple's plane (set once; the
  // triple adds a uniform base): segment maxima, q map, moment partials,
  // tile pieces
  uint32_t seg_lane, q_lane;
  uint32_t samp_lane;  // the lane's slot in the q sample, or ~0u
  int stat_lane, tile_lane;
  bool qvec;  // the lane's q-map chunk is whole and 16-byte aligned in every triple
  int qn;     // q-map cells of the lane's chunk inside the row
  bool all_rows, interior;
  float inv_full;
  int mxi;

  __device__ Stream(const StreamArgs& a, Shared& s) : A(a), sh(s) {}

  template <bool ALLROWS>
  __device__ __forceinline__ void load(int k, float* dst) {
    const T* fr = frame_ptr<T>(fbase, fc0, fc1, A.ncarry, A.plane, k);
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void*)(fr + wg_off), (short)0, kRecords, kRsrcWord3);
    int pitch = A.W * (int)sizeof(T);
    // keep the row offsets in one running scalar instead of a hoisted table
    asm volatile("" : "+s"(pitch));
    int so = 0;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int y = y0 - H + i;
      if (ALLROWS || (y >= 0 && y < A.H))
        dst[i] = buf_ld<T>(r, voff, so);
      else
        dst[i] = 0.0f;
      so += pitch;
    }
  }

  // One frame: X0, P, C hold frames k-2, k-1, k; X0 becomes the load target
  // of frame k+1 (the three rotate between calls).
  template <bool ALLROWS>
  __device__ __forceinline__ void step(int k, float* X0, const float* P, const float* C) {
    // running maximum on the signed-int view of the bits: it orders every
    // positive float correctly and maps non-positive values below them, which
    // is all max(., C) with C > 0 needs
#pragma unroll
    // (own rows only: halo rows belong to the neighbouring bands; halo
    // columns repeat pixels of the neighbouring groups, harmless for a max)
    for (int i = H; i + 1 < H + kBand; i += 2) mxi = max(mxi, max(__float_as_int(C[i]), __float_as_int(C[i + 1])));
    float dl[NR], rl[NR];
    if (k >= 2) {
#pragma unroll
      for (int i = 0; i < NR; ++i) pix3<RS>(X0[i], P[i], C[i], A.Cf, dl[i], rl[i]);
    }
    // the next frame's loads go straight into X0 (after the last frame the
    // same frame is re-read from cache: an unconditional load avoids copies)
    load<ALLROWS>(k + 1 < A.n ? k + 1 : k, X0);
    if (k < 2) return;
    const int s = k - 2;
    // vertical windows, one quantity at a time (each goes to LDS at once, so
    // only one set of window temporaries is live); per-column tile pieces
    // (sum and maximum over the band's own 16 rows) for the frequency branch
    const int ox = lane - H;
    const bool colp = A.tile_part && ox >= 0 && ox < A.out_w;
    {
      float v[kBand], t[kBand / 8];
      Win<H, kBand, false, true>::run(dl, v, t);
#pragma unroll
      for (int c = 0; c < kBand; ++c) sh.V[0][c][lcol(lane)] = v[c];
      if (colp) sh.col[0][CPAD + ox] = t[0] + t[1];
    }
    {
      float v[kBand];
      WinMaxAbs<H, kBand>::run(dl, v);
#pragma unroll
      for (int c = 0; c < kBand; ++c) sh.V[1][c][lcol(lane)] = v[c];
      if (colp) {
        // maximum over rows 0..15 from windows that tile them (2H + 1 <= 16)
        float m;
        if constexpr (2 * H + 1 <= kBand) {
          constexpr int WW = 2 * H + 1;
          m = v[H];
#pragma unroll
          for (int c = H + WW; c < kBand - 1 - H; c += WW) m = fmaxf(m, v[c]);
          m = fmaxf(m, v[kBand - 1 - H]);
        } else {
          m = fabsf(dl[H]);
#pragma unroll
          for (int i = 1; i < kBand; ++i) m = fmaxf(m, fabsf(dl[H + i]));
        }
        sh.col[1][CPAD + ox] = m;
      }
    }
    {
      float v[kBand], t[kBand / 8];
      Win<H, kBand, false>::run(rl, v, t);
#pragma unroll
      for (int c = 0; c < kBand; ++c) sh.V[2][c][lcol(lane)] = v[c];
      if (colp) sh.col[2][CPAD + ox] = t[0] + t[1];
    }
    __syncthreads();
    // horizontal: lane -> (row r, 16-column chunk ch)
    const int r = lane >> 4, ch = lane & 15;
    const int y = y0 + r;
    const int xc = x0 + NT * ch;
    const bool chv = (NT * ch < A.out_w) && (xc < A.W) && (y < A.H);
    // column 16 ch + i of the padded layout: cb + i for i < 16, cb2 + i past
    // the chunk (the next run for odd ch). The last chunk's columns 256.. read
    // words 256..263 of the row (bank-aligned with the rest; they only feed
    // outputs outside the group).
    const int cb = chv ? 16 * ch + (ch >> 1) : 0;
    const int cb2 = chv ? cb + (ch & 1) - (ch == 15 ? 8 : 0) : 0;
    // horizontal windows, one quantity at a time; the product is formed as
    // the factors arrive: pv = (sum * max) * sum_r, the association of the
    // exact recompute
    float pv[NT];
    {
      float t[NT];
      {
        float h[NH], os[NT];
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = sh.V[0][r][(i < 16 ? cb : cb2) + i];
        Win<H, NT, false>::run(h, os, nullptr);
#pragma unroll
        for (int c = 0; c < NT; ++c) t[c] = os[c];
      }
      {
        float h[NH], om[NT];
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = sh.V[1][r][(i < 16 ? cb : cb2) + i];
        WinMax<H, NT>::run(h, om);
#pragma unroll
        for (int c = 0; c < NT; ++c) t[c] = t[c] * om[c];
      }
      {
        float h[NH], orr[NT];
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = sh.V[2][r][(i < 16 ? cb : cb2) + i];
        Win<H, NT, false>::run(h, orr, nullptr);
#pragma unroll
        for (int c = 0; c < NT; ++c) pv[c] = t[c] * orr[c];
      }
    }
    float qv[NT];
    // FP64 moments: q^2 of a float is exact in double, so a constant map
    // gives exactly zero variance
    double s1 = 0.0, s2 = 0.0;
    float gmax = -INFINITY;
    // the map-writing form skips the moments when the call does not use them
    // (robust spread): no partials buffer
    const bool mom = !Q || A.stat_part != nullptr;
    if (interior) {
      // every chunk but the 16th is fully inside the image: no per-cell masks,
      // the idle chunk is dropped once per lane. The constant 1/n^2 is applied
      // after the reductions: q = p * inv with p = (S max) R, and rounding
      // p * inv is monotone, so max q = (max p) * inv exactly.
      if (mom) {
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          const float pq = pv[c];
          const double pd = (double)pq;
          s1 += pd;
          s2 = fma(pd, pd, s2);
          gmax = fmaxf(gmax, pq);
        }
      } else {
#pragma unroll
        for (int c = 0; c < NT; ++c) gmax = fmaxf(gmax, pv[c]);
      }
      const double id = (double)inv_full;
      s1 *= id;
      s2 *= id * id;
      gmax *= inv_full;
      if constexpr (Q) {
#pragma unroll
        for (int c = 0; c < NT; ++c) qv[c] = pv[c] * inv_full;
      }
      if (!chv) {
        s1 = 0.0;
        s2 = 0.0;
        gmax = -INFINITY;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const int x = xc + c;
        const bool v = chv && x < A.W;
        const float q = pv[c] * inv_count2(y, x, H, A.H, A.W);
        qv[c] = q;
        const double qm = v ? (double)q : 0.0;
        s1 += qm;
        s2 = fma(qm, qm, s2);
        gmax = v ? fmaxf(gmax, q) : gmax;
      }
    }
    // 64-cell segments = 4 consecutive chunks = one lane quad
    gmax = fmaxf(gmax, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(gmax), 0xB1, 0xF, 0xF, false)));
    gmax = fmaxf(gmax, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(gmax), 0x4E, 0xF, 0xF, false)));
    if ((ch & 3) == 0 && y < A.H && xc < A.W && NT * ch < A.out_w)
      A.seg_max[(int64_t)s * ((int64_t)A.H * nseg_row) + seg_lane] = gmax;
    if (Q && chv) {
      float* dst = A.qmap + (int64_t)s * A.plane + q_lane;
      if (qvec) {
        // whole chunk inside the row, 16-byte aligned: four 16-byte stores,
        // non-temporal (the map is read back by a later kernel, not by this one)
#pragma unroll
        for (int c = 0; c < NT; c += 4)
          __builtin_nontemporal_store(fitrig_v4f{qv[c], qv[c + 1], qv[c + 2], qv[c + 3]},
                                      reinterpret_cast<fitrig_v4f*>(dst + c));
      } else {
#pragma unroll
        for (int c = 0; c < NT; ++c)
          if (c < qn) dst[c] = qv[c];
      }
    }
    if (Q && samp_lane != ~0u) A.qsamp[(int64_t)s * A.samp_S + samp_lane] = ord_key(qv[0]);
    if (mom) {
      const double a1 = row_sum_f64(s1);
      const double a2 = row_sum_f64(s2);
      if ((lane & 15) == 15) {
        double* sp = A.stat_part + ((int64_t)s * gridDim.x + bid) * 32 + stat_lane;
        sp[0] = a1;
        sp[1] = a2;
      }
    }
    if (A.tile_part) {
      // job = (quantity qd, piece p) on 8 lanes; lane sub sums columns
      // sub, sub + 8, sub + 16, sub + 24 of the 32 columns of tile x0/32 + p
      // (zeros outside the group or the image), then the 8 lanes combine by
      // DPP (fixed order). The four jobs of a half wave start at different
      // 8-column segments, so each read touches 32 distinct banks.
      const int job = lane >> 3, sub = lane & 7;
      const int qd = job / kPieces, p = job - kPieces * (job / kPieces);
      const int qs = qd < 3 ? qd : 0;
      const int c0 = (x0 / 32 + p) * 32 - x0 + sub;  // >= -31
      const float* cv = &sh.col[qs][CPAD + c0];
      const int rot = job & 3;
      const float v0 = cv[8 * (rot & 3)], v1 = cv[8 * ((rot + 1) & 3)];
      const float v2 = cv[8 * ((rot + 2) & 3)], v3 = cv[8 * ((rot + 3) & 3)];
      float sm = (v0 + v1) + (v2 + v3);
      uint32_t mb = umax3(__float_as_uint(v0), __float_as_uint(v1), max(__float_as_uint(v2), __float_as_uint(v3)));
      sm += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sm), 0xB1, 0xF, 0xF, false));
      mb = max(mb, (uint32_t)__builtin_amdgcn_mov_dpp((int)mb, 0xB1, 0xF, 0xF, false));
      sm += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sm), 0x4E, 0xF, 0xF, false));
      mb = max(mb, (uint32_t)__builtin_amdgcn_mov_dpp((int)mb, 0x4E, 0xF, 0xF, false));
      sm += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(sm), 0x141, 0xF, 0xF, false));
      mb = max(mb, (uint32_t)__builtin_amdgcn_mov_dpp((int)mb, 0x141, 0xF, 0xF, false));
      if (sub == 0 && qd < 3)
        A.tile_part[(int64_t)s * ((int64_t)A.nbands * A.ncol * kPieces * 3) + tile_lane] =
            (double)(qd == 1 ? __uint_as_float(mb) : sm);
    }
    __syncthreads();
  }
};

template <typename T, int H, bool RS, bool Q>
__global__ __launch_bounds__(kLanes) void k_stream(StreamArgs A) {
  using S = Stream<T, H, RS, Q>;
  __shared__ typename S::Shared sh;
  S st(A, sh);
  st.fbase = A.cd->base;
  st.fc0 = A.cd->carry0;
  st.fc1 = A.cd->carry1;
  st.lane = threadIdx.x;
  st.wave = st.lane >> 6;
  tile_of(xcd_remap(blockIdx.x, gridDim.x), A.nbands, A.ncol, A.band_block, st.band, st.grp);
  st.bid = st.band * A.ncol + st.grp;
  st.y0 = st.band * kBand;
  st.x0 = st.grp * A.out_w;
  const int xin = st.x0 - H + st.lane;
  const bool colv = (st.lane < A.out_w + 2 * H) && xin >= 0 && xin < A.W;
  st.voff = colv ? st.lane * (int)sizeof(T) : kOffMasked;
  st.wg_off = (int64_t)(st.y0 - H) * A.W + (st.x0 - H);
  st.all_rows = (st.y0 - H >= 0) && (st.y0 + kBand + H <= A.H);
  st.interior = st.all_rows && (st.x0 - H >= 0) && (st.x0 + A.out_w - 1 + H < A.W);
  st.nseg_row = A.ncol * kSegsPerGroup;
  {
    const int r = st.lane >> 4, ch = st.lane & 15;  // horizontal task of the lane
    const int job = st.lane >> 3;                   // tile-piece job of the lane
    const int qd = job / kPieces, p = job - kPieces * (job / kPieces);
    st.seg_lane = (uint32_t)(st.y0 + r) * (uint32_t)st.nseg_row + (uint32_t)(st.grp * kSegsPerGroup + (ch >> 2));
    st.q_lane = (uint32_t)(st.y0 + r) * (uint32_t)A.W + (uint32_t)(st.x0 + S::NT * ch);
    // the map is 16-byte aligned; a triple's plane keeps the alignment when
    // H W is a multiple of 4
    st.qn = max(0, min(S::NT, A.W - (st.x0 + S::NT * ch)));
    st.qvec = Q && st.qn == S::NT && A.plane % 4 == 0 && st.q_lane % 4 == 0 && ((uintptr_t)A.qmap & 15) == 0;
    st.samp_lane = ~0u;
    if (Q && A.qsamp && r == 0 && st.band % A.samp_bstride == 0 && S::NT * ch < A.out_w &&
        st.x0 + S::NT * ch < A.W)
      st.samp_lane = (uint32_t)((st.band / A.samp_bstride) * A.samp_nch + st.grp * A.samp_cpg + ch);
    st.stat_lane = (st.lane >> 4) * 2;
    st.tile_lane = ((st.band * A.ncol + st.grp) * kPieces + p) * 3 + qd;
  }
  constexpr int WN = (2 * H + 1) * (2 * H + 1);
  st.inv_full = 1.0f / (float)(WN * WN);
  st.mxi = INT32_MIN;
  for (int i = st.lane; i < 3 * kBand * S::LDW; i += kLanes) (&sh.V[0][0][0])[i] = 0.0f;
  for (int i = st.lane; i < 3 * (kLanes + 2 * S::CPAD); i += kLanes) (&sh.col[0][0])[i] = 0.0f;
  __syncthreads();
  // frames k-2, k-1, k rotate through fa, fb, fc
  float fa[S::NR], fb[S::NR], fc[S::NR];
#pragma unroll
  for (int i = 0; i < S::NR; ++i) {
    fa[i] = 0.0f;
    fb[i] = 0.0f;
  }
  if (st.all_rows) {
    st.template load<true>(0, fc);
    for (int k = 0; k < A.n; k += 3) {
      st.template step<true>(k, fa, fb, fc);
      if (k + 1 < A.n) st.template step<true>(k + 1, fb, fc, fa);
      if (k + 2 < A.n) st.template step<true>(k + 2, fc, fa, fb);
    }
  } else {
    st.template load<false>(0, fc);
    for (int k = 0; k < A.n; k += 3) {
      st.template step<false>(k, fa, fb, fc);
      if (k + 1 < A.n) st.template step<false>(k + 1, fb, fc, fa);
      if (k + 2 < A.n) st.template step<false>(k + 2, fc, fa, fb);
    }
  }
  int mx = st.mxi;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
  // the last frame ended with a barrier: col is free
  int* wmx = reinterpret_cast<int*>(&sh.col[0][0]);
  if ((st.lane & 63) == 0) wmx[st.wave] = mx;
  __syncthreads();
  if (st.lane == 0) {
    int m = wmx[0];
    for (int w = 1; w < kLanes / 64; ++w) m = max(m, wmx[w]);
    // m is the largest value when any is positive, else some value <= 0
    atomicMax(A.max_key, ord_key(__int_as_float(m)));
  }
}

// ---------------------------------------------------------------------------
// Tile-mode kernel: one workgroup per (256-column chunk, tile row, triple).
// Each lane owns a column, reads the three frames of the triple over the
// tile row and accumulates sum Delta, max Delta and sum r in FP64; per tile
// piece of the chunk the columns are summed in order.
// ---------------------------------------------------------------------------
template <typename T, bool RS>
__global__ __launch_bounds__(kLanes) void k_tile(TileArgs A) {
  __shared__ double sCol[3][kLanes];
  __shared__ float sMax[kLanes / 64];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x, ty = blockIdx.y, s = blockIdx.z;
  const int x = chunk * kLanes + lane;
  const bool cv = x < A.W;
  const void *fb = A.cd->base, *fc0 = A.cd->carry0, *fc1 = A.cd->carry1;
  const T* f0 = frame_ptr<T>(fb, fc0, fc1, A.ncarry, A.plane, s);
  const T* f1 = frame_ptr<T>(fb, fc0, fc1, A.ncarry, A.plane, s + 1);
  const T* f2 = frame_ptr<T>(fb, fc0, fc1, A.ncarry, A.plane, s + 2);
  const int ya = ty * A.tile;
  const int yb = min(ya + A.tile, A.H);
  double sd = 0.0, md = 0.0, sr = 0.0;
  float mx = -INFINITY;
  if (cv) {
    for (int y = ya; y < yb; ++y) {
      const int64_t o = (int64_t)y * A.W + x;
      const float a = to_f<T>(f0[o]), b = to_f<T>(f1[o]), c = to_f<T>(f2[o]);
      mx = fmaxf(mx, fmaxf(a, fmaxf(b, c)));
      float dl, rl;
      pix3<RS>(a, b, c, A.Cf, dl, rl);
      dl = fabsf(dl);
      sd += (double)dl;
      md = fmax(md, (double)dl);
      sr += (double)rl;
    }
  }
  sCol[0][lane] = sd;
  sCol[1][lane] = md;
  sCol[2][lane] = sr;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((lane & 63) == 0) sMax[lane >> 6] = mx;
  __syncthreads();
  const int x0 = chunk * kLanes;
  for (int job = lane; job < A.pieces * 3; job += kLanes) {
    const int p = job / 3, qd = job - 3 * (job / 3);
    const int tx = x0 / A.tile + p;
    const int ca = max(tx * A.tile, x0) - x0;
    const int cb = min(min(tx * A.tile + A.tile, x0 + kLanes), A.W) - x0;
    double acc = 0.0;
    for (int c = ca; c < cb; ++c) acc = (qd == 1) ? fmax(acc, sCol[1][c]) : acc + sCol[qd][c];
    A.tile_part[((((int64_t)s * gridDim.y + ty) * A.nchunk + chunk) * A.pieces + p) * 3 + qd] = acc;
  }
  if (lane == 0) {
    float m = sMax[0];
    for (int w = 1; w < kLanes / 64; ++w) m = fmaxf(m, sMax[w]);
    atomicMax(A.max_key, ord_key(m));
  }
}

// ---------------------------------------------------------------------------
// Streaming tile-mode kernel (tile a power of two <= 32): one workgroup per (band of tpb
// whole tile rows, chunk of whole tiles); each lane owns a column, keeps the
// previous two frames of the band's rows in registers and walks every frame
// once. Per triple it accumulates, per tile
// row of the band, the column's sum Delta, max Delta and sum r (FP32 over at
// most 32 rows). For tiles of 16 and 32 the TILE lanes of a tile then combine
// their columns by a fixed butterfly of shuffles (sums in FP64, maximum
// exact), with no LDS and no barrier per triple; for smaller tiles the
// partials go through LDS and one job per tile sums its columns in FP64. The
// tile's q (Eq. (6) with the in-image count) goes to the cube.
// ---------------------------------------------------------------------------
constexpr int kTileTpbMax = 8;    // tile rows per band
template <typename T, int TILE, bool RS>
__global__ __launch_bounds__(kLanes) void k_tile_stream(TileStreamArgs A) {
  constexpr int TPB = (32 / TILE) < kTileTpbMax ? (32 / TILE) : kTileTpbMax;
  constexpr int ROWS = TPB * TILE;
  constexpr int TPC = kLanes / TILE;        // whole tiles per chunk
  static_assert(TILE <= 64 && (TILE & (TILE - 1)) == 0, "a tile's lanes lie in one wave");
  __shared__ float col[TILE >= 16 ? 1 : TPB][3][kLanes];
  __shared__ int mxs[kLanes / 64];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x % A.nchunk, band = blockIdx.x / A.nchunk;
  const int x = chunk * kLanes + lane;
  const bool cv = x < A.W;
  const int y0 = band * ROWS;
  int mxi = INT32_MIN;
  const void *fb = A.cd->base, *fc0 = A.cd->carry0, *fc1 = A.cd->carry1;
  // reads are unconditional: one buffer descriptor per frame from the band's
  // first row (32 rows fit its 2^30 bytes for every accepted width), columns
  // past the image masked to zero by the descriptor, rows past the last one
  // read that row again (a running scalar offset that stops there); the terms
  // of cells outside the image are zeroed where they are used, and a repeated
  // pixel leaves the maximum alone
  const int voff = cv ? lane * (int)sizeof(T) : kOffMasked;
  const int last = A.H - 1 - y0;  // last in-image row of the band (relative)
  auto load = [&](int k, float* dst) {
    const T* fr = frame_ptr<T>(fb, fc0, fc1, A.ncarry, A.plane, k);
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(fr + (int64_t)y0 * A.W + (int64_t)chunk * kLanes), (short)0, kRecords, kRsrcWord3);
    int pitch = A.W * (int)sizeof(T);
    asm volatile("" : "+s"(pitch));
    int so = 0;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      dst[i] = buf_ld<T>(r, voff, so);
      so += i < last ? pitch : 0;
    }
  };
  // frames k-2, k-1, k in X0, P, C; the next frame is read into N while this
  // one is reduced (the four arrays rotate between calls)
  auto step = [&](int k, const float* X0, const float* P, const float* C, float* N) {
    load(k + 1 < A.n ? k + 1 : k, N);
    float sd[TPB], md[TPB], sr[TPB];
#pragma unroll
    for (int t = 0; t < TPB; ++t) {
      sd[t] = 0.0f;
      md[t] = 0.0f;
      sr[t] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) mxi = max(mxi, __float_as_int(C[i]));
    if (k < 2) return;
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const bool in = cv && y0 + i < A.H;
      float dl, rl;
      pix3<RS>(X0[i], P[i], C[i], A.Cf, dl, rl);
      dl = in ? fabsf(dl) : 0.0f;
      rl = in ? rl : 0.0f;
      sd[i / TILE] += dl;
      md[i / TILE] = fmaxf(md[i / TILE], dl);
      sr[i / TILE] += rl;
    }
    const int s = k - 2;
    if constexpr (TILE >= 16) {
      // few tiles per chunk: the TILE lanes of a tile combine their columns
      const int j = lane / TILE;  // tile of the chunk
      const int ca = j * TILE;
      const int cb = min(ca + TILE, A.W - chunk * kLanes);  // in-image columns end
#pragma unroll
      for (int t = 0; t < TPB; ++t) {
        double a0 = (double)sd[t], a2 = (double)sr[t];
        float a1 = md[t];
#pragma unroll
        for (int off = 1; off < TILE; off <<= 1) {
          a0 += __shfl_xor(a0, off);
          a2 += __shfl_xor(a2, off);
          a1 = fmaxf(a1, __shfl_xor(a1, off));
        }
        const int ty = band * TPB + t;
        const int tx = chunk * TPC + j;
        if ((lane & (TILE - 1)) == 0 && ty < A.Ty && tx < A.Tx) {
          const double n = (double)(min(ty * TILE + TILE, A.H) - ty * TILE) * (double)(cb - ca);
          const double v = (a0 / n) * (double)a1 * (a2 / n);
          const int64_t o = ((int64_t)s * A.Ty + ty) * A.Tx + tx;
          A.cube[o] = v;
          A.cube_f[o] = (float)v;
        }
      }
    } else {
      // many tiles per chunk: per-column partials through LDS, one job per
      // (tile row, tile) summing its columns
      __syncthreads();  // the previous triple's jobs have read col
#pragma unroll
      for (int t = 0; t < TPB; ++t) {
        col[t][0][lane] = sd[t];
        col[t][1][lane] = md[t];
        col[t][2][lane] = sr[t];
      }
      __syncthreads();
      // one job per (tile row of the band, tile of the chunk)
      for (int job = lane; job < TPB * TPC; job += kLanes) {
        const int t = job / TPC, j = job - t * TPC;
        const int ty = band * TPB + t;
        const int tx = chunk * TPC + j;
        if (ty >= A.Ty || tx >= A.Tx) continue;
        const int ca = j * TILE;
        const int cb = min(ca + TILE, A.W - chunk * kLanes);
        double a0 = 0.0, a2 = 0.0;
        float a1 = 0.0f;
        for (int c = ca; c < cb; ++c) {
          a0 += (double)col[t][0][c];
          a1 = fmaxf(a1, col[t][1][c]);
          a2 += (double)col[t][2][c];
        }
        const double n = (double)(min(ty * TILE + TILE, A.H) - ty * TILE) * (double)(cb - ca);
        const double v = (a0 / n) * (double)a1 * (a2 / n);
        const int64_t o = ((int64_t)s * A.Ty + ty) * A.Tx + tx;
        A.cube[o] = v;
        A.cube_f[o] = (float)v;
      }
    }
  };
  float F0[ROWS], F1[ROWS], F2[ROWS], F3[ROWS];
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    F2[i] = 0.0f;
    F3[i] = 0.0f;
  }
  load(0, F0);
  for (int k = 0; k < A.n; k += 4) {
    step(k, F2, F3, F0, F1);
    if (k + 1 < A.n) step(k + 1, F3, F0, F1, F2);
    if (k + 2 < A.n) step(k + 2, F0, F1, F2, F3);
    if (k + 3 < A.n) step(k + 3, F1, F2, F3, F0);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mxi = max(mxi, __shfl_xor(mxi, off));
  if ((lane & 63) == 0) mxs[lane >> 6] = mxi;
  __syncthreads();
  if (lane == 0) {
    int m = mxs[0];
    for (int w = 1; w < kLanes / 64; ++w) m = max(m, mxs[w]);
    atomicMax(A.max_key, ord_key(__int_as_float(m)));
  }
}


// Stack maximum when no pass over the stack produced it (frequency branch
// only with too few triples): the new frames of the call.
template <typename T>
__global__ __launch_bounds__(256) void k_stack_max(const CallDev* cd, int64_t n, uint32_t* max_key) {
  __shared__ float sh[256];
  const T* p = (const T*)cd->base;
  float m = -INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, to_f<T>(p[i]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(max_key, ord_key(sh[0]));
}

// z > tau of Eqs. (9), (12) on q (or eta), in double precision.
__device__ __forceinline__ bool zsel(float q, double mu, double sg, double tau) {
  return ((double)q - mu) / sg > tau;
}

// Exact q of the cells of each selected segment, recomputed with the same
// arithmetic as k_stream; mask of z > tau.
template <typename T, int H, bool RS>
__global__ __launch_bounds__(64) void k_recompute(RecomputeArgs R) {
  constexpr int NV = 8 + 2 * H;
  __shared__ float sv[3][64 + 32 + 2 * kMaxHalo];
  const int lane = threadIdx.x;
  const SegLayout L = R.L;
  const void *base = R.cd->base, *c0 = R.cd->carry0, *c1 = R.cd->carry1;
  const double tau = R.cd->tau;
  const int ncarry = R.ncarry, Hh = R.H, Wh = R.W;
  const int64_t plane = R.plane;
  const float Cf = R.Cf;
  const int64_t cap = R.cap;
  const double* mu = R.mu;
  const double* sigma = R.sigma;
  uint64_t* seg_mask = R.mask;
  float* cell_q = R.cell_q;
  const int64_t* seg_entry = R.seg_entry;
  int64_t nsel = R.nsel[0];
  if (nsel > cap) nsel = cap;
  for (int64_t i = blockIdx.x; i < nsel; i += gridDim.x) {
    const int64_t e = seg_entry[i];
    const int g = (int)(e % L.nseg_row);
    const int64_t row = e / L.nseg_row;
    const int y = (int)(row % L.Ho);
    const int s = (int)(row / L.Ho);
    const int xs = seg_x0(L, g), wd = seg_width(L, g);
    const int cmin = 8 * (xs / 8) - H;
    const int ncols = 8 * ((xs + wd - 1) / 8) + 7 + H - cmin + 1;
    const int by = 8 * (y / 8);
    const T* f0 = frame_ptr<T>(base, c0, c1, ncarry, plane, s);
    const T* f1 = frame_ptr<T>(base, c0, c1, ncarry, plane, s + 1);
    const T* f2 = frame_ptr<T>(base, c0, c1, ncarry, plane, s + 2);
    // Vertical windows of row y, evaluated as output y - by of the 8-row
    // block (the association k_stream uses for that row). With the row a
    // compile-time index, the other outputs and the rows outside y's window
    // are never computed or read.
    // Reads are unconditional (indices clamped into the image) and out-of-image
    // pixels are zeroed after all of a column's reads are issued, so the reads
    // of the window's rows are in flight together.
    auto column = [&](auto CY) {
      constexpr int C = decltype(CY)::value;
      for (int cc = lane; cc < ncols; cc += 64) {
        const int col = cmin + cc;
        const bool colok = col >= 0 && col < Wh;
        const int colc = min(max(col, 0), Wh - 1);
        float ra[NV], rb[NV], rc[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const int yc = min(max(by - H + j, 0), Hh - 1);
          const int64_t o = (int64_t)yc * Wh + colc;
          ra[j] = ldg_f<T>(f0, o);
          rb[j] = ldg_f<T>(f1, o);
          rc[j] = ldg_f<T>(f2, o);
        }
        float dl[NV], rl[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
          const int yy = by - H + j;
          const bool ok = colok && yy >= 0 && yy < Hh;
          pix3<RS>(ok ? ra[j] : 0.0f, ok ? rb[j] : 0.0f, ok ? rc[j] : 0.0f, Cf, dl[j], rl[j]);
          dl[j] = fabsf(dl[j]);
        }
        float o8[8];
        Win<H, 8, false>::run(dl, o8, nullptr);
        sv[0][cc] = o8[C];
        WinMax<H, 8>::run(dl, o8);
        sv[1][cc] = o8[C];
        Win<H, 8, false>::run(rl, o8, nullptr);
        sv[2][cc] = o8[C];
      }
    };
    switch (y - by) {
      case 0: column(std::integral_constant<int, 0>{}); break;
      case 1: column(std::integral_constant<int, 1>{}); break;
      case 2: column(std::integral_constant<int, 2>{}); break;
      case 3: column(std::integral_constant<int, 3>{}); break;
      case 4: column(std::integral_constant<int, 4>{}); break;
      case 5: column(std::integral_constant<int, 5>{}); break;
      case 6: column(std::integral_constant<int, 6>{}); break;
      default: column(std::integral_constant<int, 7>{}); break;
    }
    __syncthreads();
    bool sel = false;
    float q = 0.0f;
    if (lane < wd) {
      const int x = xs + lane;
      const int bx = 8 * (x / 8);
      float hs[NV], hm[NV], hr[NV], os[8], om[8], orr[8];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const int ci = bx - H + j - cmin;
        hs[j] = sv[0][ci];
        hm[j] = sv[1][ci];
        hr[j] = sv[2][ci];
      }
      Win<H, 8, false>::run(hs, os, nullptr);
      WinMax<H, 8>::run(hm, om);
      Win<H, 8, false>::run(hr, orr, nullptr);
      const int c = x - bx;
      // same association as k_stream: ((sum * max) * sum_r) * 1/n^2
      const float inv = inv_count2(y, x, H, Hh, Wh);
      q = ((os[c] * om[c]) * orr[c]) * inv;
      sel = zsel(q, mu[s], sigma[s], tau);
    }
    const uint64_t m = __ballot(sel);
    cell_q[i * 64 + lane] = q;
    if (lane == 0) seg_mask[i] = m;
    __syncthreads();
  }
}

}  // namespace fitrig
