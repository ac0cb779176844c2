// FITrig device code for CDNA4 (gfx950): streaming index kernel, tile-mode
// kernel, statistics, exact selection by recompute, union-find components,
// image-frequency transform and radix selection for the robust spread.
//
// Method (Li, Adamek & Armour, arXiv 2509.21754):
//   Delta = ||x(s+2)-x(s+1)| - |x(s+1)-x(s)||, reference x(s+1)  Sec. 2.2.4, Eqs. (3)-(5)
//   r = min(Delta / |x_hat|, 1), x_hat = C where x(s+1) == 0       Eqs. (4)-(5)
//   q = mean(Delta) max(Delta) mean(r) over the window / tile       Eq. (2), Eq. (6)
//   z = (q - mean q) / std q per triple, select z > tau             Sec. 2.4.1, Eqs. (8)-(9)
//   eta = h(|DFT_s[q(s) - mean q]|) per tile, z on eta               Sec. 2.4.2, Eqs. (10)-(12)
//
// Window sums use 8-row / 8-column blocks aligned to absolute multiples of
// 8: a window [L, R] is suffix(block of L) + totals of whole blocks +
// prefix(block of R), with prefix / suffix defined by fixed left-to-right /
// right-to-left recurrences. The value of a cell therefore depends only on
// its absolute position, so the exact selection kernel recomputes it to the
// same bits as the streaming kernel.
#include <hip/hip_fp16.h>
#include <math.h>
#include <stdint.h>

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
//   (sum / max of the 8 positions [8j, 8j+7]).
template <int H, int NOUT, bool MAXOP>
struct Win {
  static constexpr int NIN = NOUT + 2 * H;
  static constexpr int MLO = -1;
  static constexpr int MHI = fdiv8(NOUT - 1 + H);
  static constexpr int NB = MHI - MLO + 1;
  __device__ static __forceinline__ float op(float x, float y) { return MAXOP ? fmaxf(x, y) : x + y; }

  __device__ static __forceinline__ void run(const float* a, float* o, float* tot) {
    if constexpr (H <= 2) {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        float s = a[c];
#pragma unroll
        for (int j = 1; j <= 2 * H; ++j) s = op(s, a[c + j]);
        o[c] = s;
      }
      if (tot) {
#pragma unroll
        for (int j = 0; j < NOUT / 8; ++j) {
          float s = a[H + 8 * j];
#pragma unroll
          for (int p = 1; p < 8; ++p) s = op(s, a[H + 8 * j + p]);
          tot[j] = s;
        }
      }
    } else {
      float pre[NB][8] = {};
      float suf[NB][8] = {};
#pragma unroll
      for (int mi = 0; mi < NB; ++mi) {
        const int m = mi + MLO;
        const int st = H + 8 * m;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const int idx = st + p;
          if (st >= 0 && idx < NIN) pre[mi][p] = (p == 0) ? a[idx] : op(pre[mi][p - 1], a[idx]);
        }
#pragma unroll
        for (int p = 7; p >= 0; --p) {
          const int idx = st + p;
          if (st + 7 < NIN && idx >= 0) suf[mi][p] = (p == 7) ? a[idx] : op(a[idx], suf[mi][p + 1]);
        }
      }
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        const int L = c - H, R = c + H;
        const int bs = fdiv8(L), be = fdiv8(R);
        const int ps = L - 8 * bs, pe = R - 8 * be;
        if (bs == be) {
          o[c] = (ps == 0) ? pre[bs - MLO][pe] : suf[bs - MLO][ps];
        } else {
          float s = suf[bs - MLO][ps];
#pragma unroll
          for (int m = bs + 1; m < be; ++m) s = op(s, pre[m - MLO][7]);
          o[c] = op(s, pre[be - MLO][pe]);
        }
      }
      if (tot) {
#pragma unroll
        for (int j = 0; j < NOUT / 8; ++j) tot[j] = pre[j - MLO][7];
      }
    }
  }
};

// Maximum over each aligned group of 8 lanes (DPP quad xor 1, xor 2, half-row mirror).
__device__ __forceinline__ float group8_max(float v) {
  float t = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v = fmaxf(v, t);
  t = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  v = fmaxf(v, t);
  t = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  return fmaxf(v, t);
}

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
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
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

template <bool RS>
__device__ __forceinline__ void pix_terms(float d_new, float d_old, float ref, float Cf, float& dl, float& rl) {
  dl = fabsf(fabsf(d_new) - fabsf(d_old));
  pix_ratio<RS>(dl, ref, Cf, rl);
}

// Same terms, Delta returned signed: Delta = |dd| (the absolute value is
// applied where it is consumed, as a source modifier).
template <bool RS>
__device__ __forceinline__ void pix_terms_signed(float d_new, float d_old, float ref, float Cf, float& dd,
                                                 float& rl) {
  dd = fabsf(d_new) - fabsf(d_old);
  pix_ratio<RS>(fabsf(dd), ref, Cf, rl);
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
#pragma unroll
      for (int j = 0; j + 2 < NIN; ++j) t3[j] = umax3(a[j], a[j + 1], a[j + 2]);
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        // terms: t3 at c, c+3, ... while they fit, then singles
        uint32_t acc[8];
        int nt = 0, p = c;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (p + 2 <= c + L - 1) {
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
#pragma unroll
      for (int j = 0; j + 2 < NIN; ++j) t3[j] = m3(fabsf(a[j]), fabsf(a[j + 1]), fabsf(a[j + 2]));
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {
        float acc[8];
        int nt = 0, p = c;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (p + 2 <= c + L - 1) {
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
// frame and the previous difference of its (16 + 2H) x 256 input pixels in
// registers; the next frame is loaded while the current one is reduced.
// Per triple it writes FP64 moment partials (one per wave), the maximum q
// of every 64-cell row segment, optional q map rows, and (tile == 32) the
// per-column sums of the 32-row tiles for the frequency branch.
// ---------------------------------------------------------------------------
template <typename T, int H, bool RS>
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
    float col[3][kLanes + 2 * CPAD];
    int mx[kLanes / 64];
  };

  const StreamArgs& A;
  Shared& sh;
  int lane, wave, bid, band, grp, y0, x0, nseg_row, voff;
  int64_t wg_off;
  bool all_rows, interior;
  float inv_full;
  int mxi;

  __device__ Stream(const StreamArgs& a, Shared& s) : A(a), sh(s) {}

  template <bool ALLROWS>
  __device__ __forceinline__ void load(int k, float* dst) {
    const T* fr = frame_ptr<T>(A.base, A.carry0, A.carry1, A.ncarry, A.plane, k);
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

  // One frame: P holds frame k-1 (becomes the load target of frame k+1), C
  // holds frame k; DI holds the difference of frames k-1, k-2 and DO receives
  // the difference of frames k, k-1 (the two swap between calls).
  template <bool ALLROWS>
  __device__ __forceinline__ void step(int k, float* P, const float* C, const float* DI, float* DO) {
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
      for (int i = 0; i < NR; ++i) {
        DO[i] = C[i] - P[i];
        pix_terms_signed<RS>(DO[i], DI[i], P[i], A.Cf, dl[i], rl[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NR; ++i) DO[i] = C[i] - P[i];
    }
    // the next frame's loads go straight into P (after the last frame the
    // same frame is re-read from cache: an unconditional load avoids copies)
    load<ALLROWS>(k + 1 < A.n ? k + 1 : k, P);
    if (k < 2) return;
    const int s = k - 2;
    {
      float vs[kBand], vm[kBand], vr[kBand], ts[kBand / 8], tr[kBand / 8];
      float al[NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) al[i] = fabsf(dl[i]);
      Win<H, kBand, false>::run(al, vs, ts);
      WinMaxAbs<H, kBand>::run(dl, vm);
      Win<H, kBand, false>::run(rl, vr, tr);
#pragma unroll
      for (int c = 0; c < kBand; ++c) {
        sh.V[0][c][lcol(lane)] = vs[c];
        sh.V[1][c][lcol(lane)] = vm[c];
        sh.V[2][c][lcol(lane)] = vr[c];
      }
      if (A.tile_part) {
        const int ox = lane - H;
        if (ox >= 0 && ox < A.out_w) {
          float m = fabsf(dl[H]);
#pragma unroll
          for (int i = 1; i < kBand; ++i) m = fmaxf(m, fabsf(dl[H + i]));
          sh.col[0][CPAD + ox] = ts[0] + ts[1];
          sh.col[1][CPAD + ox] = m;
          sh.col[2][CPAD + ox] = tr[0] + tr[1];
        }
      }
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
    float os[NT], om[NT], orr[NT];
    {
      // all three rows of inputs are requested before the windows run
      float h0[NH], h1[NH], h2[NH];
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        const int ci = (i < 16 ? cb : cb2) + i;
        h0[i] = sh.V[0][r][ci];
        h1[i] = sh.V[1][r][ci];
        h2[i] = sh.V[2][r][ci];
      }
      Win<H, NT, false>::run(h0, os, nullptr);
      WinMax<H, NT>::run(h1, om);
      Win<H, NT, false>::run(h2, orr, nullptr);
    }
    float qv[NT];
    // FP64 moments: q^2 of a float is exact in double, so a constant map
    // gives exactly zero variance
    double s1 = 0.0, s2 = 0.0;
    float gmax = -INFINITY;
    if (interior) {
      // every chunk but the 16th is fully inside the image: no per-cell masks,
      // the idle chunk is dropped once per lane. The constant 1/n^2 is applied
      // after the reductions: q = p * inv with p = (S max) R, and rounding
      // p * inv is monotone, so max q = (max p) * inv exactly.
      float pv[NT];
#pragma unroll
      for (int c = 0; c < NT; ++c) {
        const float pq = (os[c] * om[c]) * orr[c];
        pv[c] = pq;
        const double pd = (double)pq;
        s1 += pd;
        s2 = fma(pd, pd, s2);
        gmax = fmaxf(gmax, pq);
      }
      const double id = (double)inv_full;
      s1 *= id;
      s2 *= id * id;
      gmax *= inv_full;
      if (A.qmap) {
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
        const float q = ((os[c] * om[c]) * orr[c]) * inv_count2(y, x, H, A.H, A.W);
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
      A.seg_max[((int64_t)s * A.H + y) * nseg_row + grp * kSegsPerGroup + (ch >> 2)] = gmax;
    if (A.qmap && chv) {
      float* dst = A.qmap + ((int64_t)s * A.H + y) * A.W + xc;
      if (xc + NT <= A.W && ((uintptr_t)dst & 15) == 0) {
        // whole chunk inside the row, 16-byte aligned: four 16-byte stores
#pragma unroll
        for (int c = 0; c < NT; c += 4)
          *reinterpret_cast<float4*>(dst + c) = make_float4(qv[c], qv[c + 1], qv[c + 2], qv[c + 3]);
      } else {
#pragma unroll
        for (int c = 0; c < NT; ++c)
          if (xc + c < A.W) dst[c] = qv[c];
      }
    }
    const double a1 = row_sum_f64(s1);
    const double a2 = row_sum_f64(s2);
    if ((lane & 15) == 15) {
      double* sp = A.stat_part + (((int64_t)s * gridDim.x + bid) * 16 + (lane >> 4)) * 2;
      sp[0] = a1;
      sp[1] = a2;
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
        A.tile_part[((((int64_t)s * A.nbands + band) * A.ncol + grp) * kPieces + p) * 3 + qd] =
            (double)(qd == 1 ? __uint_as_float(mb) : sm);
    }
    __syncthreads();
  }
};

template <typename T, int H, bool RS>
__global__ __launch_bounds__(kLanes) void k_stream(StreamArgs A) {
  using S = Stream<T, H, RS>;
  __shared__ typename S::Shared sh;
  S st(A, sh);
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
  constexpr int WN = (2 * H + 1) * (2 * H + 1);
  st.inv_full = 1.0f / (float)(WN * WN);
  st.mxi = INT32_MIN;
  for (int i = st.lane; i < 3 * kBand * S::LDW; i += kLanes) (&sh.V[0][0][0])[i] = 0.0f;
  for (int i = st.lane; i < 3 * (kLanes + 2 * S::CPAD); i += kLanes) (&sh.col[0][0])[i] = 0.0f;
  __syncthreads();
  float fa[S::NR], fb[S::NR], da[S::NR], db[S::NR];
#pragma unroll
  for (int i = 0; i < S::NR; ++i) {
    fa[i] = 0.0f;
    da[i] = 0.0f;
  }
  if (st.all_rows) {
    st.template load<true>(0, fb);
    for (int k = 0; k < A.n; k += 2) {
      st.template step<true>(k, fa, fb, da, db);
      if (k + 1 < A.n) st.template step<true>(k + 1, fb, fa, db, da);
    }
  } else {
    st.template load<false>(0, fb);
    for (int k = 0; k < A.n; k += 2) {
      st.template step<false>(k, fa, fb, da, db);
      if (k + 1 < A.n) st.template step<false>(k + 1, fb, fa, db, da);
    }
  }
  int mx = st.mxi;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
  if ((st.lane & 63) == 0) sh.mx[st.wave] = mx;
  __syncthreads();
  if (st.lane == 0) {
    int m = sh.mx[0];
    for (int w = 1; w < kLanes / 64; ++w) m = max(m, sh.mx[w]);
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
  const T* f0 = frame_ptr<T>(A.base, A.carry0, A.carry1, A.ncarry, A.plane, s);
  const T* f1 = frame_ptr<T>(A.base, A.carry0, A.carry1, A.ncarry, A.plane, s + 1);
  const T* f2 = frame_ptr<T>(A.base, A.carry0, A.carry1, A.ncarry, A.plane, s + 2);
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
      pix_terms<RS>(c - b, b - a, b, A.Cf, dl, rl);
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
// previous frame and the previous difference of the band's rows in
// registers and walks every frame once. Per triple it accumulates, per tile
// row of the band, the column's sum Delta, max Delta and sum r (FP32 over at
// most 32 rows), then one job per tile sums its columns in FP64 and writes
// the tile's q (Eq. (6) with the in-image count) to the cube.
// ---------------------------------------------------------------------------
constexpr int kTileTpbMax = 8;    // tile rows per band
template <typename T, int TILE, bool RS>
__global__ __launch_bounds__(kLanes) void k_tile_stream(TileStreamArgs A) {
  constexpr int TPB = (32 / TILE) < kTileTpbMax ? (32 / TILE) : kTileTpbMax;
  constexpr int ROWS = TPB * TILE;
  constexpr int TPC = kLanes / TILE;        // whole tiles per chunk
  __shared__ float col[TPB][3][kLanes];
  __shared__ int mxs[kLanes / 64];
  const int lane = threadIdx.x;
  const int chunk = blockIdx.x % A.nchunk, band = blockIdx.x / A.nchunk;
  const int x = chunk * kLanes + lane;
  const bool cv = x < A.W;
  const int y0 = band * ROWS;
  float P[ROWS], D[ROWS];
  int mxi = INT32_MIN;
#pragma unroll
  for (int i = 0; i < ROWS; ++i) {
    P[i] = 0.0f;
    D[i] = 0.0f;
  }
  for (int k = 0; k < A.n; ++k) {
    const T* fr = frame_ptr<T>(A.base, A.carry0, A.carry1, A.ncarry, A.plane, k);
    float sd[TPB], md[TPB], sr[TPB];
#pragma unroll
    for (int t = 0; t < TPB; ++t) {
      sd[t] = 0.0f;
      md[t] = 0.0f;
      sr[t] = 0.0f;
    }
    // all rows of the frame are requested before any is used
    float C[ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int y = y0 + i;
      C[i] = (cv && y < A.H) ? to_f<T>(fr[(int64_t)y * A.W + x]) : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < ROWS; ++i) {
      const int y = y0 + i;
      const bool in = cv && y < A.H;
      const float c = C[i];
      mxi = max(mxi, __float_as_int(c));
      const float dn = c - P[i];
      if (k >= 2 && in) {
        float dl, rl;
        pix_terms<RS>(dn, D[i], P[i], A.Cf, dl, rl);
        sd[i / TILE] += dl;
        md[i / TILE] = fmaxf(md[i / TILE], dl);
        sr[i / TILE] += rl;
      }
      D[i] = dn;
      P[i] = c;
    }
    if (k < 2) continue;
    const int s = k - 2;
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

// Tile q from pieces: (sum Delta / n) max Delta (sum r / n), n = cells of the
// (possibly partial) tile in the image (Eq. (6) with the actual count).
__global__ void k_tile_merge(const double* part, int nsets, int nbands_part, int bpt, int nchunk, int cw,
                             int pieces, int tile, int H, int W, int Ty, int Tx, double* cube,
                             float* cube_f) {
  const int64_t total = (int64_t)nsets * Ty * Tx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int tx = (int)(i % Tx);
    const int ty = (int)((i / Tx) % Ty);
    const int s = (int)(i / ((int64_t)Tx * Ty));
    double sd = 0.0, mx = 0.0, sr = 0.0;
    const int b1 = min(ty * bpt + bpt, nbands_part);
    const int xa = tx * tile, xb = min(xa + tile, W);
    for (int b = ty * bpt; b < b1; ++b) {
      for (int ch = xa / cw; ch <= (xb - 1) / cw; ++ch) {
        const int p = tx - (ch * cw) / tile;
        const double* q = part + ((((int64_t)s * nbands_part + b) * nchunk + ch) * pieces + p) * 3;
        sd += q[0];
        mx = fmax(mx, q[1]);
        sr += q[2];
      }
    }
    const double n = (double)(min(ty * tile + tile, H) - ty * tile) * (double)(xb - xa);
    const double v = (sd / n) * mx * (sr / n);
    cube[i] = v;
    if (cube_f) cube_f[i] = (float)v;
  }
}

// ---------------------------------------------------------------------------
// Statistics.
// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of a workgroup (256 threads).
__device__ double wg_sum(double v, double* sh) {
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

// First stage of the per-set moments: workgroup g of set s reduces the
// contiguous slice g of the set's entries (raw values, or (sum, sum sq)
// pairs) into out[s][g][2], in a fixed order.
__global__ __launch_bounds__(256) void k_moments_part(const double* src, int64_t nparts, int raw, double* out) {
  __shared__ double sh[256];
  const int s = blockIdx.y, g = blockIdx.x, G = gridDim.x;
  const int64_t per = (nparts + G - 1) / G;
  const int64_t a = (int64_t)g * per, b = min(a + per, nparts);
  double x = 0.0, y = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) {
    if (raw) {
      const double v = src[(int64_t)s * nparts + i];
      x += v;
      y = fma(v, v, y);
    } else {
      x += src[((int64_t)s * nparts + i) * 2 + 0];
      y += src[((int64_t)s * nparts + i) * 2 + 1];
    }
  }
  x = wg_sum(x, sh);
  y = wg_sum(y, sh);
  if (threadIdx.x == 0) {
    out[((int64_t)s * G + g) * 2 + 0] = x;
    out[((int64_t)s * G + g) * 2 + 1] = y;
  }
}

// Per set: mean and population std from moment partials [set][nparts][2]
// (raw = 0) or from raw values [set][nparts] (raw = 1).
__global__ __launch_bounds__(256) void k_moments(const double* src, int64_t nparts, int raw, int64_t count,
                                                 double* mu, double* sigma, uint32_t* flags) {
  __shared__ double sh[256];
  const int s = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) {
    if (raw) {
      const double v = src[(int64_t)s * nparts + i];
      a += v;
      b = fma(v, v, b);
    } else {
      a += src[((int64_t)s * nparts + i) * 2 + 0];
      b += src[((int64_t)s * nparts + i) * 2 + 1];
    }
  }
  a = wg_sum(a, sh);
  b = wg_sum(b, sh);
  if (threadIdx.x == 0) {
    const double m = a / (double)count;
    double var = b / (double)count - m * m;
    if (!(var > 0.0)) var = 0.0;
    const double sg = sqrt(var);
    mu[s] = m;
    sigma[s] = sg;
    flags[s] = (sg > 0.0 && isfinite(sg) && isfinite(m)) ? 0u : (uint32_t)FITRIG_FLAG_SIGMA_ZERO;
  }
}

// M = max(max over the stack, C) from the order-preserving key of the maximum.
__global__ void k_max_finalize(const uint32_t* max_key, double C, double* M) {
  if (threadIdx.x == 0 && blockIdx.x == 0) M[0] = fmax((double)ord_val(max_key[0]), C);
}

__global__ void k_to_tlisi(float* map, int64_t n, const double* M) {
  const double m2 = M[0] * M[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    map[i] = (float)(1.0 - (double)map[i] / m2);
}

__global__ void k_f64_to_f32(const double* src, float* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ---------------------------------------------------------------------------
// Radix selection (exact order statistics of a float array per set) for the
// median / MAD spread. Keys: orderable bits of q (mode 0) or bits of
// float(|q - med|) (mode 1). Three passes of 11, 11, 10 bits.
// ---------------------------------------------------------------------------
struct RsState {
  uint32_t prefix;
  uint32_t known;
  int64_t rank;
};


// Selection key of a value: mode 0 -> order key of q, 1 -> bits of the
// float |q - med| (non-negative, so the bits order like the values), 2 -> the
// array already holds keys.
__device__ __forceinline__ uint32_t rs_key(float q, int mode, double m) {
  return mode == 2 ? __float_as_uint(q) : mode ? __float_as_uint((float)fabs((double)q - m)) : ord_key(q);
}

// Histogram of the next digit of the keys that match the prefix selected so
// far. nvalid (nullable): valid entries per set (arrays of per_set slots).
__global__ __launch_bounds__(256) void k_rs_hist(const float* vals, int64_t per_set, int mode, const double* med,
                                                 const RsState* st, int shift, int nbits, uint32_t* hist,
                                                 const unsigned long long* nvalid) {
  __shared__ uint32_t h[kHistBins];
  const int s = blockIdx.y;
  for (int i = threadIdx.x; i < kHistBins; i += 256) h[i] = 0;
  __syncthreads();
  const RsState S = st[s];
  const uint32_t dmask = (1u << nbits) - 1u;
  const float* v = vals + (int64_t)s * per_set;
  const double m = mode == 1 ? med[s] : 0.0;
  const int64_t n = nvalid ? min((int64_t)nvalid[s], per_set) : per_set;
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t key = rs_key(v[i], mode, m);
    if ((key & S.known) == S.prefix) {
      // keys near a middle value share their leading digits: the lanes whose
      // bin equals the first matching lane's add with one atomic
      const uint32_t bin = (key >> shift) & dmask;
      const uint32_t b0 = __builtin_amdgcn_readfirstlane(bin);
      const uint64_t same = __ballot(bin == b0);
      if (bin != b0)
        atomicAdd(&h[bin], 1u);
      else if (lane == __ffsll((unsigned long long)same) - 1)
        atomicAdd(&h[b0], (uint32_t)__popcll(same));
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= (int)dmask; i += 256)
    if (h[i]) atomicAdd(&hist[(int64_t)s * kHistBins + i], h[i]);
}

// Digit of the rank-th key: the first bin whose running count exceeds the
// rank (the last bin when none does); the histogram is cleared for the next
// digit. One workgroup of 256 per set, nbits 10 or 11.
__global__ __launch_bounds__(256) void k_rs_pick(RsState* st, uint32_t* hist, int shift, int nbits) {
  __shared__ int64_t part[256];
  const int s = blockIdx.x, t = threadIdx.x;
  const RsState S = st[s];
  uint32_t* h = hist + (int64_t)s * kHistBins;
  const int nb = 1 << nbits, per = nb / 256;
  uint32_t c[kHistBins / 256];
  int64_t own = 0;
#pragma unroll
  for (int j = 0; j < kHistBins / 256; ++j) {
    c[j] = j < per ? h[t * per + j] : 0u;
    own += c[j];
  }
  part[t] = own;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t x = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  const int64_t incl = part[t], excl = incl - own;
  int dig = -1;
  int64_t acc = excl;
  if (excl <= S.rank && S.rank < incl) {
#pragma unroll
    for (int j = 0; j < kHistBins / 256; ++j) {
      if (dig < 0 && j < per) {
        if (acc + (int64_t)c[j] > S.rank)
          dig = t * per + j;
        else
          acc += c[j];
      }
    }
  } else if (t == 255 && S.rank >= incl) {
    dig = nb - 1;  // rank beyond the count
    acc = incl;
  }
  if (dig >= 0) {
    RsState o = S;
    o.rank -= acc;
    o.prefix |= ((uint32_t)dig) << shift;
    o.known |= ((uint32_t)(nb - 1)) << shift;
    st[s] = o;
  }
  for (int j = 0; j < per; ++j) h[t * per + j] = 0u;
}

// Every set searches the same rank.
__global__ void k_rs_init_rank(RsState* st, int nsets, int64_t rank) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  RsState S;
  S.prefix = 0;
  S.known = 0;
  S.rank = rank;
  st[s] = S;
}

// Rank within the gathered keys: global rank minus the keys below them.
__global__ void k_rs_init_gathered(RsState* st, int nsets, int64_t rank, const unsigned long long* cnt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  RsState S;
  S.prefix = 0;
  S.known = 0;
  S.rank = rank - (int64_t)cnt[2 * s];
  st[s] = S;
}

// Keys of a sample of each set: sample i is value (i * mult) mod per_set
// with mult odd and coprime to per_set, so the samples spread over the set
// without following its rows or columns.
__global__ void k_rs_sample(const float* vals, int64_t per_set, int mode, const double* med, int64_t S,
                            uint64_t mult, uint32_t* samp) {
  const int s = blockIdx.y;
  const double m = mode == 1 ? med[s] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    // i < 2^20 and mult < per_set < 2^32: the product fits in 64 bits
    const uint64_t pos = ((uint64_t)i * mult) % (uint64_t)per_set;
    samp[(int64_t)s * S + i] = rs_key(vals[(int64_t)s * per_set + (int64_t)pos], mode, m);
  }
}

// selected key of each set -> bkt[2 s + which]
__global__ void k_rs_key_out(const RsState* st, int nsets, int which, uint32_t* bkt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsets) bkt[2 * s + which] = st[s].prefix;
}

// One pass over a set: keys below bkt[2s] are counted (cnt[2s]); keys in
// [bkt[2s], bkt[2s+1]] are counted (cnt[2s+1]) and the first cap of them
// gathered into gbuf[s * cap ...] (in no particular order: a selection does
// not need one). A workgroup stages its keys in LDS and appends them with one
// global atomic per flush.
// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// Each thread takes 16 keys per round (four 16-byte loads when VEC); a
// workgroup scan places the keys inside the bracket in an LDS stage, which is
// appended to the set's output with one global atomic per flush (atomics on
// one address per round would serialise the whole pass).
constexpr int kGatherStage = 4096;  // one round of keys
template <bool VEC>
__global__ __launch_bounds__(256) void k_rs_gather(const float* vals, int64_t per_set, int mode, const double* med,
                                                   const uint32_t* bkt, int64_t cap, unsigned long long* cnt,
                                                   uint32_t* gbuf) {
  constexpr int64_t kRound = 256 * 16;
  static_assert(kGatherStage >= kRound, "a stage holds one round");
  __shared__ uint32_t stage[kGatherStage];
  __shared__ uint32_t wsum[4];
  __shared__ unsigned long long gbase;
  const int s = blockIdx.y;
  const uint32_t lo = bkt[2 * s], hi = bkt[2 * s + 1];
  const float* v = vals + (int64_t)s * per_set;
  uint32_t* out = gbuf + (int64_t)s * cap;
  const double m = mode == 1 ? med[s] : 0.0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t below = 0, nst = 0;
  const int64_t step = (int64_t)gridDim.x * kRound;
  // appends the staged keys to the set's output (every thread calls it)
  auto flush = [&]() {
    if (threadIdx.x == 0) gbase = atomicAdd(cnt + 2 * s + 1, (unsigned long long)nst);
    __syncthreads();
    const unsigned long long g0 = gbase;
    for (uint32_t j = threadIdx.x; j < nst; j += 256)
      if ((int64_t)(g0 + j) < cap) out[g0 + j] = stage[j];
    nst = 0;
    __syncthreads();  // stage and gbase read before they are reused
  };
  // the values of a round: 16 per thread (four 16-byte loads when VEC)
  auto fetch = [&](int64_t base, float (&q)[16]) {
    if (VEC) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * 256 + threadIdx.x);  // per_set % 4 == 0
        const float4 x = i < per_set ? *reinterpret_cast<const float4*>(v + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        q[4 * j + 0] = x.x;
        q[4 * j + 1] = x.y;
        q[4 * j + 2] = x.z;
        q[4 * j + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int64_t i = base + (int64_t)j * 256 + threadIdx.x;
        q[j] = i < per_set ? v[i] : 0.0f;
      }
    }
  };
  auto index_of = [&](int64_t base, int j) -> int64_t {
    return VEC ? base + 4 * ((int64_t)(j >> 2) * 256 + threadIdx.x) + (j & 3) : base + (int64_t)j * 256 + threadIdx.x;
  };
  float q[16];
  int64_t base = blockIdx.x * kRound;
  if (base < per_set) fetch(base, q);
  // every thread of the workgroup runs the same rounds (barriers inside)
  for (; base < per_set; base += step) {
    // the next round's loads are in flight while this round is placed
    float nq[16];
    if (base + step < per_set) fetch(base + step, nq);
    uint32_t k[16];
    bool ok[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      ok[j] = index_of(base, j) < per_set;
      k[j] = rs_key(q[j], mode, m);
    }
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      below += (ok[j] && k[j] < lo) ? 1u : 0u;
      c += (ok[j] && k[j] >= lo && k[j] <= hi) ? 1u : 0u;
    }
    const uint32_t inc = wave_incl_scan(c);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    const uint32_t w0 = wsum[0], w1 = wsum[1], w2 = wsum[2], w3 = wsum[3];
    const uint32_t tot = w0 + w1 + w2 + w3;
    const uint32_t woff = (wave > 0 ? w0 : 0u) + (wave > 1 ? w1 : 0u) + (wave > 2 ? w2 : 0u);
    if (nst + tot > (uint32_t)kGatherStage) flush();  // uniform: nst and tot are
    if (c) {
      uint32_t p = nst + woff + inc - c;  // nst + tot <= kGatherStage
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (ok[j] && k[j] >= lo && k[j] <= hi) stage[p++] = k[j];
    }
    nst += tot;
    __syncthreads();  // stage written and wsum read by every thread
#pragma unroll
    for (int j = 0; j < 16; ++j) q[j] = nq[j];
  }
  if (nst) flush();
  // keys below the bracket: wave sums, then one atomic per workgroup
  uint32_t b = below;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) b += __shfl_xor(b, off);
  if (lane == 0) wsum[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(cnt + 2 * s, (unsigned long long)wsum[0] + wsum[1] + wsum[2] + wsum[3]);
}

// ---- one pass for both brackets (median and MAD) --------------------------
// Before the pass the median is known only to lie in the sample bracket
// [qlo, qhi]; with mhat its midpoint and w = max(mhat - qlo, qhi - mhat),
// every cell's |q - med| is within w of |q - mhat|. The MAD bracket [dlo, dhi]
// comes from the sample of |q - mhat|, so the cells whose |q - med| can fall
// in [dlo - w, dhi + w] have |q - mhat| in [dlo - 2w, dhi + 2w]: those are
// gathered, the ones below counted. After the exact median is known the
// selection is verified against the actual |med - mhat| (k_rs_mad_verify).
// Plan per set: pl[4 s + 0..3] = mhat, w, t_in, t_out.
__global__ void k_rs_mad_center(const uint32_t* bkt0, int nsets, double* pl, double* mhat) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const double lo = (double)ord_val(bkt0[2 * s]), hi = (double)ord_val(bkt0[2 * s + 1]);
  const double m = 0.5 * lo + 0.5 * hi;
  pl[4 * s + 0] = m;
  pl[4 * s + 1] = fmax(m - lo, hi - m);
  mhat[s] = m;
}

// The window as order-key bounds wk[4 s + 0..3] = kA, kB, kC, kD: inner
// cells kB < key < kC, outer cells key < kA or key > kD, the window the
// rest. The float bounds round inwards for the inner interval and outwards
// for the outer one, so inner cells have |q - mhat| < t_in and outer cells
// |q - mhat| > t_out exactly.
__global__ void k_rs_mad_window(const uint32_t* bkt1, int nsets, double* pl, uint32_t* wk) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const double m = pl[4 * s + 0], w = pl[4 * s + 1];
  const double t_in = (double)__uint_as_float(bkt1[2 * s]) - 2.0 * w;
  const double t_out = (double)__uint_as_float(bkt1[2 * s + 1]) + 2.0 * w;
  pl[4 * s + 2] = t_in;
  pl[4 * s + 3] = t_out;
  const uint32_t kA = ord_key(__double2float_rd(m - t_out)), kD = ord_key(__double2float_ru(m + t_out));
  uint32_t kB = ord_key(__double2float_ru(m - t_in)), kC = ord_key(__double2float_rd(m + t_in));
  if (!(t_in > 0.0) || kC <= kB) kB = kC = kA;  // no inner cells
  wk[4 * s + 0] = kA;
  wk[4 * s + 1] = kB;
  wk[4 * s + 2] = kC;
  wk[4 * s + 3] = kD;
}

// Median part: order keys below bkt0[2s] counted (cnt0[2s]), keys in
// [bkt0[2s], bkt0[2s+1]] counted (cnt0[2s+1]) and gathered into g0. MAD part
// (bounds wk of k_rs_mad_window): inner cells counted (cnt1[2s]), window
// cells counted (cnt1[2s+1]) and gathered (the bits of q) into g1. Two LDS
// stages, each appended with one atomic per flush. NONNEG: every value is
// +0 or positive (then its order key is its bits with the top bit set).
constexpr int kGather2Round = 256 * 8;
template <bool VEC, bool NONNEG>
__global__ __launch_bounds__(256) void k_rs_gather2(const float* vals, int64_t per_set, const uint32_t* bkt0,
                                                    const uint32_t* wk, int64_t cap0, int64_t cap1,
                                                    unsigned long long* cnt0, unsigned long long* cnt1, uint32_t* g0,
                                                    uint32_t* g1) {
  constexpr int kStage = kGather2Round;  // one round fits
  __shared__ uint32_t stage[2][kStage];
  __shared__ uint32_t wsum[4];
  __shared__ unsigned long long gbase;
  __shared__ uint32_t red[2][4];
  const int s = blockIdx.y;
  const uint32_t lo = bkt0[2 * s], hi = bkt0[2 * s + 1];
  const uint32_t kA = wk[4 * s + 0], kB = wk[4 * s + 1], kC = wk[4 * s + 2], kD = wk[4 * s + 3];
  const float* v = vals + (int64_t)s * per_set;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t below = 0, inner = 0, nst0 = 0, nst1 = 0;
  const int64_t step = (int64_t)gridDim.x * kGather2Round;
  auto flush = [&](int which, uint32_t n) {
    unsigned long long* cnt = which ? cnt1 : cnt0;
    uint32_t* out = (which ? g1 : g0) + (int64_t)s * (which ? cap1 : cap0);
    const int64_t cap = which ? cap1 : cap0;
    if (threadIdx.x == 0) gbase = atomicAdd(cnt + 2 * s + 1, (unsigned long long)n);
    __syncthreads();
    const unsigned long long b0 = gbase;
    for (uint32_t j = threadIdx.x; j < n; j += 256)
      if ((int64_t)(b0 + j) < cap) out[b0 + j] = stage[which][j];
    __syncthreads();  // stage and gbase read before they are reused
  };
  auto fetch = [&](int64_t base, float (&q)[8]) {
    if (VEC) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t i = base + 4 * ((int64_t)j * 256 + threadIdx.x);  // per_set % 4 == 0
        const float4 x = i < per_set ? *reinterpret_cast<const float4*>(v + i) : make_float4(0.f, 0.f, 0.f, 0.f);
        q[4 * j + 0] = x.x;
        q[4 * j + 1] = x.y;
        q[4 * j + 2] = x.z;
        q[4 * j + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t i = base + (int64_t)j * 256 + threadIdx.x;
        q[j] = i < per_set ? v[i] : 0.0f;
      }
    }
  };
  auto index_of = [&](int64_t base, int j) -> int64_t {
    return VEC ? base + 4 * ((int64_t)(j >> 2) * 256 + threadIdx.x) + (j & 3) : base + (int64_t)j * 256 + threadIdx.x;
  };
  float q[8];
  int64_t base = blockIdx.x * (int64_t)kGather2Round;
  if (base < per_set) fetch(base, q);
  for (; base < per_set; base += step) {
    float nq[8];
    if (base + step < per_set) fetch(base + step, nq);
    uint32_t k[8];
    uint32_t sel = 0;  // bit j: median bracket, bit 8 + j: MAD window
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const bool ok = index_of(base, j) < per_set;
      k[j] = NONNEG ? (__float_as_uint(q[j]) | 0x80000000u) : ord_key(q[j]);
      const bool in_w = k[j] > kB && k[j] < kC;
      below += (ok && k[j] < lo) ? 1u : 0u;
      inner += (ok && in_w) ? 1u : 0u;
      sel |= (ok && k[j] - lo <= hi - lo) ? (1u << j) : 0u;
      sel |= (ok && !in_w && k[j] - kA <= kD - kA) ? (1u << (8 + j)) : 0u;
    }
    // counts of both stages packed in 16-bit halves (at most 2048 each)
    const uint32_t c = (uint32_t)__popc(sel & 0xFFu) | ((uint32_t)__popc(sel >> 8) << 16);
    const uint32_t inc = wave_incl_scan(c);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    const uint32_t w0 = wsum[0], w1 = wsum[1], w2 = wsum[2], w3 = wsum[3];
    const uint32_t tot = w0 + w1 + w2 + w3;
    const uint32_t woff = (wave > 0 ? w0 : 0u) + (wave > 1 ? w1 : 0u) + (wave > 2 ? w2 : 0u);
    const uint32_t tot0 = tot & 0xFFFFu, tot1 = tot >> 16;
    // uniform decisions: nst and tot are the same in every thread
    if (nst0 + tot0 > (uint32_t)kStage) {
      flush(0, nst0);
      nst0 = 0;
    }
    if (nst1 + tot1 > (uint32_t)kStage) {
      flush(1, nst1);
      nst1 = 0;
    }
    if (c) {
      const uint32_t ex = woff + inc - c;
      uint32_t p0 = nst0 + (ex & 0xFFFFu), p1 = nst1 + (ex >> 16);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (sel & (1u << j)) stage[0][p0++] = k[j];
        if (sel & (1u << (8 + j))) stage[1][p1++] = __float_as_uint(q[j]);
      }
    }
    nst0 += tot0;
    nst1 += tot1;
    __syncthreads();  // stages written and wsum read by every thread
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = nq[j];
  }
  if (nst0) flush(0, nst0);
  if (nst1) flush(1, nst1);
  uint32_t b = below, in = inner;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    b += __shfl_xor(b, off);
    in += __shfl_xor(in, off);
  }
  if (lane == 0) {
    red[0][wave] = b;
    red[1][wave] = in;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(cnt0 + 2 * s, (unsigned long long)red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    atomicAdd(cnt1 + 2 * s, (unsigned long long)red[1][0] + red[1][1] + red[1][2] + red[1][3]);
  }
}

// The MAD selected from the gathered window is exact when every counted
// (inner) cell's key is at most the lower middle value and every cell beyond
// the window has a key above the upper one: inner cells have |q - med| <
// t_in + |med - mhat|, outer ones |q - med| > t_out - |med - mhat| (slack
// 2^-40 covers the double roundings of these bounds). bad[s] = 1 otherwise.
__global__ void k_rs_mad_verify(const double* pl, const double* med, const double* dev,
                                const unsigned long long* cnt1, int nsets, uint32_t* bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const double e = fabs(med[s] - pl[4 * s + 0]);
  const double slack = 0x1p-40;
  const float in_max = (float)((pl[4 * s + 2] + e) * (1.0 + slack));
  const float out_min = (float)((pl[4 * s + 3] - e) * (1.0 - slack));
  const bool ok_in = cnt1[2 * s] == 0 || (double)in_max <= dev[2 * s];
  const bool ok_out = (double)out_min > dev[2 * s + 1];
  bad[s] = (ok_in && ok_out && isfinite(med[s])) ? 0u : 1u;
}

// Dispersion keys of a sample of order keys: |q - med| of the sampled q.
__global__ void k_rs_sample_dev(uint32_t* samp, int64_t S, const double* med) {
  const int s = blockIdx.y;
  const double m = med[s];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t* p = samp + (int64_t)s * S + i;
    *p = rs_key(ord_val(*p), 1, m);
  }
}

__global__ void k_rs_init(RsState* st, int nsets, int64_t per_set, int which) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  RsState S;
  S.prefix = 0;
  S.known = 0;
  S.rank = which ? per_set / 2 : (per_set - 1) / 2;
  st[s] = S;
}

// The order statistic just above the selected one (rank + 1): the selected
// key itself when more than rank + 1 keys are <= it, else the smallest key
// above it. One pass: count of keys <= the selected key, minimum key above.
__global__ __launch_bounds__(256) void k_rs_next(const float* vals, int64_t per_set, int mode, const double* med,
                                                 const RsState* st, unsigned long long* cnt_le, uint32_t* min_gt,
                                                 const unsigned long long* nvalid) {
  __shared__ uint32_t sh_c[256];
  __shared__ uint32_t sh_m[256];
  const int s = blockIdx.y;
  const uint32_t sel = st[s].prefix;
  const float* v = vals + (int64_t)s * per_set;
  const double m = mode == 1 ? med[s] : 0.0;
  const int64_t n = nvalid ? min((int64_t)nvalid[s], per_set) : per_set;
  uint32_t c = 0, mn = 0xFFFFFFFFu;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t key = rs_key(v[i], mode, m);
    if (key <= sel) ++c;
    else mn = min(mn, key);
  }
  sh_c[threadIdx.x] = c;
  sh_m[threadIdx.x] = mn;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      sh_c[threadIdx.x] += sh_c[threadIdx.x + w];
      sh_m[threadIdx.x] = min(sh_m[threadIdx.x], sh_m[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(cnt_le + s, (unsigned long long)sh_c[0]);
    atomicMin(min_gt + s, sh_m[0]);
  }
}

// base (nullable): keys below the searched range, not in the counted array
__global__ void k_rs_next_store(const RsState* st, int nsets, int64_t rank_hi, int mode,
                                const unsigned long long* cnt_le, const uint32_t* min_gt,
                                const unsigned long long* base, double* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const int64_t le = (int64_t)cnt_le[s] + (base ? (int64_t)base[2 * s] : 0);
  const uint32_t k = (le >= rank_hi + 1) ? st[s].prefix : min_gt[s];
  out[2 * s + 1] = mode ? (double)__uint_as_float(k) : (double)ord_val(k);
}

// value of the selected key: mode 0 -> q, mode 1 -> |q - med| (as float)
__global__ void k_rs_store(const RsState* st, int nsets, int mode, int which, double* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const uint32_t k = st[s].prefix;
  const double v = mode ? (double)__uint_as_float(k) : (double)ord_val(k);
  out[2 * s + which] = v;
}

__global__ void k_rs_finish(const double* lohi_med, const double* lohi_dev, int nsets, double* mu, double* sigma,
                            uint32_t* flags, int dev_stage) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  if (!dev_stage) {
    mu[s] = 0.5 * (lohi_med[2 * s] + lohi_med[2 * s + 1]);
  } else {
    const double mad = 0.5 * (lohi_dev[2 * s] + lohi_dev[2 * s + 1]);
    const double sg = 1.482602218505602 * mad;
    sigma[s] = sg;
    flags[s] = (sg > 0.0 && isfinite(sg) && isfinite(mu[s])) ? 0u : (uint32_t)FITRIG_FLAG_SIGMA_ZERO;
  }
}

// ---------------------------------------------------------------------------
// Selection: segment maxima of a direct value array, flags, deterministic
// compaction, exact cell recompute, union-find components.
// ---------------------------------------------------------------------------
__global__ void k_segmax_direct(const float* vals, SegLayout L, float* seg_max) {
  const int64_t total = (int64_t)L.nsets * L.Ho * L.nseg_row;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(e % L.nseg_row);
    const int64_t row = e / L.nseg_row;  // set * Ho + y
    const int x0 = seg_x0(L, g), w = seg_width(L, g);
    float m = -INFINITY;
    const float* v = vals + row * L.Wo;
    for (int i = 0; i < w; ++i) m = fmaxf(m, v[x0 + i]);
    seg_max[e] = m;
  }
}

constexpr int kPerThread = 16;
constexpr int kChunk = 256 * kPerThread;

__device__ __forceinline__ bool zsel(float q, double mu, double sg, double tau) {
  return ((double)q - mu) / sg > tau;
}

// Two-level selection. A block is br rows of one 64-cell segment column
// (block b = (set, yb, g) in raster order); a block is flagged when the
// largest row-segment maximum in it passes the threshold. Flagged blocks are
// compacted, then their rows (ordered set, row, segment: raster order) are
// compacted to the selected row segments ("slots") whose cells are
// recomputed. With br = 1 the blocks are the row segments themselves.
struct BlkIdx {
  int s, yb, g;
};
__device__ __forceinline__ BlkIdx blk_decode(const SegLayout& L, int64_t b) {
  BlkIdx r;
  if (b < (int64_t)INT32_MAX) {
    const uint32_t u = (uint32_t)b, ns = (uint32_t)L.nseg_row, nb = (uint32_t)L.nbr;
    const uint32_t rb = u / ns;
    r.g = (int)(u - rb * ns);
    r.s = (int)(rb / nb);
    r.yb = (int)(rb - (uint32_t)r.s * nb);
  } else {
    const int64_t rb = b / L.nseg_row;
    r.g = (int)(b - rb * L.nseg_row);
    r.s = (int)(rb / L.nbr);
    r.yb = (int)(rb - (int64_t)r.s * L.nbr);
  }
  return r;
}

// Flag of every block into a byte array, one thread per block with
// consecutive threads on consecutive segments (coalesced maxima reads), and
// the number of flagged blocks per chunk of kChunk blocks.
__global__ __launch_bounds__(256) void k_blk_count(const float* seg_max, const double* mu, const double* sigma,
                                                   const uint32_t* flags, double tau, SegLayout L, uint8_t* bflag,
                                                   uint32_t* cnt) {
  __shared__ uint32_t sh[256];
  const int64_t NB = (int64_t)L.nsets * L.nbr * L.nseg_row;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t c = 0;
  for (int j = 0; j < kPerThread; ++j) {
    const int64_t b = base + (int64_t)j * 256 + threadIdx.x;
    if (b >= NB) break;
    const BlkIdx q = blk_decode(L, b);
    bool f = false;
    if (seg_width(L, q.g) > 0 && !flags[q.s]) {
      const int y0 = q.yb * L.br, y1 = min(y0 + L.br, L.Ho);
      const float* p = seg_max + ((int64_t)q.s * L.Ho + y0) * L.nseg_row + q.g;
      float m = p[0];
      for (int y = y0 + 1; y < y1; ++y) {
        p += L.nseg_row;
        m = fmaxf(m, *p);
      }
      f = zsel(m, mu[q.s], sigma[q.s], tau);
    }
    bflag[b] = f ? 1 : 0;
    c += f ? 1u : 0u;
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

struct ByteFlag {
  const uint8_t* bflag;
  __device__ bool operator()(int64_t b) const { return bflag[b] != 0; }
};

// flagged block -> list position (or -1 for every other block)
struct BlkEmit {
  int64_t* blk_entry;
  int32_t* blk_slot;
  int64_t cap;
  __device__ void operator()(int64_t b, bool f, int64_t pos) const {
    if (f && pos < cap) {
      blk_entry[pos] = b;
      blk_slot[b] = (int32_t)pos;
    } else {
      blk_slot[b] = -1;
    }
  }
};

// Range of each band (set, yb) in the flagged-block list: [start, end).
__global__ void k_blk_bands(const int64_t* blk_entry, const int64_t* nblk_p, int64_t bcap, SegLayout L,
                            int32_t* band_start, int32_t* band_end) {
  int64_t n = nblk_p[0];
  if (n > bcap) n = bcap;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t B = blk_entry[k] / L.nseg_row;
    if (k == 0 || blk_entry[k - 1] / L.nseg_row != B) band_start[B] = (int32_t)k;
    if (k + 1 == n || blk_entry[k + 1] / L.nseg_row != B) band_end[B] = (int32_t)(k + 1);
  }
}

// Row j of the flagged blocks in raster order: the rows of band B occupy
// [start*br, end*br), row r of the band's i-th block sits at
// start*br + r*nf + i (nf = blocks of the band).
struct RowOf {
  const int64_t* blk_entry;
  const int32_t* band_start;
  const int32_t* band_end;
  SegLayout L;
  // row-segment entry (set * Ho + y) * nseg_row + g, or -1 past the last row
  __device__ int64_t entry(int64_t j) const {
    const int64_t b0 = blk_entry[j / L.br];
    const int64_t B = b0 / L.nseg_row;
    const int st = band_start[B];
    const int nf = band_end[B] - st;
    const int64_t loc = j - (int64_t)st * L.br;
    const int r = (int)(loc / nf);
    const int64_t k = st + (loc - (int64_t)r * nf);
    const int64_t b = blk_entry[k];
    const int s = (int)(B / L.nbr);
    const int yb = (int)(B - (int64_t)s * L.nbr);
    const int y = yb * L.br + r;
    if (y >= L.Ho) return -1;
    return ((int64_t)s * L.Ho + y) * L.nseg_row + (b - B * L.nseg_row);
  }
};

struct RowFlag {
  RowOf ro;
  const float* seg_max;
  const double* mu;
  const double* sigma;
  double tau;
  __device__ bool operator()(int64_t j) const {
    const int64_t e = ro.entry(j);
    if (e < 0) return false;
    const int s = (int)(e / ((int64_t)ro.L.Ho * ro.L.nseg_row));
    return zsel(seg_max[e], mu[s], sigma[s], tau);
  }
};

struct RowEmit {
  RowOf ro;
  int32_t* rowslot;
  int64_t* seg_entry;
  int64_t cap;
  __device__ void operator()(int64_t j, bool f, int64_t pos) const {
    if (f && pos < cap) {
      rowslot[j] = (int32_t)pos;
      seg_entry[pos] = ro.entry(j);
    } else {
      rowslot[j] = -1;
    }
  }
};

struct RootFlag {
  const uint64_t* mask;
  const int32_t* parent;
  __device__ bool operator()(int64_t slot) const {
    return ((mask[slot >> 6] >> (slot & 63)) & 1ull) && parent[slot] == (int32_t)slot;
  }
};

struct RootEmit {
  int32_t* comp_of;
  int32_t* c_root;
  int64_t cap;
  __device__ void operator()(int64_t slot, bool f, int64_t pos) const {
    if (f) {
      comp_of[slot] = (pos < cap) ? (int32_t)pos : -1;
      if (pos < cap) c_root[pos] = (int32_t)slot;
    }
  }
};


__device__ __forceinline__ int64_t dyn_count(int64_t ne_static, const int64_t* ne_dyn, int64_t cap, int mult) {
  if (!ne_dyn) return ne_static;
  int64_t n = ne_dyn[0];
  if (n > cap) n = cap;
  return n * mult;
}

template <class F>
__global__ __launch_bounds__(256) void k_compact_count(F f, int64_t ne_static, const int64_t* ne_dyn, int64_t cap,
                                                       int mult, uint32_t* cnt) {
  __shared__ uint32_t sh[256];
  const int64_t ne = dyn_count(ne_static, ne_dyn, cap, mult);
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t c = 0;
  if (base < ne) {
    const int64_t a = base + (int64_t)threadIdx.x * kPerThread;
    for (int j = 0; j < kPerThread; ++j)
      if (a + j < ne && f(a + j)) ++c;
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

// Exclusive scan of nchunks counts in place (one workgroup of 1024); total -> out[0].
__global__ __launch_bounds__(1024) void k_compact_scan(uint32_t* cnt, int64_t nch_static, const int64_t* ne_dyn,
                                                        int64_t cap, int mult, int64_t* out) {
  __shared__ int64_t sh[1024];
  const int t = threadIdx.x;
  // only the chunks the count pass filled (dynamic element counts)
  const int64_t nchunks =
      ne_dyn ? (dyn_count(0, ne_dyn, cap, mult) + kChunk - 1) / kChunk : nch_static;
  const int64_t per = (nchunks + 1023) / 1024;
  const int64_t a = t * per, b = min(a + per, nchunks);
  int64_t loc = 0;
  for (int64_t i = a; i < b; ++i) loc += cnt[i];
  sh[t] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t run = sh[t] - loc;
  for (int64_t i = a; i < b; ++i) {
    const uint32_t c = cnt[i];
    cnt[i] = (uint32_t)run;  // offsets fit: callers cap totals below 2^32
    run += c;
  }
  if (t == 1023) out[0] = sh[1023];
}

template <class F, class E>
__global__ __launch_bounds__(256) void k_compact_write(F f, E emit, int64_t ne_static, const int64_t* ne_dyn,
                                                       int64_t cap, int mult, const uint32_t* cnt) {
  __shared__ uint32_t sh[256];
  const int64_t ne = dyn_count(ne_static, ne_dyn, cap, mult);
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  if (base >= ne) return;
  const int64_t a = base + (int64_t)threadIdx.x * kPerThread;
  uint32_t bits = 0, c = 0;
  for (int j = 0; j < kPerThread; ++j) {
    if (a + j < ne && f(a + j)) {
      bits |= 1u << j;
      ++c;
    }
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  // inclusive scan (Hillis-Steele)
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t v = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t pos = (int64_t)cnt[blockIdx.x] + sh[threadIdx.x] - c;
  for (int j = 0; j < kPerThread; ++j) {
    if (a + j >= ne) break;
    const bool fl = (bits >> j) & 1u;
    emit(a + j, fl, pos);
    if (fl) ++pos;
  }
}

// Exact q of the cells of each selected segment, recomputed with the same
// arithmetic as k_stream; mask of z > tau.
template <typename T, int H, bool RS>
__global__ __launch_bounds__(64) void k_recompute(const void* base, const void* c0, const void* c1, int ncarry,
                                                  int64_t plane, int Hh, int Wh, float Cf,
                                                  SegLayout L, const int64_t* seg_entry, const int64_t* nsel_p,
                                                  int64_t cap, const double* mu, const double* sigma, double tau,
                                                  uint64_t* seg_mask, float* cell_q) {
  constexpr int NV = 8 + 2 * H;
  __shared__ float sv[3][64 + 32 + 2 * kMaxHalo];
  const int lane = threadIdx.x;
  int64_t nsel = nsel_p[0];
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
    for (int cc = lane; cc < ncols; cc += 64) {
      const int col = cmin + cc;
      float dl[NV], rl[NV];
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        const int yy = by - H + j;
        float a = 0.0f, b = 0.0f, c = 0.0f;
        if (col >= 0 && col < Wh && yy >= 0 && yy < Hh) {
          const int64_t o = (int64_t)yy * Wh + col;
          a = to_f<T>(f0[o]);
          b = to_f<T>(f1[o]);
          c = to_f<T>(f2[o]);
        }
        pix_terms<RS>(c - b, b - a, b, Cf, dl[j], rl[j]);
      }
      float o8[8];
      Win<H, 8, false>::run(dl, o8, nullptr);
      sv[0][cc] = o8[y - by];
      WinMax<H, 8>::run(dl, o8);
      sv[1][cc] = o8[y - by];
      Win<H, 8, false>::run(rl, o8, nullptr);
      sv[2][cc] = o8[y - by];
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

// Cells of each selected segment taken from a value array (tiles / eta).
__global__ __launch_bounds__(64) void k_fill_direct(const float* vals, SegLayout L, const int64_t* seg_entry,
                                                    const int64_t* nsel_p, int64_t cap, const double* mu,
                                                    const double* sigma, double tau, uint64_t* seg_mask,
                                                    float* cell_q) {
  const int lane = threadIdx.x;
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  for (int64_t i = blockIdx.x; i < nsel; i += gridDim.x) {
    const int64_t e = seg_entry[i];
    const int g = (int)(e % L.nseg_row);
    const int64_t row = e / L.nseg_row;
    const int s = (int)(row / L.Ho);
    const int xs = seg_x0(L, g), wd = seg_width(L, g);
    float q = 0.0f;
    bool sel = false;
    if (lane < wd) {
      q = vals[row * L.Wo + xs + lane];
      sel = zsel(q, mu[s], sigma[s], tau);
    }
    const uint64_t m = __ballot(sel);
    cell_q[i * 64 + lane] = q;
    if (lane == 0) seg_mask[i] = m;
  }
}

__device__ __forceinline__ int32_t ld_parent(const int32_t* p, int64_t i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ int32_t uf_find(const int32_t* parent, int32_t p) {
  int32_t q = ld_parent(parent, p);
  while (q != p) {
    p = q;
    q = ld_parent(parent, p);
  }
  return p;
}

// Link the larger root under the smaller one; the surviving root of a
// component is its lowest slot, i.e. its lowest row-major cell.
__device__ void uf_union(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    const int32_t old = atomicMin(parent + a, b);
    if (old == a) return;
    a = old;
  }
}

__global__ void k_uf_init(const uint64_t* seg_mask, const int64_t* nsel_p, int64_t cap, int32_t* parent) {
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  const int64_t ns = nsel * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x)
    parent[i] = ((seg_mask[i >> 6] >> (i & 63)) & 1ull) ? (int32_t)i : -1;
}

struct SlotMap {
  const int32_t* blk_slot;
  const int32_t* band_start;
  const int32_t* band_end;
  const int32_t* rowslot;
};

__device__ __forceinline__ int32_t slot_at(const SlotMap& M, const uint64_t* seg_mask, const SegLayout& L,
                                           int64_t set, int y, int x) {
  if (y < 0 || y >= L.Ho || x < 0 || x >= L.Wo) return -1;
  const int g = seg_of_x(L, x);
  const int yb = y / L.br;
  const int64_t B = set * L.nbr + yb;
  const int32_t k = M.blk_slot[B * L.nseg_row + g];
  if (k < 0) return -1;
  const int st = M.band_start[B];
  const int nf = M.band_end[B] - st;
  const int32_t si = M.rowslot[(int64_t)st * L.br + (int64_t)(y - yb * L.br) * nf + (k - st)];
  if (si < 0) return -1;
  const int off = x - seg_x0(L, g);
  if (!((seg_mask[si] >> off) & 1ull)) return -1;
  return si * 64 + off;
}

__device__ __forceinline__ void slot_pos(const int64_t* seg_entry, const SegLayout& L, int64_t slot, int64_t& set,
                                         int& y, int& x) {
  const int64_t e = seg_entry[slot >> 6];
  const int g = (int)(e % L.nseg_row);
  const int64_t row = e / L.nseg_row;
  y = (int)(row % L.Ho);
  set = row / L.Ho;
  x = seg_x0(L, g) + (int)(slot & 63);
}

__global__ void k_uf_union(SlotMap M, const uint64_t* seg_mask, const int64_t* seg_entry, SegLayout L,
                           const int64_t* nsel_p, int64_t cap, int32_t* parent) {
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  const int64_t ns = nsel * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    if (!((seg_mask[i >> 6] >> (i & 63)) & 1ull)) continue;
    int64_t set;
    int y, x;
    slot_pos(seg_entry, L, i, set, y, x);
    const int dy[4] = {0, 1, 1, 1};
    const int dx[4] = {1, -1, 0, 1};
    for (int k = 0; k < 4; ++k) {
      const int32_t nb = slot_at(M, seg_mask, L, set, y + dy[k], x + dx[k]);
      if (nb >= 0) uf_union(parent, (int32_t)i, nb);
    }
  }
}

__global__ void k_uf_flatten(const int64_t* nsel_p, int64_t cap, int32_t* parent) {
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  const int64_t ns = nsel * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = parent[i];
    if (p >= 0) parent[i] = uf_find(parent, (int32_t)i);
  }
}

__global__ void k_comp_init(const int64_t* ncomp_p, int64_t cap, int32_t* npix, unsigned long long* key,
                            unsigned long long* w, int32_t* box) {
  int64_t n = ncomp_p[0];
  if (n > cap) n = cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    npix[i] = 0;
    key[i] = 0ull;
    for (int j = 0; j < 6; ++j) w[i * 6 + j] = 0ull;
    box[i * 4 + 0] = INT32_MAX;
    box[i * 4 + 1] = INT32_MAX;
    box[i * 4 + 2] = INT32_MIN;
    box[i * 4 + 3] = INT32_MIN;
  }
}

__device__ __forceinline__ void add128(unsigned long long* p, unsigned long long v) {
  const unsigned long long old = atomicAdd(p, v);
  if (old + v < old) atomicAdd(p + 1, 1ull);
}

// Per cell: component statistics with order-independent integer atomics
// (counts, bounding box, packed argmax key, 128-bit fixed-point z sums).
__global__ void k_comp_accum(const uint64_t* seg_mask, const int64_t* seg_entry, const float* cell_q, SegLayout L,
                             const int64_t* nsel_p, int64_t cap, const int32_t* parent, const int32_t* comp_of,
                             const double* mu, const double* sigma, int32_t* npix, unsigned long long* key,
                             unsigned long long* w, int32_t* box) {
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  const int64_t ns = nsel * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    if (!((seg_mask[i >> 6] >> (i & 63)) & 1ull)) continue;
    const int32_t c = comp_of[parent[i]];
    if (c < 0) continue;
    int64_t set;
    int y, x;
    slot_pos(seg_entry, L, i, set, y, x);
    const float q = cell_q[i];
    const double z = ((double)q - mu[set]) / sigma[set];
    atomicAdd(npix + c, 1);
    const uint32_t lin = (uint32_t)((int64_t)y * L.Wo + x);
    const unsigned long long k = ((unsigned long long)ord_key(q) << 32) | (unsigned long long)(0xFFFFFFFFu - lin);
    atomicMax(key + c, k);
    const unsigned long long wz = (unsigned long long)llround(z * 1048576.0);
    add128(w + c * 6 + 0, wz);
    add128(w + c * 6 + 2, wz * (unsigned long long)y);
    add128(w + c * 6 + 4, wz * (unsigned long long)x);
    atomicMin(box + c * 4 + 0, y);
    atomicMin(box + c * 4 + 1, x);
    atomicMax(box + c * 4 + 2, y);
    atomicMax(box + c * 4 + 3, x);
  }
}

__device__ __forceinline__ double u128_to_d(const unsigned long long* p) {
  return (double)p[1] * 18446744073709551616.0 + (double)p[0];
}

__global__ void k_comp_finalize(const int64_t* ncomp_p, int64_t cap, const int32_t* c_root, const int64_t* seg_entry,
                                SegLayout L, const double* mu, const double* sigma, int branch,
                                const int32_t* npix, const unsigned long long* key, const unsigned long long* w,
                                const int32_t* box, int64_t* out_base, fitrig_candidate* out, int64_t out_cap) {
  int64_t n = ncomp_p[0];
  if (n > cap) n = cap;
  const int64_t b0 = out_base[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = b0 + i;
    if (o >= out_cap) continue;
    int64_t set;
    int y, x;
    slot_pos(seg_entry, L, c_root[i], set, y, x);
    fitrig_candidate C;
    C.branch = branch;
    C.triple = (branch == FITRIG_IMAGE) ? (int32_t)set : -1;
    C.label = (int64_t)y * L.Wo + x;
    C.n_pix = npix[i];
    const unsigned long long k = key[i];
    const uint32_t lin = 0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull);
    C.peak_y = (int32_t)(lin / (uint32_t)L.Wo);
    C.peak_x = (int32_t)(lin % (uint32_t)L.Wo);
    const float pq = ord_val((uint32_t)(k >> 32));
    C.peak_q = pq;
    C.peak_z = (float)(((double)pq - mu[set]) / sigma[set]);
    C.pad0 = 0;
    const double sw = u128_to_d(w + i * 6 + 0);
    C.cy = u128_to_d(w + i * 6 + 2) / sw;
    C.cx = u128_to_d(w + i * 6 + 4) / sw;
    C.y0 = box[i * 4 + 0];
    C.x0 = box[i * 4 + 1];
    C.y1 = box[i * 4 + 2];
    C.x1 = box[i * 4 + 3];
    out[o] = C;
  }
}

__global__ void k_advance_base(int64_t* counters) {
  // counters: [1] components of this run, [3] output base
  if (threadIdx.x == 0 && blockIdx.x == 0) counters[3] += counters[1];
}

// ---------------------------------------------------------------------------
// Image-frequency branch: per tile, DFT over s of the detrended tile series,
// one-sided magnitudes k = 1..floor(n'/2), h = max or harmonic sum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_eta(const double* cube, int np, int64_t ntiles, int harm, double* eta,
                                             float* eta_f) {
  extern __shared__ double tw[];  // [2][np]: cos, sin of 2 pi m / np
  for (int m = threadIdx.x; m < np; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)np, &sn, &cs);
    tw[m] = cs;
    tw[np + m] = sn;
  }
  __syncthreads();
  const int K = np / 2;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    double mean = 0.0;
    for (int s = 0; s < np; ++s) mean += cube[(int64_t)s * ntiles + t];
    mean /= (double)np;
    double best = 0.0;
    for (int k = 1; k <= K; ++k) {
      double val = 0.0;
      const int jmax = harm == 0 ? 1 : harm;
      for (int j = 1; j <= jmax && j * k <= K; ++j) {
        const int kk = j * k;
        double re = 0.0, im = 0.0;
        int ph = 0;
        for (int s = 0; s < np; ++s) {
          const double v = cube[(int64_t)s * ntiles + t] - mean;
          re = fma(v, tw[ph], re);
          im = fma(-v, tw[np + ph], im);
          ph += kk;
          if (ph >= np) ph -= np;
        }
        val += sqrt(re * re + im * im);
      }
      if (k == 1 || val > best) best = val;
    }
    if (K < 1) best = 0.0;
    eta[t] = best;
    if (eta_f) eta_f[t] = (float)best;
  }
}

// Per-pixel form of the frequency branch: the same transform of every
// cell's series of sliding q over the triples (series held in registers,
// n' <= NP), one-sided magnitudes, h = max or harmonic sum. The twiddles of
// each frequency are tabulated in LDS in the order the sum runs (k, s), so
// one 16-byte broadcast read serves the two multiply-adds of a term.
template <int NP>
__global__ __launch_bounds__(256) void k_eta_px(const float* q, int np, int64_t plane, int harm, double* eta,
                                                float* eta_f) {
  extern __shared__ double2 tw2[];  // [K][np]: (cos, sin) of 2 pi k s / np, k = 1..K
  const int K = np / 2;
  for (int i = threadIdx.x; i < K * np; i += blockDim.x) {
    const int k = i / np + 1, s = i - (k - 1) * np;
    const int m = (int)(((int64_t)k * s) % np);
    double sn, cs;
    sincospi(2.0 * (double)m / (double)np, &sn, &cs);
    tw2[i] = make_double2(cs, sn);
  }
  __syncthreads();
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < plane; p += (int64_t)gridDim.x * blockDim.x) {
    double v[NP];
    double mean = 0.0;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      v[s] = s < np ? (double)q[(int64_t)s * plane + p] : 0.0;
      if (s < np) mean += v[s];
    }
    mean /= (double)np;
#pragma unroll
    for (int s = 0; s < NP; ++s) v[s] -= mean;
    double best = 0.0;
    int k0 = 1;
    if (harm == 0) {
      // h = max: two frequencies per pass over s (four independent chains)
      for (; k0 + 1 <= K; k0 += 2) {
        const double2* t0 = tw2 + (k0 - 1) * np;
        const double2* t1 = t0 + np;
        double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
#pragma unroll
        for (int s = 0; s < NP; ++s) {
          if (s < np) {
            const double2 w0 = t0[s], w1 = t1[s];
            re0 = fma(v[s], w0.x, re0);
            im0 = fma(-v[s], w0.y, im0);
            re1 = fma(v[s], w1.x, re1);
            im1 = fma(-v[s], w1.y, im1);
          }
        }
        const double a0 = sqrt(re0 * re0 + im0 * im0), a1 = sqrt(re1 * re1 + im1 * im1);
        if (k0 == 1 || a0 > best) best = a0;
        if (a1 > best) best = a1;
      }
    }
    for (int k = k0; k <= K; ++k) {
      double val = 0.0;
      const int jmax = harm == 0 ? 1 : harm;
      for (int j = 1; j <= jmax && j * k <= K; ++j) {
        const double2* t = tw2 + (j * k - 1) * np;
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int s = 0; s < NP; ++s) {
          if (s < np) {
            const double2 w = t[s];
            re = fma(v[s], w.x, re);
            im = fma(-v[s], w.y, im);
          }
        }
        val += sqrt(re * re + im * im);
      }
      if (k == 1 || val > best) best = val;
    }
    if (K < 1) best = 0.0;
    eta[p] = best;
    eta_f[p] = (float)best;
  }
}

}  // namespace fitrig
