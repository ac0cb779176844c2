// FITrig host runtime and C ABI: context, scratch arena, launch sequence.
//
// One fitrig_detect call enqueues, on one stream:
//   1. the streaming index kernel (sliding mode) or the tile kernel (tile
//      mode / frequency-only), which read the stack once;
//   2. per-triple spread: FP64 moments of the kernel partials (mean / std),
//      or exact radix selection on the q map (median / MAD);
//   3. image-branch selection: flags from the 64-cell segment maxima,
//      deterministic compaction, exact recompute of the flagged segments,
//      union-find 8-connected components, candidate records;
//   4. frequency branch: tile cube, eta per tile, spread of eta, selection
//      and components on the tile grid;
//   5. small device-to-host copies of counts, candidates and statistics.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <new>

#include "fitrig.h"
#include "fitrig_internal.h"
#include "fitrig_kernels.hip"

namespace {

using namespace fitrig;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

enum {
  CNT_NSEL = 0,    // segments selected in the current run
  CNT_NCOMP = 1,   // components of the current run
  CNT_OUTBASE = 3, // candidates written so far
  CNT_TRUNC = 5,   // internal capacity exceeded
  CNT_IMG = 6,     // image-branch candidates
  CNT_FREQ = 7,    // frequency-branch candidates
  CNT_NBLK = 8,    // selection blocks flagged in the current run
  CNT_N = 9
};

}  // namespace

struct fitrig_ctx {
  fitrig_config cfg;
  hipStream_t stream = nullptr;
  int32_t last_hip = 0;
  DevBuf stat_part, seg_max, seg_max2, tile_part, cube, cube_f, eta_d, eta_f, mu, sigma, flags, eta_st, M, qscratch;
  DevBuf fseries;  // frequency series over [history | call] (serving)
  DevBuf etapx_d, etapx_f;  // per-pixel spectrum maxima
  DevBuf hist, rs_state, rs_med, rs_dev, rs_next, chunk_cnt, counters, mom_tmp, max_key;
  DevBuf rs_samp, rs_gbuf, rs_bkt, rs_cnt, rs_nvalid, rs_plan;
  DevBuf seg_entry, seg_mask, cell_q, parent, comp_of, c_root, c_npix, c_key, c_w, c_box, c_out;
  DevBuf bflag, blk_entry, blk_slot, band_start, band_end, rowslot;
  int64_t seg_cap = 0, comp_cap = 0;
  void* h_stage = nullptr;
  size_t h_stage_cap = 0;
  hipEvent_t ev[FITRIG_N_PHASES + 1] = {};
  double phase_ms[FITRIG_N_PHASES] = {};
  int32_t have_times = 0;
};

namespace {

#define HIP_TRY(ctx, expr)                      \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      (ctx)->last_hip = (int32_t)e_;            \
      return (e_ == hipErrorOutOfMemory) ? FITRIG_E_NOMEM : FITRIG_E_HIP; \
    }                                           \
  } while (0)

#define LAUNCH_CHECK(ctx) HIP_TRY(ctx, hipGetLastError())

fitrig_status ensure(fitrig_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 64;
  if (b.cap >= bytes) return FITRIG_OK;
  if (b.p) {
    // the buffer may still be in use by work queued on any stream
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  bytes = (bytes + 255) & ~(size_t)255;
  HIP_TRY(ctx, hipMalloc(&b.p, bytes));
  b.cap = bytes;
  return FITRIG_OK;
}

fitrig_status ensure_host(fitrig_ctx* ctx, size_t bytes) {
  if (ctx->h_stage_cap >= bytes) return FITRIG_OK;
  if (ctx->h_stage) {
    HIP_TRY(ctx, hipHostFree(ctx->h_stage));
    ctx->h_stage = nullptr;
    ctx->h_stage_cap = 0;
  }
  bytes = std::max<size_t>(bytes, 1 << 16);
  HIP_TRY(ctx, hipHostMalloc(&ctx->h_stage, bytes, hipHostMallocDefault));
  ctx->h_stage_cap = bytes;
  return FITRIG_OK;
}

template <typename T, bool RS>
void launch_stream(int H, dim3 grid, hipStream_t st, const StreamArgs& A) {
  switch (H) {
#define CASE(h) \
  case h: hipLaunchKernelGGL((k_stream<T, h, RS>), grid, dim3(kLanes), 0, st, A); break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}

template <typename T>
void launch_tile_stream(int tile, bool rs, dim3 grid, hipStream_t st, const TileStreamArgs& A) {
  switch (tile) {
#define CASE(t)                                                                                           \
  case t:                                                                                                 \
    if (rs)                                                                                               \
      hipLaunchKernelGGL((k_tile_stream<T, t, true>), grid, dim3(kLanes), 0, st, A);                      \
    else                                                                                                  \
      hipLaunchKernelGGL((k_tile_stream<T, t, false>), grid, dim3(kLanes), 0, st, A);                     \
    break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: break;
  }
}

struct RecomputeArgs {
  const void* base;
  const void* c0;
  const void* c1;
  int ncarry;
  int64_t plane;
  int H, W;
  float Cf;
  int r_signed;
};

template <typename T, bool RS>
void launch_recompute(int halo, dim3 grid, hipStream_t st, const RecomputeArgs& R, const SegLayout& L,
                      const int64_t* seg_entry, const int64_t* nsel, int64_t cap, const double* mu,
                      const double* sigma, double tau, uint64_t* mask, float* cq) {
  switch (halo) {
#define CASE(h)                                                                                          \
  case h:                                                                                                \
    hipLaunchKernelGGL((k_recompute<T, h, RS>), grid, dim3(64), 0, st, R.base, R.c0, R.c1, R.ncarry, R.plane, \
                       R.H, R.W, R.Cf, L, seg_entry, nsel, cap, mu, sigma, tau, mask, cq);               \
    break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: break;
  }
}

int grid_for(int64_t n, int per = 256, int maxg = 8192) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_copy_stride2_u64(const unsigned long long* src, unsigned long long* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[2 * i];
}
// counters[CNT_TRUNC] |= overflow of this run; per-branch count; output base.
__global__ void k_run_done(int64_t* c, int64_t seg_cap, int64_t blk_cap, int64_t comp_cap, int branch) {
  if (threadIdx.x || blockIdx.x) return;
  if (c[CNT_NSEL] > seg_cap || c[CNT_NBLK] > blk_cap || c[CNT_NCOMP] > comp_cap) c[CNT_TRUNC] |= 1;
  const int64_t nc = c[CNT_NCOMP] < comp_cap ? c[CNT_NCOMP] : comp_cap;
  c[branch == FITRIG_IMAGE ? CNT_IMG : CNT_FREQ] += nc;
  c[CNT_OUTBASE] += nc;
}
template <typename T>
__global__ void k_stack_max(const T* p, int64_t n, uint32_t* max_key) {
  __shared__ float sh[256];
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

struct Call {
  const void* stack;      // the new frames
  const void* carry0;     // frames carried in front of them (serving), nullable
  const void* carry1;
  int ncarry;
  fitrig_dtype dtype;
  int n, H, W;            // n = ncarry + new frames
  double tau;
  float* index_map;
  float* eta_map;
  hipStream_t st;
  const FreqHist* hist;   // serving: frequency branch over the field's recent triples, nullable
};

// Mean / population std per set, two fixed-order stages.
fitrig_status moments(fitrig_ctx* ctx, hipStream_t st, const double* src, int nsets, int64_t nparts, int raw,
                      int64_t count, double* mu, double* sigma, uint32_t* flags) {
  const int G = (int)std::min<int64_t>(64, std::max<int64_t>(1, nparts / 4096));
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->mom_tmp, (size_t)nsets * G * 16)) != FITRIG_OK) return rc;
  hipLaunchKernelGGL(k_moments_part, dim3(G, nsets), dim3(256), 0, st, src, nparts, raw, (double*)ctx->mom_tmp.p);
  hipLaunchKernelGGL(k_moments, dim3(nsets), dim3(256), 0, st, (const double*)ctx->mom_tmp.p, (int64_t)G, 0, count,
                     mu, sigma, flags);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Spread by exact median / MAD of a float array [nsets][per_set].
// Exact median (mode 0) and MAD (mode 1) of every set. The order statistics
// come from a three-pass radix selection (11, 11, 10 bits) on the keys; the
// upper middle one of an even count from one more counting pass. For large
// sets the selection runs on a gathered bracket: a sample of 2^20
// keys gives two keys whose sample ranks lie 8 binomial standard deviations
// either side of the middle; one pass counts the keys below the bracket and
// gathers those inside; the bracket is checked on the host to hold both
// middle ranks (else the full-array selection runs) and the selection runs
// on the gathered keys. Same keys, same order statistics, either way.
// n_max: largest number of valid keys in a set (sizes the grids: about 64 K
// keys per workgroup, so the per-workgroup histograms merged into the global
// one stay few).
fitrig_status rs_select_middle(fitrig_ctx* ctx, hipStream_t st, const float* vals, int nsets, int64_t per_set,
                               int kmode, int vmode, const double* med, const unsigned long long* nvalid,
                               const unsigned long long* base, int64_t rank_lo, int64_t rank_hi, int64_t n_max,
                               double* out) {
  uint32_t* hist = (uint32_t*)ctx->hist.p;
  RsState* rs = (RsState*)ctx->rs_state.p;
  unsigned long long* cnt_le = (unsigned long long*)ctx->rs_next.p;
  uint32_t* min_gt = (uint32_t*)(cnt_le + nsets);
  const int shifts[3] = {21, 10, 0};
  const int nbits[3] = {11, 11, 10};
  const int gx = grid_for(n_max, 1 << 13, 1024);
  if (base)
    hipLaunchKernelGGL(k_rs_init_gathered, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, rank_lo, base);
  else
    hipLaunchKernelGGL(k_rs_init_rank, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, rank_lo);
  for (int p = 0; p < 3; ++p) {
    hipLaunchKernelGGL(k_rs_hist, dim3(gx, nsets), dim3(256), 0, st, vals, per_set, kmode, med, rs, shifts[p],
                       nbits[p], hist, nvalid);
    hipLaunchKernelGGL(k_rs_pick, dim3(nsets), dim3(256), 0, st, rs, hist, shifts[p], nbits[p]);
  }
  hipLaunchKernelGGL(k_rs_store, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, vmode, 0, out);
  if (rank_hi != rank_lo) {
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, (int64_t*)cnt_le, (int64_t)nsets, (int64_t)0);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, min_gt, (int64_t)nsets, 0xFFFFFFFFu);
    hipLaunchKernelGGL(k_rs_next, dim3(gx, nsets), dim3(256), 0, st, vals, per_set, kmode, med, rs, cnt_le, min_gt,
                       nvalid);
    hipLaunchKernelGGL(k_rs_next_store, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, rank_hi, vmode,
                       (const unsigned long long*)cnt_le, (const uint32_t*)min_gt, base, out);
  } else {
    hipLaunchKernelGGL(k_rs_store, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, vmode, 1, out);
  }
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Sample order statistics a and b of each set's sample (keys) -> bkt[2 s],
// bkt[2 s + 1].
void sample_bracket(fitrig_ctx* ctx, hipStream_t st, const uint32_t* samp, int nsets, int64_t S, int64_t a, int64_t b,
                    uint32_t* bkt) {
  RsState* rs = (RsState*)ctx->rs_state.p;
  const int shifts[3] = {21, 10, 0};
  const int nbits[3] = {11, 11, 10};
  for (int w = 0; w < 2; ++w) {
    hipLaunchKernelGGL(k_rs_init_rank, dim3((nsets + 63) / 64), dim3(64), 0, st, rs, nsets, w ? b : a);
    for (int p = 0; p < 3; ++p) {
      hipLaunchKernelGGL(k_rs_hist, dim3(grid_for(S, 1 << 13, 1024), nsets), dim3(256), 0, st, (const float*)samp, S,
                         2, (const double*)nullptr, rs, shifts[p], nbits[p], (uint32_t*)ctx->hist.p,
                         (const unsigned long long*)nullptr);
      hipLaunchKernelGGL(k_rs_pick, dim3(nsets), dim3(256), 0, st, rs, (uint32_t*)ctx->hist.p, shifts[p], nbits[p]);
    }
    hipLaunchKernelGGL(k_rs_key_out, dim3((nsets + 63) / 64), dim3(64), 0, st, (const RsState*)rs, nsets, w, bkt);
  }
}

// Robust spread per set (Sec. 2.3, median and MAD): mu = median of the
// values, sigma = 1.482602218505602 * median |q - mu| (two middle order
// statistics averaged for an even count), by exact radix selection.
// Large sets select inside brackets taken from a hashed sample: one pass
// over the values gathers the cells of both the median bracket and a MAD
// window placed around the sample median (k_rs_gather2); every bracket is
// checked by its counts (or, for the MAD window, against the exact median)
// and a failed one falls back to a per-statistic pass or to full selection.
// nonneg: every value is +0 or positive (q with |x_hat| in Eq. (4), eta).
fitrig_status robust_spread(fitrig_ctx* ctx, hipStream_t st, const float* vals, int nsets, int64_t per_set,
                            bool nonneg, double* mu, double* sigma, uint32_t* flags) {
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->hist, (size_t)nsets * kHistBins * 4)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_state, (size_t)nsets * sizeof(RsState))) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_med, (size_t)nsets * 2 * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_dev, (size_t)nsets * 2 * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_next, (size_t)nsets * 12)) != FITRIG_OK) return rc;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((int64_t)nsets * kHistBins)), dim3(256), 0, st, (uint32_t*)ctx->hist.p,
                     (int64_t)nsets * kHistBins, 0u);
  const int64_t r_lo = (per_set - 1) / 2, r_hi = per_set / 2;
  double* med_out = (double*)ctx->rs_med.p;
  double* dev_out = (double*)ctx->rs_dev.p;
  auto finish = [&](int mode) {
    hipLaunchKernelGGL(k_rs_finish, dim3((nsets + 63) / 64), dim3(64), 0, st, (const double*)med_out,
                       (const double*)dev_out, nsets, mu, sigma, flags, mode);
  };
  constexpr int64_t kSample = 1 << 20;
  if (per_set < 8 * kSample) {
    for (int mode = 0; mode < 2; ++mode) {
      if ((rc = rs_select_middle(ctx, st, vals, nsets, per_set, mode, mode, mu, nullptr, nullptr, r_lo, r_hi, per_set,
                                 mode ? dev_out : med_out)) != FITRIG_OK)
        return rc;
      finish(mode);
    }
    LAUNCH_CHECK(ctx);
    return FITRIG_OK;
  }

  const int64_t S = kSample;
  // sample i is value (i * mult) mod per_set: an odd multiplier near
  // per_set * (golden ratio - 1), made coprime to per_set
  uint64_t mult = (uint64_t)((double)per_set * 0.6180339887498949) | 1u;
  while (std::gcd(mult, (uint64_t)per_set) != 1) mult += 2;
  // sample ranks of the two middle values, widened by 8 standard deviations
  // of a binomial(S, 1/2) rank (4096 for S = 2^20)
  const int64_t d = 4 * (int64_t)std::ceil(std::sqrt((double)S));
  const int64_t a = std::max<int64_t>(0, (r_lo * S) / per_set - d);
  const int64_t b = std::min<int64_t>(S - 1, (r_hi * S) / per_set + d + 1);
  // expected median-bracket count (b - a) * per_set / S: room for four times
  // it; the MAD window is wider by the median's uncertainty: eight times
  const int64_t expect = (b - a + 1) * (per_set / S + 1);
  const int64_t cap0 = std::min<int64_t>(per_set, 4 * expect);
  const int64_t cap1 = std::min<int64_t>(per_set, 8 * expect);
  const bool vec = per_set % 4 == 0 && ((uintptr_t)vals & 15) == 0;
  if ((rc = ensure(ctx, ctx->rs_samp, (size_t)nsets * S * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_gbuf, (size_t)nsets * (cap0 + cap1) * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_bkt, (size_t)nsets * 8 * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_cnt, (size_t)nsets * (4 * 8 + 4))) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_nvalid, (size_t)nsets * 2 * 8)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_plan, (size_t)nsets * 5 * 8)) != FITRIG_OK ||
      (rc = ensure_host(ctx, (size_t)nsets * 4 * 8)) != FITRIG_OK)
    return rc;
  uint32_t* samp = (uint32_t*)ctx->rs_samp.p;
  uint32_t* bkt0 = (uint32_t*)ctx->rs_bkt.p;
  uint32_t* bkt1 = bkt0 + 2 * nsets;
  uint32_t* wk = bkt0 + 4 * nsets;
  unsigned long long* cnt0 = (unsigned long long*)ctx->rs_cnt.p;
  unsigned long long* cnt1 = cnt0 + 2 * nsets;
  unsigned long long* nv0 = (unsigned long long*)ctx->rs_nvalid.p;
  unsigned long long* nv1 = nv0 + nsets;
  uint32_t* g0 = (uint32_t*)ctx->rs_gbuf.p;
  uint32_t* g1 = g0 + (size_t)nsets * cap0;
  double* pl = (double*)ctx->rs_plan.p;
  double* mhat = pl + 4 * nsets;
  const dim3 gs(grid_for(S, 256, 1024), nsets), g1d((nsets + 63) / 64);
  unsigned long long* h = (unsigned long long*)ctx->h_stage;

  // brackets from the sample: median keys, then the MAD window around its midpoint
  hipLaunchKernelGGL(k_rs_sample, gs, dim3(256), 0, st, vals, per_set, 0, (const double*)nullptr, S, mult, samp);
  sample_bracket(ctx, st, samp, nsets, S, a, b, bkt0);
  hipLaunchKernelGGL(k_rs_mad_center, g1d, dim3(64), 0, st, (const uint32_t*)bkt0, nsets, pl, mhat);
  hipLaunchKernelGGL(k_rs_sample_dev, gs, dim3(256), 0, st, samp, S, (const double*)mhat);
  sample_bracket(ctx, st, samp, nsets, S, a, b, bkt1);
  hipLaunchKernelGGL(k_rs_mad_window, g1d, dim3(64), 0, st, (const uint32_t*)bkt1, nsets, pl, wk);
  // one pass over the values for both
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(256), 0, st, (int64_t*)cnt0, (int64_t)(4 * nsets), (int64_t)0);
  const dim3 gg(grid_for(per_set, kGather2Round * 2, 1024), nsets);
#define GATHER2(V, NN)                                                                                          \
  hipLaunchKernelGGL((k_rs_gather2<V, NN>), gg, dim3(256), 0, st, vals, per_set, (const uint32_t*)bkt0,            \
                     (const uint32_t*)wk, cap0, cap1, cnt0, cnt1, g0, g1)
  if (vec && nonneg)
    GATHER2(true, true);
  else if (vec)
    GATHER2(true, false);
  else if (nonneg)
    GATHER2(false, true);
  else
    GATHER2(false, false);
#undef GATHER2
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipMemcpyAsync(h, cnt0, (size_t)nsets * 32, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  bool ok0 = true, ok1 = true;
  int64_t max0 = 1, max1 = 1;
  for (int s = 0; s < nsets; ++s) {
    const int64_t below = (int64_t)h[2 * s], in = (int64_t)h[2 * s + 1];
    const int64_t inner = (int64_t)h[2 * nsets + 2 * s], win = (int64_t)h[2 * nsets + 2 * s + 1];
    ok0 = ok0 && in <= cap0 && below <= r_lo && r_hi < below + in;
    ok1 = ok1 && win <= cap1 && inner <= r_lo && r_hi < inner + win;
    max0 = std::max(max0, in);
    max1 = std::max(max1, win);
  }
  // median: inside the bracket (rank offsets at cnt0[2 s], counts at cnt0[2 s + 1])
  if (ok0) {
    hipLaunchKernelGGL(k_copy_stride2_u64, dim3(1), dim3(64), 0, st, (const unsigned long long*)cnt0 + 1, nv0,
                       (int64_t)nsets);
    rc = rs_select_middle(ctx, st, (const float*)g0, nsets, cap0, 2, 0, mu, nv0, cnt0, r_lo, r_hi, max0, med_out);
  } else {
    rc = rs_select_middle(ctx, st, vals, nsets, per_set, 0, 0, mu, nullptr, nullptr, r_lo, r_hi, per_set, med_out);
  }
  if (rc != FITRIG_OK) return rc;
  finish(0);
  // MAD: inside the window, then verified against the exact median
  bool mad_done = false;
  if (ok1) {
    hipLaunchKernelGGL(k_copy_stride2_u64, dim3(1), dim3(64), 0, st, (const unsigned long long*)cnt1 + 1, nv1,
                       (int64_t)nsets);
    // g1 holds the values q: keys |q - med| are formed as the passes read them
    if ((rc = rs_select_middle(ctx, st, (const float*)g1, nsets, cap1, 1, 1, mu, nv1, cnt1, r_lo, r_hi, max1,
                               dev_out)) != FITRIG_OK)
      return rc;
    uint32_t* bad = (uint32_t*)(cnt1 + 2 * nsets);  // rs_cnt holds 4 counts then one flag per set
    hipLaunchKernelGGL(k_rs_mad_verify, g1d, dim3(64), 0, st, (const double*)pl, (const double*)mu,
                       (const double*)dev_out, (const unsigned long long*)cnt1, nsets, bad);
    LAUNCH_CHECK(ctx);
    uint32_t* hb = (uint32_t*)h;
    HIP_TRY(ctx, hipMemcpyAsync(hb, bad, (size_t)nsets * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    mad_done = true;
    for (int s = 0; s < nsets; ++s) mad_done = mad_done && hb[s] == 0;
  }
  if (!mad_done) {
    // a pass of its own around the exact median
    hipLaunchKernelGGL(k_rs_sample, gs, dim3(256), 0, st, vals, per_set, 1, (const double*)mu, S, mult, samp);
    sample_bracket(ctx, st, samp, nsets, S, a, b, bkt1);
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, (int64_t*)cnt1, (int64_t)(2 * nsets), (int64_t)0);
    const dim3 g1g(grid_for(per_set, 256 * 16, 512), nsets);
    if (vec)
      hipLaunchKernelGGL(k_rs_gather<true>, g1g, dim3(256), 0, st, vals, per_set, 1, (const double*)mu,
                         (const uint32_t*)bkt1, cap1, cnt1, g1);
    else
      hipLaunchKernelGGL(k_rs_gather<false>, g1g, dim3(256), 0, st, vals, per_set, 1, (const double*)mu,
                         (const uint32_t*)bkt1, cap1, cnt1, g1);
    LAUNCH_CHECK(ctx);
    HIP_TRY(ctx, hipMemcpyAsync(h, cnt1, (size_t)nsets * 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    bool ok = true;
    int64_t mx = 1;
    for (int s = 0; s < nsets; ++s) {
      const int64_t below = (int64_t)h[2 * s], in = (int64_t)h[2 * s + 1];
      ok = ok && in <= cap1 && below <= r_lo && r_hi < below + in;
      mx = std::max(mx, in);
    }
    if (ok) {
      hipLaunchKernelGGL(k_copy_stride2_u64, dim3(1), dim3(64), 0, st, (const unsigned long long*)cnt1 + 1, nv1,
                         (int64_t)nsets);
      rc = rs_select_middle(ctx, st, (const float*)g1, nsets, cap1, 2, 1, mu, nv1, cnt1, r_lo, r_hi, mx, dev_out);
    } else {
      rc = rs_select_middle(ctx, st, vals, nsets, per_set, 1, 1, mu, nullptr, nullptr, r_lo, r_hi, per_set, dev_out);
    }
    if (rc != FITRIG_OK) return rc;
  }
  finish(1);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Deterministic compaction: count, scan, write.
template <class F, class E>
fitrig_status compact(fitrig_ctx* ctx, hipStream_t st, F f, E e, int64_t ne_static, const int64_t* ne_dyn,
                      int64_t cap, int mult, int64_t* total) {
  const int64_t ne_max = ne_dyn ? cap * mult : ne_static;
  const int64_t nch = std::max<int64_t>(1, (ne_max + kChunk - 1) / kChunk);
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->chunk_cnt, (size_t)nch * 4)) != FITRIG_OK) return rc;
  uint32_t* cnt = (uint32_t*)ctx->chunk_cnt.p;
  hipLaunchKernelGGL((k_compact_count<F>), dim3((unsigned)nch), dim3(256), 0, st, f, ne_static, ne_dyn, cap, mult,
                     cnt);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, cnt, nch, ne_dyn, cap, mult, total);
  hipLaunchKernelGGL((k_compact_write<F, E>), dim3((unsigned)nch), dim3(256), 0, st, f, e, ne_static, ne_dyn, cap,
                     mult, (const uint32_t*)cnt);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// One selection run over a segment layout: flags -> segments -> cells ->
// components -> candidate records appended at counters[CNT_OUTBASE].
fitrig_status select_run(fitrig_ctx* ctx, const Call& c, const SegLayout& L, float* seg_max, const double* mu,
                         const double* sigma, const uint32_t* flags, int branch, const float* direct_vals,
                         int halo) {
  hipStream_t st = c.st;
  int64_t* cnt = (int64_t*)ctx->counters.p;
  const int64_t NE = (int64_t)L.nsets * L.Ho * L.nseg_row;
  const int64_t cap = ctx->seg_cap;
  int64_t* seg_entry = (int64_t*)ctx->seg_entry.p;
  uint64_t* mask = (uint64_t*)ctx->seg_mask.p;
  float* cq = (float*)ctx->cell_q.p;
  int32_t* parent = (int32_t*)ctx->parent.p;
  fitrig_status rc;

  // blocks of L.br rows x one segment: flag (maxima of the block's rows),
  // compact, then compact the rows of the flagged blocks in raster order
  const int64_t NB = (int64_t)L.nsets * L.nbr * L.nseg_row;
  const int64_t nbands = (int64_t)L.nsets * L.nbr;
  const int64_t bcap = std::max<int64_t>(4096, cap / 2);
  const int64_t nchb = std::max<int64_t>(1, (NB + kChunk - 1) / kChunk);
  if ((rc = ensure(ctx, ctx->bflag, (size_t)NB)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->blk_slot, (size_t)NB * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->band_start, (size_t)nbands * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->band_end, (size_t)nbands * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->blk_entry, (size_t)bcap * 8)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rowslot, (size_t)bcap * L.br * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->chunk_cnt, (size_t)nchb * 4)) != FITRIG_OK)
    return rc;
  uint8_t* bflag = (uint8_t*)ctx->bflag.p;
  int64_t* blk_entry = (int64_t*)ctx->blk_entry.p;
  int32_t* blk_slot = (int32_t*)ctx->blk_slot.p;
  int32_t* band_start = (int32_t*)ctx->band_start.p;
  int32_t* band_end = (int32_t*)ctx->band_end.p;
  int32_t* rowslot = (int32_t*)ctx->rowslot.p;
  uint32_t* ccnt = (uint32_t*)ctx->chunk_cnt.p;
  hipLaunchKernelGGL(k_blk_count, dim3((unsigned)nchb), dim3(256), 0, st, (const float*)seg_max, mu, sigma, flags,
                     c.tau, L, bflag, ccnt);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, ccnt, nchb, (const int64_t*)nullptr, (int64_t)0, 1,
                     cnt + CNT_NBLK);
  hipLaunchKernelGGL((k_compact_write<ByteFlag, BlkEmit>), dim3((unsigned)nchb), dim3(256), 0, st,
                     ByteFlag{bflag}, BlkEmit{blk_entry, blk_slot, bcap}, NB, (const int64_t*)nullptr, (int64_t)0, 1,
                     (const uint32_t*)ccnt);
  hipLaunchKernelGGL(k_blk_bands, dim3(grid_for(bcap, 256, 2048)), dim3(256), 0, st, (const int64_t*)blk_entry,
                     (const int64_t*)(cnt + CNT_NBLK), bcap, L, band_start, band_end);
  LAUNCH_CHECK(ctx);
  const RowOf ro{blk_entry, band_start, band_end, L};
  if ((rc = compact(ctx, st, RowFlag{ro, seg_max, mu, sigma, c.tau}, RowEmit{ro, rowslot, seg_entry, cap}, 0,
                    cnt + CNT_NBLK, bcap, L.br, cnt + CNT_NSEL)) != FITRIG_OK)
    return rc;

  const int gsel = (int)std::min<int64_t>(cap, 4096);
  if (direct_vals) {
    hipLaunchKernelGGL(k_fill_direct, dim3(gsel), dim3(64), 0, st, direct_vals, L, (const int64_t*)seg_entry,
                       (const int64_t*)(cnt + CNT_NSEL), cap, mu, sigma, c.tau, mask, cq);
  } else {
    RecomputeArgs R{c.stack, c.carry0, c.carry1, c.ncarry, (int64_t)c.H * c.W, c.H, c.W, (float)ctx->cfg.C,
                    ctx->cfg.r_signed};
#define RC(T, RS) \
  launch_recompute<T, RS>(halo, dim3(gsel), st, R, L, seg_entry, cnt + CNT_NSEL, cap, mu, sigma, c.tau, mask, cq)
    const bool rs = ctx->cfg.r_signed != 0;
    switch (c.dtype) {
      case FITRIG_F32: rs ? RC(float, true) : RC(float, false); break;
      case FITRIG_F16: rs ? RC(__half, true) : RC(__half, false); break;
      default: rs ? RC(bf16_t, true) : RC(bf16_t, false); break;
    }
#undef RC
  }
  LAUNCH_CHECK(ctx);
  const int gcell = grid_for(cap * 64, 256, 4096);
  hipLaunchKernelGGL(k_uf_init, dim3(gcell), dim3(256), 0, st, (const uint64_t*)mask, (const int64_t*)(cnt + CNT_NSEL),
                     cap, parent);
  hipLaunchKernelGGL(k_uf_union, dim3(gcell), dim3(256), 0, st, SlotMap{blk_slot, band_start, band_end, rowslot},
                     (const uint64_t*)mask,
                     (const int64_t*)seg_entry, L, (const int64_t*)(cnt + CNT_NSEL), cap, parent);
  hipLaunchKernelGGL(k_uf_flatten, dim3(gcell), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NSEL), cap, parent);
  LAUNCH_CHECK(ctx);

  RootFlag rf{(const uint64_t*)mask, (const int32_t*)parent};
  RootEmit re{(int32_t*)ctx->comp_of.p, (int32_t*)ctx->c_root.p, ctx->comp_cap};
  if ((rc = compact(ctx, st, rf, re, 0, cnt + CNT_NSEL, cap, 64, cnt + CNT_NCOMP)) != FITRIG_OK) return rc;

  const int64_t ccap = ctx->comp_cap;
  const int gcomp = grid_for(ccap, 256, 4096);
  hipLaunchKernelGGL(k_comp_init, dim3(gcomp), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NCOMP), ccap,
                     (int32_t*)ctx->c_npix.p, (unsigned long long*)ctx->c_key.p, (unsigned long long*)ctx->c_w.p,
                     (int32_t*)ctx->c_box.p);
  hipLaunchKernelGGL(k_comp_accum, dim3(gcell), dim3(256), 0, st, (const uint64_t*)mask, (const int64_t*)seg_entry,
                     (const float*)cq, L, (const int64_t*)(cnt + CNT_NSEL), cap, (const int32_t*)parent,
                     (const int32_t*)ctx->comp_of.p, mu, sigma, (int32_t*)ctx->c_npix.p,
                     (unsigned long long*)ctx->c_key.p, (unsigned long long*)ctx->c_w.p, (int32_t*)ctx->c_box.p);
  hipLaunchKernelGGL(k_comp_finalize, dim3(gcomp), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NCOMP), ccap,
                     (const int32_t*)ctx->c_root.p, (const int64_t*)seg_entry, L, mu, sigma, branch,
                     (const int32_t*)ctx->c_npix.p, (const unsigned long long*)ctx->c_key.p,
                     (const unsigned long long*)ctx->c_w.p, (const int32_t*)ctx->c_box.p, cnt + CNT_OUTBASE,
                     (fitrig_candidate*)ctx->c_out.p, 2 * ccap);
  hipLaunchKernelGGL(k_run_done, dim3(1), dim3(64), 0, st, cnt, cap, bcap, ccap, branch);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

fitrig_status ensure_selection(fitrig_ctx* ctx, int64_t ne_total) {
  int64_t want = ctx->cfg.max_segments > 0 ? ctx->cfg.max_segments
                                           : std::max<int64_t>(65536, std::min<int64_t>(ne_total / 64, 1 << 22));
  if (want > ctx->seg_cap) {
    fitrig_status rc;
    const int64_t comp = 2 * want;
    if ((rc = ensure(ctx, ctx->seg_entry, want * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->seg_mask, want * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cell_q, want * 64 * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->parent, want * 64 * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->comp_of, want * 64 * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_root, comp * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_npix, comp * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_key, comp * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_w, comp * 6 * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_box, comp * 4 * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->c_out, 2 * comp * sizeof(fitrig_candidate))) != FITRIG_OK) return rc;
    ctx->seg_cap = want;
    ctx->comp_cap = comp;
  }
  return FITRIG_OK;
}

template <typename T>
fitrig_status run_tile_kernel(fitrig_ctx* ctx, const Call& c, int tile, int Ty, int nchunk, int pieces) {
  TileArgs A;
  A.base = c.stack;
  A.carry0 = c.carry0;
  A.carry1 = c.carry1;
  A.ncarry = c.ncarry;
  A.n = c.n;
  A.plane = (int64_t)c.H * c.W;
  A.H = c.H;
  A.W = c.W;
  A.tile = tile;
  A.nchunk = nchunk;
  A.pieces = pieces;
  A.r_signed = ctx->cfg.r_signed;
  A.Cf = (float)ctx->cfg.C;
  A.tile_part = (double*)ctx->tile_part.p;
  A.max_key = (uint32_t*)ctx->max_key.p;
  if (A.r_signed)
    hipLaunchKernelGGL((k_tile<T, true>), dim3(nchunk, Ty, c.n - 2), dim3(kLanes), 0, c.st, A);
  else
    hipLaunchKernelGGL((k_tile<T, false>), dim3(nchunk, Ty, c.n - 2), dim3(kLanes), 0, c.st, A);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

fitrig_status detect_impl(fitrig_ctx* ctx, const Call& c, fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                          fitrig_stats* stats) {
  const fitrig_config& cfg = ctx->cfg;
  hipStream_t st = c.st;
  const int np = c.n - 2;
  const int halo = cfg.window / 2;
  const int64_t plane = (int64_t)c.H * c.W;
  const bool img = (cfg.branches & FITRIG_IMAGE) != 0;
  // frequency branch: over this call's triples, or (with a history) over
  // the last hist->cap triples of [history | this call]
  const bool want_freq = (cfg.branches & FITRIG_FREQ) != 0;
  const bool ring = want_freq && c.hist && c.hist->cap > 0;
  const int nfreq = ring ? (int)std::min<int64_t>(c.hist->cap, (int64_t)c.hist->n_in + np) : np;
  const bool freq = want_freq && nfreq >= 4 && nfreq <= 2048;
  const bool cube_needed = freq || ring;
  // per-pixel frequency branch: series of sliding q held in registers
  const bool fpx = (cfg.branches & FITRIG_FREQ_PIXEL) != 0 && cfg.mode == FITRIG_SLIDING && np >= 4 && np <= 64;
  const bool sliding = cfg.mode == FITRIG_SLIDING;
  const int tile = cfg.tile;
  const int Ty = (c.H + tile - 1) / tile, Tx = (c.W + tile - 1) / tile;
  fitrig_status rc;

  if ((rc = ensure(ctx, ctx->counters, CNT_N * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->mu, (size_t)np * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->sigma, (size_t)np * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->flags, (size_t)np * 4)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->eta_st, 64)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->M, 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->max_key, 64)) != FITRIG_OK) return rc;
  int64_t* cnt = (int64_t*)ctx->counters.p;
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, cnt, (int64_t)CNT_N, (int64_t)0);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)ctx->max_key.p, (int64_t)1, 0u);
  const bool prof = cfg.profile != 0;
  ctx->have_times = 0;
  auto mark = [&](int i) -> fitrig_status {
    if (prof) HIP_TRY(ctx, hipEventRecord(ctx->ev[i], st));
    return FITRIG_OK;
  };
  if ((rc = mark(0)) != FITRIG_OK) return rc;
  double* mu = (double*)ctx->mu.p;
  double* sigma = (double*)ctx->sigma.p;
  uint32_t* flags = (uint32_t*)ctx->flags.p;
  double* eta_mu = (double*)ctx->eta_st.p;
  double* eta_sig = eta_mu + 1;
  uint32_t* eta_flag = (uint32_t*)(eta_mu + 2);

  // ---- pass over the stack -------------------------------------------------
  bool have_cube = false;
  bool have_max = false;
  const int out_w = out_width(halo);
  const int ncol = (c.W + out_w - 1) / out_w;
  const int nbands = (c.H + kBand - 1) / kBand;
  const int nseg_row = ncol * kSegsPerGroup;
  float* qmap = nullptr;
  const bool robust = cfg.sigma_est == FITRIG_MEDIAN_MAD;

  if ((img || fpx) && sliding) {
    const int64_t nwg = (int64_t)ncol * nbands;
    if (nwg > INT32_MAX) return FITRIG_E_INVAL;
    const bool byprod = cube_needed && tile == 32;
    if ((rc = ensure(ctx, ctx->stat_part, (size_t)np * nwg * 16 * 16)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->seg_max, (size_t)np * c.H * nseg_row * 4)) != FITRIG_OK) return rc;
    if (byprod && (rc = ensure(ctx, ctx->tile_part, (size_t)np * nbands * ncol * kPieces * 3 * 8)) != FITRIG_OK)
      return rc;
    qmap = c.index_map;
    if ((robust || fpx) && !qmap) {
      if ((rc = ensure(ctx, ctx->qscratch, (size_t)np * plane * 4)) != FITRIG_OK) return rc;
      qmap = (float*)ctx->qscratch.p;
    }
    StreamArgs A;
    A.base = c.stack;
    A.carry0 = c.carry0;
    A.carry1 = c.carry1;
    A.ncarry = c.ncarry;
    A.n = c.n;
    A.plane = plane;
    A.H = c.H;
    A.W = c.W;
    A.ncol = ncol;
    A.nbands = nbands;
    A.out_w = out_w;
    // 4-byte pixels: blocks of 8 bands, so neighbouring bands share their
    // halo rows in L2; 2-byte pixels run faster in row order
    A.band_block = c.dtype == FITRIG_F32 ? 8 : 1;
    A.r_signed = cfg.r_signed;
    A.Cf = (float)cfg.C;
    A.qmap = qmap;
    A.stat_part = (double*)ctx->stat_part.p;
    A.seg_max = (float*)ctx->seg_max.p;
    A.tile_part = byprod ? (double*)ctx->tile_part.p : nullptr;
    A.max_key = (uint32_t*)ctx->max_key.p;
    const bool rs = cfg.r_signed != 0;
    switch (c.dtype) {
      case FITRIG_F32: rs ? launch_stream<float, true>(halo, dim3((unsigned)nwg), st, A)
                          : launch_stream<float, false>(halo, dim3((unsigned)nwg), st, A); break;
      case FITRIG_F16: rs ? launch_stream<__half, true>(halo, dim3((unsigned)nwg), st, A)
                          : launch_stream<__half, false>(halo, dim3((unsigned)nwg), st, A); break;
      default: rs ? launch_stream<bf16_t, true>(halo, dim3((unsigned)nwg), st, A)
                  : launch_stream<bf16_t, false>(halo, dim3((unsigned)nwg), st, A); break;
    }
    LAUNCH_CHECK(ctx);
    have_max = true;
    if ((rc = mark(1)) != FITRIG_OK) return rc;
    if (byprod) {
      if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
      if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
      hipLaunchKernelGGL(k_tile_merge, dim3(grid_for((int64_t)np * Ty * Tx)), dim3(256), 0, st,
                         (const double*)ctx->tile_part.p, np, nbands, 2, ncol, out_w, kPieces, 32, c.H, c.W, Ty, Tx,
                         (double*)ctx->cube.p, (float*)ctx->cube_f.p);
      LAUNCH_CHECK(ctx);
      have_cube = true;
    }
    // per-triple spread
    if (img && !robust) {
      if ((rc = moments(ctx, st, (const double*)ctx->stat_part.p, np, nwg * 16, 0, plane, mu, sigma, flags)) !=
          FITRIG_OK)
        return rc;
    } else if (img) {
      if ((rc = robust_spread(ctx, st, qmap, np, plane, !cfg.r_signed, mu, sigma, flags)) != FITRIG_OK) return rc;
    }
  }

  // power-of-two tiles up to 32: streaming kernel (every frame read once);
  // other sizes: the tile kernel that reads three frames per triple
  const bool pow2_tile = tile <= 32 && (tile & (tile - 1)) == 0;
  if (!have_cube && (cube_needed || (img && !sliding)) && pow2_tile) {
    // streaming tile kernel: every frame read once, the cube written directly
    if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
    TileStreamArgs A;
    A.base = c.stack;
    A.carry0 = c.carry0;
    A.carry1 = c.carry1;
    A.ncarry = c.ncarry;
    A.n = c.n;
    A.plane = plane;
    A.H = c.H;
    A.W = c.W;
    A.tile = tile;
    A.nchunk = (c.W + kLanes - 1) / kLanes;
    const int tpb = std::min(32 / tile, kTileTpbMax);
    A.nbands = (Ty + tpb - 1) / tpb;
    A.Ty = Ty;
    A.Tx = Tx;
    A.r_signed = cfg.r_signed;
    A.Cf = (float)cfg.C;
    A.cube = (double*)ctx->cube.p;
    A.cube_f = (float*)ctx->cube_f.p;
    A.max_key = (uint32_t*)ctx->max_key.p;
    const int64_t nwg = (int64_t)A.nchunk * A.nbands;
    if (nwg > INT32_MAX) return FITRIG_E_INVAL;
    switch (c.dtype) {
      case FITRIG_F32: launch_tile_stream<float>(tile, cfg.r_signed != 0, dim3((unsigned)nwg), st, A); break;
      case FITRIG_F16: launch_tile_stream<__half>(tile, cfg.r_signed != 0, dim3((unsigned)nwg), st, A); break;
      default: launch_tile_stream<bf16_t>(tile, cfg.r_signed != 0, dim3((unsigned)nwg), st, A); break;
    }
    LAUNCH_CHECK(ctx);
    if (!have_max) {
      have_max = true;
      if ((rc = mark(1)) != FITRIG_OK) return rc;
    }
    have_cube = true;
  }
  if ((!have_cube && (cube_needed || (img && !sliding)))) {
    const int nchunk = (c.W + kLanes - 1) / kLanes;
    const int pieces = (kLanes + tile - 1) / tile + 1;
    if ((rc = ensure(ctx, ctx->tile_part, (size_t)np * Ty * nchunk * pieces * 3 * 8)) != FITRIG_OK) return rc;
    const int64_t nwg = (int64_t)np * Ty * nchunk;
    if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
    switch (c.dtype) {
      case FITRIG_F32: rc = run_tile_kernel<float>(ctx, c, tile, Ty, nchunk, pieces); break;
      case FITRIG_F16: rc = run_tile_kernel<__half>(ctx, c, tile, Ty, nchunk, pieces); break;
      default: rc = run_tile_kernel<bf16_t>(ctx, c, tile, Ty, nchunk, pieces); break;
    }
    if (!have_max) {
      have_max = true;
      if ((rc = mark(1)) != FITRIG_OK) return rc;
    }
    if (rc != FITRIG_OK) return rc;
    hipLaunchKernelGGL(k_tile_merge, dim3(grid_for((int64_t)np * Ty * Tx)), dim3(256), 0, st,
                       (const double*)ctx->tile_part.p, np, Ty, 1, nchunk, kLanes, pieces, tile, c.H, c.W, Ty, Tx,
                       (double*)ctx->cube.p, (float*)ctx->cube_f.p);
    LAUNCH_CHECK(ctx);
    have_cube = true;
  }
  if (!have_max) {
    // no pass produced the maximum (e.g. frequency branch only, n' < 4)
    const int g = 1024;
    uint32_t* mk = (uint32_t*)ctx->max_key.p;
    switch (c.dtype) {
      case FITRIG_F32:
        hipLaunchKernelGGL(k_stack_max<float>, dim3(g), dim3(256), 0, st, (const float*)c.stack, (int64_t)(c.n - c.ncarry) * plane,
                           mk);
        break;
      case FITRIG_F16:
        hipLaunchKernelGGL(k_stack_max<__half>, dim3(g), dim3(256), 0, st, (const __half*)c.stack,
                           (int64_t)(c.n - c.ncarry) * plane, mk);
        break;
      default:
        hipLaunchKernelGGL(k_stack_max<bf16_t>, dim3(g), dim3(256), 0, st, (const bf16_t*)c.stack,
                           (int64_t)(c.n - c.ncarry) * plane, mk);
        break;
    }
    if ((rc = mark(1)) != FITRIG_OK) return rc;
  }
  hipLaunchKernelGGL(k_max_finalize, dim3(1), dim3(64), 0, st, (const uint32_t*)ctx->max_key.p, cfg.C,
                     (double*)ctx->M.p);
  LAUNCH_CHECK(ctx);
  if ((rc = mark(2)) != FITRIG_OK) return rc;

  // ---- image-branch selection ---------------------------------------------
  if (img) {
    if (sliding) {
      SegLayout L{c.H, c.W, np, kSegsPerGroup, out_w, nseg_row, kBand, (c.H + kBand - 1) / kBand};
      if ((rc = ensure_selection(ctx, (int64_t)np * c.H * nseg_row)) != FITRIG_OK) return rc;
      if ((rc = select_run(ctx, c, L, (float*)ctx->seg_max.p, mu, sigma, flags, FITRIG_IMAGE, nullptr, halo)) !=
          FITRIG_OK)
        return rc;
    } else {
      const int64_t ncell = (int64_t)Ty * Tx;
      if (!robust) {
        if ((rc = moments(ctx, st, (const double*)ctx->cube.p, np, ncell, 1, ncell, mu, sigma, flags)) != FITRIG_OK)
          return rc;
      } else {
        if ((rc = robust_spread(ctx, st, (const float*)ctx->cube_f.p, np, ncell, !cfg.r_signed, mu, sigma, flags)) !=
            FITRIG_OK)
          return rc;
      }
      SegLayout L{Ty, Tx, np, 1, 64, (Tx + 63) / 64, 1, Ty};
      if ((rc = ensure(ctx, ctx->seg_max, (size_t)np * Ty * L.nseg_row * 4)) != FITRIG_OK) return rc;
      hipLaunchKernelGGL(k_segmax_direct, dim3(grid_for((int64_t)np * Ty * L.nseg_row)), dim3(256), 0, st,
                         (const float*)ctx->cube_f.p, L, (float*)ctx->seg_max.p);
      if ((rc = ensure_selection(ctx, (int64_t)np * Ty * L.nseg_row)) != FITRIG_OK) return rc;
      if ((rc = select_run(ctx, c, L, (float*)ctx->seg_max.p, mu, sigma, flags, FITRIG_IMAGE,
                           (const float*)ctx->cube_f.p, halo)) != FITRIG_OK)
        return rc;
      if (c.index_map)
        HIP_TRY(ctx, hipMemcpyAsync(c.index_map, ctx->cube_f.p, (size_t)np * ncell * 4, hipMemcpyDeviceToDevice, st));
    }
  }

  if ((rc = mark(3)) != FITRIG_OK) return rc;
  // ---- frequency branch ----------------------------------------------------
  const double* series = (const double*)ctx->cube.p;
  if (ring) {
    // the covered series: the newest slices of the history, then the newest
    // of this call's (oldest first); written back as the field's history
    const int64_t ntiles = (int64_t)Ty * Tx;
    const size_t sl = (size_t)ntiles * 8;
    const int from_call = std::min(np, nfreq);
    const int from_hist = nfreq - from_call;
    if ((rc = ensure(ctx, ctx->fseries, (size_t)nfreq * sl)) != FITRIG_OK) return rc;
    char* fs = (char*)ctx->fseries.p;
    if (from_hist > 0)
      HIP_TRY(ctx, hipMemcpyAsync(fs, (const char*)c.hist->in + (size_t)(c.hist->n_in - from_hist) * sl,
                                  (size_t)from_hist * sl, hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(fs + (size_t)from_hist * sl, (const char*)ctx->cube.p + (size_t)(np - from_call) * sl,
                                (size_t)from_call * sl, hipMemcpyDeviceToDevice, st));
    if (c.hist->out)
      HIP_TRY(ctx, hipMemcpyAsync(c.hist->out, fs, (size_t)nfreq * sl, hipMemcpyDeviceToDevice, st));
    series = (const double*)fs;
  }
  if (freq) {
    const int64_t ntiles = (int64_t)Ty * Tx;
    if ((rc = ensure(ctx, ctx->eta_d, ntiles * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->eta_f, ntiles * 4)) != FITRIG_OK) return rc;
    hipLaunchKernelGGL(k_eta, dim3(grid_for(ntiles, 256, 4096)), dim3(256), (size_t)2 * nfreq * 8, st, series, nfreq,
                       ntiles, cfg.harm, (double*)ctx->eta_d.p, (float*)ctx->eta_f.p);
    LAUNCH_CHECK(ctx);
    if (!robust) {
      if ((rc = moments(ctx, st, (const double*)ctx->eta_d.p, 1, ntiles, 1, ntiles, eta_mu, eta_sig, eta_flag)) !=
          FITRIG_OK)
        return rc;
    } else {
      if ((rc = robust_spread(ctx, st, (const float*)ctx->eta_f.p, 1, ntiles, true, eta_mu, eta_sig, eta_flag)) !=
          FITRIG_OK)
        return rc;
    }
    SegLayout L{Ty, Tx, 1, 1, 64, (Tx + 63) / 64, 1, Ty};
    // segment maxima of eta go to a region of seg_max past anything still in use
    const int64_t ne = (int64_t)Ty * L.nseg_row;
    if ((rc = ensure(ctx, ctx->seg_max2, (size_t)ne * 4)) != FITRIG_OK) return rc;
    float* smax = (float*)ctx->seg_max2.p;
    hipLaunchKernelGGL(k_segmax_direct, dim3(grid_for(ne)), dim3(256), 0, st, (const float*)ctx->eta_f.p, L, smax);
    if ((rc = ensure_selection(ctx, ne)) != FITRIG_OK) return rc;
    if ((rc = select_run(ctx, c, L, smax, eta_mu, eta_sig, eta_flag, FITRIG_FREQ, (const float*)ctx->eta_f.p, halo)) !=
        FITRIG_OK)
      return rc;
    if (c.eta_map)
      HIP_TRY(ctx, hipMemcpyAsync(c.eta_map, ctx->eta_f.p, (size_t)ntiles * 4, hipMemcpyDeviceToDevice, st));
  }

  // ---- per-pixel frequency branch -------------------------------------------
  if (fpx) {
    double* px_mu = (double*)ctx->eta_st.p + 4;
    double* px_sig = px_mu + 1;
    uint32_t* px_flag = (uint32_t*)(px_mu + 2);
    if ((rc = ensure(ctx, ctx->etapx_d, (size_t)plane * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->etapx_f, (size_t)plane * 4)) != FITRIG_OK) return rc;
    double* ed = (double*)ctx->etapx_d.p;
    float* ef = (float*)ctx->etapx_f.p;
    const dim3 g(grid_for(plane, 256, 8192)), b(256);
    const size_t lds = (size_t)(np / 2) * np * 16;  // at most 32 KB (n' <= 64)
    if (np <= 16)
      hipLaunchKernelGGL(k_eta_px<16>, g, b, lds, st, (const float*)qmap, np, plane, cfg.harm, ed, ef);
    else if (np <= 32)
      hipLaunchKernelGGL(k_eta_px<32>, g, b, lds, st, (const float*)qmap, np, plane, cfg.harm, ed, ef);
    else
      hipLaunchKernelGGL(k_eta_px<64>, g, b, lds, st, (const float*)qmap, np, plane, cfg.harm, ed, ef);
    LAUNCH_CHECK(ctx);
    if (!robust) {
      if ((rc = moments(ctx, st, (const double*)ed, 1, plane, 1, plane, px_mu, px_sig, px_flag)) != FITRIG_OK)
        return rc;
    } else {
      if ((rc = robust_spread(ctx, st, (const float*)ef, 1, plane, true, px_mu, px_sig, px_flag)) != FITRIG_OK)
        return rc;
    }
    SegLayout L{c.H, c.W, 1, 1, 64, (c.W + 63) / 64, 1, c.H};
    const int64_t ne = (int64_t)c.H * L.nseg_row;
    if ((rc = ensure(ctx, ctx->seg_max2, (size_t)ne * 4)) != FITRIG_OK) return rc;
    float* smax = (float*)ctx->seg_max2.p;
    hipLaunchKernelGGL(k_segmax_direct, dim3(grid_for(ne)), dim3(256), 0, st, (const float*)ef, L, smax);
    if ((rc = ensure_selection(ctx, ne)) != FITRIG_OK) return rc;
    if ((rc = select_run(ctx, c, L, smax, px_mu, px_sig, px_flag, FITRIG_FREQ_PIXEL, (const float*)ef, halo)) !=
        FITRIG_OK)
      return rc;
  }

  if (c.index_map && sliding && img && cfg.map_kind == FITRIG_MAP_TLISI) {
    hipLaunchKernelGGL(k_to_tlisi, dim3(grid_for((int64_t)np * plane, 256, 8192)), dim3(256), 0, st, c.index_map,
                       (int64_t)np * plane, (const double*)ctx->M.p);
    LAUNCH_CHECK(ctx);
  }

  if ((rc = mark(4)) != FITRIG_OK) return rc;
  // ---- results to the host --------------------------------------------------
  const size_t small = CNT_N * 8 + 8 + 32 + (size_t)np * (8 + 8 + 4);
  if ((rc = ensure_host(ctx, small)) != FITRIG_OK) return rc;
  char* h = (char*)ctx->h_stage;
  int64_t* h_cnt = (int64_t*)h;
  double* h_M = (double*)(h + CNT_N * 8);
  double* h_eta = (double*)(h + CNT_N * 8 + 8);
  double* h_mu = (double*)(h + CNT_N * 8 + 8 + 32);
  double* h_sig = h_mu + np;
  uint32_t* h_fl = (uint32_t*)(h_sig + np);
  HIP_TRY(ctx, hipMemcpyAsync(h_cnt, cnt, CNT_N * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h_M, ctx->M.p, 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h_eta, ctx->eta_st.p, 24, hipMemcpyDeviceToHost, st));
  if (img && sliding) {
    HIP_TRY(ctx, hipMemcpyAsync(h_mu, mu, (size_t)np * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemcpyAsync(h_sig, sigma, (size_t)np * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemcpyAsync(h_fl, flags, (size_t)np * 4, hipMemcpyDeviceToHost, st));
  } else if (img) {
    HIP_TRY(ctx, hipMemcpyAsync(h_mu, mu, (size_t)np * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemcpyAsync(h_sig, sigma, (size_t)np * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemcpyAsync(h_fl, flags, (size_t)np * 4, hipMemcpyDeviceToHost, st));
  }
  if ((rc = mark(5)) != FITRIG_OK) return rc;
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (prof) {
    for (int i = 0; i < FITRIG_N_PHASES; ++i) {
      float ms = 0.0f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
      ctx->phase_ms[i] = ms;
    }
    ctx->have_times = 1;
  }
  const int64_t total = h_cnt[CNT_OUTBASE];
  const bool trunc_internal = h_cnt[CNT_TRUNC] != 0;
  const int64_t ncopy = std::min<int64_t>(total, cand_cap);
  if (ncopy > 0 && cand) {
    HIP_TRY(ctx, hipMemcpyAsync(cand, ctx->c_out.p, (size_t)ncopy * sizeof(fitrig_candidate),
                                hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  *n_cand = total;
  if (stats) {
    stats->M = *h_M;
    stats->n_triples = np;
    stats->eta_mu = freq ? h_eta[0] : 0.0;
    stats->eta_sigma = freq ? h_eta[1] : 0.0;
    stats->n_image_cand = h_cnt[CNT_IMG];
    stats->n_freq_cand = h_cnt[CNT_FREQ];
    for (int s = 0; s < np; ++s) {
      const uint32_t tf = trunc_internal ? FITRIG_FLAG_TRUNC : 0u;
      if (stats->mu) stats->mu[s] = img ? h_mu[s] : 0.0;
      if (stats->sigma) stats->sigma[s] = img ? h_sig[s] : 0.0;
      if (stats->flags) stats->flags[s] = (img ? h_fl[s] : 0u) | tf;
    }
  }
  if (trunc_internal || total > cand_cap) return FITRIG_E_TRUNC;
  return FITRIG_OK;
}

fitrig_status validate_cfg(const fitrig_config* c) {
  if (!c || c->abi_version != FITRIG_ABI_VERSION) return FITRIG_E_INVAL;
  if (c->mode != FITRIG_SLIDING && c->mode != FITRIG_TILES) return FITRIG_E_INVAL;
  if (c->window < 1 || c->window % 2 == 0 || c->window > 2 * kMaxHalo + 1) return FITRIG_E_INVAL;
  if (c->tile < 1) return FITRIG_E_INVAL;
  if (c->branches < 1 || c->branches > 7) return FITRIG_E_INVAL;
  if ((c->branches & FITRIG_FREQ_PIXEL) && c->mode != FITRIG_SLIDING) return FITRIG_E_INVAL;
  if (c->sigma_est != FITRIG_MEAN_STD && c->sigma_est != FITRIG_MEDIAN_MAD) return FITRIG_E_INVAL;
  if (c->harm < 0 || c->harm == 1 || c->harm > 64) return FITRIG_E_INVAL;
  if (c->r_signed != 0 && c->r_signed != 1) return FITRIG_E_INVAL;
  if (c->map_kind != FITRIG_MAP_QTILDE && c->map_kind != FITRIG_MAP_TLISI) return FITRIG_E_INVAL;
  if (!(c->C > 0.0) || !isfinite(c->C)) return FITRIG_E_INVAL;
  if (c->max_pixels < 0 || c->max_snap < 0 || c->max_segments < 0) return FITRIG_E_INVAL;
  if (c->profile != 0 && c->profile != 1) return FITRIG_E_INVAL;
  return FITRIG_OK;
}

}  // namespace

extern "C" {

void fitrig_config_default(fitrig_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->abi_version = FITRIG_ABI_VERSION;
  cfg->mode = FITRIG_SLIDING;
  cfg->window = 7;
  cfg->tile = 32;
  cfg->branches = FITRIG_IMAGE | FITRIG_FREQ;
  cfg->sigma_est = FITRIG_MEAN_STD;
  cfg->harm = 0;
  cfg->r_signed = 0;
  cfg->map_kind = FITRIG_MAP_QTILDE;
  cfg->device = 0;
  cfg->C = 1e-6;
}

int32_t fitrig_abi_version(void) { return FITRIG_ABI_VERSION; }

int32_t fitrig_phase_times(const fitrig_ctx* ctx, double* ms, int32_t cap) {
  if (!ctx || !ms) return -1;
  if (!ctx->have_times) return 0;
  const int32_t n = cap < FITRIG_N_PHASES ? cap : FITRIG_N_PHASES;
  for (int32_t i = 0; i < n; ++i) ms[i] = ctx->phase_ms[i];
  return n < 0 ? 0 : n;
}

const char* fitrig_status_string(fitrig_status s) {
  switch (s) {
    case FITRIG_OK: return "ok";
    case FITRIG_E_INVAL: return "invalid argument";
    case FITRIG_E_NOMEM: return "out of memory";
    case FITRIG_E_HIP: return "HIP runtime error";
    case FITRIG_E_TRUNC: return "results truncated (capacity exceeded)";
    case FITRIG_E_BUSY: return "admission refused (busy)";
    case FITRIG_E_NOTREADY: return "result not ready";
    default: return "unknown status";
  }
}

int32_t fitrig_last_hip_error(const fitrig_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

fitrig_status fitrig_create(const fitrig_config* cfg, fitrig_ctx** out) {
  if (!out) return FITRIG_E_INVAL;
  *out = nullptr;
  fitrig_status rc = validate_cfg(cfg);
  if (rc != FITRIG_OK) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return FITRIG_E_INVAL;
  fitrig_ctx* ctx = new (std::nothrow) fitrig_ctx();
  if (!ctx) return FITRIG_E_NOMEM;
  ctx->cfg = *cfg;
  hipError_t e = hipSetDevice(cfg->device);
  // blocking stream: ordered after the legacy default stream, where callers
  // commonly produce the stack
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->stream, hipStreamDefault);
  for (int i = 0; e == hipSuccess && i <= FITRIG_N_PHASES; ++i) e = hipEventCreate(&ctx->ev[i]);
  if (e != hipSuccess) {
    fitrig_destroy(ctx);
    return FITRIG_E_HIP;
  }
  // Scratch sized from the capacity hints, so warm calls allocate nothing.
  if (cfg->max_pixels > 0 && cfg->max_snap >= 3) {
    const int64_t np = cfg->max_snap - 2;
    const int halo = cfg->window / 2;
    const int64_t Wd = (int64_t)ceil(sqrt((double)cfg->max_pixels));
    const int out_w = out_width(halo);
    const int64_t ncol = (Wd + out_w - 1) / out_w + 1;
    const int64_t nbands = (Wd + kBand - 1) / kBand + 1;
    const int64_t nwg = ncol * nbands;
    const int64_t nseg = np * (cfg->max_pixels / out_w + Wd) * kSegsPerGroup;
    if ((rc = ensure(ctx, ctx->stat_part, (size_t)(np * nwg * 16 * 16))) != FITRIG_OK ||
        (rc = ensure(ctx, ctx->seg_max, (size_t)(nseg * 4))) != FITRIG_OK ||
        (rc = ensure_selection(ctx, nseg)) != FITRIG_OK) {
      fitrig_destroy(ctx);
      return rc;
    }
  }
  *out = ctx;
  return FITRIG_OK;
}

fitrig_status fitrig_destroy(fitrig_ctx* ctx) {
  if (!ctx) return FITRIG_E_INVAL;
  (void)hipSetDevice(ctx->cfg.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  DevBuf* bufs[] = {&ctx->etapx_d, &ctx->etapx_f, &ctx->fseries, &ctx->mom_tmp, &ctx->max_key, &ctx->seg_max2, &ctx->stat_part, &ctx->seg_max,  &ctx->tile_part, &ctx->cube,    &ctx->cube_f,
                    &ctx->eta_d,     &ctx->eta_f,    &ctx->mu,        &ctx->sigma,    &ctx->flags,   &ctx->eta_st,
                    &ctx->M,         &ctx->qscratch, &ctx->hist,      &ctx->rs_state, &ctx->rs_med,  &ctx->rs_dev,
                    &ctx->chunk_cnt, &ctx->counters, &ctx->seg_entry, &ctx->seg_mask, &ctx->cell_q,  &ctx->parent,
                    &ctx->comp_of,   &ctx->c_root,   &ctx->c_npix,    &ctx->c_key,    &ctx->c_w,     &ctx->c_box,
                    &ctx->c_out,     &ctx->bflag,    &ctx->blk_entry, &ctx->blk_slot, &ctx->band_start,
                    &ctx->band_end,  &ctx->rowslot,  &ctx->rs_next,  &ctx->rs_samp,  &ctx->rs_gbuf,
                    &ctx->rs_bkt,    &ctx->rs_cnt,   &ctx->rs_nvalid, &ctx->rs_plan};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  for (int i = 0; i <= FITRIG_N_PHASES; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  delete ctx;
  return FITRIG_OK;
}

fitrig_status fitrig_detect(fitrig_ctx* ctx, const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H,
                            int32_t W, double sigma, fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                            float* index_map, float* eta_map, fitrig_stats* stats, void* hip_stream) {
  if (!ctx || !stack || !n_cand) return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  if (n_snap < 3 || H < 1 || W < 1) return FITRIG_E_INVAL;
  if ((uint64_t)H * (uint64_t)W >= (1ull << 32)) return FITRIG_E_INVAL;
  if (!(sigma > 0.0) || !isfinite(sigma)) return FITRIG_E_INVAL;
  if (cand_cap < 0 || (cand_cap > 0 && !cand)) return FITRIG_E_INVAL;
  *n_cand = 0;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FITRIG_E_HIP;
  Call c;
  c.stack = stack;
  c.carry0 = c.carry1 = nullptr;
  c.ncarry = 0;
  c.dtype = dtype;
  c.n = n_snap;
  c.H = H;
  c.W = W;
  c.tau = sigma;
  c.index_map = index_map;
  c.eta_map = eta_map;
  c.st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  c.hist = nullptr;
  return detect_impl(ctx, c, cand, cand_cap, n_cand, stats);
}

}  // extern "C"

namespace fitrig {

// Detect over [carried frames][new frames] (serving). The carried frames
// have the dtype and size of the stack.
fitrig_status detect_frames(fitrig_ctx* ctx, const void* carry0, const void* carry1, int ncarry, const void* stack,
                            fitrig_dtype dtype, int32_t n_new, int32_t H, int32_t W, double sigma,
                            fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand, fitrig_stats* stats,
                            void* hip_stream, const FreqHist* hist) {
  if (!ctx || !stack || !n_cand || ncarry < 0 || ncarry > 2) return FITRIG_E_INVAL;
  if (hist && (hist->n_in < 0 || hist->cap < 0 || hist->cap > 2048 || hist->n_in > hist->cap ||
               (hist->n_in > 0 && !hist->in)))
    return FITRIG_E_INVAL;
  if ((ncarry >= 1 && !carry0) || (ncarry == 2 && !carry1)) return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  if (n_new < 1 || ncarry + n_new < 3 || H < 1 || W < 1) return FITRIG_E_INVAL;
  if ((uint64_t)H * (uint64_t)W >= (1ull << 32)) return FITRIG_E_INVAL;
  if (!(sigma > 0.0) || !isfinite(sigma)) return FITRIG_E_INVAL;
  if (cand_cap < 0 || (cand_cap > 0 && !cand)) return FITRIG_E_INVAL;
  *n_cand = 0;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FITRIG_E_HIP;
  Call c;
  c.stack = stack;
  c.carry0 = carry0;
  c.carry1 = carry1;
  c.ncarry = ncarry;
  c.dtype = dtype;
  c.n = ncarry + n_new;
  c.H = H;
  c.W = W;
  c.tau = sigma;
  c.index_map = nullptr;
  c.eta_map = nullptr;
  c.st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  c.hist = hist;
  return detect_impl(ctx, c, cand, cand_cap, n_cand, stats);
}

hipStream_t ctx_stream(fitrig_ctx* ctx) { return ctx->stream; }
int32_t& ctx_last_hip(fitrig_ctx* ctx) { return ctx->last_hip; }

// Device bytes a context needs for one call of this size (admission).
int64_t scratch_estimate(const fitrig_config& cfg, int n, int H, int W) {
  const int64_t np = n - 2, plane = (int64_t)H * W;
  const int out_w = out_width(cfg.window / 2);
  const int64_t ncol = (W + out_w - 1) / out_w, nbands = (H + kBand - 1) / kBand;
  const int64_t nwg = ncol * nbands;
  const int64_t nseg = np * H * ncol * kSegsPerGroup;
  const int64_t segcap = cfg.max_segments > 0 ? cfg.max_segments : std::max<int64_t>(65536, std::min<int64_t>(nseg / 64, 1 << 22));
  const int64_t Ty = (H + cfg.tile - 1) / cfg.tile, Tx = (W + cfg.tile - 1) / cfg.tile;
  int64_t b = np * nwg * 256 + nseg * 4 + np * nbands * ncol * kPieces * 24 + np * Ty * Tx * 12;
  b += segcap * (8 + 8 + 64 * 12) + 2 * segcap * (4 + 4 + 8 + 48 + 16 + 2 * (int64_t)sizeof(fitrig_candidate));
  // median / MAD: the value map, plus the bracket gathers (about 4 % of it)
  if (cfg.sigma_est == FITRIG_MEDIAN_MAD) b += np * plane * 4 + np * plane / 2;
  // per-pixel frequency branch: the q map and the per-pixel spectrum maxima
  if (cfg.branches & FITRIG_FREQ_PIXEL) b += np * plane * 4 + plane * 12;
  return b;
}

}  // namespace fitrig
