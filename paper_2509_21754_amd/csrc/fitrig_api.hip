// FITrig host runtime and C ABI: context, scratch, launch sequence.
//
// One fitrig_detect call enqueues, on one stream:
//   0. the call record (stack pointers, tau, history pointers) into device
//      memory, which the kernels read;
//   1. the streaming index kernel (sliding mode) or the tile kernel (tile
//      mode / frequency-only), which read the stack once;
//   2. per-triple spread: FP64 moments of the kernel partials (mean / std),
//      or exact radix selection on the q map (median / MAD), every path
//      decision taken on the device;
//   3. image-branch selection: flags from the 64-cell segment maxima,
//      deterministic compaction, exact recompute of the flagged segments,
//      union-find 8-connected components, candidate records;
//   4. frequency branches: tile cube, eta per tile, spread of eta, selection
//      and components on the tile grid; per-pixel spectra on the matrix cores;
//   5. results packed into host-visible memory.
// Scratch sizes come from a sizing pass over the same sequence (no launch),
// so buffers grow, if at all, before anything of the call is enqueued.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <condition_variable>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "fitrig.h"
#include "fitrig_internal.h"
#include "fitrig_kernels.hip"

// Scratch of the allocation-free entry (fitrig_detect_noalloc): one array in
// the library's device code, so each GPU the library runs on holds its own
// copy until the process ends. Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): it uses the
// per-device address taken with hipGetSymbolAddress at fitrig_create.
static __device__ __align__(256) char scratch[FITRIG_NOALLOC_SCRATCH_BYTES];

namespace {

using namespace fitrig;

// Device address of `scratch` on each device (null until set up), the HIP
// error of a failed lookup, and a lock per device that serialises the
// allocation-free calls sharing that device's array.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_setup_mu;
void* g_scratch_ptr[kMaxDevices] = {};
int32_t g_scratch_err[kMaxDevices] = {};
std::mutex g_scratch_call_mu[kMaxDevices];

// Once per device, with that device current.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_setup_mu);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_scratch_ptr[dev] = p;
    g_scratch_err[dev] = 0;
  } else {
    g_scratch_err[dev] = e != hipSuccess ? (int32_t)e : (int32_t)hipErrorInvalidSymbol;
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;   // bytes owned (or carved from the arena)
  size_t want = 0;  // bytes the sizing pass asked for
};

// Host outputs of an asynchronous call, written by a host function on the
// call's stream once the results are in host-visible memory.
struct AsyncOut {
  fitrig_ctx* ctx;
  fitrig_candidate* cand;
  int64_t cand_cap;
  int64_t* n_cand;
  fitrig_stats* stats;
  double* mu;
  double* sigma;
  uint32_t* flags;
  int np;
  uint32_t ran;
  ResultLayout R;
  bool captured;  // recorded into a graph: replays reuse it, freed with the context
  bool direct;    // the records went straight into cand (page-locked)
};

// A launch sequence captured for one call shape (serving slots).
struct GraphKey {
  int n, H, W, ncarry, dtype, hist_cap, hist_n_in, hist_out, px_cap, px_n;
  int64_t cand_cap;
  int maps;  // bit 0: index map, bit 1: eta map, bit 2: per-pixel eta map (the kernels chosen depend on them)
  bool operator==(const GraphKey& o) const {
    return n == o.n && H == o.H && W == o.W && ncarry == o.ncarry && dtype == o.dtype && hist_cap == o.hist_cap &&
           hist_n_in == o.hist_n_in && hist_out == o.hist_out && px_cap == o.px_cap && px_n == o.px_n &&
           cand_cap == o.cand_cap && maps == o.maps;
  }
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  uint64_t gen;
  int64_t last_use;
};
constexpr size_t kMaxGraphs = 64;

}  // namespace

struct fitrig_ctx {
  fitrig_config cfg;
  hipStream_t stream = nullptr;
  int32_t last_hip = 0;
  bool sizing = false;      // sizing pass: record sizes, enqueue nothing
  bool in_arena = false;    // scratch carved from a fixed device arena (allocation-free entry)
  char* arena = nullptr;
  size_t arena_cap = 0;
  DevBuf call, stat_part, seg_max, seg_max2, tile_part, cube, cube_f, eta_d, eta_f, mu, sigma, flags, eta_st, M;
  DevBuf qscratch, fseries, etapx_f, pxpart, tw, tw_px, mom_tmp, max_key;
  DevBuf hist, rs_state, rs_med, rs_dev, rs_next, chunk_cnt, counters;
  DevBuf rs_samp, rs_gbuf, rs_bkt, rs_cnt, rs_nvalid, rs_plan, rs_gate;
  DevBuf seg_entry, seg_mask, cell_q, parent, comp_of, c_root, c_npix, c_key, c_w, c_box, c_out;
  DevBuf bflag, blk_entry, blk_slot, band_start, band_end, rowslot;
  DevBuf res_dev;           // results for the allocation-free entry (device memory)
  int64_t seg_cap = 0, comp_cap = 0;
  // host-visible results (mapped pinned memory)
  char* h_stage = nullptr;
  char* h_stage_dev = nullptr;
  size_t h_stage_cap = 0, h_want = 0;
  hipEvent_t ev[FITRIG_N_PHASES + 1] = {};
  bool ev_recorded = false;
  std::vector<AsyncOut*> captured_outs;
  // serving slot: calls are synchronous on the context's own stream, so
  // scratch growth waits for that stream only; launch sequences are captured
  // into HIP graphs per call shape and replayed
  bool serving = false;
  bool use_graphs = false;
  hipGraph_t rec_graph = nullptr;       // set while a launch sequence is built as a graph
  hipGraphNode_t rec_last = nullptr;    // its last node (nodes form one chain)
  hipError_t launch_err = hipSuccess;   // first launch error since the last check
  uint64_t gen = 0;  // bumps whenever scratch moves (graphs hold its addresses)
  std::vector<GraphEntry> graphs;
  int64_t graph_clock = 0;
  int64_t graph_replays = 0;
};

namespace {
// Every scratch buffer of a context (sizing, growth, arena carving, release).
DevBuf fitrig_ctx::* const kBufs[] = {
    &fitrig_ctx::call,      &fitrig_ctx::stat_part, &fitrig_ctx::seg_max,    &fitrig_ctx::seg_max2,
    &fitrig_ctx::tile_part, &fitrig_ctx::cube,      &fitrig_ctx::cube_f,     &fitrig_ctx::eta_d,
    &fitrig_ctx::eta_f,     &fitrig_ctx::mu,        &fitrig_ctx::sigma,      &fitrig_ctx::flags,
    &fitrig_ctx::eta_st,    &fitrig_ctx::M,         &fitrig_ctx::qscratch,   &fitrig_ctx::fseries,
    &fitrig_ctx::etapx_f,   &fitrig_ctx::pxpart,    &fitrig_ctx::tw,         &fitrig_ctx::tw_px,
    &fitrig_ctx::mom_tmp,   &fitrig_ctx::max_key,   &fitrig_ctx::hist,       &fitrig_ctx::rs_state,
    &fitrig_ctx::rs_med,    &fitrig_ctx::rs_dev,    &fitrig_ctx::rs_next,    &fitrig_ctx::chunk_cnt,
    &fitrig_ctx::counters,  &fitrig_ctx::rs_samp,   &fitrig_ctx::rs_gbuf,    &fitrig_ctx::rs_bkt,
    &fitrig_ctx::rs_cnt,    &fitrig_ctx::rs_nvalid, &fitrig_ctx::rs_plan,    &fitrig_ctx::rs_gate,
    &fitrig_ctx::seg_entry, &fitrig_ctx::seg_mask,  &fitrig_ctx::cell_q,     &fitrig_ctx::parent,
    &fitrig_ctx::comp_of,   &fitrig_ctx::c_root,    &fitrig_ctx::c_npix,     &fitrig_ctx::c_key,
    &fitrig_ctx::c_w,       &fitrig_ctx::c_box,     &fitrig_ctx::c_out,      &fitrig_ctx::bflag,
    &fitrig_ctx::blk_entry, &fitrig_ctx::blk_slot,  &fitrig_ctx::band_start, &fitrig_ctx::band_end,
    &fitrig_ctx::rowslot,   &fitrig_ctx::res_dev};
constexpr size_t kNBufs = sizeof(kBufs) / sizeof(kBufs[0]);
}  // namespace

namespace {

#define HIP_TRY(ctx, expr)                      \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      (ctx)->last_hip = (int32_t)e_;            \
      return (e_ == hipErrorOutOfMemory) ? FITRIG_E_NOMEM : FITRIG_E_HIP; \
    }                                           \
  } while (0)

// Launches a kernel (args: pointers to its argument values), or, while a
// graph is being built (ctx->rec_graph), appends it as a kernel node after
// the previous node. Graphs are built node by node rather than by stream
// capture, which would forbid device-wide synchronisation in every other
// thread of the process while it lasts.
hipError_t launch_raw(fitrig_ctx* ctx, const void* fn, dim3 g, dim3 b, size_t sh, hipStream_t st, void** args) {
  if (!fn) return hipErrorInvalidDeviceFunction;
  if (!ctx->rec_graph) return hipLaunchKernel(fn, g, b, args, sh, st);
  hipKernelNodeParams p;
  memset(&p, 0, sizeof(p));
  p.func = const_cast<void*>(fn);
  p.gridDim = g;
  p.blockDim = b;
  p.sharedMemBytes = (unsigned int)sh;
  p.kernelParams = args;
  p.extra = nullptr;
  hipGraphNode_t n = nullptr;
  const hipError_t e =
      hipGraphAddKernelNode(&n, ctx->rec_graph, ctx->rec_last ? &ctx->rec_last : nullptr, ctx->rec_last ? 1 : 0, &p);
  if (e == hipSuccess) ctx->rec_last = n;
  return e;
}

// Device-to-device copy on the stream, or a copy node while building a graph.
hipError_t copy_d2d(fitrig_ctx* ctx, void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!ctx->rec_graph) return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  hipGraphNode_t n = nullptr;
  const hipError_t e = hipGraphAddMemcpyNode1D(&n, ctx->rec_graph, ctx->rec_last ? &ctx->rec_last : nullptr,
                                               ctx->rec_last ? 1 : 0, dst, src, bytes, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) ctx->rec_last = n;
  return e;
}

// Typed front end of launch_raw: the arguments are converted to the kernel's
// parameter types and passed by address.
template <typename... P, typename... A, size_t... I>
hipError_t launch_k_impl(fitrig_ctx* ctx, void (*k)(P...), dim3 g, dim3 b, size_t sh, hipStream_t st,
                         std::index_sequence<I...>, A&&... a) {
  std::tuple<std::decay_t<P>...> vals(static_cast<std::decay_t<P>>(std::forward<A>(a))...);
  void* ptrs[sizeof...(P) + 1] = {(void*)&std::get<I>(vals)...};
  return launch_raw(ctx, (const void*)k, g, b, sh, st, ptrs);
}
template <typename... P, typename... A>
hipError_t launch_k(fitrig_ctx* ctx, void (*k)(P...), dim3 g, dim3 b, size_t sh, hipStream_t st, A&&... a) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  return launch_k_impl(ctx, k, g, b, sh, st, std::index_sequence_for<P...>{}, std::forward<A>(a)...);
}

void note_launch(fitrig_ctx* ctx, hipError_t e) {
  if (e != hipSuccess && ctx->launch_err == hipSuccess) ctx->launch_err = e;
}

// Launch only in the launch pass.
#define KL(k, g, b, sh, st, ...)                                        \
  do {                                                                  \
    if (!ctx->sizing) note_launch(ctx, launch_k(ctx, k, g, b, sh, st, __VA_ARGS__)); \
  } while (0)
#define LAUNCH_CHECK(ctx)                                               \
  do {                                                                  \
    if (!(ctx)->sizing) {                                               \
      hipError_t le_ = (ctx)->launch_err;                               \
      (ctx)->launch_err = hipSuccess;                                   \
      if (le_ == hipSuccess && !(ctx)->rec_graph) le_ = hipGetLastError(); \
      HIP_TRY(ctx, le_);                                                \
    }                                                                   \
  } while (0)

// Records (sizing pass) or checks (launch pass) a scratch buffer's size.
fitrig_status ensure(fitrig_ctx* ctx, DevBuf& b, size_t bytes) {
  bytes = (std::max<size_t>(bytes, 64) + 255) & ~(size_t)255;
  if (ctx->sizing) {
    b.want = std::max(b.want, bytes);
    return FITRIG_OK;
  }
  return b.cap >= bytes ? FITRIG_OK : FITRIG_E_NOMEM;  // the sizing pass covers every request
}

fitrig_status ensure_host(fitrig_ctx* ctx, size_t bytes) {
  if (ctx->sizing) ctx->h_want = std::max(ctx->h_want, bytes);
  return FITRIG_OK;
}

// Grows the buffers the sizing pass asked for (before anything of the call is
// enqueued). Earlier calls may still use the old buffers, so growth waits for
// the device; it is refused while the stream is capturing.
fitrig_status provision(fitrig_ctx* ctx, hipStream_t st) {
  if (ctx->in_arena) {
    size_t off = 0;
    for (DevBuf fitrig_ctx::* m : kBufs) {
      DevBuf& b = ctx->*m;
      b.p = b.want ? ctx->arena + off : nullptr;
      b.cap = b.want;
      off += b.want;
    }
    return off <= ctx->arena_cap ? FITRIG_OK : FITRIG_E_SCRATCH;
  }
  bool grow = ctx->h_want > ctx->h_stage_cap;
  for (DevBuf fitrig_ctx::* m : kBufs) grow = grow || (ctx->*m).want > (ctx->*m).cap;
  if (!grow) return FITRIG_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(ctx, hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return FITRIG_E_INVAL;
  // a serving slot's calls all ran synchronously on its own stream
  if (ctx->serving)
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  else
    HIP_TRY(ctx, hipDeviceSynchronize());
  ++ctx->gen;
  for (DevBuf fitrig_ctx::* m : kBufs) {
    DevBuf& b = ctx->*m;
    if (b.want <= b.cap) continue;
    if (b.p) HIP_TRY(ctx, hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    HIP_TRY(ctx, hipMalloc(&b.p, b.want));
    b.cap = b.want;
  }
  if (ctx->h_want > ctx->h_stage_cap) {
    if (ctx->h_stage) HIP_TRY(ctx, hipHostFree(ctx->h_stage));
    ctx->h_stage = ctx->h_stage_dev = nullptr;
    ctx->h_stage_cap = 0;
    const size_t bytes = std::max<size_t>(ctx->h_want, 1 << 16);
    HIP_TRY(ctx, hipHostMalloc((void**)&ctx->h_stage, bytes, hipHostMallocMapped));
    HIP_TRY(ctx, hipHostGetDevicePointer((void**)&ctx->h_stage_dev, ctx->h_stage, 0));
    ctx->h_stage_cap = bytes;
  }
  return FITRIG_OK;
}

void clear_wants(fitrig_ctx* ctx) {
  for (DevBuf fitrig_ctx::* m : kBufs) (ctx->*m).want = 0;
  ctx->h_want = 0;
}

int grid_for(int64_t n, int per = 256, int maxg = 8192) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

// Kernels templated on the storage type: one argument struct by value (the
// stack maximum: three arguments).
bool dispatch_stream(fitrig_ctx* ctx, int dt, int halo, bool rs, dim3 g, hipStream_t st, const StreamArgs& A) {
  const bool q = A.qmap != nullptr;
  const void* fn = dt == FITRIG_F32 ? kernel_stream_f32(halo, rs, q)
                   : dt == FITRIG_F16 ? kernel_stream_f16(halo, rs, q)
                                      : kernel_stream_bf16(halo, rs, q);
  if (!fn) return false;
  void* a[] = {(void*)&A};
  note_launch(ctx, launch_raw(ctx, fn, g, dim3(kLanes), 0, st, a));
  return true;
}
bool dispatch_tile_stream(fitrig_ctx* ctx, int dt, int tile, bool rs, dim3 g, hipStream_t st,
                          const TileStreamArgs& A) {
  const void* fn = dt == FITRIG_F32 ? kernel_tile_stream_f32(tile, rs)
                   : dt == FITRIG_F16 ? kernel_tile_stream_f16(tile, rs)
                                      : kernel_tile_stream_bf16(tile, rs);
  if (!fn) return false;
  void* a[] = {(void*)&A};
  note_launch(ctx, launch_raw(ctx, fn, g, dim3(kLanes), 0, st, a));
  return true;
}
bool dispatch_tile(fitrig_ctx* ctx, int dt, bool rs, dim3 g, hipStream_t st, const TileArgs& A) {
  const void* fn = dt == FITRIG_F32 ? kernel_tile_f32(rs) : dt == FITRIG_F16 ? kernel_tile_f16(rs) : kernel_tile_bf16(rs);
  if (!fn) return false;
  void* a[] = {(void*)&A};
  note_launch(ctx, launch_raw(ctx, fn, g, dim3(kLanes), 0, st, a));
  return true;
}
bool dispatch_recompute(fitrig_ctx* ctx, int dt, int halo, bool rs, dim3 g, hipStream_t st, const RecomputeArgs& R) {
  const void* fn = dt == FITRIG_F32 ? kernel_recompute_f32(halo, rs)
                   : dt == FITRIG_F16 ? kernel_recompute_f16(halo, rs)
                                      : kernel_recompute_bf16(halo, rs);
  if (!fn) return false;
  void* a[] = {(void*)&R};
  note_launch(ctx, launch_raw(ctx, fn, g, dim3(64), 0, st, a));
  return true;
}
bool dispatch_stack_max(fitrig_ctx* ctx, int dt, dim3 g, hipStream_t st, const CallDev* cd, int64_t n,
                        uint32_t* mk) {
  const void* fn = dt == FITRIG_F32 ? kernel_stack_max_f32() : dt == FITRIG_F16 ? kernel_stack_max_f16()
                                                                                 : kernel_stack_max_bf16();
  if (!fn) return false;
  void* a[] = {(void*)&cd, (void*)&n, (void*)&mk};
  note_launch(ctx, launch_raw(ctx, fn, g, dim3(256), 0, st, a));
  return true;
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
  float* eta_px_map;
  hipStream_t st;
  const FreqHist* hist;   // serving: frequency branch over the field's recent triples, nullable
  int64_t cand_cap;       // candidates delivered to the host
};

// What runs for a call, from the config and the shape.
struct Plan {
  int np;
  bool sliding, img, robust, freq, ring, fpx, pring, cube_needed, qpass;
  int nfreq;
  int npx;  // series length of the per-pixel branch
};

Plan make_plan(const fitrig_config& cfg, const Call& c) {
  Plan p;
  p.np = c.n - 2;
  p.sliding = cfg.mode == FITRIG_SLIDING;
  p.img = (cfg.branches & FITRIG_IMAGE) != 0;
  p.robust = cfg.sigma_est == FITRIG_MEDIAN_MAD;
  // frequency branch: over this call's triples, or (with a history) over
  // the last hist->cap triples of [history | this call]
  const bool want_freq = (cfg.branches & FITRIG_FREQ) != 0;
  p.ring = want_freq && c.hist && c.hist->cap > 0;
  p.nfreq = p.ring ? (int)std::min<int64_t>(c.hist->cap, (int64_t)c.hist->n_in + p.np) : p.np;
  p.freq = want_freq && p.nfreq >= 4 && !(c.hist && c.hist->defer);
  // per-pixel branch: over this call's maps, or (serving) over the last
  // px_cap of [the field's kept maps | this call's]
  const bool want_px = (cfg.branches & FITRIG_FREQ_PIXEL) != 0 && p.sliding;
  p.pring = want_px && c.hist && c.hist->px_cap > 0;
  p.npx = p.pring ? (int)std::min<int64_t>(c.hist->px_cap, (int64_t)c.hist->px_n + p.np) : p.np;
  p.fpx = want_px && p.npx >= 4 && !(c.hist && c.hist->defer);
  // the tile cube: frequency branch, history, tile-mode image branch or map
  p.cube_needed = p.freq || p.ring || (!p.sliding && (p.img || c.index_map));
  // the streaming sliding pass: image branch, per-pixel spectra (or their
  // kept maps) or the map
  p.qpass = p.sliding && (p.img || p.fpx || p.pring || c.index_map);
  return p;
}

ResultLayout result_layout(int np, int64_t cap) {
  ResultLayout R;
  R.off_cnt = 0;
  R.off_scalars = CNT_N * 8;
  R.off_mu = R.off_scalars + (1 + ES_N) * 8;
  R.off_sigma = R.off_mu + (int64_t)np * 8;
  R.off_flags = R.off_sigma + (int64_t)np * 8;
  R.off_cand = (R.off_flags + (int64_t)np * 4 + 7) & ~(int64_t)7;
  R.bytes = R.off_cand + cap * (int64_t)sizeof(fitrig_candidate);
  return R;
}

// Mean / population std per set, two fixed-order stages.
fitrig_status moments(fitrig_ctx* ctx, hipStream_t st, const double* src, int nsets, int64_t nparts, int raw,
                      int64_t count, double* mu, double* sigma, uint32_t* flags) {
  const int G = (int)std::min<int64_t>(64, std::max<int64_t>(1, nparts / 4096));
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->mom_tmp, (size_t)nsets * G * 16)) != FITRIG_OK) return rc;
  KL(k_moments_part, dim3(G, nsets), dim3(256), 0, st, src, nparts, raw, (double*)ctx->mom_tmp.p);
  KL(k_moments, dim3(nsets), dim3(256), 0, st, (const double*)ctx->mom_tmp.p, (int64_t)G, 0, count, mu, sigma,
     flags);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Exact order statistics rank_lo (and rank_hi) of the keys of every set whose
// gate entry equals `want` (gate null: every set). Three-pass radix
// selection (11, 11, 10 bits); the upper middle one of an even count from one
// more counting pass. n_max: largest number of valid keys in a set (sizes the
// grids: about 8 K keys per workgroup).
fitrig_status rs_select_middle(fitrig_ctx* ctx, hipStream_t st, const float* vals, int nsets, int64_t per_set,
                               int kmode, int vmode, const double* med, const unsigned long long* nvalid,
                               const unsigned long long* base, int64_t rank_lo, int64_t rank_hi, int64_t n_max,
                               double* out, const uint32_t* gate, uint32_t want, const uint32_t* kb = nullptr) {
  uint32_t* hist = (uint32_t*)ctx->hist.p;
  RsState* rs = (RsState*)ctx->rs_state.p;
  unsigned long long* cnt_le = (unsigned long long*)ctx->rs_next.p;
  uint32_t* min_gt = (uint32_t*)(cnt_le + nsets);
  const int shifts[3] = {21, 10, 0};
  const int nbits[3] = {11, 11, 10};
  const int gx = grid_for(n_max, 1 << 13, 1024);
  const dim3 g1((nsets + 63) / 64);
  if (base)
    KL(k_rs_init_gathered, g1, dim3(64), 0, st, rs, nsets, rank_lo, base, kb, gate, want);
  else
    KL(k_rs_init_rank, g1, dim3(64), 0, st, rs, nsets, rank_lo, gate, want);
  // upper middle value (even counts): from the last digit's histogram when
  // it holds it, else by a counting pass over the values (need[s] = 1)
  const bool two = rank_hi != rank_lo;
  uint32_t* need = min_gt + nsets;
  if (two) {
    KL(k_fill_i64, dim3(1), dim3(64), 0, st, (int64_t*)cnt_le, (int64_t)nsets, (int64_t)0);
    KL(k_fill_u32, dim3(1), dim3(64), 0, st, min_gt, (int64_t)nsets, 0xFFFFFFFFu);
    KL(k_fill_u32, dim3(1), dim3(64), 0, st, need, (int64_t)nsets, 1u);
  }
  for (int p = 0; p < 3; ++p) {
    KL(k_rs_hist, dim3(gx, nsets), dim3(256), 0, st, vals, per_set, kmode, med, (const RsState*)rs, shifts[p],
       nbits[p], hist, nvalid, gate, want);
    const RsNext nx = (two && p == 2) ? RsNext{cnt_le, min_gt, need} : RsNext{nullptr, nullptr, nullptr};
    KL(k_rs_pick, dim3(nsets), dim3(256), 0, st, rs, hist, shifts[p], nbits[p], gate, want, nx);
  }
  KL(k_rs_store, g1, dim3(64), 0, st, (const RsState*)rs, nsets, vmode, 0, out, gate, want);
  if (two) {
    KL(k_rs_next, dim3(gx, nsets), dim3(256), 0, st, vals, per_set, kmode, med, (const RsState*)rs, cnt_le, min_gt,
       nvalid, gate, want, (const uint32_t*)need);
    KL(k_rs_next_store, g1, dim3(64), 0, st, (const RsState*)rs, nsets, rank_hi, vmode,
       (const unsigned long long*)cnt_le, (const uint32_t*)min_gt, base, out, gate, want);
  } else {
    KL(k_rs_store, g1, dim3(64), 0, st, (const RsState*)rs, nsets, vmode, 1, out, gate, want);
  }
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Sample order statistics a and b of each set's sample (keys) -> bkt[2 s],
// bkt[2 s + 1].
void sample_bracket(fitrig_ctx* ctx, hipStream_t st, const uint32_t* samp, int nsets, int64_t S, int64_t a, int64_t b,
                    uint32_t* bkt, const uint32_t* gate, uint32_t want) {
  RsState* rs = (RsState*)ctx->rs_state.p;
  const int shifts[3] = {21, 10, 0};
  const int nbits[3] = {11, 11, 10};
  const dim3 g1((nsets + 63) / 64);
  for (int w = 0; w < 2; ++w) {
    KL(k_rs_init_rank, g1, dim3(64), 0, st, rs, nsets, w ? b : a, gate, want);
    for (int p = 0; p < 3; ++p) {
      KL(k_rs_hist, dim3(grid_for(S, 1 << 13, 1024), nsets), dim3(256), 0, st, (const float*)samp, S, 2,
         (const double*)nullptr, (const RsState*)rs, shifts[p], nbits[p], (uint32_t*)ctx->hist.p,
         (const unsigned long long*)nullptr, gate, want);
      KL(k_rs_pick, dim3(nsets), dim3(256), 0, st, rs, (uint32_t*)ctx->hist.p, shifts[p], nbits[p], gate, want,
         RsNext{nullptr, nullptr, nullptr});
    }
    KL(k_rs_key_out, g1, dim3(64), 0, st, (const RsState*)rs, nsets, w, bkt, gate, want);
  }
}

// Robust spread per set (median and MAD): mu = median of the values,
// sigma = 1.482602218505602 * median |q - mu| (two middle order statistics
// averaged for an even count), by exact radix selection.
// Large sets select inside brackets taken from a hashed sample: one pass
// over the values gathers the cells of both the median bracket and a MAD
// window placed around the sample median (k_rs_gather2). Each set's path is
// decided on the device: a bracket that misses a middle rank or overflows
// its buffer sends the set to the full-array selection (median) or to a
// fallback bracket pass around the exact median, and from there to the full
// selection (MAD). The host enqueues every path; kernels of a path skip the
// sets not on it. Same keys, same order statistics on every path.
// nonneg: every value is +0 or positive (q with |x_hat| in Eq. (4), eta).
fitrig_status robust_spread(fitrig_ctx* ctx, hipStream_t st, const float* vals, int nsets, int64_t per_set,
                            bool nonneg, double* mu, double* sigma, uint32_t* flags, int64_t pre_S = 0) {
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->hist, (size_t)nsets * kHistBins * 4)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_state, (size_t)nsets * sizeof(RsState))) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_med, (size_t)nsets * 2 * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_dev, (size_t)nsets * 2 * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->rs_next, (size_t)nsets * 16)) != FITRIG_OK) return rc;
  KL(k_fill_u32, dim3(grid_for((int64_t)nsets * kHistBins)), dim3(256), 0, st, (uint32_t*)ctx->hist.p,
     (int64_t)nsets * kHistBins, 0u);
  const int64_t r_lo = (per_set - 1) / 2, r_hi = per_set / 2;
  double* med_out = (double*)ctx->rs_med.p;
  double* dev_out = (double*)ctx->rs_dev.p;
  const dim3 g1d((nsets + 63) / 64);
  auto finish = [&](int mode) {
    KL(k_rs_finish, g1d, dim3(64), 0, st, (const double*)med_out, (const double*)dev_out, nsets, mu, sigma, flags,
       mode);
  };
  constexpr int64_t kSample = kRsSample;
  if (per_set < 8 * kSample) {
    for (int mode = 0; mode < 2; ++mode) {
      if ((rc = rs_select_middle(ctx, st, vals, nsets, per_set, mode, mode, mu, nullptr, nullptr, r_lo, r_hi, per_set,
                                 mode ? dev_out : med_out, nullptr, 0u)) != FITRIG_OK)
        return rc;
      finish(mode);
    }
    LAUNCH_CHECK(ctx);
    return FITRIG_OK;
  }

  // pre_S > 0: the sample (pre_S order keys per set, at least 2^20 and below
  // 2^21) is already in rs_samp, written by the index pass on a grid of cells
  // 16 or more apart; otherwise 2^20 hashed positions are read from the values
  const int64_t S = pre_S > 0 ? pre_S : kSample;
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
      (rc = ensure(ctx, ctx->rs_bkt, (size_t)nsets * 10 * 4)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_cnt, (size_t)nsets * 4 * 8)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_nvalid, (size_t)nsets * 2 * 8)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_plan, (size_t)nsets * 5 * 8)) != FITRIG_OK ||
      (rc = ensure(ctx, ctx->rs_gate, (size_t)nsets * 2 * 4)) != FITRIG_OK)
    return rc;
  uint32_t* samp = (uint32_t*)ctx->rs_samp.p;
  uint32_t* bkt0 = (uint32_t*)ctx->rs_bkt.p;
  uint32_t* bkt1 = bkt0 + 2 * nsets;
  uint32_t* wk = bkt0 + 4 * nsets;
  uint32_t* dkb = bkt0 + 8 * nsets;  // bounds of the MAD window's keys
  unsigned long long* cnt0 = (unsigned long long*)ctx->rs_cnt.p;
  unsigned long long* cnt1 = cnt0 + 2 * nsets;
  unsigned long long* nv0 = (unsigned long long*)ctx->rs_nvalid.p;
  unsigned long long* nv1 = nv0 + nsets;
  uint32_t* g0 = (uint32_t*)ctx->rs_gbuf.p;
  uint32_t* g1 = g0 + (size_t)nsets * cap0;
  double* pl = (double*)ctx->rs_plan.p;
  double* mhat = pl + 4 * nsets;
  uint32_t* gate_med = (uint32_t*)ctx->rs_gate.p;
  uint32_t* gate_mad = gate_med + nsets;
  const dim3 gs(grid_for(S, 256, 1024), nsets);

  // brackets from the sample: median keys, then the MAD window around its midpoint
  if (pre_S <= 0)
    KL(k_rs_sample, gs, dim3(256), 0, st, vals, per_set, 0, (const double*)nullptr, S, mult, samp,
       (const uint32_t*)nullptr, 0u);
  sample_bracket(ctx, st, samp, nsets, S, a, b, bkt0, nullptr, 0u);
  KL(k_rs_mad_center, g1d, dim3(64), 0, st, (const uint32_t*)bkt0, nsets, pl, mhat);
  KL(k_rs_sample_dev, gs, dim3(256), 0, st, samp, S, (const double*)mhat, (const uint32_t*)nullptr, 0u);
  sample_bracket(ctx, st, samp, nsets, S, a, b, bkt1, nullptr, 0u);
  KL(k_rs_mad_window, g1d, dim3(64), 0, st, (const uint32_t*)bkt1, nsets, pl, wk);
  // one pass over the values for both
  KL(k_fill_i64, dim3(1), dim3(256), 0, st, (int64_t*)cnt0, (int64_t)(4 * nsets), (int64_t)0);
  const dim3 gg(grid_for(per_set, kGather2Round * 2, 1024), nsets);
#define GATHER2(V, NN)                                                                                        \
  KL((k_rs_gather2<V, NN>), gg, dim3(256), 0, st, vals, per_set, (const uint32_t*)bkt0, (const uint32_t*)wk, cap0, \
     cap1, cnt0, cnt1, g0, g1)
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
  KL(k_rs_plan, g1d, dim3(64), 0, st, (const unsigned long long*)cnt0, nsets, cap0, r_lo, r_hi, gate_med, 0u,
     kPathGathered, kPathFull, nv0);
  KL(k_rs_plan, g1d, dim3(64), 0, st, (const unsigned long long*)cnt1, nsets, cap1, r_lo, r_hi, gate_mad, 0u,
     kPathGathered, kPathFallback, nv1);
  // median: inside the bracket (rank offsets at cnt0[2 s]), or over the whole set
  if ((rc = rs_select_middle(ctx, st, (const float*)g0, nsets, cap0, 2, 0, mu, nv0, cnt0, r_lo, r_hi, cap0, med_out,
                             gate_med, kPathGathered, bkt0)) != FITRIG_OK ||
      (rc = rs_select_middle(ctx, st, vals, nsets, per_set, 0, 0, mu, nullptr, nullptr, r_lo, r_hi, per_set, med_out,
                             gate_med, kPathFull)) != FITRIG_OK)
    return rc;
  finish(0);
  // MAD inside the window (g1 holds the values q: keys |q - med| are formed
  // as the passes read them), then verified against the exact median
  KL(k_rs_mad_keybounds, g1d, dim3(64), 0, st, (const double*)pl, (const double*)mu, (const uint32_t*)wk, nsets,
     (const uint32_t*)gate_mad, kPathGathered, dkb);
  if ((rc = rs_select_middle(ctx, st, (const float*)g1, nsets, cap1, 1, 1, mu, nv1, cnt1, r_lo, r_hi, cap1, dev_out,
                             gate_mad, kPathGathered, dkb)) != FITRIG_OK)
    return rc;
  KL(k_rs_mad_verify, g1d, dim3(64), 0, st, (const double*)pl, (const double*)mu, (const double*)dev_out,
     (const unsigned long long*)cnt1, nsets, gate_mad);
  // fallback: a bracket pass of its own around the exact median
  KL(k_rs_sample, gs, dim3(256), 0, st, vals, per_set, 1, (const double*)mu, S, mult, samp, (const uint32_t*)gate_mad,
     kPathFallback);
  sample_bracket(ctx, st, samp, nsets, S, a, b, bkt1, gate_mad, kPathFallback);
  KL(k_fill_i64, dim3(1), dim3(64), 0, st, (int64_t*)cnt1, (int64_t)(2 * nsets), (int64_t)0);
  const dim3 g1g(grid_for(per_set, 256 * 16, 512), nsets);
  if (vec)
    KL(k_rs_gather<true>, g1g, dim3(256), 0, st, vals, per_set, 1, (const double*)mu, (const uint32_t*)bkt1, cap1,
       cnt1, g1, (const uint32_t*)gate_mad, kPathFallback);
  else
    KL(k_rs_gather<false>, g1g, dim3(256), 0, st, vals, per_set, 1, (const double*)mu, (const uint32_t*)bkt1, cap1,
       cnt1, g1, (const uint32_t*)gate_mad, kPathFallback);
  KL(k_rs_plan, g1d, dim3(64), 0, st, (const unsigned long long*)cnt1, nsets, cap1, r_lo, r_hi, gate_mad,
     kPathFallback, kPathFallback, kPathFull, nv1);
  if ((rc = rs_select_middle(ctx, st, (const float*)g1, nsets, cap1, 2, 1, mu, nv1, cnt1, r_lo, r_hi, cap1, dev_out,
                             gate_mad, kPathFallback, bkt1)) != FITRIG_OK ||
      (rc = rs_select_middle(ctx, st, vals, nsets, per_set, 1, 1, mu, nullptr, nullptr, r_lo, r_hi, per_set, dev_out,
                             gate_mad, kPathFull)) != FITRIG_OK)
    return rc;
  finish(1);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Deterministic compaction: count, scan, write. The element count is read on
// the device (ne_dyn, at most cap * mult entries); the grid and the chunk
// counts are sized from that bound. The bound, not the pointer, decides the
// size: in the sizing pass of a fresh context the counters are not allocated
// yet and ne_dyn may be a null offset.
template <class F, class E>
fitrig_status compact(fitrig_ctx* ctx, hipStream_t st, F f, E e, int64_t ne_static, const int64_t* ne_dyn,
                      int64_t cap, int mult, int64_t* total) {
  const int64_t ne_max = cap > 0 ? cap * mult : ne_static;
  const int64_t nch = std::max<int64_t>(1, (ne_max + kChunk - 1) / kChunk);
  fitrig_status rc;
  if ((rc = ensure(ctx, ctx->chunk_cnt, (size_t)nch * 4)) != FITRIG_OK) return rc;
  uint32_t* cnt = (uint32_t*)ctx->chunk_cnt.p;
  KL((k_compact_count<F>), dim3((unsigned)nch), dim3(256), 0, st, f, ne_static, ne_dyn, cap, mult, cnt);
  KL(k_compact_scan, dim3(1), dim3(1024), 0, st, cnt, nch, ne_dyn, cap, mult, total);
  KL((k_compact_write<F, E>), dim3((unsigned)nch), dim3(256), 0, st, f, e, ne_static, ne_dyn, cap, mult,
     (const uint32_t*)cnt);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// One selection run over a segment layout: flags -> segments -> cells ->
// components -> candidate records appended at counters[CNT_OUTBASE].
fitrig_status select_run(fitrig_ctx* ctx, const Call& c, const SegLayout& L, float* seg_max, const double* mu,
                         const double* sigma, const uint32_t* flags, int branch, const float* direct_vals,
                         int halo) {
  hipStream_t st = c.st;
  const CallDev* cd = (const CallDev*)ctx->call.p;
  int64_t* cnt = (int64_t*)ctx->counters.p;
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
  KL(k_blk_count, dim3((unsigned)nchb), dim3(256), 0, st, (const float*)seg_max, mu, sigma, flags, cd, L, bflag, ccnt);
  KL(k_compact_scan, dim3(1), dim3(1024), 0, st, ccnt, nchb, (const int64_t*)nullptr, (int64_t)0, 1, cnt + CNT_NBLK);
  KL((k_compact_write<ByteFlag, BlkEmit>), dim3((unsigned)nchb), dim3(256), 0, st, ByteFlag{bflag},
     BlkEmit{blk_entry, blk_slot, bcap}, NB, (const int64_t*)nullptr, (int64_t)0, 1, (const uint32_t*)ccnt);
  KL(k_blk_bands, dim3(grid_for(bcap, 256, 2048)), dim3(256), 0, st, (const int64_t*)blk_entry,
     (const int64_t*)(cnt + CNT_NBLK), bcap, L, band_start, band_end);
  LAUNCH_CHECK(ctx);
  const RowOf ro{blk_entry, band_start, band_end, L};
  if ((rc = compact(ctx, st, RowFlag{ro, seg_max, mu, sigma, cd}, RowEmit{ro, rowslot, seg_entry, cap}, 0,
                    cnt + CNT_NBLK, bcap, L.br, cnt + CNT_NSEL)) != FITRIG_OK)
    return rc;

  const int gsel = (int)std::min<int64_t>(cap, 4096);
  // recompute: one wave per segment, grid-stride; 8192 waves put 8 on each
  // SIMD, which hides the latency of the frame reads
  const int grec = (int)std::min<int64_t>(cap, 8192);
  if (direct_vals) {
    KL(k_fill_direct, dim3(gsel), dim3(64), 0, st, direct_vals, L, (const int64_t*)seg_entry,
       (const int64_t*)(cnt + CNT_NSEL), cap, mu, sigma, cd, mask, cq);
  } else if (!ctx->sizing) {
    RecomputeArgs R;
    R.cd = cd;
    R.ncarry = c.ncarry;
    R.plane = (int64_t)c.H * c.W;
    R.H = c.H;
    R.W = c.W;
    R.Cf = (float)ctx->cfg.C;
    R.L = L;
    R.seg_entry = seg_entry;
    R.nsel = cnt + CNT_NSEL;
    R.cap = cap;
    R.mu = mu;
    R.sigma = sigma;
    R.mask = mask;
    R.cell_q = cq;
    if (!dispatch_recompute(ctx, c.dtype, halo, ctx->cfg.r_signed != 0, dim3(grec), st, R)) return FITRIG_E_INVAL;
  }
  LAUNCH_CHECK(ctx);
  const int gcell = grid_for(cap * 64, 256, 4096);
  KL(k_uf_init, dim3(gcell), dim3(256), 0, st, (const uint64_t*)mask, (const int64_t*)(cnt + CNT_NSEL), cap, parent);
  KL(k_uf_union, dim3(gcell), dim3(256), 0, st, SlotMap{blk_slot, band_start, band_end, rowslot},
     (const uint64_t*)mask, (const int64_t*)seg_entry, L, (const int64_t*)(cnt + CNT_NSEL), cap, parent);
  KL(k_uf_flatten, dim3(gcell), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NSEL), cap, parent);
  LAUNCH_CHECK(ctx);

  RootFlag rf{(const uint64_t*)mask, (const int32_t*)parent};
  RootEmit re{(int32_t*)ctx->comp_of.p, (int32_t*)ctx->c_root.p, ctx->comp_cap};
  if ((rc = compact(ctx, st, rf, re, 0, cnt + CNT_NSEL, cap, 64, cnt + CNT_NCOMP)) != FITRIG_OK) return rc;

  const int64_t ccap = ctx->comp_cap;
  const int gcomp = grid_for(ccap, 256, 4096);
  KL(k_comp_init, dim3(gcomp), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NCOMP), ccap, (int32_t*)ctx->c_npix.p,
     (unsigned long long*)ctx->c_key.p, (unsigned long long*)ctx->c_w.p, (int32_t*)ctx->c_box.p);
  KL(k_comp_accum, dim3(gcell), dim3(256), 0, st, (const uint64_t*)mask, (const int64_t*)seg_entry, (const float*)cq,
     L, (const int64_t*)(cnt + CNT_NSEL), cap, (const int32_t*)parent, (const int32_t*)ctx->comp_of.p, mu, sigma,
     (int32_t*)ctx->c_npix.p, (unsigned long long*)ctx->c_key.p, (unsigned long long*)ctx->c_w.p,
     (int32_t*)ctx->c_box.p);
  KL(k_comp_finalize, dim3(gcomp), dim3(256), 0, st, (const int64_t*)(cnt + CNT_NCOMP), ccap,
     (const int32_t*)ctx->c_root.p, (const int64_t*)seg_entry, L, mu, sigma, branch, (const int32_t*)ctx->c_npix.p,
     (const unsigned long long*)ctx->c_key.p, (const unsigned long long*)ctx->c_w.p, (const int32_t*)ctx->c_box.p,
     cnt + CNT_OUTBASE, (fitrig_candidate*)ctx->c_out.p, 3 * ccap);
  KL(k_run_done, dim3(1), dim3(64), 0, st, cnt, cap, bcap, ccap, branch);
  LAUNCH_CHECK(ctx);
  return FITRIG_OK;
}

// Selection capacity in 64-cell segments for ne_total candidate segments
// (grows only; the component records hold three runs: image, tile and
// per-pixel frequency branches).
fitrig_status ensure_selection(fitrig_ctx* ctx, int64_t ne_total) {
  int64_t want = ctx->cfg.max_segments > 0 ? ctx->cfg.max_segments
                                           : std::max<int64_t>(65536, std::min<int64_t>(ne_total / 64, 1 << 22));
  want = std::max(want, ctx->seg_cap);
  const int64_t comp = 2 * want;
  fitrig_status rc;
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
  if ((rc = ensure(ctx, ctx->c_out, 3 * comp * sizeof(fitrig_candidate))) != FITRIG_OK) return rc;
  // both passes: the selection runs after this size their buffers from it
  // (the sizing pass's values are restored when it ends)
  ctx->seg_cap = want;
  ctx->comp_cap = comp;
  return FITRIG_OK;
}

// The call record (stack pointers, tau, history pointers) the kernels read.
void write_call(fitrig_ctx* ctx, const Call& c) {
  CallDev v;
  v.base = c.stack;
  v.carry0 = c.carry0;
  v.carry1 = c.carry1;
  v.hist_in = c.hist ? c.hist->in : nullptr;
  v.hist_out = c.hist ? c.hist->out : nullptr;
  v.tau = c.tau;
  v.px_ring = c.hist ? c.hist->px_ring : nullptr;
  v.px_start = c.hist ? c.hist->px_start : 0;
  v.px_pad = 0;
  KL(k_set_call, dim3(1), dim3(64), 0, c.st, (CallDev*)ctx->call.p, v);
}

// Enqueues the whole path of one call (or, in the sizing pass, records the
// scratch it needs). with_call: also write the call record first.
fitrig_status enqueue(fitrig_ctx* ctx, const Call& c, bool with_call) {
  const fitrig_config& cfg = ctx->cfg;
  hipStream_t st = c.st;
  const Plan P = make_plan(cfg, c);
  const int np = P.np;
  const int halo = cfg.window / 2;
  const int64_t plane = (int64_t)c.H * c.W;
  const int tile = cfg.tile;
  const int Ty = (c.H + tile - 1) / tile, Tx = (c.W + tile - 1) / tile;
  fitrig_status rc;

  if ((rc = ensure(ctx, ctx->call, sizeof(CallDev))) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->counters, CNT_N * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->mu, (size_t)np * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->sigma, (size_t)np * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->flags, (size_t)np * 4)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->eta_st, ES_N * 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->M, 8)) != FITRIG_OK) return rc;
  if ((rc = ensure(ctx, ctx->max_key, 64)) != FITRIG_OK) return rc;
  CallDev* cd = (CallDev*)ctx->call.p;
  int64_t* cnt = (int64_t*)ctx->counters.p;
  if (with_call) write_call(ctx, c);
  KL(k_fill_i64, dim3(1), dim3(64), 0, st, cnt, (int64_t)CNT_N, (int64_t)0);
  KL(k_fill_i64, dim3(1), dim3(64), 0, st, (int64_t*)ctx->eta_st.p, (int64_t)ES_N, (int64_t)0);
  KL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)ctx->max_key.p, (int64_t)1, 0u);
  KL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)ctx->flags.p, (int64_t)np, 0u);
  bool prof = cfg.profile != 0 && !ctx->sizing && !ctx->rec_graph;
  if (prof) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(ctx, hipStreamIsCapturing(st, &cs));
    prof = cs == hipStreamCaptureStatusNone;
  }
  if (!ctx->sizing) ctx->ev_recorded = prof;
  // named host ranges of the phases being enqueued (rocprofv3 --marker-trace);
  // the guard closes the open one on every return
  struct PhaseRange {
    bool on, open = false;
    void to(const char* name) {
      if (!on) return;
      if (open) roctxRangePop();
      roctxRangePushA(name);
      open = true;
    }
    ~PhaseRange() {
      if (open) roctxRangePop();
    }
  } range{!ctx->sizing};
  static const char* const kPhaseName[5] = {"fitrig: index pass", "fitrig: spread", "fitrig: image selection",
                                            "fitrig: frequency branches", "fitrig: results"};
  auto mark = [&](int i) -> fitrig_status {
    range.to(kPhaseName[i]);
    if (prof) HIP_TRY(ctx, hipEventRecord(ctx->ev[i], st));
    return FITRIG_OK;
  };
  if ((rc = mark(0)) != FITRIG_OK) return rc;
  double* mu = (double*)ctx->mu.p;
  double* sigma = (double*)ctx->sigma.p;
  uint32_t* flags = (uint32_t*)ctx->flags.p;
  double* est = (double*)ctx->eta_st.p;
  uint32_t* eflags = (uint32_t*)(est + ES_FLAGS);

  // ---- pass over the stack -------------------------------------------------
  bool have_cube = false;
  bool have_max = false;
  const int out_w = out_width(halo);
  const int ncol = (c.W + out_w - 1) / out_w;
  const int nbands = (c.H + kBand - 1) / kBand;
  const int nseg_row = ncol * kSegsPerGroup;
  float* qmap = nullptr;

  if (P.qpass) {
    const int64_t nwg = (int64_t)ncol * nbands;
    if (nwg > INT32_MAX) return FITRIG_E_INVAL;
    const bool byprod = P.cube_needed && tile == 32;
    if ((rc = ensure(ctx, ctx->stat_part, (size_t)np * nwg * 16 * 16)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->seg_max, (size_t)np * c.H * nseg_row * 4)) != FITRIG_OK) return rc;
    if (byprod && (rc = ensure(ctx, ctx->tile_part, (size_t)np * nbands * ncol * kPieces * 3 * 8)) != FITRIG_OK)
      return rc;
    qmap = c.index_map;
    if (((P.img && P.robust) || P.fpx || P.pring) && !qmap) {
      if ((rc = ensure(ctx, ctx->qscratch, (size_t)np * plane * 4)) != FITRIG_OK) return rc;
      qmap = (float*)ctx->qscratch.p;
    }
    // robust spread of a large q map: the index pass writes its bracket
    // sample, q at the first cell of every 16-cell chunk of the first row of
    // every bstride-th band (cells 16 or more apart, so the windows of
    // sampled cells do not overlap), with bstride set for 2^20 to 2^21 samples
    // per triple; smaller maps keep the hashed sample of the map
    int64_t pre_S = 0;
    int samp_bstride = 1, samp_cpg = 0, samp_nch = 0;
    if (P.img && P.robust && plane >= 8 * (int64_t)kRsSample) {
      samp_cpg = (out_w + 15) / 16;
      const int last_w = c.W - (ncol - 1) * out_w;
      samp_nch = samp_cpg * (ncol - 1) + std::min(samp_cpg, (last_w + 15) / 16);
      const int64_t grid = (int64_t)nbands * samp_nch;
      if (grid >= kRsSample) {
        samp_bstride = (int)std::max<int64_t>(1, grid / kRsSample);
        pre_S = (int64_t)((nbands + samp_bstride - 1) / samp_bstride) * samp_nch;
        if ((rc = ensure(ctx, ctx->rs_samp, (size_t)np * pre_S * 4)) != FITRIG_OK) return rc;
      }
    }
    if (!ctx->sizing) {
      StreamArgs A;
      A.cd = cd;
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
      // moment partials only when the call takes the mean/std spread of q
      // (the map-free form always writes them)
      A.stat_part = (qmap && !(P.img && !P.robust)) ? nullptr : (double*)ctx->stat_part.p;
      A.seg_max = (float*)ctx->seg_max.p;
      A.tile_part = byprod ? (double*)ctx->tile_part.p : nullptr;
      A.max_key = (uint32_t*)ctx->max_key.p;
      A.qsamp = nullptr;
      A.samp_S = 0;
      A.samp_bstride = 1;
      A.samp_cpg = 0;
      A.samp_nch = 0;
      if (pre_S > 0) {
        A.qsamp = (uint32_t*)ctx->rs_samp.p;
        A.samp_S = pre_S;
        A.samp_bstride = samp_bstride;
        A.samp_cpg = samp_cpg;
        A.samp_nch = samp_nch;
      }
      if (!dispatch_stream(ctx, c.dtype, halo, cfg.r_signed != 0, dim3((unsigned)nwg), st, A)) return FITRIG_E_INVAL;
    }
    LAUNCH_CHECK(ctx);
    have_max = true;
    if ((rc = mark(1)) != FITRIG_OK) return rc;
    if (byprod) {
      if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
      if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
      KL(k_tile_merge, dim3(grid_for((int64_t)np * Ty * Tx)), dim3(256), 0, st, (const double*)ctx->tile_part.p, np,
         nbands, 2, ncol, out_w, kPieces, 32, c.H, c.W, Ty, Tx, (double*)ctx->cube.p, (float*)ctx->cube_f.p);
      LAUNCH_CHECK(ctx);
      have_cube = true;
    }
    // per-triple spread
    if (P.img && !P.robust) {
      if ((rc = moments(ctx, st, (const double*)ctx->stat_part.p, np, nwg * 16, 0, plane, mu, sigma, flags)) !=
          FITRIG_OK)
        return rc;
    } else if (P.img) {
      if ((rc = robust_spread(ctx, st, qmap, np, plane, !cfg.r_signed, mu, sigma, flags, pre_S)) != FITRIG_OK)
        return rc;
    }
  }

  // power-of-two tiles up to 32: streaming kernel (every frame read once);
  // other sizes: the tile kernel that reads three frames per triple
  const bool pow2_tile = tile <= 32 && (tile & (tile - 1)) == 0;
  if (!have_cube && P.cube_needed && pow2_tile) {
    if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
    TileStreamArgs A;
    A.cd = cd;
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
    if (!ctx->sizing && !dispatch_tile_stream(ctx, c.dtype, tile, cfg.r_signed != 0, dim3((unsigned)nwg), st, A))
      return FITRIG_E_INVAL;
    LAUNCH_CHECK(ctx);
    if (!have_max) {
      have_max = true;
      if ((rc = mark(1)) != FITRIG_OK) return rc;
    }
    have_cube = true;
  }
  if (!have_cube && P.cube_needed) {
    const int nchunk = (c.W + kLanes - 1) / kLanes;
    const int pieces = (kLanes + tile - 1) / tile + 1;
    if ((rc = ensure(ctx, ctx->tile_part, (size_t)np * Ty * nchunk * pieces * 3 * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cube, (size_t)np * Ty * Tx * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->cube_f, (size_t)np * Ty * Tx * 4)) != FITRIG_OK) return rc;
    TileArgs A;
    A.cd = cd;
    A.ncarry = c.ncarry;
    A.n = c.n;
    A.plane = plane;
    A.H = c.H;
    A.W = c.W;
    A.tile = tile;
    A.nchunk = nchunk;
    A.pieces = pieces;
    A.r_signed = cfg.r_signed;
    A.Cf = (float)cfg.C;
    A.tile_part = (double*)ctx->tile_part.p;
    A.max_key = (uint32_t*)ctx->max_key.p;
    if (!ctx->sizing && !dispatch_tile(ctx, c.dtype, cfg.r_signed != 0, dim3(nchunk, Ty, np), st, A))
      return FITRIG_E_INVAL;
    LAUNCH_CHECK(ctx);
    if (!have_max) {
      have_max = true;
      if ((rc = mark(1)) != FITRIG_OK) return rc;
    }
    KL(k_tile_merge, dim3(grid_for((int64_t)np * Ty * Tx)), dim3(256), 0, st, (const double*)ctx->tile_part.p, np, Ty,
       1, nchunk, kLanes, pieces, tile, c.H, c.W, Ty, Tx, (double*)ctx->cube.p, (float*)ctx->cube_f.p);
    LAUNCH_CHECK(ctx);
    have_cube = true;
  }
  if (!have_max) {
    // no pass produced the maximum (frequency branch only with too few triples)
    if (!ctx->sizing &&
        !dispatch_stack_max(ctx, c.dtype, dim3(1024), st, cd, (int64_t)(c.n - c.ncarry) * plane, (uint32_t*)ctx->max_key.p))
      return FITRIG_E_INVAL;
    if ((rc = mark(1)) != FITRIG_OK) return rc;
  }
  KL(k_max_finalize, dim3(1), dim3(64), 0, st, (const uint32_t*)ctx->max_key.p, cfg.C, (double*)ctx->M.p);
  LAUNCH_CHECK(ctx);
  if ((rc = mark(2)) != FITRIG_OK) return rc;

  // ---- image-branch selection ---------------------------------------------
  if (P.img) {
    if (P.sliding) {
      SegLayout L{c.H, c.W, np, kSegsPerGroup, out_w, nseg_row, kBand, (c.H + kBand - 1) / kBand};
      if ((rc = ensure_selection(ctx, (int64_t)np * c.H * nseg_row)) != FITRIG_OK) return rc;
      if ((rc = select_run(ctx, c, L, (float*)ctx->seg_max.p, mu, sigma, flags, FITRIG_IMAGE, nullptr, halo)) !=
          FITRIG_OK)
        return rc;
    } else {
      const int64_t ncell = (int64_t)Ty * Tx;
      if (!P.robust) {
        if ((rc = moments(ctx, st, (const double*)ctx->cube.p, np, ncell, 1, ncell, mu, sigma, flags)) != FITRIG_OK)
          return rc;
      } else {
        if ((rc = robust_spread(ctx, st, (const float*)ctx->cube_f.p, np, ncell, !cfg.r_signed, mu, sigma, flags)) !=
            FITRIG_OK)
          return rc;
      }
      SegLayout L{Ty, Tx, np, 1, 64, (Tx + 63) / 64, 1, Ty};
      if ((rc = ensure(ctx, ctx->seg_max, (size_t)np * Ty * L.nseg_row * 4)) != FITRIG_OK) return rc;
      KL(k_segmax_direct, dim3(grid_for((int64_t)np * Ty * L.nseg_row * 16)), dim3(256), 0, st, (const float*)ctx->cube_f.p,
         L, (float*)ctx->seg_max.p);
      if ((rc = ensure_selection(ctx, (int64_t)np * Ty * L.nseg_row)) != FITRIG_OK) return rc;
      if ((rc = select_run(ctx, c, L, (float*)ctx->seg_max.p, mu, sigma, flags, FITRIG_IMAGE,
                           (const float*)ctx->cube_f.p, halo)) != FITRIG_OK)
        return rc;
    }
  }
  if (c.index_map && !P.sliding && !ctx->sizing)
    HIP_TRY(ctx, copy_d2d(ctx, c.index_map, ctx->cube_f.p, (size_t)np * Ty * Tx * 4, st));

  if ((rc = mark(3)) != FITRIG_OK) return rc;
  // ---- frequency branch ----------------------------------------------------
  const double* series = (const double*)ctx->cube.p;
  if (P.ring) {
    // the covered series: the newest slices of the history, then the newest
    // of this call's (oldest first); written back as the field's history
    const int64_t ntiles = (int64_t)Ty * Tx;
    const int from_call = std::min(np, P.nfreq);
    const int from_hist = P.nfreq - from_call;
    if ((rc = ensure(ctx, ctx->fseries, (size_t)P.nfreq * ntiles * 8)) != FITRIG_OK) return rc;
    double* fs = (double*)ctx->fseries.p;
    const int64_t tot = (int64_t)P.nfreq * ntiles;
    KL(k_hist_in, dim3(grid_for(tot)), dim3(256), 0, st, (const CallDev*)cd,
       (int64_t)(c.hist->n_in - from_hist) * ntiles, (int64_t)from_hist * ntiles, (const double*)ctx->cube.p,
       (int64_t)(np - from_call) * ntiles, (int64_t)from_call * ntiles, fs);
    if (c.hist->out) KL(k_hist_out, dim3(grid_for(tot)), dim3(256), 0, st, (const CallDev*)cd, (const double*)fs, tot);
    LAUNCH_CHECK(ctx);
    series = fs;
  }
  if (P.freq) {
    const int64_t ntiles = (int64_t)Ty * Tx;
    if ((rc = ensure(ctx, ctx->eta_d, ntiles * 8)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->eta_f, ntiles * 4)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->tw, (size_t)P.nfreq * 16)) != FITRIG_OK) return rc;
    KL(k_twiddle, dim3(grid_for(P.nfreq)), dim3(256), 0, st, P.nfreq, (double2*)ctx->tw.p);
    // long series: a workgroup per tile (twiddles, series and magnitudes in LDS)
    const size_t blk_lds = (size_t)P.nfreq * 16 + (size_t)P.nfreq * 8 + (size_t)(P.nfreq / 2) * 8;
    if (P.nfreq >= 128 && blk_lds <= 60 * 1024) {
      KL(k_eta_blk, dim3((unsigned)std::min<int64_t>(ntiles, 65536)), dim3(256), blk_lds, st, series, P.nfreq,
         ntiles, cfg.harm, (const double2*)ctx->tw.p, (double*)ctx->eta_d.p, (float*)ctx->eta_f.p);
    } else if (P.nfreq <= 64) {
      // short series: held in registers
#define ETA_REG(NPM)                                                                                           \
  KL(k_eta_reg<NPM>, dim3(grid_for(ntiles, 256, 4096)), dim3(256), 0, st, series, P.nfreq, ntiles, cfg.harm, \
     (const double2*)ctx->tw.p, (double*)ctx->eta_d.p, (float*)ctx->eta_f.p)
      if (P.nfreq <= 32)
        ETA_REG(32);
      else
        ETA_REG(64);
#undef ETA_REG
    } else {
      KL(k_eta, dim3(grid_for(ntiles, 256, 4096)), dim3(256), 0, st, series, P.nfreq, ntiles, cfg.harm,
         (const double2*)ctx->tw.p, (double*)ctx->eta_d.p, (float*)ctx->eta_f.p);
    }
    LAUNCH_CHECK(ctx);
    if (!P.robust) {
      if ((rc = moments(ctx, st, (const double*)ctx->eta_d.p, 1, ntiles, 1, ntiles, est + ES_MU, est + ES_SIG,
                        eflags)) != FITRIG_OK)
        return rc;
    } else {
      if ((rc = robust_spread(ctx, st, (const float*)ctx->eta_f.p, 1, ntiles, true, est + ES_MU, est + ES_SIG,
                              eflags)) != FITRIG_OK)
        return rc;
    }
    SegLayout L{Ty, Tx, 1, 1, 64, (Tx + 63) / 64, 1, Ty};
    const int64_t ne = (int64_t)Ty * L.nseg_row;
    if ((rc = ensure(ctx, ctx->seg_max2, (size_t)ne * 4)) != FITRIG_OK) return rc;
    float* smax = (float*)ctx->seg_max2.p;
    KL(k_segmax_direct, dim3(grid_for(ne * 16)), dim3(256), 0, st, (const float*)ctx->eta_f.p, L, smax);
    if ((rc = ensure_selection(ctx, ne)) != FITRIG_OK) return rc;
    if ((rc = select_run(ctx, c, L, smax, est + ES_MU, est + ES_SIG, eflags, FITRIG_FREQ, (const float*)ctx->eta_f.p,
                         halo)) != FITRIG_OK)
      return rc;
    if (c.eta_map && !ctx->sizing)
      HIP_TRY(ctx, copy_d2d(ctx, c.eta_map, ctx->eta_f.p, (size_t)ntiles * 4, st));
  }

  // ---- per-pixel frequency branch -------------------------------------------
  // the series: the field's kept maps (serving), then the call's last ones
  const int px_from_call = P.pring ? std::min(np, P.npx) : np;
  const int px_from_ring = P.pring ? P.npx - px_from_call : 0;
  const int px_cap = P.pring ? c.hist->px_cap : 1;
  const int px_first = P.pring ? c.hist->px_n - px_from_ring : 0;  // held maps skipped (oldest)
  if (P.fpx) {
    const int nps = P.npx;
    const int K = nps / 2;
    const int nmb = (K + 15) / 16;  // blocks of 16 frequencies (cosine and sine accumulators each)
    const int mbg = nmb <= 1 ? 1 : 2;
    const int64_t ntile = (plane + 63) / 64;
    const int G = (int)std::min<int64_t>(ntile, 8192);
    const size_t lds = (size_t)nps * 16 + (cfg.harm ? (size_t)K * 64 * 4 : 0);
    if (lds > 65536) return FITRIG_E_INVAL;
    float* ef = c.eta_px_map;
    if (!ef) {
      if ((rc = ensure(ctx, ctx->etapx_f, (size_t)plane * 4)) != FITRIG_OK) return rc;
      ef = (float*)ctx->etapx_f.p;
    }
    if ((rc = ensure(ctx, ctx->pxpart, (size_t)G * 16)) != FITRIG_OK) return rc;
    if ((rc = ensure(ctx, ctx->tw_px, (size_t)nps * 16)) != FITRIG_OK) return rc;
    KL(k_twiddle, dim3(grid_for(nps)), dim3(256), 0, st, nps, (double2*)ctx->tw_px.p);
    const float* qcall = qmap + (int64_t)(np - px_from_call) * plane;
    // 16-byte loads of four pixels: rows of the maps start 16-byte aligned
    const bool vec = plane % 4 == 0 && ((uintptr_t)qcall & 15) == 0;
    // loads run 4 step groups (16 series steps) ahead, 2 for short series
    const bool deep = (nps / 2 + 4) / 4 >= 4;
    // short series: one pass of at most 16 frequencies and one round of step
    // groups, no field ring (weights and row offsets fixed per lane)
    const int tgroups = (nps / 2 + 4) / 4, dpre = deep ? 4 : 2;
    const bool shortk = px_from_ring == 0 && nmb == 1 && (tgroups + dpre - 1) / dpre * dpre == dpre;
#define EPX2(MB, V, DD, RG)                                                                                     \
  KL((k_eta_px<MB, V, DD, RG>), dim3(G), dim3(64), lds, st, qcall, nps, plane, cfg.harm,                          \
     (const double2*)ctx->tw_px.p, ef, (double*)ctx->pxpart.p, (const CallDev*)cd, px_from_ring, px_first, px_cap)
#define EPX(MB, V, DD)                                                                                 \
  do {                                                                                                 \
    if (px_from_ring > 0)                                                                              \
      EPX2(MB, V, DD, true);                                                                           \
    else if (MB == 1 && shortk)                                                                        \
      KL((k_eta_px_short<V, DD>), dim3(G), dim3(64), lds, st, qcall, nps, plane, cfg.harm,             \
         (const double2*)ctx->tw_px.p, ef, (double*)ctx->pxpart.p);                                    \
    else                                                                                               \
      EPX2(MB, V, DD, false);                                                                          \
  } while (0)
    if (deep) {
      if (vec) {
        if (mbg == 1) EPX(1, true, 4); else EPX(2, true, 4);
      } else {
        if (mbg == 1) EPX(1, false, 4); else EPX(2, false, 4);
      }
    } else {
      if (vec) {
        if (mbg == 1) EPX(1, true, 2); else EPX(2, true, 2);
      } else {
        if (mbg == 1) EPX(1, false, 2); else EPX(2, false, 2);
      }
    }
#undef EPX
#undef EPX2
    LAUNCH_CHECK(ctx);
    double* px_mu = est + ES_PXMU;
    double* px_sig = est + ES_PXSIG;
    uint32_t* px_flag = eflags + 1;
    if (!P.robust) {
      if ((rc = moments(ctx, st, (const double*)ctx->pxpart.p, 1, G, 0, plane, px_mu, px_sig, px_flag)) != FITRIG_OK)
        return rc;
    } else {
      if ((rc = robust_spread(ctx, st, (const float*)ef, 1, plane, true, px_mu, px_sig, px_flag)) != FITRIG_OK)
        return rc;
    }
    SegLayout L{c.H, c.W, 1, 1, 64, (c.W + 63) / 64, 1, c.H};
    const int64_t ne = (int64_t)c.H * L.nseg_row;
    if ((rc = ensure(ctx, ctx->seg_max2, (size_t)ne * 4)) != FITRIG_OK) return rc;
    float* smax = (float*)ctx->seg_max2.p;
    KL(k_segmax_direct, dim3(grid_for(ne * 16)), dim3(256), 0, st, (const float*)ef, L, smax);
    if ((rc = ensure_selection(ctx, ne)) != FITRIG_OK) return rc;
    if ((rc = select_run(ctx, c, L, smax, px_mu, px_sig, px_flag, FITRIG_FREQ_PIXEL, (const float*)ef, halo)) !=
        FITRIG_OK)
      return rc;
  }

  if (P.pring) {
    // the call's last maps join the field's ring (after the branch read it)
    const int nap = std::min(np, px_cap);
    KL(k_px_ring_append, dim3(grid_for((int64_t)nap * plane, 256, 8192)), dim3(256), 0, st, (const CallDev*)cd,
       (const float*)(qmap + (int64_t)(np - nap) * plane), plane, nap, c.hist->px_n, px_cap);
    LAUNCH_CHECK(ctx);
  }

  if (c.index_map && P.sliding && cfg.map_kind == FITRIG_MAP_TLISI) {
    KL(k_to_tlisi, dim3(grid_for((int64_t)np * plane, 256, 8192)), dim3(256), 0, st, c.index_map, (int64_t)np * plane,
       (const double*)ctx->M.p);
    LAUNCH_CHECK(ctx);
  }
  if ((rc = mark(4)) != FITRIG_OK) return rc;
  return FITRIG_OK;
}

// Packs the results into host-visible memory (dst: a device-visible pointer).
fitrig_status enqueue_results(fitrig_ctx* ctx, const Call& c, char* dst, const ResultLayout& R, int64_t cap,
                              fitrig_candidate* cand_dst = nullptr) {
  const int np = c.n - 2;
  KL(k_pack_results, dim3(grid_for(std::max<int64_t>(cap, 1) * 9 + 64, 256, 256)), dim3(256), 0, c.st,
     (const int64_t*)ctx->counters.p, (const double*)ctx->M.p, (const double*)ctx->eta_st.p,
     (const double*)ctx->mu.p, (const double*)ctx->sigma.p, (const uint32_t*)ctx->flags.p, np,
     (const fitrig_candidate*)ctx->c_out.p, cap, R, dst, cand_dst);
  LAUNCH_CHECK(ctx);
  if (ctx->cfg.profile && ctx->ev_recorded && !ctx->sizing) HIP_TRY(ctx, hipEventRecord(ctx->ev[5], c.st));
  return FITRIG_OK;
}

// Host outputs from the results (after the stream reached them): counters
// cnt, scalars sc (M, then the frequency statistics), per-triple hmu, hsg,
// hfl and the candidate records hcand. A piece may already be the caller's
// array (the allocation-free entry copies into them directly).
fitrig_status unpack_pieces(const int64_t* cnt, const double* sc, const double* hmu, const double* hsg,
                            const uint32_t* hfl, const fitrig_candidate* hcand, int np, uint32_t ran,
                            fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand, fitrig_stats* stats,
                            double* mu_o, double* sg_o, uint32_t* fl_o) {
  const int64_t total = cnt[CNT_OUTBASE];
  const bool trunc_internal = cnt[CNT_TRUNC] != 0;
  const int64_t ncopy = std::min<int64_t>(total, cand_cap);
  if (ncopy > 0 && cand && cand != hcand) memcpy(cand, hcand, (size_t)ncopy * sizeof(fitrig_candidate));
  *n_cand = total;
  const fitrig_status status = (trunc_internal || total > cand_cap) ? FITRIG_E_TRUNC : FITRIG_OK;
  if (stats) {
    const bool img = (ran & FITRIG_IMAGE) != 0;
    const uint32_t* ef = (const uint32_t*)(sc + 1 + ES_FLAGS);
    stats->M = sc[0];
    stats->n_triples = np;
    stats->status = status;
    stats->eta_mu = (ran & FITRIG_FREQ) ? sc[1 + ES_MU] : 0.0;
    stats->eta_sigma = (ran & FITRIG_FREQ) ? sc[1 + ES_SIG] : 0.0;
    stats->eta_px_mu = (ran & FITRIG_FREQ_PIXEL) ? sc[1 + ES_PXMU] : 0.0;
    stats->eta_px_sigma = (ran & FITRIG_FREQ_PIXEL) ? sc[1 + ES_PXSIG] : 0.0;
    stats->n_image_cand = cnt[CNT_IMG];
    stats->n_freq_cand = cnt[CNT_FREQ];
    stats->n_freq_px_cand = cnt[CNT_FPX];
    stats->ran = ran;
    stats->eta_flags = ((ran & FITRIG_FREQ) ? (ef[0] & 0xFFu) : 0u) | ((ran & FITRIG_FREQ_PIXEL) ? (ef[1] & 0xFFu) << 8 : 0u);
    const uint32_t tf = trunc_internal ? FITRIG_FLAG_TRUNC : 0u;
    for (int s = 0; s < np; ++s) {
      if (mu_o) mu_o[s] = img ? hmu[s] : 0.0;
      if (sg_o) sg_o[s] = img ? hsg[s] : 0.0;
      if (fl_o) fl_o[s] = (img ? hfl[s] : 0u) | tf;
    }
  }
  return status;
}

// Host outputs from the packed results in host-visible memory h.
// direct: the candidate records were written into cand by the device
fitrig_status unpack_results(const char* h, const ResultLayout& R, int np, uint32_t ran, fitrig_candidate* cand,
                             int64_t cand_cap, int64_t* n_cand, fitrig_stats* stats, double* mu_o, double* sg_o,
                             uint32_t* fl_o, bool direct = false) {
  return unpack_pieces((const int64_t*)(h + R.off_cnt), (const double*)(h + R.off_scalars),
                       (const double*)(h + R.off_mu), (const double*)(h + R.off_sigma),
                       (const uint32_t*)(h + R.off_flags),
                       direct ? cand : (const fitrig_candidate*)(h + R.off_cand), np, ran, cand, cand_cap, n_cand,
                       stats, mu_o, sg_o, fl_o);
}

void async_done(void* p) {
  AsyncOut* o = (AsyncOut*)p;
  (void)unpack_results(o->ctx->h_stage, o->R, o->np, o->ran, o->cand, o->cand_cap, o->n_cand, o->stats, o->mu,
                       o->sigma, o->flags, o->direct);
  if (!o->captured) delete o;
}

uint32_t branches_ran(const fitrig_config& cfg, const Call& c) {
  const Plan P = make_plan(cfg, c);
  return (P.img ? FITRIG_IMAGE : 0u) | (P.freq ? FITRIG_FREQ : 0u) | (P.fpx ? FITRIG_FREQ_PIXEL : 0u);
}

fitrig_status check_shape(const fitrig_config& cfg, const Call& c) {
  const size_t bpp = c.dtype == FITRIG_F32 ? 4 : 2;
  // the streaming kernels address a workgroup's rows (at most 32) through one
  // buffer descriptor of 2^30 bytes starting at its first row
  if ((uint64_t)c.W * bpp * (uint64_t)(kBand + 2 * kMaxHalo + 1) >= (1ull << 30)) return FITRIG_E_INVAL;
  const Plan P = make_plan(cfg, c);
  // per-pixel spectra: the twiddle table (and, for harmonic sums, the
  // magnitudes of 64 pixels) in the 64 KB of LDS of one workgroup
  if (P.fpx && P.npx > (cfg.harm ? 448 : 4096)) return FITRIG_E_INVAL;
  return FITRIG_OK;
}

// Records the scratch (and host-visible result bytes) one call needs,
// enqueueing nothing; the selection capacities it sets on the way are put
// back, the launch pass derives the same ones.
fitrig_status sizing_pass(fitrig_ctx* ctx, const Call& c, size_t result_bytes) {
  const int64_t seg_cap = ctx->seg_cap, comp_cap = ctx->comp_cap;
  clear_wants(ctx);
  // buffers not allocated yet get a stand-in address for the pass, so the
  // pointer arithmetic of the sequence stays defined (nothing is
  // dereferenced or launched while sizing)
  bool stand_in[kNBufs];
  for (size_t i = 0; i < kNBufs; ++i) {
    DevBuf& b = ctx->*kBufs[i];
    stand_in[i] = b.p == nullptr;
    if (stand_in[i]) b.p = (void*)(uintptr_t)(1u << 20);
  }
  ctx->sizing = true;
  fitrig_status rc = enqueue(ctx, c, true);
  for (size_t i = 0; i < kNBufs; ++i)
    if (stand_in[i]) (ctx->*kBufs[i]).p = nullptr;
  // results: host-visible memory, or (allocation-free entry) device scratch
  if (rc == FITRIG_OK) rc = ctx->in_arena ? ensure(ctx, ctx->res_dev, result_bytes) : ensure_host(ctx, result_bytes);
  ctx->sizing = false;
  ctx->seg_cap = seg_cap;
  ctx->comp_cap = comp_cap;
  return rc;
}

// The whole call: sizing pass, scratch growth, launch pass, results.
// Device address of the caller's candidate array when it is page-locked host
// memory mapped for the device (then the records are written there
// directly), else null.
fitrig_candidate* mapped_cand(fitrig_candidate* cand) {
  if (!cand) return nullptr;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, cand) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory reports an error
    return nullptr;
  }
  return at.type == hipMemoryTypeHost ? (fitrig_candidate*)at.devicePointer : nullptr;
}

fitrig_status detect_impl(fitrig_ctx* ctx, const Call& c, fitrig_candidate* cand, int64_t* n_cand,
                          fitrig_stats* stats, bool async) {
  fitrig_status rc = check_shape(ctx->cfg, c);
  if (rc != FITRIG_OK) return rc;
  const int np = c.n - 2;
  const int64_t cap = c.cand_cap;
  const ResultLayout R = result_layout(np, cap);
  // sizing pass
  rc = sizing_pass(ctx, c, (size_t)R.bytes);
  if (rc != FITRIG_OK) return rc;
  if ((rc = provision(ctx, c.st)) != FITRIG_OK) return rc;
  // launch pass (the caller's array is not queried while the stream is
  // being captured: a graph keeps the staging copy)
  hipStreamCaptureStatus cap_st = hipStreamCaptureStatusNone;
  const bool capturing = hipStreamIsCapturing(c.st, &cap_st) == hipSuccess && cap_st != hipStreamCaptureStatusNone;
  fitrig_candidate* cand_dev = capturing ? nullptr : mapped_cand(cand);
  if ((rc = enqueue(ctx, c, true)) != FITRIG_OK) return rc;
  if ((rc = enqueue_results(ctx, c, ctx->h_stage_dev, R, cap, cand_dev)) != FITRIG_OK) return rc;
  const uint32_t ran = branches_ran(ctx->cfg, c);
  if (!async) {
    HIP_TRY(ctx, hipStreamSynchronize(c.st));
    return unpack_results(ctx->h_stage, R, np, ran, cand, cap, n_cand, stats, stats ? stats->mu : nullptr,
                          stats ? stats->sigma : nullptr, stats ? stats->flags : nullptr, cand_dev != nullptr);
  }
  AsyncOut* o = new (std::nothrow) AsyncOut();
  if (!o) return FITRIG_E_NOMEM;
  o->ctx = ctx;
  o->cand = cand;
  o->cand_cap = cap;
  o->n_cand = n_cand;
  o->stats = stats;
  o->mu = stats ? stats->mu : nullptr;
  o->sigma = stats ? stats->sigma : nullptr;
  o->flags = stats ? stats->flags : nullptr;
  o->np = np;
  o->ran = ran;
  o->R = R;
  o->direct = cand_dev != nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(c.st, &cs);
  o->captured = e == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (e == hipSuccess) e = hipLaunchHostFunc(c.st, async_done, o);
  if (e != hipSuccess) {
    delete o;
    ctx->last_hip = (int32_t)e;
    return FITRIG_E_HIP;
  }
  if (o->captured) ctx->captured_outs.push_back(o);
  return FITRIG_OK;
}

void drop_graph(GraphEntry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  e.exec = nullptr;
}

// The whole call as a replay of the launch sequence built as a graph for its
// shape (synchronous on c.st). The sequence reads the per-call values from
// the call record, which is written before each replay; scratch addresses
// are built in, so a graph is valid for the context's current generation of
// scratch only. When building or instantiation fails the context goes back
// to direct launches for good.
fitrig_status detect_graph(fitrig_ctx* ctx, const Call& c, fitrig_candidate* cand, int64_t* n_cand,
                           fitrig_stats* stats) {
  fitrig_status rc = check_shape(ctx->cfg, c);
  if (rc != FITRIG_OK) return rc;
  const int np = c.n - 2;
  const int64_t cap = c.cand_cap;
  const ResultLayout R = result_layout(np, cap);
  if ((rc = sizing_pass(ctx, c, (size_t)R.bytes)) != FITRIG_OK) return rc;
  if ((rc = provision(ctx, c.st)) != FITRIG_OK) return rc;
  for (size_t i = 0; i < ctx->graphs.size();) {
    if (ctx->graphs[i].gen != ctx->gen) {
      drop_graph(ctx->graphs[i]);
      ctx->graphs.erase(ctx->graphs.begin() + (std::ptrdiff_t)i);
    } else {
      ++i;
    }
  }
  const GraphKey key{c.n, c.H, c.W, c.ncarry, (int)c.dtype, c.hist ? c.hist->cap : 0, c.hist ? c.hist->n_in : 0,
                     (c.hist && c.hist->out) ? 1 + (c.hist->defer ? 1 : 0) : 0, c.hist ? c.hist->px_cap : 0,
                     c.hist ? c.hist->px_n : 0, cap,
                     (c.index_map ? 1 : 0) | (c.eta_map ? 2 : 0) | (c.eta_px_map ? 4 : 0)};
  GraphEntry* e = nullptr;
  for (GraphEntry& g : ctx->graphs)
    if (g.key == key) e = &g;
  if (!e) {
    hipGraph_t g = nullptr;
    hipError_t he = hipGraphCreate(&g, 0);
    if (he == hipSuccess) {
      ctx->rec_graph = g;
      ctx->rec_last = nullptr;
      ctx->launch_err = hipSuccess;
      rc = enqueue(ctx, c, false);
      if (rc == FITRIG_OK) rc = enqueue_results(ctx, c, ctx->h_stage_dev, R, cap);
      ctx->rec_graph = nullptr;
      ctx->rec_last = nullptr;
      ctx->launch_err = hipSuccess;
    }
    hipGraphExec_t x = nullptr;
    if (he == hipSuccess && rc == FITRIG_OK) he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (he != hipSuccess || rc != FITRIG_OK || !x) {
      if (x) (void)hipGraphExecDestroy(x);
      (void)hipGetLastError();
      ctx->use_graphs = false;
      return detect_impl(ctx, c, cand, n_cand, stats, false);
    }
    if (ctx->graphs.size() >= kMaxGraphs) {
      size_t lru = 0;
      for (size_t i = 1; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].last_use < ctx->graphs[lru].last_use) lru = i;
      drop_graph(ctx->graphs[lru]);
      ctx->graphs.erase(ctx->graphs.begin() + (std::ptrdiff_t)lru);
    }
    ctx->graphs.push_back(GraphEntry{key, x, ctx->gen, 0});
    e = &ctx->graphs.back();
  }
  e->last_use = ++ctx->graph_clock;
  write_call(ctx, c);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipGraphLaunch(e->exec, c.st));
  HIP_TRY(ctx, hipStreamSynchronize(c.st));
  ++ctx->graph_replays;
  return unpack_results(ctx->h_stage, R, np, branches_ran(ctx->cfg, c), cand, cap, n_cand, stats,
                        stats ? stats->mu : nullptr, stats ? stats->sigma : nullptr, stats ? stats->flags : nullptr);
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

fitrig_status check_args(const void* stack, fitrig_dtype dtype, int32_t H, int32_t W, double sigma,
                         fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand) {
  if (!stack || !n_cand) return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  if (H < 1 || W < 1 || (uint64_t)H * (uint64_t)W >= (1ull << 32)) return FITRIG_E_INVAL;
  if (!(sigma > 0.0) || !isfinite(sigma)) return FITRIG_E_INVAL;
  if (cand_cap < 0 || (cand_cap > 0 && !cand)) return FITRIG_E_INVAL;
  return FITRIG_OK;
}

// Scratch for a stack of the capacity hints' size (square image of
// max_pixels, max_snap frames), through the sizing pass.
fitrig_status presize(fitrig_ctx* ctx) {
  const fitrig_config& cfg = ctx->cfg;
  if (cfg.max_pixels <= 0 || cfg.max_snap < 3) return FITRIG_OK;
  const int64_t side = (int64_t)ceil(sqrt((double)cfg.max_pixels));
  if (side >= (1 << 16)) return FITRIG_OK;
  Call c;
  memset(&c, 0, sizeof(c));
  c.stack = (const void*)(uintptr_t)256;  // sizing only: never dereferenced
  c.dtype = FITRIG_F32;
  c.n = cfg.max_snap;
  c.H = (int)side;
  c.W = (int)side;
  c.tau = 1.0;
  c.st = ctx->stream;
  c.cand_cap = 65536;
  if (check_shape(cfg, c) != FITRIG_OK) return FITRIG_OK;
  const fitrig_status rc = sizing_pass(ctx, c, (size_t)result_layout(c.n - 2, c.cand_cap).bytes);
  if (rc != FITRIG_OK) return rc;
  return provision(ctx, ctx->stream);
}

// The allocation-free call: the context's own buffers are set aside, the
// call's scratch (and its device results) is carved from this device's
// static array, and the results are copied into the caller's host memory.
fitrig_status detect_noalloc_impl(fitrig_ctx* ctx, const Call& c, fitrig_candidate* cand, int64_t* n_cand,
                                  fitrig_stats* stats) {
  const int dev = ctx->cfg.device;
  if (dev < 0 || dev >= kMaxDevices) return FITRIG_E_INVAL;
  void* base = g_scratch_ptr[dev];
  if (!base) {
    ctx->last_hip = g_scratch_err[dev];
    return FITRIG_E_HIP;
  }
  fitrig_status rc = check_shape(ctx->cfg, c);
  if (rc != FITRIG_OK) return rc;
  const int np = c.n - 2;
  const int64_t cap = c.cand_cap;
  const ResultLayout R = result_layout(np, cap);
  std::lock_guard<std::mutex> lk(g_scratch_call_mu[dev]);
  DevBuf saved[kNBufs];
  for (size_t i = 0; i < kNBufs; ++i) saved[i] = ctx->*kBufs[i];
  const int64_t seg_cap = ctx->seg_cap, comp_cap = ctx->comp_cap;
  ctx->seg_cap = ctx->comp_cap = 0;
  ctx->in_arena = true;
  ctx->arena = (char*)base;
  ctx->arena_cap = FITRIG_NOALLOC_SCRATCH_BYTES;
  int64_t hcnt[CNT_N] = {};
  double hsc[1 + ES_N] = {};
  const uint32_t ran = branches_ran(ctx->cfg, c);
  auto run = [&]() -> fitrig_status {
    fitrig_status r = sizing_pass(ctx, c, (size_t)R.bytes);
    if (r != FITRIG_OK) return r;
    if ((r = provision(ctx, c.st)) != FITRIG_OK) return r;
    if ((r = enqueue(ctx, c, true)) != FITRIG_OK) return r;
    const char* res = (const char*)ctx->res_dev.p;
    if ((r = enqueue_results(ctx, c, (char*)ctx->res_dev.p, R, cap)) != FITRIG_OK) return r;
    HIP_TRY(ctx, hipMemcpyAsync(hcnt, res + R.off_cnt, sizeof(hcnt), hipMemcpyDeviceToHost, c.st));
    HIP_TRY(ctx, hipMemcpyAsync(hsc, res + R.off_scalars, sizeof(hsc), hipMemcpyDeviceToHost, c.st));
    if (stats && np > 0) {
      if (stats->mu)
        HIP_TRY(ctx, hipMemcpyAsync(stats->mu, res + R.off_mu, (size_t)np * 8, hipMemcpyDeviceToHost, c.st));
      if (stats->sigma)
        HIP_TRY(ctx, hipMemcpyAsync(stats->sigma, res + R.off_sigma, (size_t)np * 8, hipMemcpyDeviceToHost, c.st));
      if (stats->flags)
        HIP_TRY(ctx, hipMemcpyAsync(stats->flags, res + R.off_flags, (size_t)np * 4, hipMemcpyDeviceToHost, c.st));
    }
    HIP_TRY(ctx, hipStreamSynchronize(c.st));
    const int64_t ncopy = std::min<int64_t>(hcnt[CNT_OUTBASE], cap);
    if (ncopy > 0 && cand) {
      HIP_TRY(ctx, hipMemcpyAsync(cand, res + R.off_cand, (size_t)ncopy * sizeof(fitrig_candidate),
                                  hipMemcpyDeviceToHost, c.st));
      HIP_TRY(ctx, hipStreamSynchronize(c.st));
    }
    return FITRIG_OK;
  };
  rc = run();
  if (rc != FITRIG_OK) {
    // nothing of a failed call may still use the array when it is released
    // to the next call (and the caller's buffers must be settled)
    (void)hipStreamSynchronize(c.st);
  }
  for (size_t i = 0; i < kNBufs; ++i) ctx->*kBufs[i] = saved[i];
  ctx->seg_cap = seg_cap;
  ctx->comp_cap = comp_cap;
  ctx->in_arena = false;
  ctx->arena = nullptr;
  ctx->arena_cap = 0;
  if (rc != FITRIG_OK) return rc;
  return unpack_pieces(hcnt, hsc, stats ? stats->mu : nullptr, stats ? stats->sigma : nullptr,
                       stats ? stats->flags : nullptr, cand, np, ran, cand, cap, n_cand, stats,
                       stats ? stats->mu : nullptr, stats ? stats->sigma : nullptr, stats ? stats->flags : nullptr);
}

// A call of this shape for the sizing pass (the stack pointer is a stand-in,
// never dereferenced).
Call shape_call(int ncarry, int n_new, int H, int W, fitrig_dtype dtype, const FreqHist* hist, int64_t cand_cap,
                hipStream_t st) {
  Call c;
  memset(&c, 0, sizeof(c));
  c.stack = (const void*)(uintptr_t)256;
  c.carry0 = ncarry >= 1 ? c.stack : nullptr;
  c.carry1 = ncarry >= 2 ? c.stack : nullptr;
  c.ncarry = ncarry;
  c.dtype = dtype;
  c.n = ncarry + n_new;
  c.H = H;
  c.W = W;
  c.tau = 1.0;
  c.hist = hist;
  c.cand_cap = cand_cap;
  c.st = st;
  return c;
}

// Sizing pass of a host-only context with ctx's config (nothing allocated or
// launched); false when the shape is not a valid call.
bool size_shape(const fitrig_config& cfg, const Call& c, fitrig_ctx& tmp) {
  tmp.cfg = cfg;
  tmp.cfg.profile = 0;
  if (c.n < 3 || check_shape(cfg, c) != FITRIG_OK) return false;
  return sizing_pass(&tmp, c, (size_t)result_layout(c.n - 2, c.cand_cap).bytes) == FITRIG_OK;
}

// Device memory and streams of one host-resident call, released on scope exit.
// Pageable input: chunks are copied by host threads into two page-locked
// staging buffers ahead of the device, and each transfer goes from a staging
// buffer, so transfers overlap the path as they do from page-locked input.
// The filler thread refills a buffer once the transfer out of it has
// completed; the caller's thread waits for a chunk to be staged before it
// issues its transfer.
struct Stager {
  int dev = 0;
  char* buf[2] = {nullptr, nullptr};
  hipEvent_t out[2] = {nullptr, nullptr};  // transfer out of buffer b done
  std::mutex mu;
  std::condition_variable cv;
  int staged = 0;   // chunks copied into a buffer
  int issued = 0;   // chunks whose transfer has been enqueued
  bool stop = false;
  bool failed = false;
  std::thread th;
  void finish() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    if (th.joinable()) th.join();
  }
  ~Stager() {
    finish();
    (void)hipSetDevice(dev);
    for (int b = 0; b < 2; ++b) {
      if (out[b]) (void)hipEventSynchronize(out[b]);
      if (out[b]) (void)hipEventDestroy(out[b]);
      if (buf[b]) (void)hipHostFree(buf[b]);
    }
  }
};

// memcpy of n bytes split over up to 16 host threads
void parallel_copy(char* dst, const char* src, size_t n) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int T = (int)std::min<size_t>(std::min(16u, hw), std::max<size_t>(1, n >> 24));
  if (T <= 1) {
    memcpy(dst, src, n);
    return;
  }
  std::vector<std::thread> ts;
  const size_t part = (n + T - 1) / T;
  for (int t = 1; t < T; ++t) {
    const size_t a = (size_t)t * part, b = std::min(n, a + part);
    if (a < b) ts.emplace_back([=] { memcpy(dst + a, src + a, b - a); });
  }
  memcpy(dst, src, std::min(n, part));
  for (std::thread& x : ts) x.join();
}

struct HostPipe {
  int dev = 0;
  char* buf = nullptr;      // nbuf chunk buffers of cap_frames frames
  double* hist = nullptr;   // tile cube of every triple so far (frequency branch)
  hipStream_t copy = nullptr;
  hipEvent_t ev[4] = {};
  Stager* stage = nullptr;  // pageable input only
  ~HostPipe() {
    delete stage;  // stops the filler thread first
    (void)hipSetDevice(dev);
    if (copy) (void)hipStreamSynchronize(copy);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (copy) (void)hipStreamDestroy(copy);
    if (buf) (void)hipFree(buf);
    if (hist) (void)hipFree(hist);
  }
};

// A stack in host memory, streamed in chunks of frames: the copy of chunk
// i + 1 (on a stream of its own) overlaps the path over chunk i, which
// carries the two frames before it and extends the tile-cube history; the
// frequency branch runs on the last chunk over the whole history.
fitrig_status detect_host_impl(fitrig_ctx* ctx, const char* host, fitrig_dtype dtype, int n, int H, int W,
                               double tau, int L, fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                               float* eta_map, fitrig_stats* stats) {
  const fitrig_config& cfg = ctx->cfg;
  if (cfg.branches & FITRIG_FREQ_PIXEL) return FITRIG_E_INVAL;
  const size_t fb = (size_t)H * W * (dtype == FITRIG_F32 ? 4 : 2);
  const int L0 = std::min(n, std::max(L, 3));  // the first chunk needs three frames
  const int nbuf = L >= 2 ? 3 : 4;             // chunk i reads the buffers of chunks i, i-1 (and i-2 when L = 1)
  std::vector<int> start;
  for (int s0 = 0; s0 < n; s0 += (s0 == 0 ? L0 : L)) start.push_back(s0);
  const int nch = (int)start.size();
  auto len = [&](int i) { return (i + 1 < nch ? start[i + 1] : n) - start[i]; };
  const int np_all = n - 2;
  const int tile = cfg.tile;
  const int64_t ntiles = (int64_t)((H + tile - 1) / tile) * ((W + tile - 1) / tile);
  const bool freq = (cfg.branches & FITRIG_FREQ) != 0;
  HostPipe P;
  P.dev = cfg.device;
  HIP_TRY(ctx, hipMalloc((void**)&P.buf, (size_t)nbuf * L0 * fb));
  if (freq) HIP_TRY(ctx, hipMalloc((void**)&P.hist, (size_t)np_all * ntiles * 8));
  HIP_TRY(ctx, hipStreamCreateWithFlags(&P.copy, hipStreamNonBlocking));
  for (int i = 0; i < nbuf; ++i) HIP_TRY(ctx, hipEventCreateWithFlags(&P.ev[i], hipEventDisableTiming));
  auto frame_dev = [&](int f) -> const char* {  // device address of frame f (its chunk resident)
    int j = nch - 1;
    while (start[j] > f) --j;
    return P.buf + (size_t)(j % nbuf) * L0 * fb + (size_t)(f - start[j]) * fb;
  };
  // page-locked input is copied straight from the caller's memory; pageable
  // input through the stager
  bool pinned = false;
  {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, host) == hipSuccess) {
      if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeArray) return FITRIG_E_INVAL;
      pinned = at.type == hipMemoryTypeHost;
    } else {
      (void)hipGetLastError();  // unregistered memory may report an error
    }
  }
  if (!pinned) {
    P.stage = new (std::nothrow) Stager;
    if (!P.stage) return FITRIG_E_NOMEM;
    Stager& S = *P.stage;
    S.dev = cfg.device;
    for (int b = 0; b < 2; ++b) {
      if (hipHostMalloc((void**)&S.buf[b], (size_t)L0 * fb, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        S.buf[b] = nullptr;
        return FITRIG_E_NOMEM;
      }
      HIP_TRY(ctx, hipEventCreateWithFlags(&S.out[b], hipEventDisableTiming));
    }
    S.th = std::thread([&S, &start, len, host, fb, nch] {
      (void)hipSetDevice(S.dev);
      for (int j = 0; j < nch; ++j) {
        const int b = j & 1;
        {
          // buffer b is free once the transfer of chunk j - 2 is enqueued and done
          std::unique_lock<std::mutex> lk(S.mu);
          S.cv.wait(lk, [&] { return S.stop || S.issued >= j - 1; });
          if (S.stop) return;
        }
        if (j >= 2 && hipEventSynchronize(S.out[b]) != hipSuccess) {
          std::lock_guard<std::mutex> lk(S.mu);
          S.failed = true;
          S.cv.notify_all();
          return;
        }
        parallel_copy(S.buf[b], host + (size_t)start[j] * fb, (size_t)len(j) * fb);
        {
          std::lock_guard<std::mutex> lk(S.mu);
          S.staged = j + 1;
        }
        S.cv.notify_all();
      }
    });
  }
  auto copy_in = [&](int i) -> fitrig_status {
    char* dst = P.buf + (size_t)(i % nbuf) * L0 * fb;
    if (pinned) {
      HIP_TRY(ctx, hipMemcpyAsync(dst, host + (size_t)start[i] * fb, (size_t)len(i) * fb, hipMemcpyHostToDevice,
                                  P.copy));
    } else {
      Stager& S = *P.stage;
      {
        std::unique_lock<std::mutex> lk(S.mu);
        S.cv.wait(lk, [&] { return S.failed || S.staged > i; });
        if (S.failed) return FITRIG_E_HIP;
      }
      HIP_TRY(ctx, hipMemcpyAsync(dst, S.buf[i & 1], (size_t)len(i) * fb, hipMemcpyHostToDevice, P.copy));
      HIP_TRY(ctx, hipEventRecord(S.out[i & 1], P.copy));
      {
        std::lock_guard<std::mutex> lk(S.mu);
        S.issued = i + 1;
      }
      S.cv.notify_all();
    }
    HIP_TRY(ctx, hipEventRecord(P.ev[i % nbuf], P.copy));
    return FITRIG_OK;
  };
  fitrig_status rc;
  // scratch for the largest chunk call up front (first chunk, then a chunk
  // with two carried frames and the longest history), so no call grows it
  {
    FreqHist h0{P.hist, 0, np_all, P.hist, nch > 1 ? 1 : 0};
    Call c0 = shape_call(0, L0, H, W, dtype, freq ? &h0 : nullptr, cand_cap, ctx->stream);
    if ((rc = check_shape(cfg, c0)) != FITRIG_OK) return rc;
    if ((rc = sizing_pass(ctx, c0, (size_t)result_layout(c0.n - 2, cand_cap).bytes)) != FITRIG_OK ||
        (rc = provision(ctx, ctx->stream)) != FITRIG_OK)
      return rc;
    if (nch > 1) {
      FreqHist h1{P.hist, np_all - L, np_all, P.hist, 0};
      Call c1 = shape_call(2, L, H, W, dtype, freq ? &h1 : nullptr, cand_cap, ctx->stream);
      if ((rc = sizing_pass(ctx, c1, (size_t)result_layout(c1.n - 2, cand_cap).bytes)) != FITRIG_OK ||
          (rc = provision(ctx, ctx->stream)) != FITRIG_OK)
        return rc;
    }
  }
  if ((rc = copy_in(0)) != FITRIG_OK) return rc;
  int64_t total = 0, written = 0;
  int done_triples = 0;
  fitrig_status status = FITRIG_OK;
  double M = -INFINITY;
  fitrig_stats last;
  memset(&last, 0, sizeof(last));
  int64_t n_img = 0;
  uint32_t ran = 0;
  for (int i = 0; i < nch; ++i) {
    if (i + 1 < nch && (rc = copy_in(i + 1)) != FITRIG_OK) return rc;
    HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, P.ev[i % nbuf], 0));
    Call c;
    memset(&c, 0, sizeof(c));
    c.stack = P.buf + (size_t)(i % nbuf) * L0 * fb;
    c.ncarry = i == 0 ? 0 : 2;
    c.carry0 = i == 0 ? nullptr : frame_dev(start[i] - 2);
    c.carry1 = i == 0 ? nullptr : frame_dev(start[i] - 1);
    c.dtype = dtype;
    c.n = c.ncarry + len(i);
    c.H = H;
    c.W = W;
    c.tau = tau;
    c.eta_map = i + 1 == nch ? eta_map : nullptr;
    c.st = ctx->stream;
    const FreqHist h{P.hist, done_triples, np_all, P.hist, i + 1 < nch ? 1 : 0};
    c.hist = freq ? &h : nullptr;
    const int64_t room = std::max<int64_t>(0, cand_cap - written);
    c.cand_cap = room;
    const int np = c.n - 2;
    fitrig_stats st;
    memset(&st, 0, sizeof(st));
    st.mu = stats && stats->mu ? stats->mu + done_triples : nullptr;
    st.sigma = stats && stats->sigma ? stats->sigma + done_triples : nullptr;
    st.flags = stats && stats->flags ? stats->flags + done_triples : nullptr;
    int64_t nc = 0;
    rc = detect_impl(ctx, c, room > 0 ? cand + written : nullptr, &nc, &st, false);
    if (rc != FITRIG_OK && rc != FITRIG_E_TRUNC) return rc;
    if (rc == FITRIG_E_TRUNC) status = FITRIG_E_TRUNC;
    const int64_t k = std::min(nc, room);
    for (int64_t j = 0; j < k; ++j)
      if (cand[written + j].branch == FITRIG_IMAGE) cand[written + j].triple += done_triples;
    written += k;
    total += nc;
    n_img += st.n_image_cand;
    ran |= st.ran;
    M = std::max(M, st.M);
    last = st;
    done_triples += np;
  }
  *n_cand = total;
  if (total > cand_cap) status = FITRIG_E_TRUNC;
  if (stats) {
    stats->M = M;
    stats->n_triples = np_all;
    stats->status = status;
    stats->eta_mu = last.eta_mu;
    stats->eta_sigma = last.eta_sigma;
    stats->n_image_cand = n_img;
    stats->n_freq_cand = last.n_freq_cand;
    stats->n_freq_px_cand = 0;
    stats->eta_px_mu = 0.0;
    stats->eta_px_sigma = 0.0;
    stats->ran = (ran & FITRIG_IMAGE) | (last.ran & FITRIG_FREQ);
    stats->eta_flags = last.eta_flags;
  }
  return status;
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
  if (!ctx->ev_recorded) return 0;
  const int32_t n = cap < FITRIG_N_PHASES ? cap : FITRIG_N_PHASES;
  for (int32_t i = 0; i < n; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[i + 1]) != hipSuccess) return 0;
    ms[i] = t;
  }
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
    case FITRIG_E_SCRATCH: return "the call needs more scratch than the allocation-free entry's static array holds";
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
  // address of the allocation-free entry's array on this device (once per
  // device; a failed lookup shows only in that entry, as E_HIP)
  scratch_setup(cfg->device);
  // scratch sized from the capacity hints, so warm calls allocate nothing
  if ((rc = presize(ctx)) != FITRIG_OK) {
    fitrig_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return FITRIG_OK;
}

fitrig_status fitrig_destroy(fitrig_ctx* ctx) {
  if (!ctx) return FITRIG_E_INVAL;
  (void)hipSetDevice(ctx->cfg.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (GraphEntry& g : ctx->graphs) drop_graph(g);
  if (!ctx->in_arena)
    for (DevBuf fitrig_ctx::* m : kBufs)
      if ((ctx->*m).p) (void)hipFree((ctx->*m).p);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  for (int i = 0; i <= FITRIG_N_PHASES; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  for (AsyncOut* o : ctx->captured_outs) delete o;
  delete ctx;
  return FITRIG_OK;
}

fitrig_status fitrig_detect(fitrig_ctx* ctx, const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H,
                            int32_t W, double sigma, fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                            float* index_map, float* eta_map, float* eta_px_map, fitrig_stats* stats,
                            void* hip_stream) {
  if (!ctx) return FITRIG_E_INVAL;
  fitrig_status rc = check_args(stack, dtype, H, W, sigma, cand, cand_cap, n_cand);
  if (rc != FITRIG_OK) return rc;
  if (n_snap < 3) return FITRIG_E_INVAL;
  if (!hip_stream) *n_cand = 0;
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
  c.eta_px_map = eta_px_map;
  c.st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  c.hist = nullptr;
  c.cand_cap = cand_cap;
  return detect_impl(ctx, c, cand, n_cand, stats, hip_stream != nullptr);
}

fitrig_status fitrig_detect_noalloc(fitrig_ctx* ctx, const void* stack, fitrig_dtype dtype, int32_t n_snap,
                                    int32_t H, int32_t W, double sigma, fitrig_candidate* cand, int64_t cand_cap,
                                    int64_t* n_cand, float* index_map, float* eta_map, float* eta_px_map,
                                    fitrig_stats* stats, void* hip_stream) {
  if (!ctx) return FITRIG_E_INVAL;
  fitrig_status rc = check_args(stack, dtype, H, W, sigma, cand, cand_cap, n_cand);
  if (rc != FITRIG_OK) return rc;
  if (n_snap < 3) return FITRIG_E_INVAL;
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
  c.eta_px_map = eta_px_map;
  c.st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  c.hist = nullptr;
  c.cand_cap = cand_cap;
  return detect_noalloc_impl(ctx, c, cand, n_cand, stats);
}

fitrig_status fitrig_detect_host(fitrig_ctx* ctx, const void* host_stack, fitrig_dtype dtype, int32_t n_snap,
                                 int32_t H, int32_t W, double sigma, int32_t chunk_frames, fitrig_candidate* cand,
                                 int64_t cand_cap, int64_t* n_cand, float* eta_map, fitrig_stats* stats) {
  if (!ctx) return FITRIG_E_INVAL;
  fitrig_status rc = check_args(host_stack, dtype, H, W, sigma, cand, cand_cap, n_cand);
  if (rc != FITRIG_OK) return rc;
  if (n_snap < 3 || chunk_frames < 1) return FITRIG_E_INVAL;
  *n_cand = 0;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FITRIG_E_HIP;
  return detect_host_impl(ctx, (const char*)host_stack, dtype, n_snap, H, W, sigma, chunk_frames, cand, cand_cap,
                          n_cand, eta_map, stats);
}

}  // extern "C"

namespace fitrig {

// Detect over [carried frames][new frames] (serving, synchronous on the
// context's stream). The carried frames have the dtype and size of the stack.
fitrig_status detect_frames(fitrig_ctx* ctx, const void* carry0, const void* carry1, int ncarry, const void* stack,
                            fitrig_dtype dtype, int32_t n_new, int32_t H, int32_t W, double sigma,
                            fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand, fitrig_stats* stats,
                            void* hip_stream, const FreqHist* hist) {
  if (!ctx || ncarry < 0 || ncarry > 2) return FITRIG_E_INVAL;
  fitrig_status rc = check_args(stack, dtype, H, W, sigma, cand, cand_cap, n_cand);
  if (rc != FITRIG_OK) return rc;
  if (hist && (hist->n_in < 0 || hist->cap < 0 || hist->cap > 2048 || hist->n_in > hist->cap ||
               (hist->n_in > 0 && !hist->in) || hist->px_cap < 0 || hist->px_cap > 2048 || hist->px_n < 0 ||
               hist->px_n > hist->px_cap || (hist->px_cap > 0 && (!hist->px_ring || hist->px_start < 0 ||
                                                                  hist->px_start >= hist->px_cap))))
    return FITRIG_E_INVAL;
  if ((ncarry >= 1 && !carry0) || (ncarry == 2 && !carry1)) return FITRIG_E_INVAL;
  if (n_new < 1 || ncarry + n_new < 3) return FITRIG_E_INVAL;
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
  c.eta_px_map = nullptr;
  c.st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
  c.hist = hist;
  c.cand_cap = cand_cap;
  if (ctx->use_graphs) return detect_graph(ctx, c, cand, n_cand, stats);
  return detect_impl(ctx, c, cand, n_cand, stats, false);
}

// A serving slot runs on a non-blocking stream of its own (captures must not
// be joined by work on the legacy default stream; the server orders each
// request after that stream with an event recorded at submit).
fitrig_status ctx_set_serving(fitrig_ctx* ctx, bool graphs) {
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FITRIG_E_HIP;
  hipStream_t s = nullptr;
  HIP_TRY(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (ctx->stream) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
  }
  ctx->stream = s;
  ctx->serving = true;
  ctx->use_graphs = graphs;
  return FITRIG_OK;
}
bool ctx_uses_graphs(const fitrig_ctx* ctx) { return ctx->use_graphs; }
int64_t ctx_graph_replays(const fitrig_ctx* ctx) { return ctx->graph_replays; }

// Device bytes the context holds (scratch buffers and mapped result memory).
int64_t ctx_device_bytes(const fitrig_ctx* ctx) {
  int64_t b = (int64_t)ctx->h_stage_cap;
  for (DevBuf fitrig_ctx::* m : kBufs) b += (int64_t)(ctx->*m).cap;
  return b;
}


// Sizes ctx's scratch for a call of this shape (allocates, before serving).
fitrig_status ctx_presize_for(fitrig_ctx* ctx, int ncarry, int n_new, int H, int W, fitrig_dtype dtype,
                              const FreqHist* hist, int64_t cand_cap) {
  const Call c = shape_call(ncarry, n_new, H, W, dtype, hist, cand_cap, ctx->stream);
  if (c.n < 3 || check_shape(ctx->cfg, c) != FITRIG_OK) return FITRIG_E_INVAL;
  if (hipSetDevice(ctx->cfg.device) != hipSuccess) return FITRIG_E_HIP;
  const fitrig_status rc = sizing_pass(ctx, c, (size_t)result_layout(c.n - 2, cand_cap).bytes);
  if (rc != FITRIG_OK) return rc;
  return provision(ctx, ctx->stream);
}

// Exact device bytes one call of this shape needs (the sizing pass of a
// host-only context: nothing is allocated or launched).
int64_t call_scratch_bytes(const fitrig_config& cfg, int ncarry, int n_new, int H, int W, fitrig_dtype dtype,
                           const FreqHist* hist, int64_t cand_cap) {
  fitrig_ctx tmp;
  if (!size_shape(cfg, shape_call(ncarry, n_new, H, W, dtype, hist, cand_cap, nullptr), tmp)) return 0;
  int64_t b = (int64_t)std::max<size_t>(tmp.h_want, 1 << 16);
  for (DevBuf fitrig_ctx::* m : kBufs) b += (int64_t)(tmp.*m).want;
  return b;
}

hipStream_t ctx_stream(fitrig_ctx* ctx) { return ctx->stream; }
int32_t& ctx_last_hip(fitrig_ctx* ctx) { return ctx->last_hip; }

}  // namespace fitrig
