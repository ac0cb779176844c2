// Internal declarations shared by the FITrig device code and its host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fitrig {

// Output rows per band of the streaming kernel, lanes (input columns) per
// workgroup, 64-cell row segments per column group.
constexpr int kBand = 16;
constexpr int kLanes = 256;
constexpr int kSegsPerGroup = 4;
constexpr int64_t kRsSample = 1 << 20;  // bracket sample of the robust spread (values per set)
constexpr int kMaxHalo = 8;          // window <= 17
constexpr int kPieces = 9;           // 32-wide tile pieces a column group can touch
constexpr int kHistBins = 2048;      // radix-select digit bins (11 bits)

// Output columns of a column group: 15 full 16-column chunks (the 256 lanes
// also cover the halo of up to 8 columns on each side).
inline int out_width(int /*halo*/) { return kLanes - 16; }

// Values of one call that change between calls of the same shape. The
// kernels read them from device memory (written by a one-thread kernel at the
// start of each call), so a recorded launch sequence (a HIP graph) serves
// every call of its shape once this record is rewritten.
struct CallDev {
  const void* base;      // first frame of the new stack
  const void* carry0;    // frames carried in front of the stack (serving), nullable
  const void* carry1;
  const double* hist_in; // serving: frequency history [n_in][Ty][Tx] (nullable)
  double* hist_out;      // serving: receives the covered slices (nullable)
  double tau;            // threshold of Eqs. (9), (12)
  float* px_ring;        // serving: ring of per-pixel q maps [cap][H][W] (nullable)
  int32_t px_start;      // ring slot of the oldest map held
  int32_t px_pad;
};

// Streaming index kernel arguments (one launch covers every triple).
struct StreamArgs {
  const CallDev* cd;     // frame pointers
  int32_t ncarry;
  int32_t n;             // total frames seen by the kernel = ncarry + new frames
  int64_t plane;         // H * W
  int32_t H, W;
  int32_t ncol, nbands, out_w;
  int32_t band_block;    // workgroup order: blocks of this many bands (1 = row order)
  int32_t r_signed;
  float Cf;
  float* qmap;           // nullable [n-2][H][W]
  double* stat_part;     // [n-2][nwg][2]  (sum q, sum q^2); nullable when qmap is set
  float* seg_max;        // [n-2][H][ncol*4]
  double* tile_part;     // nullable [n-2][nbands][ncol][kPieces][3]
  uint32_t* max_key;     // order-preserving key of the stack maximum (atomic max)
  // nullable (map-writing form only): order keys of q on a sample grid, the
  // first cell of every 16-cell chunk in the first row of every samp_bstride-th
  // band, [n-2][samp_S] (index: band / samp_bstride * samp_nch + group *
  // samp_cpg + chunk)
  uint32_t* qsamp;
  int64_t samp_S;
  int32_t samp_bstride, samp_cpg, samp_nch;
};

// Generic tile-mode kernel arguments (re-reads the three frames of a triple).
struct TileArgs {
  const CallDev* cd;
  int32_t ncarry;
  int32_t n;
  int64_t plane;
  int32_t H, W;
  int32_t tile;
  int32_t nchunk;        // ceil(W / 256)
  int32_t pieces;        // tiles a 256-column chunk can touch
  int32_t r_signed;
  float Cf;
  double* tile_part;     // [n-2][Ty][nchunk][pieces][3]
  uint32_t* max_key;     // order-preserving key of the stack maximum (atomic max)
};

// Streaming tile-mode kernel arguments (tile a power of two <= 32): one
// workgroup per band of whole tile rows and chunk of 256 columns, every frame
// read once.
struct TileStreamArgs {
  const CallDev* cd;
  int32_t ncarry;
  int32_t n;
  int64_t plane;
  int32_t H, W;
  int32_t tile;
  int32_t nchunk, nbands;
  int32_t Ty, Tx;
  int32_t r_signed;
  float Cf;
  double* cube;          // [n-2][Ty][Tx]
  float* cube_f;         // [n-2][Ty][Tx]
  uint32_t* max_key;     // order-preserving key of the stack maximum (atomic max)
};

// Layout of the 64-cell row segments a selection works on.
struct SegLayout {
  int32_t Ho, Wo;        // cell grid of one set (one triple)
  int32_t nsets;         // number of sets (triples)
  int32_t spg;           // segments per column group
  int32_t gw;            // column-group width (cells)
  int32_t nseg_row;      // segments per row
  int32_t br;            // rows per selection block (a block is br rows of one segment)
  int32_t nbr;           // blocks per column of segments: ceil(Ho / br)
};

__host__ __device__ inline int seg_x0(const SegLayout& L, int g) {
  return (g / L.spg) * L.gw + (g % L.spg) * 64;
}
__host__ __device__ inline int seg_width(const SegLayout& L, int g) {
  int x0 = seg_x0(L, g);
  int w = L.gw - (g % L.spg) * 64;
  if (w > 64) w = 64;
  if (x0 + w > L.Wo) w = L.Wo - x0;
  return w < 0 ? 0 : w;
}
__host__ __device__ inline int seg_of_x(const SegLayout& L, int x) {
  return (x / L.gw) * L.spg + (x % L.gw) / 64;
}

// Arguments of the exact recompute of selected segments (sliding mode).
struct RecomputeArgs {
  const CallDev* cd;
  int32_t ncarry;
  int64_t plane;
  int32_t H, W;
  float Cf;
  SegLayout L;
  const int64_t* seg_entry;
  const int64_t* nsel;   // segments selected (device)
  int64_t cap;
  const double* mu;
  const double* sigma;
  uint64_t* mask;
  float* cell_q;
};

// Device counters of one call.
enum {
  CNT_NSEL = 0,    // segments selected in the current selection run
  CNT_NCOMP = 1,   // components of the current run
  CNT_OUTBASE = 3, // candidates written so far
  CNT_TRUNC = 5,   // internal capacity exceeded
  CNT_IMG = 6,     // image-branch candidates
  CNT_FREQ = 7,    // tile frequency-branch candidates
  CNT_NBLK = 8,    // selection blocks flagged in the current run
  CNT_FPX = 9,     // per-pixel frequency-branch candidates
  CNT_N = 10
};

// Frequency-branch statistics of one call (doubles; the last one holds two
// uint32 flag words: tile branch, per-pixel branch).
enum { ES_MU = 0, ES_SIG = 1, ES_PXMU = 2, ES_PXSIG = 3, ES_FLAGS = 4, ES_N = 5 };

// Byte offsets of a call's results in host-visible memory.
struct ResultLayout {
  int64_t off_cnt;      // int64[CNT_N]
  int64_t off_scalars;  // double M, then the ES_N words of the frequency statistics
  int64_t off_mu;       // double[n']
  int64_t off_sigma;    // double[n']
  int64_t off_flags;    // uint32[n']
  int64_t off_cand;     // fitrig_candidate[cap]
  int64_t bytes;
};

// Kernels templated on the storage type, per type (fitrig_launch.hip): the
// host handle of the instantiation for the given parameters, null if none.
const void* kernel_stream_f32(int halo, bool r_signed, bool qmap);
const void* kernel_stream_f16(int halo, bool r_signed, bool qmap);
const void* kernel_stream_bf16(int halo, bool r_signed, bool qmap);
const void* kernel_tile_stream_f32(int tile, bool r_signed);
const void* kernel_tile_stream_f16(int tile, bool r_signed);
const void* kernel_tile_stream_bf16(int tile, bool r_signed);
const void* kernel_tile_f32(bool r_signed);
const void* kernel_tile_f16(bool r_signed);
const void* kernel_tile_bf16(bool r_signed);
const void* kernel_recompute_f32(int halo, bool r_signed);
const void* kernel_recompute_f16(int halo, bool r_signed);
const void* kernel_recompute_bf16(int halo, bool r_signed);
const void* kernel_stack_max_f32();
const void* kernel_stack_max_f16();
const void* kernel_stack_max_bf16();

}  // namespace fitrig

#include "fitrig.h"

namespace fitrig {
// Tile-cube history of a field for the frequency branch (serving): the
// branch covers the last `cap` triples of [history | this call's triples].
//   in:  device, FP64 [n_in][Ty][Tx], oldest first (nullable when n_in = 0)
//   out: device, receives the covered slices, [min(cap, n_in + n')][Ty][Tx]
//        (may be the same memory as `in`)
struct FreqHist {
  const double* in;
  int n_in;
  int cap;
  double* out;
  int defer;  // 1: only extend the history; the branch runs on a later call
  // per-pixel branch: ring of the sliding q maps of the field's last px_cap
  // triples (device, [px_cap][H][W] FP32); px_n maps held, the oldest at
  // slot px_start; the call appends its own maps (0 = not kept)
  float* px_ring;
  int px_cap;
  int px_start;
  int px_n;
};

// Host-side entry points shared between translation units of the library.
fitrig_status detect_frames(fitrig_ctx* ctx, const void* carry0, const void* carry1, int ncarry, const void* stack,
                            fitrig_dtype dtype, int32_t n_new, int32_t H, int32_t W, double sigma,
                            fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand, fitrig_stats* stats,
                            void* hip_stream, const FreqHist* hist);
hipStream_t ctx_stream(fitrig_ctx* ctx);
// serving slots: synchronous calls on the context's stream, launch sequences
// replayed from HIP graphs captured per call shape (graphs = true)
fitrig_status ctx_set_serving(fitrig_ctx* ctx, bool graphs);
bool ctx_uses_graphs(const fitrig_ctx* ctx);
int64_t ctx_graph_replays(const fitrig_ctx* ctx);
int64_t ctx_device_bytes(const fitrig_ctx* ctx);
int64_t call_scratch_bytes(const fitrig_config& cfg, int ncarry, int n_new, int H, int W, fitrig_dtype dtype,
                           const FreqHist* hist, int64_t cand_cap);
fitrig_status ctx_presize_for(fitrig_ctx* ctx, int ncarry, int n_new, int H, int W, fitrig_dtype dtype,
                              const FreqHist* hist, int64_t cand_cap);

int32_t& ctx_last_hip(fitrig_ctx* ctx);
}  // namespace fitrig
