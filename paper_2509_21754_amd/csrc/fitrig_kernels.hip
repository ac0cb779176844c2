// FITrig device code that does not depend on the storage type: tile-cube
// merge, statistics, radix selection for the robust spread, the selection
// pipeline (segment flags, compaction, union-find components), the
// image-frequency transforms and result delivery. Included by the host
// runtime (fitrig_api.hip), which launches these kernels.
//
// Method (Li, Adamek & Armour, arXiv 2509.21754):
//   z = (q - mean q) / std q per triple, select z > tau             Sec. 2.4.1, Eqs. (8)-(9)
//   eta = h(|DFT_s[q(s) - mean q]|) per tile or pixel, z on eta      Sec. 2.4.2, Eqs. (10)-(12)
#include "fitrig_device.h"

namespace fitrig {

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

// Selection paths of a set (gate values): order statistics from the keys
// gathered in a bracket, from a fallback bracket pass, or from the whole set.
constexpr uint32_t kPathGathered = 1;
constexpr uint32_t kPathFallback = 2;
constexpr uint32_t kPathFull = 3;


// Per-set gate: the kernels of one selection path run for a set only when
// its entry equals `want` (null gate: every set). The path of each set is
// decided on the device, so no host round trip sits inside the spread.
__device__ __forceinline__ bool gated_off(const uint32_t* gate, int s, uint32_t want) {
  return gate != nullptr && gate[s] != want;
}

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
                                                 const unsigned long long* nvalid, const uint32_t* gate, uint32_t want) {
  __shared__ uint32_t h[kHistBins];
  const int s = blockIdx.y;
  if (gated_off(gate, s, want)) return;
  const RsState S = st[s];
  const uint32_t dmask = (1u << nbits) - 1u;
  if (((S.known >> shift) & dmask) == dmask) return;  // digit known from the start
  for (int i = threadIdx.x; i < kHistBins; i += 256) h[i] = 0;
  __syncthreads();
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
// Upper middle value from the last digit's histogram (nullable in k_rs_pick):
// the key after the selected one is the same key while the selected bin has
// more keys, else the next non-empty bin's key; only when neither is in the
// histogram does need[s] stay 1 (then k_rs_next counts over the values).
// Written for k_rs_next_store: cnt_le huge (same key) or 0 with min_gt.
struct RsNext {
  unsigned long long* cnt_le;
  uint32_t* min_gt;
  uint32_t* need;
};

__global__ __launch_bounds__(256) void k_rs_pick(RsState* st, uint32_t* hist, int shift, int nbits, const uint32_t* gate,
                                                 uint32_t want, RsNext nx) {
  __shared__ int64_t part[256];
  __shared__ int nxt_sh[256];
  __shared__ int sdig;
  __shared__ int64_t srem;
  __shared__ uint32_t scnt;
  const int s = blockIdx.x, t = threadIdx.x;
  if (gated_off(gate, s, want)) return;
  const RsState S = st[s];
  if (((S.known >> shift) & ((1u << nbits) - 1u)) == ((1u << nbits) - 1u)) return;  // known from the start
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
  uint32_t cdig = 0;
  if (excl <= S.rank && S.rank < incl) {
#pragma unroll
    for (int j = 0; j < kHistBins / 256; ++j) {
      if (dig < 0 && j < per) {
        if (acc + (int64_t)c[j] > S.rank) {
          dig = t * per + j;
          cdig = c[j];
        } else {
          acc += c[j];
        }
      }
    }
  } else if (t == 255 && S.rank >= incl) {
    dig = nb - 1;  // rank beyond the count
    acc = incl;
  }
  if (nx.need) {
    if (t == 0) sdig = -1;
    __syncthreads();
    if (dig >= 0) {
      sdig = dig;
      srem = S.rank - acc;
      scnt = cdig;
    }
    __syncthreads();
    const int d = sdig;
    int nxt = INT32_MAX;
#pragma unroll
    for (int j = 0; j < kHistBins / 256; ++j) {
      const int b = t * per + j;
      if (j < per && b > d && c[j] != 0u && b < nxt) nxt = b;
    }
    nxt_sh[t] = nxt;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (t < w) nxt_sh[t] = min(nxt_sh[t], nxt_sh[t + w]);
      __syncthreads();
    }
    if (t == 0 && d >= 0) {
      if (srem + 1 < (int64_t)scnt) {
        nx.cnt_le[s] = 1ull << 62;  // the upper middle is the selected key
        nx.need[s] = 0u;
      } else if (nxt_sh[0] != INT32_MAX) {
        nx.cnt_le[s] = 0ull;
        nx.min_gt[s] = (S.prefix & ~(((uint32_t)(nb - 1)) << shift)) | ((uint32_t)nxt_sh[0] << shift);
        nx.need[s] = 0u;
      }
    }
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
__global__ void k_rs_init_rank(RsState* st, int nsets, int64_t rank, const uint32_t* gate, uint32_t want) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gated_off(gate, s, want)) return;
  RsState S;
  S.prefix = 0;
  S.known = 0;
  S.rank = rank;
  st[s] = S;
}

// Rank within the gathered keys: global rank minus the keys below them.
// kb (nullable): bounds kb[2 s] <= key <= kb[2 s + 1] of every gathered key;
// the digits (11, 11, 10 bits from the top) inside the common leading bits
// of the two bounds are the same in every gathered key, so they start known
// (their passes are skipped).
__global__ void k_rs_init_gathered(RsState* st, int nsets, int64_t rank, const unsigned long long* cnt,
                                   const uint32_t* kb, const uint32_t* gate, uint32_t want) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gated_off(gate, s, want)) return;
  RsState S;
  S.prefix = 0;
  S.known = 0;
  if (kb && kb[2 * s] <= kb[2 * s + 1]) {
    const uint32_t d = kb[2 * s] ^ kb[2 * s + 1];
    const int common = d ? __clz((int)d) : 32;
    uint32_t known = 0;
    if (common >= 11) known |= 0xFFE00000u;
    if (common >= 22) known |= 0x001FFC00u;
    if (common >= 32) known = 0xFFFFFFFFu;
    S.known = known;
    S.prefix = kb[2 * s] & known;
  }
  S.rank = rank - (int64_t)cnt[2 * s];
  st[s] = S;
}

// Bounds of the MAD keys bits((float)|q - med|) of the cells gathered in the
// MAD window (k_rs_mad_window: |q - mhat| at most t_out, and at least t_in
// when the window has inner cells, kB != kC, up to the FP32 rounding of the
// window's bounds) once the median med is exact: |q - med| is within
// e = |med - mhat| of |q - mhat|. The bounds are widened by 2^-20 of
// |mhat| + t_out + e, far beyond every rounding involved.
__global__ void k_rs_mad_keybounds(const double* pl, const double* med, const uint32_t* wk, int nsets,
                                   const uint32_t* gate, uint32_t want, uint32_t* kb) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gated_off(gate, s, want)) return;
  const double mh = pl[4 * s + 0], t_in = pl[4 * s + 2], t_out = pl[4 * s + 3];
  const bool inner = wk[4 * s + 1] != wk[4 * s + 2];
  const double e = fabs(med[s] - mh);
  const double slack = (fabs(mh) + fabs(t_out) + e) * 0x1p-20;
  const double lo = (inner && t_in > 0.0) ? fmax(0.0, t_in - e - slack) : 0.0;
  const double hi = t_out + e + slack;
  const bool ok = isfinite(lo) && isfinite(hi) && hi >= lo;
  kb[2 * s] = ok ? __float_as_uint(__double2float_rd(lo)) : 1u;
  kb[2 * s + 1] = ok ? __float_as_uint(__double2float_ru(hi)) : 0u;  // lo > hi: no seed
}

// Keys of a sample of each set: sample i is value (i * mult) mod per_set
// with mult odd and coprime to per_set, so the samples spread over the set
// without following its rows or columns.
__global__ void k_rs_sample(const float* vals, int64_t per_set, int mode, const double* med, int64_t S,
                            uint64_t mult, uint32_t* samp, const uint32_t* gate, uint32_t want) {
  const int s = blockIdx.y;
  if (gated_off(gate, s, want)) return;
  const double m = mode == 1 ? med[s] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    // i < 2^21 and mult < per_set < 2^32: the product fits in 64 bits
    const uint64_t pos = ((uint64_t)i * mult) % (uint64_t)per_set;
    samp[(int64_t)s * S + i] = rs_key(vals[(int64_t)s * per_set + (int64_t)pos], mode, m);
  }
}

// selected key of each set -> bkt[2 s + which]
__global__ void k_rs_key_out(const RsState* st, int nsets, int which, uint32_t* bkt, const uint32_t* gate,
                             uint32_t want) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsets && !gated_off(gate, s, want)) bkt[2 * s + which] = st[s].prefix;
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
                                                   uint32_t* gbuf, const uint32_t* gate, uint32_t want) {
  if (gated_off(gate, blockIdx.y, want)) return;
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
constexpr int kGather2PT = 8;  // values per thread per round (16 measured slower)
constexpr int kGather2Round = 256 * kGather2PT;
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
  constexpr int PT = kGather2PT;
  static_assert(PT % 4 == 0 && PT <= 16, "two selection bits per value in 32 bits; 16-bit round counts");
  // Every read is in range and unconditional: past the end the address is
  // clamped to the set's last values, which the ok flags below ignore. (A
  // per-lane condition on the read would put the round's prefetch behind a
  // branch, and the wait for the current round would then also wait for it.)
  auto fetch = [&](int64_t base, float (&q)[PT]) {
    if (VEC) {
#pragma unroll
      for (int j = 0; j < PT / 4; ++j) {
        const int64_t i = min(base + 4 * ((int64_t)j * 256 + threadIdx.x), per_set - 4);  // per_set % 4 == 0
        // read once: non-temporal
        const fitrig_v4f x = __builtin_nontemporal_load(reinterpret_cast<const fitrig_v4f*>(v + i));
        q[4 * j + 0] = x.x;
        q[4 * j + 1] = x.y;
        q[4 * j + 2] = x.z;
        q[4 * j + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < PT; ++j) q[j] = v[min(base + (int64_t)j * 256 + threadIdx.x, per_set - 1)];
    }
  };
  auto index_of = [&](int64_t base, int j) -> int64_t {
    return VEC ? base + 4 * ((int64_t)(j >> 2) * 256 + threadIdx.x) + (j & 3) : base + (int64_t)j * 256 + threadIdx.x;
  };
  // one round: place this round's values (q, read one round earlier)
  auto round = [&](const float (&q)[PT], int64_t base) {
    uint32_t k[PT];
    uint32_t sel = 0;  // bit j: median bracket, bit PT + j: MAD window
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const bool ok = index_of(base, j) < per_set;
      k[j] = NONNEG ? (__float_as_uint(q[j]) | 0x80000000u) : ord_key(q[j]);
      const bool in_w = k[j] > kB && k[j] < kC;
      below += (ok && k[j] < lo) ? 1u : 0u;
      inner += (ok && in_w) ? 1u : 0u;
      sel |= (ok && k[j] - lo <= hi - lo) ? (1u << j) : 0u;
      sel |= (ok && !in_w && k[j] - kA <= kD - kA) ? (1u << (PT + j)) : 0u;
    }
    // counts of both stages packed in 16-bit halves (at most 256 PT each)
    const uint32_t c = (uint32_t)__popc(sel & ((1u << PT) - 1u)) | ((uint32_t)__popc(sel >> PT) << 16);
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
      for (int j = 0; j < PT; ++j) {
        if (sel & (1u << j)) stage[0][p0++] = k[j];
        if (sel & (1u << (PT + j))) stage[1][p1++] = __float_as_uint(q[j]);
      }
    }
    nst0 += tot0;
    nst1 += tot1;
    __syncthreads();  // stages written and wsum read by every thread
  };
  // Two buffers in turn (no register copies between rounds): the next
  // round's reads are issued, a scheduling barrier keeps this round's work
  // after them, then the round is placed. Past the last round the reads are
  // clamped and unused. Every thread runs the same rounds.
  float qa[PT], qb[PT];
  int64_t base = blockIdx.x * (int64_t)kGather2Round;
  if (base < per_set) fetch(base, qa);
  while (base < per_set) {
    fetch(base + step, qb);
    __builtin_amdgcn_sched_barrier(0);
    round(qa, base);
    base += step;
    if (base >= per_set) break;
    fetch(base + step, qa);
    __builtin_amdgcn_sched_barrier(0);
    round(qb, base);
    base += step;
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
                                const unsigned long long* cnt1, int nsets, uint32_t* gate_mad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gate_mad[s] != kPathGathered) return;
  const double e = fabs(med[s] - pl[4 * s + 0]);
  const double slack = 0x1p-40;
  const float in_max = (float)((pl[4 * s + 2] + e) * (1.0 + slack));
  const float out_min = (float)((pl[4 * s + 3] - e) * (1.0 - slack));
  const bool ok_in = cnt1[2 * s] == 0 || (double)in_max <= dev[2 * s];
  const bool ok_out = (double)out_min > dev[2 * s + 1];
  // a failed check sends the set to the fallback pass around the exact median
  if (!(ok_in && ok_out && isfinite(med[s]))) gate_mad[s] = kPathFallback;
}

// Path of each set after a bracket pass: the gathered keys when the bracket
// holds both middle ranks and fitted its buffer, else `otherwise`. Also the
// number of valid gathered keys (rank offsets stay in cnt[2 s]).
__global__ void k_rs_plan(const unsigned long long* cnt, int nsets, int64_t cap, int64_t r_lo, int64_t r_hi,
                          uint32_t* gate, uint32_t only, uint32_t take, uint32_t otherwise, unsigned long long* nvalid) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || (only != 0u && gate[s] != only)) return;
  const int64_t below = (int64_t)cnt[2 * s], in = (int64_t)cnt[2 * s + 1];
  const bool ok = in <= cap && below <= r_lo && r_hi < below + in;
  gate[s] = ok ? take : otherwise;
  nvalid[s] = cnt[2 * s + 1];
}

// Dispersion keys of a sample of order keys: |q - med| of the sampled q.
__global__ void k_rs_sample_dev(uint32_t* samp, int64_t S, const double* med, const uint32_t* gate, uint32_t want) {
  const int s = blockIdx.y;
  if (gated_off(gate, s, want)) return;
  const double m = med[s];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t* p = samp + (int64_t)s * S + i;
    *p = rs_key(ord_val(*p), 1, m);
  }
}

// The order statistic just above the selected one (rank + 1): the selected
// key itself when more than rank + 1 keys are <= it, else the smallest key
// above it. One pass: count of keys <= the selected key, minimum key above.
__global__ __launch_bounds__(256) void k_rs_next(const float* vals, int64_t per_set, int mode, const double* med,
                                                 const RsState* st, unsigned long long* cnt_le, uint32_t* min_gt,
                                                 const unsigned long long* nvalid, const uint32_t* gate,
                                                 uint32_t want, const uint32_t* need) {
  __shared__ uint32_t sh_c[256];
  __shared__ uint32_t sh_m[256];
  const int s = blockIdx.y;
  if (gated_off(gate, s, want) || (need && !need[s])) return;
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
                                const unsigned long long* base, double* out, const uint32_t* gate, uint32_t want) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gated_off(gate, s, want)) return;
  const int64_t le = (int64_t)cnt_le[s] + (base ? (int64_t)base[2 * s] : 0);
  const uint32_t k = (le >= rank_hi + 1) ? st[s].prefix : min_gt[s];
  out[2 * s + 1] = mode ? (double)__uint_as_float(k) : (double)ord_val(k);
}

// value of the selected key: mode 0 -> q, mode 1 -> |q - med| (as float)
__global__ void k_rs_store(const RsState* st, int nsets, int mode, int which, double* out, const uint32_t* gate,
                           uint32_t want) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets || gated_off(gate, s, want)) return;
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
// 16 threads per segment, 4 consecutive cells each (a segment's 64 cells are
// read as 256 contiguous bytes), then a maximum over the 16 lanes.
__global__ __launch_bounds__(256) void k_segmax_direct(const float* vals, SegLayout L, float* seg_max) {
  const int64_t total = (int64_t)L.nsets * L.Ho * L.nseg_row;
  const int sub = threadIdx.x & 15;
  // every lane of a 16-lane group runs the same iterations: the shuffles
  // below see the whole group
  for (int64_t e = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4; e < total;
       e += ((int64_t)gridDim.x * blockDim.x) >> 4) {
    const int g = (int)(e % L.nseg_row);
    const int64_t row = e / L.nseg_row;  // set * Ho + y
    const int x0 = seg_x0(L, g), w = seg_width(L, g);
    const float* v = vals + row * L.Wo + x0;
    float m = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * sub + j;
      if (i < w) m = fmaxf(m, v[i]);
    }
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (sub == 0) seg_max[e] = m;
  }
}

constexpr int kPerThread = 16;
constexpr int kChunk = 256 * kPerThread;

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
                                                   const uint32_t* flags, const CallDev* cd, SegLayout L,
                                                   uint8_t* bflag, uint32_t* cnt) {
  __shared__ uint32_t sh[256];
  const double tau = cd->tau;
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
      float m;
      if (y1 - y0 == kBand) {
        // a whole block: every row requested before the first is used
        float v[kBand];
#pragma unroll
        for (int i = 0; i < kBand; ++i) v[i] = p[(int64_t)i * L.nseg_row];
        m = v[0];
#pragma unroll
        for (int i = 1; i < kBand; ++i) m = fmaxf(m, v[i]);
      } else {
        m = p[0];
        for (int y = y0 + 1; y < y1; ++y) {
          p += L.nseg_row;
          m = fmaxf(m, *p);
        }
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
  const CallDev* cd;
  __device__ bool operator()(int64_t j) const {
    const int64_t e = ro.entry(j);
    if (e < 0) return false;
    const int s = (int)(e / ((int64_t)ro.L.Ho * ro.L.nseg_row));
    return zsel(seg_max[e], mu[s], sigma[s], cd->tau);
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

// Cells of each selected segment taken from a value array (tiles / eta).
__global__ __launch_bounds__(64) void k_fill_direct(const float* vals, SegLayout L, const int64_t* seg_entry,
                                                    const int64_t* nsel_p, int64_t cap, const double* mu,
                                                    const double* sigma, const CallDev* cd, uint64_t* seg_mask,
                                                    float* cell_q) {
  const int lane = threadIdx.x;
  const double tau = cd->tau;
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

// Each selected cell starts linked to the first cell of its run of selected
// cells in the slot (the run's lowest slot, so every parent is at most its
// cell and a root is its set's lowest slot): the horizontal unions inside a
// slot are made here.
__global__ void k_uf_init(const uint64_t* seg_mask, const int64_t* nsel_p, int64_t cap, int32_t* parent) {
  int64_t nsel = nsel_p[0];
  if (nsel > cap) nsel = cap;
  const int64_t ns = nsel * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = seg_mask[i >> 6];
    const int off = (int)(i & 63);
    // unselected cells before off; the run starts after the last of them
    const uint64_t gap = ~m & ((1ull << off) - 1ull);
    const int start = gap ? 64 - __clzll((long long)gap) : 0;
    parent[i] = ((m >> off) & 1ull) ? (int32_t)((i & ~63ll) + start) : -1;
  }
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
    const uint64_t m = seg_mask[i >> 6];
    const int off = (int)(i & 63);
    if (!((m >> off) & 1ull)) continue;
    int64_t set;
    int y, x;
    slot_pos(seg_entry, L, i, set, y, x);
    // 8-connectivity from the upper cell of each pair. The right neighbour
    // inside the slot is in the same run (linked at init); across the slot's
    // last cell it is looked up. Below: the cell under x; the lower-left and
    // lower-right cells only from the run's first and last cells (under any
    // other cell of the run they are under its run neighbour).
    const bool first = off == 0 || !((m >> (off - 1)) & 1ull);
    const bool last = off == 63 || !((m >> (off + 1)) & 1ull);
    const int g = seg_of_x(L, x);
    if (off == seg_width(L, g) - 1) {
      const int32_t nb = slot_at(M, seg_mask, L, set, y, x + 1);
      if (nb >= 0) uf_union(parent, (int32_t)i, nb);
    }
    {
      const int32_t nb = slot_at(M, seg_mask, L, set, y + 1, x);
      if (nb >= 0) uf_union(parent, (int32_t)i, nb);
    }
    if (first) {
      const int32_t nb = slot_at(M, seg_mask, L, set, y + 1, x - 1);
      if (nb >= 0) uf_union(parent, (int32_t)i, nb);
    }
    if (last) {
      const int32_t nb = slot_at(M, seg_mask, L, set, y + 1, x + 1);
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
  // the stride and ns are multiples of 64 and blocks are whole waves: every
  // wave holds the 64 cells of one slot (one row of one set) per iteration
  const int lane = threadIdx.x & 63;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns; i += (int64_t)gridDim.x * blockDim.x) {
    bool act = (seg_mask[i >> 6] >> lane) & 1ull;
    const int32_t c = act ? comp_of[parent[i]] : -1;
    act = act && c >= 0;
    const uint64_t am = __ballot(act);
    if (!am) continue;
    int64_t set;
    int y, x;
    slot_pos(seg_entry, L, i, set, y, x);
    const float q = act ? cell_q[i] : 0.0f;
    const double z = ((double)q - mu[set]) / sigma[set];
    const uint32_t lin = (uint32_t)((int64_t)y * L.Wo + x);
    const unsigned long long k =
        act ? ((unsigned long long)ord_key(q) << 32) | (unsigned long long)(0xFFFFFFFFu - lin) : 0ull;
    const unsigned long long wz = act ? (unsigned long long)llround(z * 1048576.0) : 0ull;
    const unsigned long long wy = wz * (unsigned long long)y, wx = wz * (unsigned long long)x;
    const int lead = __ffsll((unsigned long long)am) - 1;
    const int32_t c0 = __shfl(c, lead);
    if (__ballot(act && c != c0) == 0) {
      // one component in the slot's row: integer totals of the wave (exact,
      // so the same as per-cell atomics), added by one lane
      unsigned long long km = k;
      unsigned long long lo[3] = {wz, wy, wx}, hi[3] = {0ull, 0ull, 0ull};
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long ko = __shfl_xor(km, o);
        km = ko > km ? ko : km;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const unsigned long long l2 = __shfl_xor(lo[j], o), h2 = __shfl_xor(hi[j], o);
          const unsigned long long sl = lo[j] + l2;
          hi[j] += h2 + (sl < l2 ? 1ull : 0ull);
          lo[j] = sl;
        }
      }
      if (lane == lead) {
        atomicAdd(npix + c0, (int)__popcll(am));
        atomicMax(key + c0, km);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          unsigned long long* p = w + c0 * 6 + 2 * j;
          const unsigned long long old = atomicAdd(p, lo[j]);
          const unsigned long long h = hi[j] + (old + lo[j] < old ? 1ull : 0ull);
          if (h) atomicAdd(p + 1, h);
        }
        const int xs = x - lane;  // the slot's first cell
        atomicMin(box + c0 * 4 + 0, y);
        atomicMin(box + c0 * 4 + 1, xs + lead);
        atomicMax(box + c0 * 4 + 2, y);
        atomicMax(box + c0 * 4 + 3, xs + 63 - __clzll((long long)am));
      }
      continue;
    }
    if (!act) continue;
    atomicAdd(npix + c, 1);
    atomicMax(key + c, k);
    add128(w + c * 6 + 0, wz);
    add128(w + c * 6 + 2, wy);
    add128(w + c * 6 + 4, wx);
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



// ---------------------------------------------------------------------------
// Image-frequency branch (Sec. 2.4.2, Eq. (10)): per series, DFT over s of
// the mean-removed series, one-sided magnitudes k = 1..floor(n'/2),
// h = max or harmonic sum.
// ---------------------------------------------------------------------------
// tw[m] = (cos, sin)(2 pi m / n'), m = 0..n'-1 (the phase k s is reduced
// modulo n' exactly before the table is read).
__global__ void k_twiddle(int np, double2* tw) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < np; m += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)np, &sn, &cs);
    tw[m] = make_double2(cs, sn);
  }
}

// Tile branch: one thread per tile, direct FP64 sums in the order of Eq. (10).
__global__ __launch_bounds__(256) void k_eta(const double* cube, int np, int64_t ntiles, int harm, const double2* tw,
                                             double* eta, float* eta_f) {
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
          const double2 w = tw[ph];
          re = fma(v, w.x, re);
          im = fma(-v, w.y, im);
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

// Tile branch for series of at most NPMAX values: k_eta with the tile's
// series read once into registers (k_eta reads it again for every
// frequency). The twiddle index depends only on the loop counters: every lane
// reads the same LDS word (a broadcast). Mean, mean removal and every sum are
// k_eta's, in the same order, so eta is the same.
template <int NPMAX>
__global__ __launch_bounds__(256) void k_eta_reg(const double* cube, int np, int64_t ntiles, int harm,
                                                 const double2* twg, double* eta, float* eta_f) {
  __shared__ double2 tw[NPMAX];
  for (int i = threadIdx.x; i < np; i += blockDim.x) tw[i] = twg[i];
  __syncthreads();
  const int K = np / 2;
  const int jmax = harm == 0 ? 1 : harm;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles; t += (int64_t)gridDim.x * blockDim.x) {
    double x[NPMAX];
    const double* p = cube + t;
#pragma unroll
    for (int s = 0; s < NPMAX; ++s) {
      // one running address; past the series it stays on the last value
      // (read again, replaced by zero below), so every read is in range
      asm volatile("" : "+v"(p));
      x[s] = *p;
      p += s + 1 < np ? ntiles : 0;
    }
    double mean = 0.0;
#pragma unroll
    for (int s = 0; s < NPMAX; ++s)
      if (s < np) mean += x[s];
    mean /= (double)np;
    // the mean-removed series, zero past its end: the extra products of the
    // sums below add exact zeros
#pragma unroll
    for (int s = 0; s < NPMAX; ++s) x[s] = s < np ? x[s] - mean : 0.0;
    double best = 0.0;
    for (int k = 1; k <= K; ++k) {
      double val = 0.0;
      for (int j = 1; j <= jmax && j * k <= K; ++j) {
        const int kk = j * k;
        double re = 0.0, im = 0.0;
        int ph = 0;
#pragma unroll
        for (int s = 0; s < NPMAX; ++s) {
          const double2 w = tw[ph];
          re = fma(x[s], w.x, re);
          im = fma(-x[s], w.y, im);
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

// Tile branch for long series: one workgroup per tile, the threads over the
// frequencies. The series (mean removed; the mean summed serially in s, as in
// k_eta), the twiddles and the magnitudes |X_k| sit in LDS; each |X_k| is
// formed once (k_eta forms |X_jk| again for every harmonic sum that uses it),
// then each thread takes the harmonic sums of its frequencies and the block
// takes their maximum. Per frequency the arithmetic and its order are k_eta's,
// so eta is the same.
__global__ __launch_bounds__(256) void k_eta_blk(const double* cube, int np, int64_t ntiles, int harm,
                                                 const double2* twg, double* eta, float* eta_f) {
  extern __shared__ double2 lds_e[];  // [np] twiddles, [np] series, [K] magnitudes
  __shared__ double red[256];
  __shared__ double smean;
  double2* tw = lds_e;
  double* ser = (double*)(lds_e + np);
  double* amp = ser + np;
  const int K = np / 2;
  const int tid = threadIdx.x;
  for (int i = tid; i < np; i += 256) tw[i] = twg[i];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    for (int s = tid; s < np; s += 256) ser[s] = cube[(int64_t)s * ntiles + t];
    __syncthreads();
    if (tid == 0) {
      double mean = 0.0;
      for (int s = 0; s < np; ++s) mean += ser[s];
      smean = mean / (double)np;
    }
    __syncthreads();
    const double mean = smean;
    for (int k = 1 + tid; k <= K; k += 256) {
      double re = 0.0, im = 0.0;
      int ph = 0;
      for (int s = 0; s < np; ++s) {
        const double v = ser[s] - mean;
        const double2 w = tw[ph];
        re = fma(v, w.x, re);
        im = fma(-v, w.y, im);
        ph += k;
        if (ph >= np) ph -= np;
      }
      amp[k - 1] = sqrt(re * re + im * im);
    }
    __syncthreads();
    // harmonic sums (j = 1 .. harm, jk <= K, in order of j) and their maximum
    double best = 0.0;
    bool have = false;
    const int jmax = harm == 0 ? 1 : harm;
    for (int k = 1 + tid; k <= K; k += 256) {
      double val = 0.0;
      for (int j = 1; j <= jmax && j * k <= K; ++j) val += amp[j * k - 1];
      if (!have || val > best) best = val;
      have = true;
    }
    red[tid] = have ? best : -1.0;  // magnitudes are >= 0
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
      __syncthreads();
    }
    if (tid == 0) {
      const double b = K < 1 ? 0.0 : red[0];
      eta[t] = b;
      if (eta_f) eta_f[t] = (float)b;
    }
    __syncthreads();  // ser, amp and red are reused by the next tile
  }
}

typedef double fitrig_v4d __attribute__((ext_vector_type(4)));

// f(integral_constant<int, I>) for I = B .. E - 1, unrolled at compile time.
template <int B, int E, class F>
__device__ __forceinline__ void fitrig_static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    fitrig_static_for<B + 1, E>(f);
  }
}
typedef __attribute__((address_space(1))) float fitrig_gf;        // global memory
typedef __attribute__((address_space(1))) fitrig_v4f fitrig_gv4f;

// Per-pixel form of Eq. (10) on the matrix cores. The series of a pixel is
// real, so with u_s = x_s + x_(n'-s) and v_s = x_s - x_(n'-s) for
// 0 < s < n' / 2 (u_s = x_s, v_s = 0 at s = 0 and s = n' / 2) the transform at
// frequency k is
//   Re = sum_{s=0}^{floor(n'/2)} u_s cos(2 pi k s / n'),
//   Im = -sum_{s=1}^{floor(n'/2)} v_s sin(2 pi k s / n'),
// half the products of the unfolded sum. u and v of FP32 q are exact in
// FP64. For a tile of 64 pixels both are FP64 matrix products D = T U:
// v_mfma_f64_16x16x4 takes 16 rows x 4 folded steps (A: lane i + 16 kk holds
// T[i][kk], the cosine or sine of 2 pi f s / n' for the row's frequency f) and
// 4 steps x 16 pixels (B: lane n + 16 kk holds u or v of step kk, pixel
// column n) and accumulates D, whose register r of lane n + 16 c holds row
// 4 r + c of pixel column n. A block of 16 rows is 16 consecutive
// frequencies, with one accumulator for the cosine rows (B = u) and one for
// the sine rows (B = v): register r of lane n + 16 c then holds Re (resp. Im)
// of frequency 16 b + 4 r + c + 1 of pixel column n. A lane's four pixel
// columns are the four pixels of one 16-byte load, so a block of 16 columns
// is pixels p0 + 4 n + j. The series is not mean-removed: for k >= 1 the
// weights of a row sum to zero, so the mean contributes only the FP64
// rounding of that sum (the products of exact FP64 u, v and FP64 twiddles are
// accumulated in FP64). MBG blocks of 16 frequencies are accumulated per pass
// over the series. The loads run D step groups ahead of the products, along
// the wave's whole walk (tiles, passes, groups; the group count padded to a
// multiple of D with empty groups), so they cross pass and tile boundaries
// and about D groups of loads are in flight per wave. Per block of the grid (one wave) the FP64 sum
// and sum of squares of its pixels' eta go to part[2 b], part[2 b + 1].
template <int MBG, bool VEC, int D, bool RING, bool SHORT>
__device__ __forceinline__ void eta_px_body(const float* q, int np, int64_t plane, int harm, const double2* twg,
                                            float* eta_f, double* part, const CallDev* cd, int n_ring,
                                            int ring_first, int ring_cap) {
  extern __shared__ double2 lds_tw[];         // [np] twiddles, then [K][64] float magnitudes (harmonic sums)
  float* ak = (float*)(lds_tw + np);
  const int lane = threadIdx.x;
  const int n = lane & 15, kk = lane >> 4;
  const int K = np / 2;
  const int L = np / 2;                // last folded step
  const int nmb = (K + 15) / 16;
  const int T = (L + 4) / 4;           // step groups covering s = 0 .. L
  for (int i = lane; i < np; i += 64) lds_tw[i] = twg[i];
  __syncthreads();
  // series step s: the newest n_ring of the field's kept maps (held from slot
  // px_start, oldest first; serving), then the call's. px_start < ring_cap and
  // ring_first + n_ring <= ring_cap, so one wrap suffices. Branch-free: the
  // loop below keeps its accumulators in place only without branches.
  const int rbase = n_ring > 0 ? cd->px_start + ring_first : 0;
  const float* ring = n_ring > 0 ? cd->px_ring : q;
  auto row_of = [&](int s) -> const float* {
    const bool in_ring = s < n_ring;
    int v = rbase + s;
    v = v >= ring_cap ? v - ring_cap : v;
    return (in_ring ? ring : q) + (int64_t)(in_ring ? v : s - n_ring) * plane;
  };
  // raw values of step group t for this lane: x_s and its partner x_(n'-s).
  // Every load reads a valid step and pixel (clamped); values of pixels past
  // the plane are never stored. Steps without a value or a partner are zeroed
  // where the values are used, not here: a select on a load's result would
  // make the wave wait for that load at once and undo the prefetch.
  // 32-bit wave-uniform tile and plane arithmetic (plane < 2^32, so tiles
  // < 2^26): 64-bit compares and multiplies would run on the vector ALU
  const int ntile = (int)((plane + 63) / 64);
  const uint32_t plane32 = (uint32_t)plane;
  const int gsz = gridDim.x;
  auto fetch = [&](int t, int tile, float4& xs, float4& xp) {
    const uint32_t tc = (uint32_t)(tile < ntile ? tile : ntile - 1);
    const int64_t p0 = (int64_t)tc * 64;
    const int s = 4 * t + kk;
    // rows read: x_s and x_(n'-s); a step without a partner reads its own
    // row twice (u = 2 x_s, v = 0 exactly; its weight is halved where the
    // values are used), a step past the series any valid row (weight zero)
    const int s1 = min(s, np - 1);
    const int s2 = (s > 0 && 2 * s < np) ? np - s : s1;
    // global address space: generic (flat) loads would also count against
    // the LDS counter, so every wait for a twiddle read would wait for all
    // prefetched rows
    const fitrig_gf* g1;
    const fitrig_gf* g2;
    if constexpr (RING) {
      g1 = (const fitrig_gf*)(row_of(s1) + p0);
      g2 = (const fitrig_gf*)(row_of(s2) + p0);
    } else {
      // one 32 x 32 -> 64-bit multiply-add per row
      const fitrig_gf* base = (const fitrig_gf*)q + p0;
      g1 = base + (uint64_t)(uint32_t)s1 * plane32;
      g2 = base + (uint64_t)(uint32_t)s2 * plane32;
    }
    const uint32_t rem = plane32 - tc * 64u;  // pixels from p0 to the end of the plane (>= 1)
    if (VEC) {
      // plane % 4 == 0: a 16-byte group of pixels is wholly inside or outside
      const int o = min(4 * n, (int)min(rem - 4u, 60u));
      // read once: non-temporal
      const fitrig_v4f av = __builtin_nontemporal_load((const fitrig_gv4f*)(g1 + o));
      const fitrig_v4f bv = __builtin_nontemporal_load((const fitrig_gv4f*)(g2 + o));
      xs = make_float4(av.x, av.y, av.z, av.w);
      xp = make_float4(bv.x, bv.y, bv.z, bv.w);
    } else {
      const int lim = (int)min(rem - 1u, 63u);
      int o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = min(4 * n + j, lim);
      xs = make_float4(g1[o[0]], g1[o[1]], g1[o[2]], g1[o[3]]);
      xp = make_float4(g2[o[0]], g2[o[1]], g2[o[2]], g2[o[3]]);
    }
  };
  // Short series (SHORT: one pass of at most 16 frequencies, one round of D
  // step groups, no ring): a lane's weights are the same for every tile, so
  // they are set once (no twiddle read, index update or weight factor per
  // step group).
  double wcs[D], wss[D];
  if constexpr (SHORT) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int s = 4 * d + kk;
      const double2 w = lds_tw[(int)(((int64_t)(n + 1) * s) % np)];
      const double sc = s > L ? 0.0 : (s > 0 && 2 * s < np) ? 1.0 : 0.5;
      // rows of frequencies above K get zero weights: their magnitudes are 0
      const bool fv = n + 1 <= K;
      wcs[d] = fv ? w.x * sc : 0.0;
      wss[d] = fv ? w.y : 0.0;
    }
  }
  const int Tp = (T + D - 1) / D * D;
  // prefetch cursor (wave-uniform): tile, pass (first block), group
  int ftile = blockIdx.x;
  int fg = 0, fs = 0;
  // branch-free (selects): branches would split the unrolled loop body and
  // make the compiler copy the prefetch slots at the back edge
  auto advance = [&]() {
    const bool w1 = fs + 1 == Tp;
    fs = w1 ? 0 : fs + 1;
    const int g1 = fg + (w1 ? MBG : 0);
    const bool w2 = g1 >= nmb;
    fg = w2 ? 0 : g1;
    ftile += w2 ? gsz : 0;
  };
  float4 bs[D], bp[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    fetch(fs, ftile, bs[d], bp[d]);
    advance();
  }
  double s1 = 0.0, s2 = 0.0;
  for (int tile = blockIdx.x; tile < ntile; tile += gsz) {
    const int64_t p0 = (int64_t)tile * 64;
    double best[4] = {0.0, 0.0, 0.0, 0.0};  // max over k of |X_k|^2 (pixel p0 + 4 n + j)
    for (int g = 0; g < nmb; g += MBG) {
      fitrig_v4d ac[MBG][4], as[MBG][4];  // written by the pass's first step group
      int idx[MBG], stp[MBG];
#pragma unroll
      for (int m = 0; m < MBG; ++m) {
        const int f = 16 * (g + m) + n + 1;  // frequency of this lane's A row
        idx[m] = (int)(((int64_t)f * kk) % np);
        stp[m] = (int)(((int64_t)f * 4) % np);
      }
      // one step group (slot DC of the group t .. t + D - 1); the first group
      // of a pass starts its products from a zero accumulator instead of
      // clearing 64 registers per tile
      auto group = [&](auto FIRSTC, auto DC, int t) {
        constexpr bool FIRST = decltype(FIRSTC)::value;
        constexpr int d = decltype(DC)::value;
        const int s = 4 * (t + d) + kk;
        // cosine weight factor: 1 for a pair, 1/2 for x_0 and x_(n'/2) (read
        // twice, u = 2 x_s), 0 past the series; the sine rows see v = 0
        // wherever there is no pair. Rows of frequencies above K are never read.
        const double sc = s > L ? 0.0 : (s > 0 && 2 * s < np) ? 1.0 : 0.5;
        const float4 cs = bs[d], cp = bp[d];
        double u[4] = {(double)cs.x + (double)cp.x, (double)cs.y + (double)cp.y, (double)cs.z + (double)cp.z,
                       (double)cs.w + (double)cp.w};
        double v[4] = {(double)cs.x - (double)cp.x, (double)cs.y - (double)cp.y, (double)cs.z - (double)cp.z,
                       (double)cs.w - (double)cp.w};
        // the slot is free: the group D ahead goes into it. u and v are
        // materialised first and the load cannot move above the empty asm,
        // so the new value can take the old one's registers (otherwise the
        // back edge copies them, and a copy waits for its load)
        asm volatile("" : "+v"(u[0]), "+v"(u[1]), "+v"(u[2]), "+v"(u[3]), "+v"(v[0]), "+v"(v[1]), "+v"(v[2]),
                     "+v"(v[3])
                     :
                     : "memory");
        fetch(fs, ftile, bs[d], bp[d]);
        advance();
#pragma unroll
        for (int m = 0; m < MBG; ++m) {
          double wc, ws;
          if constexpr (SHORT) {
            wc = wcs[d];
            ws = wss[d];
          } else {
            const double2 w = lds_tw[idx[m]];
            wc = w.x * sc;
            ws = w.y;
            idx[m] += stp[m];
            if (idx[m] >= np) idx[m] -= np;
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if constexpr (FIRST) {
              const fitrig_v4d zero = {0.0, 0.0, 0.0, 0.0};
              ac[m][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc, u[j], zero, 0, 0, 0);
              as[m][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ws, v[j], zero, 0, 0, 0);
            } else {
              ac[m][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc, u[j], ac[m][j], 0, 0, 0);
              as[m][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ws, v[j], as[m][j], 0, 0, 0);
            }
          }
        }
      };
      fitrig_static_for<0, D>([&](auto DC) { group(std::integral_constant<bool, DC.value == 0>{}, DC, 0); });
      if constexpr (!SHORT)
        for (int t = D; t < Tp; t += D) fitrig_static_for<0, D>([&](auto DC) { group(std::false_type{}, DC, t); });
      // register r: Re / Im of frequency 16 (g + m) + 4 r + kk + 1 (the test
      // of harm is uniform and taken once, not per element)
      if (harm == 0) {
        // per pixel: the maximum over this pass's rows first (values of
        // arithmetic, no canonicalisation), then one maximum with best
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double mj = 0.0;
#pragma unroll
          for (int m = 0; m < MBG; ++m) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int f = 16 * (g + m) + 4 * r + kk + 1;
              double a2 = fma(ac[m][j][r], ac[m][j][r], as[m][j][r] * as[m][j][r]);
              if constexpr (!SHORT) a2 = f > K ? 0.0 : a2;  // SHORT: those rows are 0
              mj = (m == 0 && r == 0) ? a2 : fmax(mj, a2);
            }
          }
          best[j] = fmax(best[j], mj);
        }
      } else {
#pragma unroll
        for (int m = 0; m < MBG; ++m) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int f = 16 * (g + m) + 4 * r + kk + 1;
            if (f > K) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              ak[(f - 1) * 64 + 4 * n + j] =
                  (float)sqrt(fma(ac[m][j][r], ac[m][j][r], as[m][j][r] * as[m][j][r]));
          }
        }
      }
    }
    if (harm == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        best[j] = fmax(best[j], __shfl_xor(best[j], 16));
        best[j] = fmax(best[j], __shfl_xor(best[j], 32));
      }
      // lane n + 16 kk finishes pixel p0 + 4 n + kk (one square root per lane)
      const double bj = kk == 0 ? best[0] : kk == 1 ? best[1] : kk == 2 ? best[2] : best[3];
      const int64_t p = p0 + 4 * n + kk;
      if (p < plane) {
        const double e = sqrt(bj);
        eta_f[p] = (float)e;
        s1 += e;
        s2 = fma(e, e, s2);
      }
    } else {
      __syncthreads();
      const int64_t p = p0 + lane;
      double bv = 0.0;
      for (int k = 1; k <= K; ++k) {
        double val = 0.0;
        for (int j = 1; j <= harm && j * k <= K; ++j) val += (double)ak[(j * k - 1) * 64 + lane];
        if (k == 1 || val > bv) bv = val;
      }
      if (p < plane) {
        eta_f[p] = (float)bv;
        s1 += bv;
        s2 = fma(bv, bv, s2);
      }
      __syncthreads();
    }
  }
  // fixed-order wave sums
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  if (lane == 0) {
    part[2 * (int64_t)blockIdx.x] = s1;
    part[2 * (int64_t)blockIdx.x + 1] = s2;
  }
}

template <int MBG, bool VEC, int D, bool RING>
__global__ __launch_bounds__(64) void k_eta_px(const float* q, int np, int64_t plane, int harm, const double2* twg,
                                               float* eta_f, double* part, const CallDev* cd, int n_ring,
                                               int ring_first, int ring_cap) {
  eta_px_body<MBG, VEC, D, RING, false>(q, np, plane, harm, twg, eta_f, part, cd, n_ring, ring_first, ring_cap);
}

// Short series (one pass of at most 16 frequencies, one round of step groups,
// no field ring): weights set once per wave.
template <bool VEC, int D>
__global__ __launch_bounds__(64) void k_eta_px_short(
    const float* q, int np, int64_t plane, int harm, const double2* twg, float* eta_f, double* part) {
  eta_px_body<1, VEC, D, false, true>(q, np, plane, harm, twg, eta_f, part, nullptr, 0, 0, 1);
}

// ---------------------------------------------------------------------------
// Call record, result delivery, small fills and copies.
// ---------------------------------------------------------------------------
__global__ void k_set_call(CallDev* d, CallDev v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *d = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// counters[CNT_TRUNC] |= overflow of this run; per-branch count; output base.
__global__ void k_run_done(int64_t* c, int64_t seg_cap, int64_t blk_cap, int64_t comp_cap, int branch) {
  if (threadIdx.x || blockIdx.x) return;
  if (c[CNT_NSEL] > seg_cap || c[CNT_NBLK] > blk_cap || c[CNT_NCOMP] > comp_cap) c[CNT_TRUNC] |= 1;
  const int64_t nc = c[CNT_NCOMP] < comp_cap ? c[CNT_NCOMP] : comp_cap;
  c[branch == FITRIG_IMAGE ? CNT_IMG : branch == FITRIG_FREQ ? CNT_FREQ : CNT_FPX] += nc;
  c[CNT_OUTBASE] += nc;
}

// Frequency series over [history | this call] (serving): slices
// n_in - from_hist .. n_in - 1 of the history, then the call's last
// from_call slices of the cube, into fs; afterwards (k_hist_out) fs becomes
// the field's history.
__global__ void k_hist_in(const CallDev* cd, int64_t hist_off, int64_t n_hist, const double* cube, int64_t cube_off,
                          int64_t n_call, double* fs) {
  const double* h = cd->hist_in;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_hist + n_call;
       i += (int64_t)gridDim.x * blockDim.x)
    fs[i] = i < n_hist ? h[hist_off + i] : cube[cube_off + (i - n_hist)];
}
// The call's last n maps appended to the field's ring of per-pixel q maps
// (slots after the n_held maps kept from slot px_start).
__global__ void k_px_ring_append(const CallDev* cd, const float* q, int64_t plane, int n, int n_held, int cap) {
  const int64_t tot = (int64_t)n * plane;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i / plane);
    const int64_t p = i - (int64_t)j * plane;
    const int slot = (cd->px_start + n_held + j) % cap;
    cd->px_ring[(int64_t)slot * plane + p] = q[i];
  }
}

__global__ void k_hist_out(const CallDev* cd, const double* fs, int64_t n) {
  double* h = cd->hist_out;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    h[i] = fs[i];
}

// Results of a call into host-visible memory: counters, M, the frequency
// statistics, per-triple mu / sigma / flags and min(total, cap) candidates
// (layout in ResultLayout). Only the records that exist cross the bus.
// cand_dst (nullable): the caller's page-locked candidate array (its device
// address), written directly instead of the staging copy
__global__ void k_pack_results(const int64_t* cnt, const double* M, const double* eta_st, const double* mu,
                               const double* sigma, const uint32_t* flags, int np, const fitrig_candidate* cand,
                               int64_t cap, ResultLayout R, char* dst, fitrig_candidate* cand_dst) {
  int64_t ncand = cnt[CNT_OUTBASE];
  if (ncand > cap) ncand = cap;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
  int64_t* hc = (int64_t*)(dst + R.off_cnt);
  for (int64_t i = tid; i < CNT_N; i += nth) hc[i] = cnt[i];
  uint64_t* hd = (uint64_t*)(dst + R.off_scalars);
  if (tid == 0) {
    hd[0] = __double_as_longlong(M[0]);
    for (int i = 0; i < ES_N; ++i) hd[1 + i] = ((const uint64_t*)eta_st)[i];
  }
  double* hmu = (double*)(dst + R.off_mu);
  double* hsg = (double*)(dst + R.off_sigma);
  uint32_t* hfl = (uint32_t*)(dst + R.off_flags);
  for (int64_t i = tid; i < np; i += nth) {
    hmu[i] = mu[i];
    hsg[i] = sigma[i];
    hfl[i] = flags[i];
  }
  const uint64_t* src = (const uint64_t*)cand;
  uint64_t* out = cand_dst ? (uint64_t*)cand_dst : (uint64_t*)(dst + R.off_cand);
  const int64_t words = ncand * (int64_t)(sizeof(fitrig_candidate) / 8);
  for (int64_t i = tid; i < words; i += nth) out[i] = src[i];
}


}  // namespace fitrig
