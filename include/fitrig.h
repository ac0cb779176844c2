/*
 * fitrig.h - C ABI of the MI355X (gfx950) FITrig trigger library.
 *
 * The library computes, for a stack of fast-imaging snapshots, the
 * transient-oriented index tLISI of Li, Adamek & Armour ("FITrig",
 * arXiv 2509.21754), per pixel (sliding window) or per tile, then the
 * per-triple spread, the N-sigma selection, 8-connected candidate
 * components and the image-frequency branch:
 *
 *   triple s (0-based) = snapshots s, s+1, s+2; reference = snapshot s+1;
 *   D(s) = |x(s+1) - x(s)|, Delta = |D(s) - D(s+1)|          Sec. 2.2.4, Eq. (3)
 *   x_hat = x(s+1), or C where x(s+1) == 0                  Eq. (5)
 *   r = min(Delta / |x_hat|, 1)                             Eq. (4)
 *   tLISI = 1 - mean(Delta) max(Delta) mean(r) / M^2,
 *   M = max(max over the stack, C)                          Eq. (2), Eq. (6)
 *   z = (mu - tLISI) / sigma per triple; select z > tau     Sec. 2.4.1, Eqs. (8)-(9)
 *   eta = h(|F_s[q(s) - mean q]|) per tile, z on eta        Sec. 2.4.2, Eqs. (10)-(12)
 *
 * The index map holds q = mean(Delta) max(Delta) mean(r) (tLISI = 1 - q/M^2);
 * the z-score of Eq. (8) is computed on q, which is the same number.
 *
 * All device pointers are HIP device memory of the device named in the
 * config. Every call returns a fitrig_status (0 = OK, < 0 = error).
 * Threading: a context is not thread-safe; use one per host thread.
 * Determinism: results depend only on the inputs and the config, and are
 * bitwise reproducible on the same GPU and build.
 */
#ifndef FITRIG_H
#define FITRIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FITRIG_ABI_VERSION 4

typedef int32_t fitrig_status;
#define FITRIG_OK 0
#define FITRIG_E_INVAL (-1)   /* bad argument: see each call */
#define FITRIG_E_NOMEM (-2)   /* a device or host allocation failed */
#define FITRIG_E_HIP (-3)     /* a HIP call failed; fitrig_last_hip_error gives the code */
#define FITRIG_E_TRUNC (-4)   /* more results than the given or internal capacity */
#define FITRIG_E_BUSY (-5)    /* serving: admission refused on a non-blocking submit */
#define FITRIG_E_NOTREADY (-6)/* serving: result not ready on a non-blocking poll */
#define FITRIG_E_SCRATCH (-7) /* fitrig_detect_noalloc: the call needs more than FITRIG_NOALLOC_SCRATCH_BYTES */

typedef enum { FITRIG_F32 = 0, FITRIG_F16 = 1, FITRIG_BF16 = 2 } fitrig_dtype;

/* index mode */
#define FITRIG_SLIDING 0      /* odd window x window centred on every pixel, clipped at the edge */
#define FITRIG_TILES 1        /* non-overlapping tile x tile tiles, row-major (Sec. 2.2.1, Alg. 1) */
/* branches (bitmask) */
#define FITRIG_IMAGE 1        /* image-domain selection, Sec. 2.4.1 */
#define FITRIG_FREQ 2         /* image-frequency selection, Sec. 2.4.2 (needs n_snap - 2 >= 4) */
#define FITRIG_FREQ_PIXEL 4   /* the same transform and selection per cell of the sliding index maps
                                 (sliding mode only; needs n_snap - 2 >= 4; n_snap - 2 <= 4096,
                                 or <= 448 with a harmonic sum) */
/* spread estimator */
#define FITRIG_MEAN_STD 0     /* mean and population std (Eq. (8)) */
#define FITRIG_MEDIAN_MAD 1   /* median and 1.482602218505602 * MAD */
/* what the optional index map holds */
#define FITRIG_MAP_QTILDE 0   /* q = mean(Delta) max(Delta) mean(r) */
#define FITRIG_MAP_TLISI 1    /* 1 - q / M^2 (one extra pass over the map) */
/* per-triple flags */
#define FITRIG_FLAG_SIGMA_ZERO 1u  /* zero or non-finite spread: no selection */
#define FITRIG_FLAG_TRUNC 2u       /* internal selection capacity exceeded */

typedef struct {
  int32_t abi_version;  /* must be FITRIG_ABI_VERSION */
  int32_t mode;         /* FITRIG_SLIDING (default) or FITRIG_TILES */
  int32_t window;       /* sliding window, odd, 1..17 (default 7) */
  int32_t tile;         /* tile size for FITRIG_TILES and for the frequency branch (default 32) */
  int32_t branches;     /* FITRIG_IMAGE | FITRIG_FREQ | FITRIG_FREQ_PIXEL (default IMAGE | FREQ) */
  int32_t sigma_est;    /* FITRIG_MEAN_STD (default) or FITRIG_MEDIAN_MAD */
  int32_t harm;         /* 0: eta = max magnitude (default); h >= 2: harmonic sum of h terms */
  int32_t r_signed;     /* 0: divide by |x_hat| (default); 1: by the signed x_hat (literal Eq. (4)) */
  int32_t map_kind;     /* FITRIG_MAP_QTILDE (default) or FITRIG_MAP_TLISI */
  int32_t device;       /* HIP device ordinal (default 0) */
  double C;             /* the constant of Eqs. (2), (5); > 0 (default 1e-6) */
  int64_t max_pixels;   /* capacity hint H*W used to size scratch at create (0 = grow on demand) */
  int32_t max_snap;     /* capacity hint n_snap (0 = grow on demand) */
  int32_t profile;      /* 1: time each phase of fitrig_detect with HIP events (see fitrig_phase_times) */
  int64_t max_segments; /* selection capacity in 64-cell row segments (0 = automatic) */
} fitrig_config;

/* One candidate: an 8-connected component of selected cells. */
typedef struct {
  int32_t branch;       /* FITRIG_IMAGE, FITRIG_FREQ or FITRIG_FREQ_PIXEL (in that order) */
  int32_t triple;       /* first snapshot s of the triple; -1 for the frequency branches */
  int64_t label;        /* lowest row-major cell index y * width + x of the component */
  int32_t n_pix;        /* cells in the component (pixels, or tiles for tile mode / FREQ) */
  int32_t peak_y, peak_x; /* cell of the largest z (ties: lowest index) */
  float peak_z;         /* z at the peak */
  float peak_q;         /* q (or eta) at the peak */
  int32_t pad0;
  double cy, cx;        /* z-weighted centroid in cell units */
  int32_t y0, x0, y1, x1; /* inclusive bounding box */
} fitrig_candidate;

/* Optional per-call statistics (host memory owned by the caller). */
typedef struct {
  double M;             /* max(max over the stack, C) */
  int32_t n_triples;    /* out: n_snap - 2 */
  int32_t status;       /* out: the call's result, FITRIG_OK or FITRIG_E_TRUNC (for an
                           asynchronous call this is where truncation shows) */
  double* mu;           /* in: array of >= n_snap - 2, out: per-triple location of q (nullable) */
  double* sigma;        /* in: array of >= n_snap - 2, out: per-triple spread of q (nullable) */
  uint32_t* flags;      /* in: array of >= n_snap - 2, out: FITRIG_FLAG_* (nullable) */
  double eta_mu;        /* tile frequency branch: location of eta (0 if not run) */
  double eta_sigma;     /* tile frequency branch: spread of eta (0 if not run) */
  int64_t n_image_cand; /* candidates from the image branch */
  int64_t n_freq_cand;  /* candidates from the tile frequency branch */
  int64_t n_freq_px_cand; /* candidates from the per-pixel frequency branch */
  double eta_px_mu;     /* per-pixel frequency branch: location of eta (0 if not run) */
  double eta_px_sigma;  /* per-pixel frequency branch: spread of eta (0 if not run) */
  uint32_t ran;         /* out: the branches that ran (FITRIG_IMAGE | FITRIG_FREQ | FITRIG_FREQ_PIXEL);
                           a requested frequency branch does not run when n_snap - 2 < 4 */
  uint32_t eta_flags;   /* out: FITRIG_FLAG_SIGMA_ZERO of the tile branch (bit 0) and of the
                           per-pixel branch (bit 8) */
} fitrig_stats;

typedef struct fitrig_ctx fitrig_ctx;

/* Fills cfg with the defaults listed above. */
void fitrig_config_default(fitrig_config* cfg);

/*
 * Creates a context on cfg->device: a HIP stream and a scratch arena sized
 * from the capacity hints. The context owns both.
 * Errors: E_INVAL (null pointer, ABI mismatch, bad mode/window/tile/branches/
 * sigma_est/harm, C <= 0, bad device), E_NOMEM, E_HIP.
 */
fitrig_status fitrig_create(const fitrig_config* cfg, fitrig_ctx** out);

/*
 * Runs the whole path on one stack.
 *   stack      device, [n_snap][H][W] row-major, dtype as given, read only
 *   n_snap     >= 3 (the frequency branches run only when n_snap - 2 >= 4)
 *   H, W       >= 1, H * W < 2^32, W * (bytes per pixel) * 33 < 2^30 for every
 *              window (a workgroup's rows are addressed within 2^30 bytes of its
 *              first row: W <= 8134407 in FP32, 16268815 in FP16/BF16)
 *   sigma      the threshold tau of Eqs. (9), (12); finite and > 0
 *   cand       host, cand_cap records (nullable when cand_cap == 0); when it
 *              is page-locked memory mapped for the device (hipHostMalloc)
 *              and the stream is not being captured, the device writes the
 *              records there directly, otherwise they are copied from the
 *              library's staging memory
 *   n_cand     host, out: total number of candidates (always written)
 *   index_map  device, nullable: [n_snap-2][H][W] floats (sliding) or
 *              [n_snap-2][ceil(H/tile)][ceil(W/tile)] (tiles); written
 *              whenever given, whichever branches run
 *   eta_map    device, nullable: [ceil(H/tile)][ceil(W/tile)] floats (tile
 *              frequency branch)
 *   eta_px_map device, nullable: [H][W] floats, the per-pixel spectrum
 *              eta of every cell (FITRIG_FREQ_PIXEL)
 *   stats      host, nullable
 *   hip_stream NULL: the call runs on the context's stream (a blocking
 *              stream: it starts after work queued earlier on the legacy
 *              default stream, where the stack may have been written) and
 *              returns when every output is written.
 *              Non-NULL, a hipStream_t: the call is asynchronous. It
 *              enqueues the whole path on that stream and returns; the
 *              device maps, cand, *n_cand and *stats (and the arrays stats
 *              points to) are written when the stream reaches the end of
 *              the call (the host outputs by a host function the call
 *              enqueues), so the caller keeps them alive and reads them
 *              after synchronising the stream. Such a call may be captured
 *              into a HIP graph; every replay rewrites the same outputs.
 * Candidates come in canonical order: image branch by (triple, label), then
 * the tile frequency branch by label, then the per-pixel frequency branch by
 * label. Scratch is sized from the capacity hints at create; a call that
 * needs more grows it before enqueueing anything (a device-wide
 * synchronisation), except on a capturing stream, where it returns E_INVAL
 * instead. With adequate hints a call allocates nothing. Calls on one
 * context must be ordered: one stream per context, or the caller orders them.
 * Returns (synchronous call): OK, or E_TRUNC (more candidates than cand_cap:
 * the first cand_cap are written and *n_cand holds the total; or the
 * internal selection capacity was exceeded, flagged FITRIG_FLAG_TRUNC).
 * An asynchronous call returns OK once enqueued; the result status then
 * appears in stats->status (and *n_cand > cand_cap shows truncation).
 * Errors: E_INVAL (argument outside the ranges above, unknown dtype, a
 * per-pixel series longer than the FITRIG_FREQ_PIXEL limits, scratch growth
 * while capturing), E_NOMEM, E_HIP.
 */
fitrig_status fitrig_detect(fitrig_ctx* ctx, const void* stack, fitrig_dtype dtype,
                            int32_t n_snap, int32_t H, int32_t W, double sigma,
                            fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                            float* index_map, float* eta_map, float* eta_px_map,
                            fitrig_stats* stats, void* hip_stream);

/*
 * Allocation-free variant of fitrig_detect, for callers that cannot allocate
 * device memory during a call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). It runs the same kernels on the
 * same arguments and writes the same outputs as fitrig_detect, but its
 * scratch, including the packed device results, is carved from one static
 * device array of FITRIG_NOALLOC_SCRATCH_BYTES per GPU that the library
 * holds until the process ends (its address on ctx's device is taken once,
 * at fitrig_create). The call allocates nothing: no hipMalloc, hipFree or
 * pinned host memory, and none of the context's own buffers are used or
 * grown.
 *   Arguments as fitrig_detect. The call is always synchronous: it runs on
 *   hip_stream (NULL = the context's stream) and returns when every output
 *   is written (host outputs are copied from the device results).
 *   Limit: everything one call needs beyond its inputs and outputs must fit
 *   in FITRIG_NOALLOC_SCRATCH_BYTES (the default selection capacity alone
 *   takes about 90 MB; the median/MAD spread and per-pixel spectra also
 *   need an [n_snap-2][H][W] float map unless index_map is given). A larger
 *   call returns E_SCRATCH and enqueues nothing.
 *   Sharing: every call on a GPU uses that GPU's one array, which keeps the
 *   last call's contents; each call clears what it needs zeroed. Calls that
 *   overlap on one GPU would race on the array, so the library serialises
 *   them per device with a lock held for the whole call.
 * Returns OK or E_TRUNC as fitrig_detect. Errors: E_INVAL (as fitrig_detect),
 * E_SCRATCH, E_HIP (including a failed lookup of the array's address).
 */
#define FITRIG_NOALLOC_SCRATCH_BYTES (256ull << 20)
fitrig_status fitrig_detect_noalloc(fitrig_ctx* ctx, const void* stack, fitrig_dtype dtype,
                                    int32_t n_snap, int32_t H, int32_t W, double sigma,
                                    fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                                    float* index_map, float* eta_map, float* eta_px_map,
                                    fitrig_stats* stats, void* hip_stream);

/*
 * Stacks in host memory, streamed to the device in chunks of frames. The
 * paper's real-time design moves each snapshot over PCIe while the trigger
 * kernel works on the previous one (Sec. 3.2); here the copy of chunk i + 1
 * runs on a stream of its own while the whole path runs over chunk i. A
 * chunk carries the two frames before it (its first two triples reach back
 * into the previous chunk) and extends a device copy of the tile cube of
 * every triple so far, so the frequency branch runs once, on the last chunk,
 * over the whole series. Every result equals fitrig_detect's on the same
 * stack in device memory, bit for bit.
 *   host_stack   host, [n_snap][H][W] row-major, dtype as given. Page-locked
 *                memory (hipHostMalloc, a pinned torch tensor) is copied
 *                directly; pageable memory is copied by host threads into two
 *                page-locked staging buffers of chunk_frames frames ahead of
 *                the device (for stacks that cannot be page-locked whole). In
 *                both cases the copies overlap the kernels. A device pointer
 *                is E_INVAL.
 *   chunk_frames frames per copy (>= 1; the first chunk holds at least 3)
 *   cand, cand_cap, n_cand, eta_map (device, nullable), stats: as
 *                fitrig_detect (no index maps: they would not fit the point
 *                of streaming)
 * The call allocates (and frees) 3 chunk buffers (4 when chunk_frames = 1),
 * for pageable input the 2 staging buffers and one filler thread, and, for
 * the frequency branch, an (n_snap-2) * ceil(H/tile) * ceil(W/tile) FP64
 * history; it is synchronous on the context's stream.
 * Errors: E_INVAL (as fitrig_detect, chunk_frames < 1, FITRIG_FREQ_PIXEL in
 * the config), E_NOMEM, E_HIP.
 */
fitrig_status fitrig_detect_host(fitrig_ctx* ctx, const void* host_stack, fitrig_dtype dtype, int32_t n_snap,
                                 int32_t H, int32_t W, double sigma, int32_t chunk_frames,
                                 fitrig_candidate* cand, int64_t cand_cap, int64_t* n_cand,
                                 float* eta_map, fitrig_stats* stats);

/* Releases the context and its device memory. Errors: E_INVAL (null). */
fitrig_status fitrig_destroy(fitrig_ctx* ctx);

/* Text of a status code (static storage). */
const char* fitrig_status_string(fitrig_status s);

/* The last HIP error code seen by the context (0 = none). */
int32_t fitrig_last_hip_error(const fitrig_ctx* ctx);

/*
 * Phase durations of the last fitrig_detect on ctx, in milliseconds, measured
 * with HIP events recorded on the call's stream (config profile = 1; not
 * recorded while the stream is capturing):
 *   [0] pass over the stack (streaming index kernel or tile kernel)
 *   [1] per-triple spread
 *   [2] image-branch selection and components
 *   [3] frequency branch
 *   [4] result copies to the host
 * Writes min(cap, FITRIG_N_PHASES) values; returns the number written, or
 * 0 when profiling is off or the last call has not completed, -1 on a null
 * pointer.
 */
#define FITRIG_N_PHASES 5
int32_t fitrig_phase_times(const fitrig_ctx* ctx, double* ms, int32_t cap);

/* Library ABI version (FITRIG_ABI_VERSION of the build). */
int32_t fitrig_abi_version(void);

/* ---- sub-cell localisation ---------------------------------------------------
 * The paper localises a source inside the selected tiles by interpolating the
 * tile values (the spectrum matrix eta) with a bilinear, spline, bicubic or
 * Makima cubic interpolant and taking the interpolated maximum (Sec. 2.4.2;
 * Sec. 3.1 uses a spline on eta). For each peak cell (py[i], px[i]) of a value
 * map (eta_map from fitrig_detect, or an index map), the 5 x 5 cells around
 * it (indices clamped into the map, so edge values repeat) are interpolated
 * along x for each row and then along y, the surface is evaluated at
 * (py + a / sub, px + b / sub) for a, b = -sub .. sub, and the grid point of
 * the largest value is returned (ties: smallest a, then smallest b).
 * Methods, on unit-spaced nodes:
 *   BILINEAR  straight lines between nodes;
 *   BICUBIC   cubic convolution with Keys' kernel, a = -1/2;
 *   SPLINE    cubic spline through the 5 nodes, not-a-knot end conditions;
 *   MAKIMA    modified Akima piecewise cubic (end slopes extended linearly).
 * map: device FP32 [H][W] row-major (read only). py, px: host int32 [n].
 * out: host double [3 n]: y, x, interpolated value per peak. hip_stream:
 * hipStream_t (NULL = legacy default stream) on the current device; the call
 * returns when out is written. Arithmetic in FP64.
 * Errors: E_INVAL (n < 0, H or W < 1, sub outside 1..64, unknown method, null
 * pointers with n > 0, a peak outside the map), E_NOMEM, E_HIP. n = 0 does
 * nothing. */
#define FITRIG_INTERP_BILINEAR 0
#define FITRIG_INTERP_BICUBIC 1
#define FITRIG_INTERP_SPLINE 2
#define FITRIG_INTERP_MAKIMA 3
fitrig_status fitrig_interp_peaks(const float* map, int32_t H, int32_t W, const int32_t* py, const int32_t* px,
                                  int32_t n, int32_t method, int32_t sub, double* out, void* hip_stream);

/* ---- window sums from full-image prefix sums (comparison variant) ----------
 * The index maps of fitrig_detect's sliding mode with the window sums of
 * Delta and r (Sec. 2.3, Eq. (6)) read from integral images instead of
 * summed directly: S = I(y2+1, x2+1) - I(y1, x2+1) - I(y2+1, x1) + I(y1, x1)
 * over the clipped window, I(y, x) = sum over y' < y, x' < x. The integral
 * image grows with the image (about H W mean), so its four-corner difference
 * needs FP64 beyond a few thousand pixels on a side (prefix_bits = 64); FP32
 * (prefix_bits = 32) shows the loss. fitrig_detect never uses this path: its
 * direct sums of at most 17 terms have no such growth. The window maximum is
 * exact (separable); q = (S_Delta / n) max (S_r / n) in the prefix precision.
 *   index_map  device float [n_snap-2][H][W] (q, as fitrig_detect's)
 *   window, r_signed, C: as fitrig_config
 * Runs on hip_stream (NULL: the legacy default stream) and returns when the
 * map is written; allocates 2 (H+1)(W+1) prefix values and 3 H W floats for
 * the call. Errors: E_INVAL (null pointers, sizes as fitrig_detect, even or
 * non-positive window, prefix_bits not 32 or 64, r_signed not 0 or 1,
 * C <= 0), E_NOMEM, E_HIP. */
fitrig_status fitrig_index_prefix(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H, int32_t W,
                                  int32_t window, int32_t prefix_bits, int32_t r_signed, double C,
                                  float* index_map, void* hip_stream);

/* ---- snapshot accumulation -------------------------------------------------
 * For very short sampling periods adjacent snapshots are nearly the same and
 * their differences nearly blank; the paper then applies the method to sums
 * of adjacent snapshots, combined until adjacent sums differ enough
 * (Sec. 3.3.2, Fig. accum: the combination is a plain sum). The paper gives
 * no criterion; this library uses one factor K for the whole stack (so the
 * accumulated series stays uniformly sampled for the frequency branch):
 *   Y_j  = sum_{k = jK}^{jK+K-1} X_k, j = 0 .. P-1, P = floor(n_snap / K)
 *          (FP32, added in frame order; the last n_snap - PK snapshots are
 *          dropped)
 *   c_j  = sum_p |Y_{j+1}(p) - Y_j(p)| / sum_p |Y_j(p)| over all pixels
 *   C(K) = median of c_0 .. c_{P-2} (mean of the two middle values for an
 *          even count; NaN when P < 2)
 *   automatic K = the smallest K <= k_max with P >= 3 and C(K) >= gamma,
 *          else the largest K <= k_max with P >= 3.
 * The accumulated stack is an FP32 stack for fitrig_detect.
 */

/* out: device float [n_snap / K][H][W]. stack: device, dtype as given.
 * Enqueued on hip_stream (NULL: the legacy default stream); returns once
 * enqueued. Errors: E_INVAL (null pointers, sizes as fitrig_detect, K < 1,
 * K > n_snap, unknown dtype), E_HIP. */
fitrig_status fitrig_accumulate(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H, int32_t W,
                                int32_t K, float* out, void* hip_stream);

/* The automatic factor. K_out: host, the chosen K. contrast: host, nullable,
 * k_max doubles C(1) .. C(k_max). Runs on hip_stream (NULL: the legacy
 * default stream) and returns when the results are written; allocates a
 * small device buffer for the duration of the call. Each C(K) reads the
 * stack about twice.
 * Errors: E_INVAL (null pointers, sizes as fitrig_detect, n_snap outside
 * 3 .. 65536, k_max < 1, gamma negative or not finite, unknown dtype),
 * E_NOMEM, E_HIP. */
fitrig_status fitrig_accum_factor(const void* stack, fitrig_dtype dtype, int32_t n_snap, int32_t H, int32_t W,
                                  double gamma, int32_t k_max, int32_t* K_out, double* contrast,
                                  void* hip_stream);

/* ---- serving form ----------------------------------------------------------
 * A real-time trigger loop: requests are snapshot stacks of a field (a
 * fixed sky position and image size). The server keeps each field's last two
 * snapshots and its running maximum M resident on the device (the paper
 * estimates M from past snapshots in real time, Sec. 2.2.4), so a request's
 * first two triples reach back into the previous request and triples are
 * numbered per field. With freq_window > 0 it also keeps the tile cube of
 * the field's last freq_window triples, and each request's frequency branch
 * (Sec. 2.3) transforms that window of the field's history rather than the
 * request's own triples alone. Requests are admitted while a slot and the memory
 * budget allow; admitted requests of different fields run concurrently on
 * separate streams, requests of one field run in submission order. Each
 * result is identical to running the same frames alone.
 */
typedef struct fitrig_server fitrig_server;

typedef struct {
  fitrig_config base;   /* index / selection settings of every request. With
                           capacity hints (max_pixels > 0, max_snap >= 3) every
                           slot's scratch is sized at create for a square image
                           of max_pixels with max_snap new frames and the
                           longest history, so such requests run without
                           allocating. A slot that meets a larger request grows
                           (waiting for its own stream only) and keeps that
                           scratch. */
  int32_t n_slots;      /* requests on the device at once (default 4) */
  int32_t max_fields;   /* fields with resident state (default 64); a new field
                           beyond it evicts the least recently used idle field */
  int64_t mem_budget;   /* device bytes for slot scratch plus field state; 0 = no limit.
                           Admission bounds the device use: resident field state
                           plus, per slot, the larger of the scratch it holds
                           (sized from the base capacity hints at create, grown
                           to the largest request it ran) and the exact scratch
                           of the largest queued or running request */
  int64_t cand_cap;     /* candidates kept per result (default 65536) */
  int32_t freq_window;  /* 0 (default): a request's frequency branch covers its
                           own triples; 1..2048: it covers the field's last
                           freq_window triples (FP64 tile cube kept per field,
                           freq_window * ceil(H/tile) * ceil(W/tile) * 8 bytes,
                           counted in mem_budget). The branch runs once the
                           covered series has at least 4 triples. The
                           per-pixel branch (FITRIG_FREQ_PIXEL, sliding mode)
                           likewise covers the field's last freq_window
                           triples, from a ring of the field's FP32 index maps
                           (freq_window * H * W * 4 bytes, counted in
                           mem_budget). */
  int32_t graphs;       /* 1 (default): each slot captures its launch sequence
                           into a HIP graph per request shape (frames, size,
                           dtype, carried frames, history length) and replays
                           it; 0: direct launches */
} fitrig_server_config;

typedef struct {
  int64_t ticket;
  int64_t field_id;
  fitrig_status status;     /* status of the run (as fitrig_detect) */
  int32_t n_triples;        /* triples analysed, including those reaching into the previous request */
  int64_t first_triple;     /* field-wide index of the first of them */
  int64_t n_cand;           /* total candidates (records beyond cand_cap are not kept) */
  const fitrig_candidate* cand; /* min(n_cand, cand_cap) records, owned by the server until released */
  double M;                 /* running max(max over every frame of the field so far, C) */
  int64_t t_submit_ns, t_start_ns, t_done_ns; /* steady-clock stamps: submit, launch, results on the host */
  int32_t freq_triples;     /* triples the frequency branch covered: the field's
                               triples first_triple + n_triples - freq_triples ..
                               first_triple + n_triples - 1 (0 = it did not run) */
  int32_t replayed;         /* 1: the request ran as a replay of a captured graph */
} fitrig_result;

/* Fills cfg with the defaults above. */
void fitrig_server_config_default(fitrig_server_config* cfg);

/* Creates the server: one context and stream per slot, worker threads.
 * Errors: E_INVAL (null, bad base config, n_slots < 1, max_fields < 1,
 * cand_cap < 0, mem_budget < 0, freq_window outside 0..2048, graphs not 0 or
 * 1), E_NOMEM (also: the slots' scratch sized from the capacity hints alone
 * exceeds mem_budget), E_HIP. */
fitrig_status fitrig_server_create(const fitrig_server_config* cfg, fitrig_server** out);

/* Submits a stack (device, [n_snap][H][W], must stay valid and unchanged
 * until the request is done; work queued on the legacy default stream before
 * the submit, where the stack may have been written, completes before the
 * request reads it). A field keeps its size and dtype; a request of
 * another size or dtype resets the field's state. blocking = 1 waits for
 * admission; blocking = 0 returns E_BUSY when the request does not fit now.
 * *ticket identifies the request.
 * Errors: E_INVAL (null, n_snap < 1, a field's first request with n_snap < 3,
 * sizes as fitrig_detect, sigma not finite or <= 0, a new size or dtype for a
 * field with requests in flight), E_BUSY (non-blocking and not admitted; the
 * request alone exceeds mem_budget; max_fields fields all have requests in
 * flight), E_NOMEM. */
fitrig_status fitrig_submit(fitrig_server* srv, int64_t field_id, const void* stack, fitrig_dtype dtype,
                            int32_t n_snap, int32_t H, int32_t W, double sigma, int32_t blocking,
                            int64_t* ticket);

/* Result of a ticket. wait = 1 blocks until it is done; wait = 0 returns
 * E_NOTREADY while it runs. Errors: E_INVAL (unknown or released ticket). */
fitrig_status fitrig_poll(fitrig_server* srv, int64_t ticket, int32_t wait, fitrig_result* out);

/* Frees a finished ticket's result memory. Errors: E_INVAL (unknown ticket),
 * E_NOTREADY (still running). */
fitrig_status fitrig_release(fitrig_server* srv, int64_t ticket);

/* Waits for every request, then frees the server. Errors: E_INVAL (null). */
fitrig_status fitrig_server_destroy(fitrig_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* FITRIG_H */
