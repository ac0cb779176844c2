// FITrig serving form: a trigger loop over fields (sky position + image size).
//
// Per field the server keeps the last two snapshots (device), the running
// maximum M and, when freq_window > 0, the tile cube (q~ per tile, which does
// not depend on M) of the field's last freq_window triples, so every request
// continues the field's sequence of triples, its M estimate from past
// snapshots (the paper's real-time rule for M, Sec. 2.2.4) and the time
// series the frequency branch transforms (Sec. 2.3). Requests are admitted
// while a bound on the device memory in use fits the budget (resident field
// state plus, per slot, the larger of its retained scratch and the exact
// scratch of the largest queued or running request); admitted requests wait
// for one of n_slots worker slots, each with its own context and HIP stream,
// so requests of different fields run concurrently on the device. A slot
// replays the launch sequence it captured into a HIP graph for the request's
// shape. A field's requests run in submission order. Results are bitwise
// those of running the same frames alone (the kernels are deterministic and
// each slot owns its scratch).
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fitrig.h"
#include "fitrig_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t dtype_bytes(fitrig_dtype d) { return d == FITRIG_F32 ? 4 : 2; }

struct Req {
  int64_t ticket = 0, field = 0;
  const void* stack = nullptr;
  fitrig_dtype dtype = FITRIG_F32;
  int n = 0, H = 0, W = 0;
  double tau = 0.0;
  int64_t mem = 0;  // exact scratch bytes of the request (admission, while queued or running)
  hipEvent_t ready = nullptr;  // recorded on the legacy default stream at submit
  int replayed = 0;
  int64_t t_submit = 0, t_start = 0, t_done = 0;
  bool done = false;
  fitrig_status status = FITRIG_OK;
  std::vector<fitrig_candidate> cand;
  int64_t n_cand = 0;
  int n_triples = 0;
  int64_t first_triple = 0;
  int freq_triples = 0;
  double M = 0.0;
};

struct Field {
  int H = 0, W = 0;
  fitrig_dtype dtype = FITRIG_F32;
  char* carry = nullptr;     // two frames on the device
  size_t frame_bytes = 0;
  double* ring = nullptr;    // tile-cube slices of the latest triples, oldest first
  size_t ring_bytes = 0;     // capacity: freq_window slices
  int nring = 0;             // slices held
  float* pxring = nullptr;   // per-pixel branch: q maps of the latest triples (a ring)
  size_t pxring_bytes = 0;   // capacity: freq_window maps
  int px_start = 0, px_n = 0;  // slot of the oldest map held, maps held
  int ncarry = 0;            // frames held (0..2) once every submitted request has run
  int64_t frames_seen = 0;   // frames of finished requests
  int64_t frames_submitted = 0;
  double M = -INFINITY;
  int64_t last_use = 0;      // submit counter of the field's latest request
  bool busy = false;         // a request of this field is ready or running
  std::deque<int64_t> pending;
};

}  // namespace

struct fitrig_server {
  fitrig_server_config cfg;
  std::mutex mu;
  std::condition_variable cv_ready, cv_done;
  std::deque<int64_t> ready;
  std::unordered_map<int64_t, Req*> reqs;
  std::unordered_map<int64_t, Field> fields;
  std::vector<std::thread> workers;
  std::vector<fitrig_ctx*> ctxs;
  int64_t next_ticket = 1;
  int64_t use_clock = 0;
  std::multiset<int64_t> inflight;  // scratch bytes of the queued and running requests
  std::vector<int64_t> retained;    // device bytes each slot's context holds
  int64_t mem_fields = 0;   // resident field state
  int outstanding = 0;      // admitted, not finished
  bool stop = false;
};

namespace {

// Bound on the device bytes in use once every admitted request has run, with
// `need` the largest scratch of a queued or running request: any of them may
// run on any slot, and a slot keeps the largest scratch it has held.
int64_t device_bound(const fitrig_server* S, int64_t need) {
  int64_t b = S->mem_fields;
  for (int64_t r : S->retained) b += std::max(r, need);
  return b;
}

// Device bytes of a field's resident state.
size_t field_bytes(const Field& f) { return 2 * f.frame_bytes + f.ring_bytes + f.pxring_bytes; }

void free_field(Field& f) {
  if (f.carry) (void)hipFree(f.carry);
  if (f.ring) (void)hipFree(f.ring);
  if (f.pxring) (void)hipFree(f.pxring);
  f.pxring = nullptr;
  f.carry = nullptr;
  f.ring = nullptr;
}

void worker_main(fitrig_server* S, int slot) {
  fitrig_ctx* ctx = S->ctxs[slot];
  (void)hipSetDevice(S->cfg.base.device);
  std::vector<fitrig_candidate> buf((size_t)std::max<int64_t>(S->cfg.cand_cap, 1));
  for (;;) {
    Req* r = nullptr;
    const void *c0 = nullptr, *c1 = nullptr;
    int nc = 0;
    int64_t first = 0;
    fitrig::FreqHist fh{nullptr, 0, 0, nullptr, 0};
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_ready.wait(lk, [&] { return S->stop || !S->ready.empty(); });
      if (S->ready.empty()) return;
      const int64_t t = S->ready.front();
      S->ready.pop_front();
      r = S->reqs[t];
      Field& f = S->fields[r->field];
      nc = f.ncarry;
      if (nc >= 1) c0 = f.carry + (2 - nc) * f.frame_bytes;
      if (nc == 2) c1 = f.carry + f.frame_bytes;
      first = f.frames_seen - nc;
      if (f.ring) fh = fitrig::FreqHist{f.ring, f.nring, S->cfg.freq_window, f.ring, 0};
      if (f.pxring) {
        fh.px_ring = f.pxring;
        fh.px_cap = S->cfg.freq_window;
        fh.px_start = f.px_start;
        fh.px_n = f.px_n;
      }
    }
    r->t_start = now_ns();
    fitrig_stats st;
    memset(&st, 0, sizeof(st));
    int64_t ncand = 0;
    const int64_t replays0 = fitrig::ctx_graph_replays(ctx);
    // the slot's stream does not wait on the legacy default stream by itself
    hipError_t we = hipStreamWaitEvent(fitrig::ctx_stream(ctx), r->ready, 0);
    fitrig_status rc = we != hipSuccess ? FITRIG_E_HIP : fitrig::detect_frames(ctx, c0, c1, nc, r->stack, r->dtype, r->n, r->H, r->W, r->tau,
                                             buf.data(), S->cfg.cand_cap, &ncand, &st, nullptr,
                                             (fh.cap || fh.px_cap) ? &fh : nullptr);
    r->replayed = fitrig::ctx_graph_replays(ctx) > replays0 ? 1 : 0;
    // the field keeps the last two frames of [carried | new]
    Field* fp;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      fp = &S->fields[r->field];
    }
    const size_t fb = fp->frame_bytes;
    hipStream_t hs = fitrig::ctx_stream(ctx);
    hipError_t he = hipSuccess;
    if (r->n >= 2) {
      he = hipMemcpyAsync(fp->carry, (const char*)r->stack + (size_t)(r->n - 2) * fb, 2 * fb,
                          hipMemcpyDeviceToDevice, hs);
    } else {  // one new frame: [previous newest, new]
      if (nc >= 1)
        he = hipMemcpyAsync(fp->carry, fp->carry + fb, fb, hipMemcpyDeviceToDevice, hs);
      if (he == hipSuccess)
        he = hipMemcpyAsync(fp->carry + fb, r->stack, fb, hipMemcpyDeviceToDevice, hs);
    }
    if (he == hipSuccess) he = hipStreamSynchronize(hs);
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    if (he != hipSuccess && (rc == FITRIG_OK || rc == FITRIG_E_TRUNC)) {
      fitrig::ctx_last_hip(ctx) = (int32_t)he;
      rc = FITRIG_E_HIP;
    }
    const int64_t kept = std::min<int64_t>(ncand, S->cfg.cand_cap);
    r->cand.assign(buf.begin(), buf.begin() + kept);
    for (fitrig_candidate& c : r->cand)  // field-wide triple numbers
      if (c.branch == FITRIG_IMAGE) c.triple = (int32_t)(c.triple + first);
    r->t_done = now_ns();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      Field& f = S->fields[r->field];
      r->status = rc;
      r->n_cand = ncand;
      r->n_triples = nc + r->n - 2 > 0 ? nc + r->n - 2 : 0;
      r->first_triple = first;
      if (f.pxring) {
        // the ring gained the run's last min(n_triples, window) maps
        const bool ok = rc == FITRIG_OK || rc == FITRIG_E_TRUNC;
        const int cap = S->cfg.freq_window;
        const int nap = std::min(r->n_triples, cap);
        const int n_new = (int)std::min<int64_t>(cap, (int64_t)f.px_n + r->n_triples);
        f.px_start = ok ? (f.px_start + f.px_n + nap - n_new) % cap : 0;
        f.px_n = ok ? n_new : 0;
      }
      if (f.ring) {
        // the history holds what the run wrote; after a failed run it is dropped
        const bool ok = rc == FITRIG_OK || rc == FITRIG_E_TRUNC;
        f.nring = ok ? (int)std::min<int64_t>(S->cfg.freq_window, (int64_t)f.nring + r->n_triples) : 0;
        r->freq_triples = (ok && (S->cfg.base.branches & FITRIG_FREQ) && f.nring >= 4) ? f.nring : 0;
      } else {
        r->freq_triples = ((S->cfg.base.branches & FITRIG_FREQ) && r->n_triples >= 4) ? r->n_triples : 0;
      }
      f.M = fmax(f.M, st.M);
      r->M = f.M;
      f.frames_seen += r->n;
      f.ncarry = (int)std::min<int64_t>(2, nc + r->n);
      S->retained[slot] = fitrig::ctx_device_bytes(ctx);
      auto it = S->inflight.find(r->mem);
      if (it != S->inflight.end()) S->inflight.erase(it);
      S->outstanding -= 1;
      r->done = true;
      f.busy = false;
      if (!f.pending.empty()) {
        S->ready.push_back(f.pending.front());
        f.pending.pop_front();
        f.busy = true;
        S->cv_ready.notify_one();
      }
    }
    S->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

void fitrig_server_config_default(fitrig_server_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  fitrig_config_default(&cfg->base);
  cfg->n_slots = 4;
  cfg->max_fields = 64;
  cfg->mem_budget = 0;
  cfg->cand_cap = 65536;
  cfg->freq_window = 0;
  cfg->graphs = 1;
}

fitrig_status fitrig_server_create(const fitrig_server_config* cfg, fitrig_server** out) {
  if (!cfg || !out) return FITRIG_E_INVAL;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 64 || cfg->max_fields < 1 || cfg->cand_cap < 0 || cfg->mem_budget < 0 ||
      cfg->freq_window < 0 || cfg->freq_window > 2048 || cfg->base.tile < 1 || (cfg->graphs != 0 && cfg->graphs != 1))
    return FITRIG_E_INVAL;
  fitrig_server* S = new (std::nothrow) fitrig_server();
  if (!S) return FITRIG_E_NOMEM;
  S->cfg = *cfg;
  S->cfg.base.profile = 0;
  for (int i = 0; i < cfg->n_slots; ++i) {
    fitrig_ctx* c = nullptr;
    const fitrig_status rc = fitrig_create(&S->cfg.base, &c);
    if (rc != FITRIG_OK) {
      for (fitrig_ctx* x : S->ctxs) fitrig_destroy(x);
      delete S;
      return rc;
    }
    S->ctxs.push_back(c);
    const fitrig_status rs = fitrig::ctx_set_serving(c, cfg->graphs != 0);
    if (rs != FITRIG_OK) {
      for (fitrig_ctx* x : S->ctxs) fitrig_destroy(x);
      delete S;
      return rs;
    }
  }
  // with capacity hints every slot is sized at create for a square image of
  // max_pixels with max_snap new frames after two carried ones and the
  // longest frequency history, so requests up to that size do not grow it
  const fitrig_config& b = S->cfg.base;
  if (b.max_pixels > 0 && b.max_snap >= 3) {
    const int side = (int)ceil(sqrt((double)b.max_pixels));
    const bool ring = S->cfg.freq_window > 0 && (b.branches & FITRIG_FREQ) != 0;
    const bool pxr = S->cfg.freq_window > 0 && (b.branches & FITRIG_FREQ_PIXEL) != 0 && b.mode == FITRIG_SLIDING;
    const fitrig::FreqHist hs{(const double*)(uintptr_t)256, ring ? S->cfg.freq_window : 0,
                              ring ? S->cfg.freq_window : 0, (double*)(uintptr_t)256, 0,
                              pxr ? (float*)(uintptr_t)256 : nullptr, pxr ? S->cfg.freq_window : 0, 0,
                              pxr ? S->cfg.freq_window : 0};
    for (fitrig_ctx* c : S->ctxs) {
      const fitrig_status rc = fitrig::ctx_presize_for(c, 2, b.max_snap, side, side, FITRIG_F32,
                                                       (ring || pxr) ? &hs : nullptr, S->cfg.cand_cap);
      if (rc != FITRIG_OK) {
        for (fitrig_ctx* x : S->ctxs) fitrig_destroy(x);
        delete S;
        return rc;
      }
    }
  }
  for (fitrig_ctx* c : S->ctxs) S->retained.push_back(fitrig::ctx_device_bytes(c));
  if (cfg->mem_budget > 0 && device_bound(S, 0) > cfg->mem_budget) {
    for (fitrig_ctx* x : S->ctxs) fitrig_destroy(x);
    delete S;
    return FITRIG_E_NOMEM;
  }
  for (int i = 0; i < cfg->n_slots; ++i) S->workers.emplace_back(worker_main, S, i);
  *out = S;
  return FITRIG_OK;
}

fitrig_status fitrig_submit(fitrig_server* S, int64_t field_id, const void* stack, fitrig_dtype dtype, int32_t n_snap,
                            int32_t H, int32_t W, double sigma, int32_t blocking, int64_t* ticket) {
  if (!S || !stack || !ticket) return FITRIG_E_INVAL;
  if (dtype != FITRIG_F32 && dtype != FITRIG_F16 && dtype != FITRIG_BF16) return FITRIG_E_INVAL;
  if (n_snap < 1 || H < 1 || W < 1 || (uint64_t)H * (uint64_t)W >= (1ull << 32)) return FITRIG_E_INVAL;
  if (!(sigma > 0.0) || !isfinite(sigma)) return FITRIG_E_INVAL;
  const int64_t t_submit = now_ns();
  const size_t fb = (size_t)H * W * dtype_bytes(dtype);
  const int tile = S->cfg.base.tile;
  const bool keep_ring = S->cfg.freq_window > 0 && (S->cfg.base.branches & FITRIG_FREQ) != 0;
  const size_t rb = keep_ring ? (size_t)S->cfg.freq_window * ((H + tile - 1) / tile) * ((W + tile - 1) / tile) * 8 : 0;
  const bool keep_px = S->cfg.freq_window > 0 && (S->cfg.base.branches & FITRIG_FREQ_PIXEL) != 0 &&
                       S->cfg.base.mode == FITRIG_SLIDING;
  const size_t pb = keep_px ? (size_t)S->cfg.freq_window * (size_t)H * W * 4 : 0;
  const int64_t budget = S->cfg.mem_budget;
  std::unique_lock<std::mutex> lk(S->mu);
  // the field's state and the charge are re-read after every wait, so
  // concurrent submits to the same field see each other
  bool fresh, resize;
  int64_t mem, field_mem;
  for (;;) {
    auto it = S->fields.find(field_id);
    fresh = it == S->fields.end();
    const Field* f0 = fresh ? nullptr : &it->second;
    resize = f0 && (f0->H != H || f0->W != W || f0->dtype != dtype);
    if (resize && (f0->busy || !f0->pending.empty())) return FITRIG_E_INVAL;
    const int64_t carried = (f0 && !resize) ? std::min<int64_t>(2, f0->frames_submitted) : 0;
    if (carried + n_snap < 3) return FITRIG_E_INVAL;
    field_mem = (fresh || resize) ? (int64_t)(2 * fb + rb + pb) : 0;
    // exact scratch of the request (the histories at their longest)
    const fitrig::FreqHist hs{(const double*)(uintptr_t)256, keep_ring ? S->cfg.freq_window : 0,
                              keep_ring ? S->cfg.freq_window : 0, (double*)(uintptr_t)256, 0,
                              keep_px ? (float*)(uintptr_t)256 : nullptr, keep_px ? S->cfg.freq_window : 0, 0,
                              keep_px ? S->cfg.freq_window : 0};
    mem = fitrig::call_scratch_bytes(S->cfg.base, (int)carried, n_snap, H, W, dtype,
                                     (keep_ring || keep_px) ? &hs : nullptr, S->cfg.cand_cap);
    if (mem <= 0) return FITRIG_E_INVAL;
    if (budget > 0 && field_mem + device_bound(S, mem) > budget) return FITRIG_E_BUSY;
    const int64_t top = S->inflight.empty() ? mem : std::max(mem, *S->inflight.rbegin());
    if (budget == 0 || field_mem + device_bound(S, top) <= budget) break;
    if (!blocking) return FITRIG_E_BUSY;
    S->cv_done.wait(lk);
  }
  if (fresh && (int64_t)S->fields.size() >= S->cfg.max_fields) {
    // evict the least recently used idle field (its carried frames and M)
    auto lru = S->fields.end();
    for (auto jt = S->fields.begin(); jt != S->fields.end(); ++jt)
      if (!jt->second.busy && jt->second.pending.empty() &&
          (lru == S->fields.end() || jt->second.last_use < lru->second.last_use))
        lru = jt;
    if (lru == S->fields.end()) return FITRIG_E_BUSY;
    free_field(lru->second);
    S->mem_fields -= (int64_t)field_bytes(lru->second);
    S->fields.erase(lru);
  }
  Field* f = fresh ? nullptr : &S->fields[field_id];
  // (re)create the field state
  if (fresh || resize) {
    Field& nf = S->fields[field_id];
    if (nf.carry || nf.ring || nf.pxring) {
      free_field(nf);
      S->mem_fields -= (int64_t)field_bytes(nf);
    }
    nf = Field();
    nf.H = H;
    nf.W = W;
    nf.dtype = dtype;
    nf.frame_bytes = fb;
    nf.ring_bytes = rb;
    nf.pxring_bytes = pb;
    if (hipSetDevice(S->cfg.base.device) != hipSuccess || hipMalloc((void**)&nf.carry, 2 * fb) != hipSuccess ||
        (rb && hipMalloc((void**)&nf.ring, rb) != hipSuccess) ||
        (pb && hipMalloc((void**)&nf.pxring, pb) != hipSuccess)) {
      free_field(nf);
      S->fields.erase(field_id);
      return FITRIG_E_NOMEM;
    }
    S->mem_fields += (int64_t)field_bytes(nf);
    f = &nf;
  }
  Req* r = new (std::nothrow) Req();
  if (!r) return FITRIG_E_NOMEM;
  // work queued on the legacy default stream before the submit (where the
  // stack may have been written) completes before the request reads it
  if (hipSetDevice(S->cfg.base.device) != hipSuccess ||
      hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(r->ready, nullptr) != hipSuccess) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    delete r;
    return FITRIG_E_HIP;
  }
  r->ticket = S->next_ticket++;
  r->field = field_id;
  r->stack = stack;
  r->dtype = dtype;
  r->n = n_snap;
  r->H = H;
  r->W = W;
  r->tau = sigma;
  r->mem = mem;
  r->t_submit = t_submit;
  S->reqs[r->ticket] = r;
  S->inflight.insert(mem);
  S->outstanding += 1;
  f->frames_submitted += n_snap;
  f->last_use = ++S->use_clock;
  if (!f->busy) {
    f->busy = true;
    S->ready.push_back(r->ticket);
    S->cv_ready.notify_one();
  } else {
    f->pending.push_back(r->ticket);
  }
  *ticket = r->ticket;
  return FITRIG_OK;
}

fitrig_status fitrig_poll(fitrig_server* S, int64_t ticket, int32_t wait, fitrig_result* out) {
  if (!S || !out) return FITRIG_E_INVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return FITRIG_E_INVAL;
  Req* r = it->second;
  if (!r->done) {
    if (!wait) return FITRIG_E_NOTREADY;
    S->cv_done.wait(lk, [&] { return r->done; });
  }
  out->ticket = r->ticket;
  out->field_id = r->field;
  out->status = r->status;
  out->n_triples = r->n_triples;
  out->first_triple = r->first_triple;
  out->n_cand = r->n_cand;
  out->cand = r->cand.empty() ? nullptr : r->cand.data();
  out->M = r->M;
  out->freq_triples = r->freq_triples;
  out->replayed = r->replayed;
  out->t_submit_ns = r->t_submit;
  out->t_start_ns = r->t_start;
  out->t_done_ns = r->t_done;
  return FITRIG_OK;
}

fitrig_status fitrig_release(fitrig_server* S, int64_t ticket) {
  if (!S) return FITRIG_E_INVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return FITRIG_E_INVAL;
  if (!it->second->done) return FITRIG_E_NOTREADY;
  delete it->second;
  S->reqs.erase(it);
  return FITRIG_OK;
}

fitrig_status fitrig_server_destroy(fitrig_server* S) {
  if (!S) return FITRIG_E_INVAL;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->outstanding == 0; });
    S->stop = true;
  }
  S->cv_ready.notify_all();
  for (std::thread& t : S->workers) t.join();
  for (fitrig_ctx* c : S->ctxs) fitrig_destroy(c);
  for (auto& kv : S->fields) free_field(kv.second);
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return FITRIG_OK;
}

}  // extern "C"
