// Host-only exercise of the runtime's argument checks, sizing passes and
// result unpacking, built with AddressSanitizer and UndefinedBehaviorSanitizer
// (no GPU: nothing is allocated on or launched to a device). Seeded fuzzing
// over shapes and configurations; exits non-zero on a failed expectation.
#include "../../paper_2509_21754_amd/csrc/fitrig_api.hip"

#include <cstdio>
#include <random>

namespace fitrig {
// The launch pass never runs here; the kernel handles are not needed.
const void* kernel_stream_f32(int, bool, bool) { return nullptr; }
const void* kernel_stream_f16(int, bool, bool) { return nullptr; }
const void* kernel_stream_bf16(int, bool, bool) { return nullptr; }
const void* kernel_tile_stream_f32(int, bool) { return nullptr; }
const void* kernel_tile_stream_f16(int, bool) { return nullptr; }
const void* kernel_tile_stream_bf16(int, bool) { return nullptr; }
const void* kernel_tile_f32(bool) { return nullptr; }
const void* kernel_tile_f16(bool) { return nullptr; }
const void* kernel_tile_bf16(bool) { return nullptr; }
const void* kernel_recompute_f32(int, bool) { return nullptr; }
const void* kernel_recompute_f16(int, bool) { return nullptr; }
const void* kernel_recompute_bf16(int, bool) { return nullptr; }
const void* kernel_stack_max_f32() { return nullptr; }
const void* kernel_stack_max_f16() { return nullptr; }
const void* kernel_stack_max_bf16() { return nullptr; }
}  // namespace fitrig

static int failures = 0;
#define EXPECT(c)                                                  \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                  \
    }                                                              \
  } while (0)

int main() {
  std::mt19937_64 rng(12345);
  auto pick = [&](int lo, int hi) { return lo + (int)(rng() % (uint64_t)(hi - lo + 1)); };
  // status strings and defaults
  for (int c = -8; c <= 1; ++c) EXPECT(fitrig_status_string(c) != nullptr);
  fitrig_config cfg;
  fitrig_config_default(&cfg);
  EXPECT(validate_cfg(&cfg) == FITRIG_OK);
  EXPECT(validate_cfg(nullptr) == FITRIG_E_INVAL);
  int64_t sized = 0;
  for (int it = 0; it < 3000; ++it) {
    fitrig_config_default(&cfg);
    cfg.mode = pick(0, 1);
    cfg.window = 2 * pick(0, 8) + 1;
    cfg.tile = pick(0, 3) == 0 ? pick(1, 70) : (1 << pick(0, 6));
    cfg.branches = pick(1, 7);
    if (cfg.mode == FITRIG_TILES) cfg.branches &= ~FITRIG_FREQ_PIXEL;
    if (!cfg.branches) cfg.branches = FITRIG_IMAGE;
    cfg.sigma_est = pick(0, 1);
    cfg.harm = pick(0, 2) ? 0 : pick(2, 8);
    cfg.r_signed = pick(0, 1);
    cfg.max_segments = pick(0, 3) ? 0 : pick(1, 1 << 16);
    // occasionally an invalid field
    const int bad = pick(0, 20);
    if (bad == 0) cfg.window = 2 * pick(1, 9);
    if (bad == 1) cfg.tile = 0;
    if (bad == 2) cfg.harm = 1;
    if (bad == 3) cfg.C = -1.0;
    const fitrig_status v = validate_cfg(&cfg);
    EXPECT((bad <= 3) == (v != FITRIG_OK));
    if (v != FITRIG_OK) continue;
    const int H = pick(0, 3) ? pick(1, 700) : pick(1, 5000);
    const int W = pick(0, 3) ? pick(1, 700) : pick(1, 5000);
    const int n = pick(3, pick(0, 5) ? 40 : 300);
    const int ncarry = pick(0, 2);
    const fitrig_dtype dt = (fitrig_dtype)pick(0, 2);
    const int hcap = pick(0, 2) ? 0 : pick(1, 64);
    fitrig::FreqHist h{(const double*)(uintptr_t)256, hcap ? pick(0, hcap) : 0, hcap, (double*)(uintptr_t)256,
                       pick(0, 1)};
    const int64_t cap = pick(0, 1 << 17);
    const int64_t b = fitrig::call_scratch_bytes(cfg, ncarry, std::max(1, n - ncarry), H, W, dt, hcap ? &h : nullptr,
                                                 cap);
    const Call c = shape_call(ncarry, std::max(1, n - ncarry), H, W, dt, hcap ? &h : nullptr, cap, nullptr);
    const bool ok_shape = check_shape(cfg, c) == FITRIG_OK;
    EXPECT(ok_shape == (b > 0));
    if (b > 0) sized += 1;
    // unpack a synthetic packed result of this shape
    const int np = c.n - 2;
    const int64_t kc = std::min<int64_t>(cap, 300);
    const ResultLayout R = result_layout(np, kc);
    std::vector<char> packed((size_t)R.bytes, 0);
    int64_t* cnt = (int64_t*)(packed.data() + R.off_cnt);
    cnt[CNT_OUTBASE] = pick(0, (int)kc + 5);
    cnt[CNT_TRUNC] = pick(0, 1);
    std::vector<fitrig_candidate> out((size_t)std::max<int64_t>(kc, 1));
    std::vector<double> mu(np), sg(np);
    std::vector<uint32_t> fl(np);
    fitrig_stats st;
    memset(&st, 0, sizeof(st));
    st.mu = mu.data();
    st.sigma = sg.data();
    st.flags = fl.data();
    int64_t nc = -1;
    const fitrig_status us = unpack_results(packed.data(), R, np, branches_ran(cfg, c), out.data(), kc, &nc, &st,
                                            st.mu, st.sigma, st.flags);
    EXPECT(nc == cnt[CNT_OUTBASE]);
    EXPECT((us == FITRIG_E_TRUNC) == (cnt[CNT_TRUNC] != 0 || nc > kc));
  }
  std::printf("host sizing: %lld shapes sized, %d failures\n", (long long)sized, failures);
  return failures ? 1 : 0;
}
