// Autotuner of the H*v launch: times every admissible (variant, grid size,
// columns per lane) on the caller's buffers with HIP events, times the four
// fastest again with more launches, and keeps the fastest in the handle; subsequent ftlm_apply / ftlm_run launches with the same
// precision and column count use it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "ftlm_internal.hpp"

using namespace ftlm;

extern "C" {

int ftlm_hamiltonian_set_tuning(ftlm_hamiltonian *h, int32_t precision, int32_t n_cols, int32_t variant,
                                int32_t grid_cap, int32_t kc) {
  if (!h || (precision != FTLM_C128 && precision != FTLM_C64) || n_cols < 1 || n_cols > 64 || variant < 0 ||
      variant > 6 || grid_cap < 0 || kc < 0) {
    set_error("bad tuning arguments");
    return FTLM_EINVAL;
  }
  HvTuning &t = h->dev.tune[precision][n_cols];
  t.variant = variant;
  t.grid_cap = grid_cap;
  t.kc = kc;
  return FTLM_OK;
}

int ftlm_hamiltonian_autotune(ftlm_hamiltonian *h, int32_t precision, int32_t n_cols, const void *v, void *w,
                              void *stream, int32_t *variant, int32_t *grid_cap, int32_t *kc,
                              float *best_ms) {
  if (!h || !v || !w || (precision != FTLM_C128 && precision != FTLM_C64) || n_cols < 1 || n_cols > 64) {
    set_error("bad autotune arguments");
    return FTLM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const HamGeom &g = h->dev.geom;
  struct Cand {
    int variant, cap, kc;
  };
  std::vector<Cand> cands;
  const int caps[4] = {512, 1024, 2048, 4096};
  for (int cap : caps) {
    for (int k : {1, 2, 4, 8})
      if (n_cols % k == 0) cands.push_back({1, cap, k});
    if (n_cols == 1) cands.push_back({2, cap, 0});
    if (n_cols == 1 && g.spin_half && g.n >= kTileBits) cands.push_back({3, cap, 0});
    if (n_cols == 1 && cap <= 2048) cands.push_back({4, cap, 0});
    if (n_cols == 1 && cap <= 2048 && g.spin_half && g.n > kTileBits &&
        !(precision == FTLM_C64 ? h->dev.tw32 : h->dev.tw64).passes.empty())
      for (int groups : {1, 2, 4}) cands.push_back({5, cap, groups});
    // stream kernel: 1024 or 256 threads per block, chunks of 1, 4, 16 or 64 tiles per
    // XCD, the mixed pairs' partner tiles read directly or staged in LDS
    if (n_cols == 1 && cap <= 2048 && (precision == FTLM_C64 ? h->dev.sp32 : h->dev.sp64).ok)
      for (int st : {0, 1})
        for (int nt : {0, 1})
          for (int ch : {0, 2, 4, 6}) cands.push_back({6, cap, nt | (ch << 4) | (st << 8)});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("hipEventCreate failed");
    return FTLM_EHIP;
  }
  const HvTuning saved = h->dev.tune[precision][n_cols];
  float best = FLT_MAX;
  Cand bestc{0, 0, 0};
  int rc = FTLM_OK;
  // mean time of reps launches after one warm-up launch; < 0 if the shape is
  // inadmissible, NaN on a HIP error
  auto time_cand = [&](const Cand &c, int reps) -> float {
    HvLaunch L{};
    L.precision = precision;
    L.K = n_cols;
    L.v = v;
    L.w = w;
    L.variant = c.variant;
    L.grid_cap = c.cap;
    L.kc = c.kc;
    if (launch_hv(h->dev, L, s) != FTLM_OK) return -1.0f;
    if (hipEventRecord(e0, s) != hipSuccess) return NAN;
    for (int r = 0; r < reps; r++) launch_hv(h->dev, L, s);
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return NAN;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return ms / (float)reps;
  };
  // a quick pass over every candidate, then the four fastest again with more
  // launches each (neighbouring grid sizes often differ by a few per cent,
  // within the noise of three launches)
  std::vector<std::pair<float, int>> timed;
  for (size_t i = 0; i < cands.size() && !rc; i++) {
    const float ms = time_cand(cands[i], 3);
    if (std::isnan(ms)) rc = FTLM_EHIP;
    else if (ms >= 0) timed.push_back({ms, (int)i});
  }
  std::sort(timed.begin(), timed.end());
  for (size_t r = 0; r < timed.size() && r < 4 && !rc; r++) {
    const float ms = time_cand(cands[timed[r].second], 10);
    if (std::isnan(ms)) rc = FTLM_EHIP;
    else if (ms >= 0 && ms < best) {
      best = ms;
      bestc = cands[timed[r].second];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    h->dev.tune[precision][n_cols] = saved;
    set_error("autotune timing failed");
    return rc;
  }
  if (best == FLT_MAX) {
    set_error("no admissible H*v configuration");
    return FTLM_EINVAL;
  }
  HvTuning &t = h->dev.tune[precision][n_cols];
  t.variant = bestc.variant;
  t.grid_cap = bestc.cap;
  t.kc = bestc.kc;
  if (variant) *variant = bestc.variant;
  if (grid_cap) *grid_cap = bestc.cap;
  if (kc) *kc = bestc.kc;
  if (best_ms) *best_ms = best;
  return FTLM_OK;
}

}  // extern "C"
