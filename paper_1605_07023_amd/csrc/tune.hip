// Autotuning (Merry 2016, Section 4): a small data set is gridded with each
// candidate work decomposition (coarsening factors, tile shape, visibilities
// per work-group, kernel variant) and the fastest is kept.  This translation
// unit holds the timing sweep; the winner goes to the library's tuning memo
// (api.hip), which calls without a tuning read.  The candidate list, and
// keeping tunings across processes, are the caller's.
#include <cmath>
#include <vector>

#include "internal.h"

using namespace gr;

extern "C" gr_status gr_bin(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                            int32_t support, int32_t height, int32_t width, int32_t seg_len, void* bins,
                            size_t bins_bytes, void* stream);
extern "C" gr_status gr_grid_records(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                                     const gr_kernel* kernel, void* grid, int32_t height, int32_t width,
                                     const gr_tuning* tuning, void* stream);
extern "C" size_t gr_bin_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height, int32_t width,
                               int32_t seg_len);

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" gr_status gr_autotune(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                                 const gr_kernel* kernel, void* grid, int32_t height, int32_t width,
                                 void* bins, size_t bins_bytes, const gr_tuning* candidates,
                                 int32_t n_candidates, int32_t reps, float* times_ms, int32_t* best,
                                 void* stream) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  if (candidates == nullptr || n_candidates < 1 || times_ms == nullptr || best == nullptr)
    return fail(GR_EINVAL, "gr_autotune: candidates, times_ms and best must be non-NULL, n_candidates >= 1");
  if (reps < 1 || reps > 1000) return fail(GR_EINVAL, "gr_autotune: reps must be in 1..1000");
  if (grid == nullptr || (n_vis > 0 && (records == nullptr || wvis == nullptr)))
    return fail(GR_EINVAL, "gr_autotune: grid, records and wvis must be non-NULL");
  hipStream_t s = (hipStream_t)stream;
  EventPair ev;
  if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
    return fail(GR_EDEVICE, "gr_autotune: hipEventCreate failed");
  int best_i = -1;
  float best_t = INFINITY;
  for (int c = 0; c < n_candidates; ++c) {
    const gr_tuning& t = candidates[c];
    times_ms[c] = INFINITY;
    const int variant = t.variant == 1 ? 1 : 2;
    auto run = [&]() -> gr_status {
      if (variant == 1) return gr_grid_records(records, wvis, n_vis, n_pol, kernel, grid, height, width, &t, stream);
      const size_t need = gr_bin_bytes(n_vis, n_pol, kernel->support, height, width, t.vis_per_wg);
      if (need == 0 || bins == nullptr || bins_bytes < need) return fail(GR_ENOMEM, "gr_autotune: bins too small");
      gr_status r = gr_bin(records, wvis, n_vis, n_pol, kernel->support, height, width, t.vis_per_wg, bins,
                           bins_bytes, stream);
      if (r != GR_OK) return r;
      return grid_binned(bins, n_vis, n_pol, kernel, t.vis_per_wg, grid, height, width, stream, t.wg_v);
    };
    // warm-up call; unsupported candidates are skipped with time +inf
    if (run() != GR_OK) continue;
    if (hipEventRecord(ev.a, s) != hipSuccess) return fail(GR_EDEVICE, "gr_autotune: event record failed");
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = run() == GR_OK;
    if (hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
      return fail(GR_EDEVICE, "gr_autotune: event synchronisation failed");
    float ms = 0.f;
    if (!ok || hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) continue;
    times_ms[c] = ms / reps;
    if (times_ms[c] < best_t) {
      best_t = times_ms[c];
      best_i = c;
    }
  }
  *best = best_i;
  if (best_i < 0) return fail(GR_EUNSUPPORTED, "gr_autotune: no candidate ran");
  // remember the winner for calls without a tuning: slot 0 (gr_grid) takes the
  // fastest candidate, slot 1 (gr_grid_records) the fastest VALU one
  gr_tuning win = candidates[best_i];
  win.variant = win.variant == 1 ? 1 : 2;
  memo_store(n_pol, *kernel, height, width, 0, win);
  int best_v1 = -1;
  for (int c = 0; c < n_candidates; ++c)
    if (candidates[c].variant == 1 && std::isfinite(times_ms[c]) && (best_v1 < 0 || times_ms[c] < times_ms[best_v1]))
      best_v1 = c;
  if (best_v1 >= 0) memo_store(n_pol, *kernel, height, width, 1, candidates[best_v1]);
  set_error("");
  return GR_OK;
}
