// C-ABI entry points: host-side validation, workspace layout, dispatch.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "internal.h"

namespace gr {

namespace {
thread_local std::string g_last_error;
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

void set_error(const std::string& msg) { g_last_error = msg; }

gr_status fail(gr_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

gr_status ensure_lds_limit(const void* fn, size_t bytes, const char* what) {
  // hipFuncSetAttribute is issued once per (kernel, device) and size increase:
  // later launches, including ones captured into a graph, skip it.
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> done;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GR_EDEVICE, std::string(what) + ": no device");
  std::lock_guard<std::mutex> lock(mu);
  size_t& have = done[{fn, dev}];
  if (bytes <= have) return GR_OK;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess)
    return fail(GR_EDEVICE, std::string(what) + ": hipFuncSetAttribute: " + hipGetErrorString(e));
  have = bytes;
  return GR_OK;
}

gr_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return GR_OK;
}

gr_status validate_kernel(const gr_kernel* k, bool need_taps) {
  if (k == nullptr) return fail(GR_EINVAL, "kernel descriptor is NULL");
  if (k->kind != GR_SEPARABLE && k->kind != GR_TABLE2D && k->kind != GR_MLP)
    return fail(GR_EUNSUPPORTED, "kernel.kind must be GR_SEPARABLE, GR_TABLE2D or GR_MLP");
  if (k->kind == GR_TABLE2D && !k->taps_complex)
    return fail(GR_EUNSUPPORTED, "GR_TABLE2D kernels must have complex taps");
  if (k->kind == GR_MLP && (!k->taps_complex || k->tap_dtype != GR_F32))
    return fail(GR_EUNSUPPORTED, "GR_MLP kernels are complex with an FP32 weight blob");
  if (k->support < 2 || k->support > 64 || (k->support & 1))
    return fail(GR_EINVAL, "kernel.support must be even, 2..64");
  if (!pow2(k->oversample) || k->oversample > kMaxOversample)
    return fail(GR_EINVAL, "kernel.oversample must be a power of two <= 128");
  if (k->n_planes < 1 || k->n_planes > kMaxPlanes)
    return fail(GR_EINVAL, "kernel.n_planes must be in 1..32767");
  if (k->n_planes > 1 && (!std::isfinite(k->w_min) || !std::isfinite(k->inv_dw)))
    return fail(GR_EINVAL, "kernel.w_min / inv_dw must be finite");
  if (k->tap_dtype != GR_F32 && k->tap_dtype != GR_F16 && k->tap_dtype != GR_BF16)
    return fail(GR_EINVAL, "kernel.tap_dtype must be GR_F32, GR_F16 or GR_BF16");
  if (need_taps && k->taps == nullptr) return fail(GR_EINVAL, "kernel.taps is NULL");
  return GR_OK;
}

namespace {

gr_status validate_grid(int n_pol, int height, int width, int support) {
  if (n_pol != 1 && n_pol != 4) return fail(GR_EINVAL, "n_pol must be 1 or 4");
  if (height < support || width < support || height > kMaxGrid || width > kMaxGrid)
    return fail(GR_EINVAL, "grid height/width must be in [support, 32768]");
  return GR_OK;
}

}  // namespace

}  // namespace gr

using namespace gr;

extern "C" const char* gr_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t gr_version(void) { return 1; }

namespace gr {

// ---- tuning memo: the autotuner's winners, per device and problem class
namespace {
struct MemoKey {
  int dev, n_pol, kind, cplx, dtype, support, side, slot;
  bool operator<(const MemoKey& o) const {
    const int a[8] = {dev, n_pol, kind, cplx, dtype, support, side, slot};
    const int b[8] = {o.dev, o.n_pol, o.kind, o.cplx, o.dtype, o.support, o.side, o.slot};
    for (int i = 0; i < 8; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};
std::mutex g_memo_mu;
std::map<MemoKey, gr_tuning> g_memo;

MemoKey memo_key(int n_pol, const gr_kernel& k, int height, int width, int slot) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  int side = 1;
  while (side < std::max(height, width)) side <<= 1;
  return MemoKey{dev, n_pol, k.kind, k.taps_complex != 0, k.tap_dtype, k.support, side, slot};
}
}  // namespace

void memo_store(int n_pol, const gr_kernel& k, int height, int width, int slot, const gr_tuning& t) {
  std::lock_guard<std::mutex> lock(g_memo_mu);
  g_memo[memo_key(n_pol, k, height, width, slot)] = t;
}

bool memo_find(int n_pol, const gr_kernel& k, int height, int width, int slot, gr_tuning* out) {
  std::lock_guard<std::mutex> lock(g_memo_mu);
  const auto it = g_memo.find(memo_key(n_pol, k, height, width, slot));
  if (it == g_memo.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace gr

namespace {

int seg_len_of(const gr_tuning* t) { return t && t->vis_per_wg > 0 ? t->vis_per_wg : kDefaultSegLen; }

// the tuning a call uses: the caller's, else the memo's entry for the call's
// class, else NULL (library defaults); `slot` 0 for gr_grid, 1 for gr_grid_records
const gr_tuning* resolve_tuning(const gr_tuning* t, int n_pol, const gr_kernel& k, int height, int width,
                                int slot, gr_tuning* buf) {
  if (t != nullptr) return t;
  return memo_find(n_pol, k, height, width, slot, buf) ? buf : nullptr;
}

bool valid_slot(int slot) { return slot == 0 || slot == 1; }

// variant actually used by gr_grid: 1 = VALU work-item kernel on the input order,
// 2 = MFMA kernel on the binned stream
int pick_variant(const gr_kernel& k, int n_pol, const gr_tuning* t) {
  if (k.kind != GR_SEPARABLE) return 2;        // only the binned path handles other kinds
  const int want = t ? t->variant : 0;
  if (want == 1 || want == 2) return want;
  size_t lds;
  const std::string saved = g_last_error;
  const bool mfma_ok = plan_mfma(k, n_pol, &lds) == GR_OK;
  g_last_error = saved;
  return mfma_ok ? 2 : 1;
}

size_t pre_bytes(int64_t n_vis, int n_pol) {
  return align256(sizeof(Record) * (size_t)n_vis) + align256(sizeof(float2) * (size_t)n_vis * n_pol);
}

// gr_grid's variant-1 workspace: the preprocessed stream, then the VALU
// kernel's work counter
size_t valu_ws_bytes(int64_t n_vis, int n_pol) { return pre_bytes(n_vis, n_pol) + 256; }

}  // namespace

namespace gr {
// binned gridder for the kernel's kind
gr_status launch_binned(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                        float2* grid, int height, int width, hipStream_t stream, int ng) {
  if (k.kind == GR_TABLE2D) return launch_table2d(bins, L, n_pol, k, grid, height, width, stream);
  if (k.kind == GR_MLP) return launch_grid_mlp(bins, L, n_pol, k, grid, height, width, stream);
  return launch_mfma(bins, L, n_pol, k, grid, height, width, stream, ng);
}
}  // namespace gr

extern "C" size_t gr_bin_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                               int32_t width, int32_t seg_len) {
  if (n_vis < 0 || n_pol < 1 || support < 2 || support > 56 || height < 1 || width < 1) return 0;
  return bin_layout(n_vis, n_pol, support, height, width, seg_len > 0 ? seg_len : kDefaultSegLen).bytes;
}

extern "C" size_t gr_preprocess_bin_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                                          int32_t width, int32_t seg_len) {
  if (n_vis < 0 || n_pol < 1 || support < 2 || support > 56 || height < 1 || width < 1) return 0;
  return bin_layout(n_vis, n_pol, support, height, width, seg_len > 0 ? seg_len : kDefaultSegLen).bytes +
         align256(sizeof(Record) * (size_t)n_vis);
}

extern "C" size_t gr_grid_workspace_bytes(int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                                          int32_t height, int32_t width, const gr_tuning* tuning) {
  if (n_vis < 0 || n_pol < 1 || kernel == nullptr || height < 1 || width < 1) return 0;
  gr_tuning memo_t;
  tuning = resolve_tuning(tuning, n_pol, *kernel, height, width, 0, &memo_t);
  if (pick_variant(*kernel, n_pol, tuning) == 2) {   // fused preprocess and bin
    if (kernel->support > kMaxBinnedSupport) return 0;  // gr_grid refuses such a call
    return bin_layout(n_vis, n_pol, kernel->support, height, width, seg_len_of(tuning)).bytes +
           align256(sizeof(Record) * (size_t)n_vis);
  }
  return valu_ws_bytes(n_vis, n_pol);
}

namespace {
// arguments common to gr_preprocess and gr_preprocess_bin
gr_status validate_raw_inputs(const char* who, const double* uvw, const void* vis, int32_t vis_dtype,
                              const float* vis_scale, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                              double inv_cell_u, double inv_cell_v, int32_t height, int32_t width) {
  gr_status st = validate_kernel(kernel, false);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (n_vis < 0) return fail(GR_EINVAL, "n_vis must be >= 0");
  if (n_vis > 0 && (uvw == nullptr || vis == nullptr))
    return fail(GR_EINVAL, std::string(who) + ": uvw and vis must be non-NULL");
  if (vis_dtype != GR_F32 && vis_dtype != GR_F16)
    return fail(GR_EINVAL, "vis_dtype must be GR_F32 (complex64) or GR_F16 (scaled half pairs)");
  if (vis_dtype == GR_F16 && n_vis > 0 && vis_scale == nullptr)
    return fail(GR_EINVAL, "GR_F16 visibilities need vis_scale");
  if (!std::isfinite(inv_cell_u) || !std::isfinite(inv_cell_v) || inv_cell_u <= 0 || inv_cell_v <= 0)
    return fail(GR_EINVAL, "inv_cell_u / inv_cell_v must be finite and > 0");
  return GR_OK;
}
}  // namespace

extern "C" gr_status gr_preprocess(const double* uvw, const void* vis, int32_t vis_dtype,
                                   const float* vis_scale, const float* weights, int64_t n_vis,
                                   int32_t n_pol, const gr_kernel* kernel, double inv_cell_u,
                                   double inv_cell_v, int32_t height, int32_t width,
                                   void* records, void* wvis, int64_t* dev_stats, void* stream) {
  gr_status st = validate_raw_inputs("gr_preprocess", uvw, vis, vis_dtype, vis_scale, n_vis, n_pol, kernel,
                                     inv_cell_u, inv_cell_v, height, width);
  if (st != GR_OK) return st;
  if (n_vis > 0 && (records == nullptr || wvis == nullptr))
    return fail(GR_EINVAL, "gr_preprocess: records and wvis must be non-NULL");
  return launch_preprocess(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, *kernel, inv_cell_u,
                           inv_cell_v, height, width, reinterpret_cast<Record*>(records),
                           reinterpret_cast<float2*>(wvis), dev_stats, (hipStream_t)stream);
}

extern "C" gr_status gr_grid_records(const void* records, const void* wvis, int64_t n_vis,
                                     int32_t n_pol, const gr_kernel* kernel, void* grid,
                                     int32_t height, int32_t width, const gr_tuning* tuning,
                                     void* stream) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (n_vis < 0) return fail(GR_EINVAL, "n_vis must be >= 0");
  if (grid == nullptr) return fail(GR_EINVAL, "grid is NULL");
  if (n_vis > 0 && (records == nullptr || wvis == nullptr))
    return fail(GR_EINVAL, "records and wvis must be non-NULL");
  if (tuning && tuning->variant != 0 && tuning->variant != 1)
    return fail(GR_EUNSUPPORTED, "gr_grid_records runs the VALU work-item kernel (variant 0 or 1)");
  if (kernel->kind != GR_SEPARABLE)
    return fail(GR_EUNSUPPORTED, "gr_grid_records needs a separable kernel");
  gr_tuning memo_t;
  tuning = resolve_tuning(tuning, n_pol, *kernel, height, width, 1, &memo_t);
  RomeinPlan plan;
  if ((st = plan_romein(*kernel, n_pol, tuning, &plan)) != GR_OK) return st;
  return launch_romein(reinterpret_cast<const Record*>(records), reinterpret_cast<const float2*>(wvis),
                       n_vis, n_pol, *kernel, reinterpret_cast<float2*>(grid), height, width, plan,
                       (hipStream_t)stream);
}

extern "C" gr_status gr_bin(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                            int32_t support, int32_t height, int32_t width, int32_t seg_len,
                            void* bins, size_t bins_bytes, void* stream) {
  if (n_pol != 1 && n_pol != 4) return fail(GR_EINVAL, "n_pol must be 1 or 4");
  if (support < 2 || support > 56 || (support & 1)) return fail(GR_EINVAL, "gr_bin: support must be even, 2..56");
  if (height < support || width < support || height > kMaxGrid || width > kMaxGrid)
    return fail(GR_EINVAL, "grid height/width must be in [support, 32768]");
  if (n_vis < 0 || n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_bin: n_vis must be in [0, 2^31)");
  if (n_vis > 0 && (records == nullptr || wvis == nullptr)) return fail(GR_EINVAL, "records and wvis must be non-NULL");
  if (bins == nullptr) return fail(GR_EINVAL, "bins is NULL");
  const BinLayout L = bin_layout(n_vis, n_pol, support, height, width, seg_len > 0 ? seg_len : kDefaultSegLen);
  if (bins_bytes < L.bytes) return fail(GR_ENOMEM, "bins buffer too small (see gr_bin_bytes)");
  return launch_bin(reinterpret_cast<const Record*>(records), reinterpret_cast<const float2*>(wvis), n_vis,
                    n_pol, L, bins, (hipStream_t)stream);
}

extern "C" gr_status gr_preprocess_bin(const double* uvw, const void* vis, int32_t vis_dtype,
                                       const float* vis_scale, const float* weights, int64_t n_vis,
                                       int32_t n_pol, const gr_kernel* kernel, double inv_cell_u,
                                       double inv_cell_v, int32_t height, int32_t width, int32_t seg_len,
                                       void* bins, size_t bins_bytes, int64_t* dev_stats, void* stream) {
  gr_status st = validate_raw_inputs("gr_preprocess_bin", uvw, vis, vis_dtype, vis_scale, n_vis, n_pol, kernel,
                                     inv_cell_u, inv_cell_v, height, width);
  if (st != GR_OK) return st;
  if (kernel->support > 56) return fail(GR_EINVAL, "gr_preprocess_bin: support must be <= 56");
  if (n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_preprocess_bin: n_vis must be in [0, 2^31)");
  if (bins == nullptr) return fail(GR_EINVAL, "bins is NULL");
  const BinLayout L = bin_layout(n_vis, n_pol, kernel->support, height, width,
                                 seg_len > 0 ? seg_len : kDefaultSegLen);
  if (bins_bytes < L.bytes + align256(sizeof(Record) * (size_t)n_vis))
    return fail(GR_ENOMEM, "bins buffer too small (see gr_preprocess_bin_bytes)");
  auto* rec_tmp = reinterpret_cast<Record*>(reinterpret_cast<char*>(bins) + L.bytes);
  return launch_preprocess_bin(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, *kernel, inv_cell_u,
                               inv_cell_v, height, width, L, bins, rec_tmp, dev_stats, (hipStream_t)stream);
}

extern "C" size_t gr_compress_workspace_bytes(int64_t n_vis) {
  return n_vis < 0 ? 0 : compress_workspace_bytes(n_vis);
}

extern "C" gr_status gr_compress(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                                 void* out_records, void* out_wvis, int64_t* out_count, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  if (n_pol != 1 && n_pol != 4) return fail(GR_EINVAL, "n_pol must be 1 or 4");
  if (n_vis < 0 || n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_compress: n_vis must be in [0, 2^31)");
  if (n_vis > 0 && (records == nullptr || wvis == nullptr || out_records == nullptr || out_wvis == nullptr))
    return fail(GR_EINVAL, "gr_compress: records, wvis, out_records and out_wvis must be non-NULL");
  if (workspace == nullptr) return fail(GR_EINVAL, "gr_compress: workspace is NULL");
  if (workspace_bytes < compress_workspace_bytes(n_vis))
    return fail(GR_ENOMEM, "gr_compress: workspace too small (see gr_compress_workspace_bytes)");
  // the outputs are written while the inputs are still read: they must not overlap
  auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
    const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
  };
  const size_t rb = sizeof(Record) * (size_t)n_vis, wb = sizeof(float2) * (size_t)n_vis * n_pol;
  if (n_vis > 0 && (overlap(out_records, rb, records, rb) || overlap(out_records, rb, wvis, wb) ||
                    overlap(out_wvis, wb, records, rb) || overlap(out_wvis, wb, wvis, wb)))
    return fail(GR_EINVAL, "gr_compress: outputs must not overlap the inputs");
  return launch_compress(reinterpret_cast<const Record*>(records), reinterpret_cast<const float2*>(wvis), n_vis,
                         n_pol, reinterpret_cast<Record*>(out_records), reinterpret_cast<float2*>(out_wvis),
                         out_count, workspace, (hipStream_t)stream);
}

extern "C" size_t gr_wslice_partition_workspace_bytes(int64_t n_vis, int32_t n_slices) {
  if (n_vis < 0 || n_slices < 1 || n_slices > 255) return 0;
  return wslice_workspace_bytes(n_vis, n_slices);
}

extern "C" gr_status gr_wslice_partition(const double* uvw, const void* vis, const float* weights, int64_t n_vis,
                                         int32_t n_pol, double w_first, double inv_width, int32_t n_slices,
                                         double* uvw_out, void* vis_out, float* weights_out,
                                         int64_t* slice_offsets, void* workspace, size_t workspace_bytes,
                                         void* stream) {
  if (n_pol != 1 && n_pol != 4) return fail(GR_EINVAL, "n_pol must be 1 or 4");
  if (n_vis < 0 || n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_wslice_partition: n_vis must be in [0, 2^31)");
  if (n_slices < 1 || n_slices > 255) return fail(GR_EINVAL, "gr_wslice_partition: n_slices must be in [1, 255]");
  if (!std::isfinite(w_first) || !std::isfinite(inv_width) || inv_width <= 0)
    return fail(GR_EINVAL, "gr_wslice_partition: w_first must be finite and inv_width finite and > 0");
  if (slice_offsets == nullptr) return fail(GR_EINVAL, "gr_wslice_partition: slice_offsets is NULL");
  if (n_vis > 0 && (uvw == nullptr || vis == nullptr || uvw_out == nullptr || vis_out == nullptr))
    return fail(GR_EINVAL, "gr_wslice_partition: uvw, vis, uvw_out and vis_out must be non-NULL");
  if (n_vis > 0 && ((weights == nullptr) != (weights_out == nullptr)))
    return fail(GR_EINVAL, "gr_wslice_partition: weights_out must be given exactly when weights is");
  if (workspace == nullptr) return fail(GR_EINVAL, "gr_wslice_partition: workspace is NULL");
  if (workspace_bytes < wslice_workspace_bytes(n_vis, n_slices))
    return fail(GR_ENOMEM, "gr_wslice_partition: workspace too small (see gr_wslice_partition_workspace_bytes)");
  // the outputs are written while the inputs are still read: they must not overlap
  auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
    const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && pa < pb + nb && pb < pa + na;
  };
  const size_t ub = 3 * sizeof(double) * (size_t)n_vis, vb = sizeof(float2) * (size_t)n_vis * n_pol;
  const size_t wb = weights ? sizeof(float) * (size_t)n_vis * n_pol : 0;
  const void* ins[3] = {uvw, vis, weights};
  const size_t in_b[3] = {ub, vb, wb};
  const void* outs[3] = {uvw_out, vis_out, weights_out};
  const size_t out_b[3] = {ub, vb, wb};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      if (n_vis > 0 && overlap(outs[a], out_b[a], ins[b], in_b[b]))
        return fail(GR_EINVAL, "gr_wslice_partition: outputs must not overlap the inputs");
    if (n_vis > 0 && overlap(slice_offsets, sizeof(int64_t) * (size_t)(n_slices + 1), ins[a], in_b[a]))
      return fail(GR_EINVAL, "gr_wslice_partition: slice_offsets must not overlap the inputs");
  }
  return launch_wslice_partition(uvw, reinterpret_cast<const float2*>(vis), weights, n_vis, n_pol, w_first,
                                 inv_width, n_slices, uvw_out, reinterpret_cast<float2*>(vis_out), weights_out,
                                 slice_offsets, workspace, (hipStream_t)stream);
}

extern "C" size_t gr_grid_aterm_workspace_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                                                int32_t width) {
  if (n_vis < 0 || n_pol < 1 || support < 2 || support > 56 || height < 1 || width < 1) return 0;
  return bin_layout(n_vis, n_pol, support, height, width, kDefaultSegLen, aterm_window(support)).bytes +
         align256(sizeof(Record) * (size_t)n_vis);
}

extern "C" gr_status gr_grid_aterm(const double* uvw, const void* vis, int32_t vis_dtype, const float* vis_scale,
                                   const float* weights, const int32_t* kernel_id, int32_t n_ids, int64_t n_vis,
                                   int32_t n_pol, const gr_kernel* kernel, double inv_cell_u, double inv_cell_v,
                                   void* grid, int32_t height, int32_t width, void* workspace,
                                   size_t workspace_bytes, int64_t* dev_stats, void* stream) {
  gr_status st = validate_raw_inputs("gr_grid_aterm", uvw, vis, vis_dtype, vis_scale, n_vis, n_pol, kernel,
                                     inv_cell_u, inv_cell_v, height, width);
  if (st != GR_OK) return st;
  if ((st = validate_kernel(kernel, true)) != GR_OK) return st;
  if (kernel->kind != GR_TABLE2D)
    return fail(GR_EUNSUPPORTED, "gr_grid_aterm takes a GR_TABLE2D kernel (taps [n_ids][planes][O][O][n_pol][S][S])");
  if (kernel->support > 56) return fail(GR_EUNSUPPORTED, "gr_grid_aterm: support must be <= 56");
  if (n_ids < 1 || (int64_t)n_ids * kernel->n_planes > kMaxPlanes)
    return fail(GR_EINVAL, "gr_grid_aterm: n_ids must be >= 1 with n_ids x n_planes <= 32767");
  if (n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_grid_aterm: n_vis must be in [0, 2^31)");
  if (n_vis > 0 && kernel_id == nullptr) return fail(GR_EINVAL, "gr_grid_aterm: kernel_id is NULL");
  if (grid == nullptr) return fail(GR_EINVAL, "grid is NULL");
  const BinLayout L = bin_layout(n_vis, n_pol, kernel->support, height, width, kDefaultSegLen,
                                 aterm_window(kernel->support));
  const size_t need = L.bytes + align256(sizeof(Record) * (size_t)n_vis);
  if (workspace == nullptr) return fail(GR_EINVAL, "gr_grid_aterm: workspace is NULL");
  if (workspace_bytes < need)
    return fail(GR_ENOMEM, "gr_grid_aterm: workspace too small (see gr_grid_aterm_workspace_bytes)");
  auto* rec_tmp = reinterpret_cast<Record*>(reinterpret_cast<char*>(workspace) + L.bytes);
  if ((st = launch_preprocess_bin(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, *kernel, inv_cell_u,
                                  inv_cell_v, height, width, L, workspace, rec_tmp, dev_stats, (hipStream_t)stream,
                                  kernel_id, n_ids)) != GR_OK)
    return st;
  return launch_aterm(workspace, L, n_pol, *kernel, reinterpret_cast<float2*>(grid), height, width,
                      (hipStream_t)stream);
}

extern "C" size_t gr_degrid_workspace_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                                            int32_t width, int32_t seg_len) {
  return gr_preprocess_bin_bytes(n_vis, n_pol, support, height, width, seg_len);
}

extern "C" gr_status gr_degrid(const double* uvw, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                               double inv_cell_u, double inv_cell_v, const void* grid, int32_t height,
                               int32_t width, void* vis_out, int32_t seg_len, void* workspace,
                               size_t workspace_bytes, int64_t* dev_stats, void* stream) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (n_vis < 0 || n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "gr_degrid: n_vis must be in [0, 2^31)");
  if (n_vis > 0 && (uvw == nullptr || vis_out == nullptr))
    return fail(GR_EINVAL, "gr_degrid: uvw and vis_out must be non-NULL");
  if (grid == nullptr) return fail(GR_EINVAL, "gr_degrid: grid is NULL");
  if (!std::isfinite(inv_cell_u) || !std::isfinite(inv_cell_v) || inv_cell_u <= 0 || inv_cell_v <= 0)
    return fail(GR_EINVAL, "inv_cell_u / inv_cell_v must be finite and > 0");
  size_t lds = 0;
  if ((st = plan_degrid(*kernel, n_pol, &lds)) != GR_OK) return st;
  if (seg_len > 4096) return fail(GR_EINVAL, "gr_degrid: seg_len must be <= 4096");
  const BinLayout L = bin_layout(n_vis, n_pol, kernel->support, height, width,
                                 seg_len > 0 ? seg_len : kDefaultSegLen);
  const size_t need = L.bytes + align256(sizeof(Record) * (size_t)n_vis);
  if (n_vis > 0 && workspace == nullptr) return fail(GR_EINVAL, "gr_degrid: workspace is NULL");
  if (workspace_bytes < need) return fail(GR_ENOMEM, "gr_degrid: workspace too small (see gr_degrid_workspace_bytes)");
  if (n_vis == 0) return GR_OK;
  auto* rec_tmp = reinterpret_cast<Record*>(reinterpret_cast<char*>(workspace) + L.bytes);
  if ((st = launch_degrid_bin(uvw, n_vis, n_pol, *kernel, inv_cell_u, inv_cell_v, height, width, L, workspace,
                              rec_tmp, reinterpret_cast<float2*>(vis_out), dev_stats, (hipStream_t)stream)) != GR_OK)
    return st;
  return launch_degrid(workspace, L, n_pol, *kernel, reinterpret_cast<const float2*>(grid), height, width,
                       reinterpret_cast<float2*>(vis_out), n_vis, (hipStream_t)stream);
}

extern "C" gr_status gr_grid_binned(const void* bins, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                                    int32_t seg_len, void* grid, int32_t height, int32_t width, void* stream) {
  return grid_binned(bins, n_vis, n_pol, kernel, seg_len, grid, height, width, stream, -1);
}

gr_status gr::grid_binned(const void* bins, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel, int32_t seg_len,
                          void* grid, int32_t height, int32_t width, void* stream, int ng) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (n_vis < 0 || n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "n_vis must be in [0, 2^31)");
  if (grid == nullptr || bins == nullptr) return fail(GR_EINVAL, "grid and bins must be non-NULL");
  if (kernel->support > kMaxBinnedSupport) return fail(GR_EUNSUPPORTED, "the binned gridders need support <= 56");
  const BinLayout L = bin_layout(n_vis, n_pol, kernel->support, height, width,
                                 seg_len > 0 ? seg_len : kDefaultSegLen);
  if (ng < 0) {   // the row groups per wave of the memo's variant-2 entry, else the default
    gr_tuning t;
    ng = memo_find(n_pol, *kernel, height, width, 0, &t) && t.variant == 2 ? t.wg_v : 0;
  }
  return launch_binned(bins, L, n_pol, *kernel, reinterpret_cast<float2*>(grid), height, width,
                       (hipStream_t)stream, ng);
}

extern "C" gr_status gr_grid(const double* uvw, const void* vis, int32_t vis_dtype,
                             const float* vis_scale, const float* weights, int64_t n_vis,
                             int32_t n_pol, const gr_kernel* kernel, double inv_cell_u,
                             double inv_cell_v, void* grid, int32_t height, int32_t width,
                             const gr_tuning* tuning, void* workspace, size_t workspace_bytes,
                             int64_t* dev_stats, void* stream) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (n_vis < 0) return fail(GR_EINVAL, "n_vis must be >= 0");
  if (grid == nullptr) return fail(GR_EINVAL, "grid is NULL");
  gr_tuning memo_t;
  tuning = resolve_tuning(tuning, n_pol, *kernel, height, width, 0, &memo_t);
  if (tuning && (tuning->variant < 0 || tuning->variant > 2))
    return fail(GR_EUNSUPPORTED, "tuning.variant not available in this build");
  const int variant = pick_variant(*kernel, n_pol, tuning);
  if (variant == 2 && kernel->support > kMaxBinnedSupport)
    return fail(GR_EUNSUPPORTED, "the binned gridders need support <= 56");
  const size_t need = gr_grid_workspace_bytes(n_vis, n_pol, kernel, height, width, tuning);
  if (n_vis > 0 && workspace == nullptr) return fail(GR_EINVAL, "workspace is NULL");
  if (workspace_bytes < need) return fail(GR_ENOMEM, "workspace too small (see gr_grid_workspace_bytes)");
  RomeinPlan plan;
  size_t lds;
  if (variant == 1 && (st = plan_romein(*kernel, n_pol, tuning, &plan)) != GR_OK) return st;
  if (variant == 2) {
    if (kernel->kind == GR_SEPARABLE && (st = plan_mfma(*kernel, n_pol, &lds)) != GR_OK) return st;
    if (kernel->support > 56) return fail(GR_EUNSUPPORTED, "the binned gridders need support <= 56");
    if (n_vis > 0x7fffffffLL) return fail(GR_EINVAL, "n_vis must be < 2^31 for the binned gridders");
  }
  if (variant == 1) {
    auto* rec = reinterpret_cast<Record*>(workspace);
    auto* wv = reinterpret_cast<float2*>(reinterpret_cast<char*>(workspace) +
                                         align256(sizeof(Record) * (size_t)n_vis));
    st = gr_preprocess(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel, inv_cell_u,
                       inv_cell_v, height, width, rec, wv, dev_stats, stream);
    if (st != GR_OK) return st;
    auto* counter = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) + pre_bytes(n_vis, n_pol));
    return launch_romein(rec, wv, n_vis, n_pol, *kernel, reinterpret_cast<float2*>(grid), height, width,
                         plan, (hipStream_t)stream, counter);
  }
  // binned path: preprocess and bin fused, then the binned gridder
  st = gr_preprocess_bin(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel, inv_cell_u, inv_cell_v,
                         height, width, seg_len_of(tuning), workspace, workspace_bytes, dev_stats, stream);
  if (st != GR_OK) return st;
  const BinLayout L = bin_layout(n_vis, n_pol, kernel->support, height, width, seg_len_of(tuning));
  return launch_binned(workspace, L, n_pol, *kernel, reinterpret_cast<float2*>(grid), height, width,
                       (hipStream_t)stream, tuning && tuning->variant == 2 ? tuning->wg_v : 0);
}

extern "C" gr_status gr_tuning_memo_put(int32_t n_pol, const gr_kernel* kernel, int32_t height, int32_t width,
                                        int32_t slot, const gr_tuning* tuning) {
  gr_status st = validate_kernel(kernel, false);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (!valid_slot(slot)) return fail(GR_EINVAL, "gr_tuning_memo_put: slot must be 0 or 1");
  if (tuning == nullptr) return fail(GR_EINVAL, "gr_tuning_memo_put: tuning is NULL");
  if (tuning->variant < 0 || tuning->variant > 2 || (slot == 1 && tuning->variant == 2))
    return fail(GR_EINVAL, "gr_tuning_memo_put: variant must be 0..2 (0 or 1 in slot 1)");
  memo_store(n_pol, *kernel, height, width, slot, *tuning);
  return GR_OK;
}

extern "C" gr_status gr_tuning_memo_get(int32_t n_pol, const gr_kernel* kernel, int32_t height, int32_t width,
                                        int32_t slot, gr_tuning* out) {
  gr_status st = validate_kernel(kernel, false);
  if (st != GR_OK) return st;
  if ((st = validate_grid(n_pol, height, width, kernel->support)) != GR_OK) return st;
  if (!valid_slot(slot)) return fail(GR_EINVAL, "gr_tuning_memo_get: slot must be 0 or 1");
  if (out == nullptr) return fail(GR_EINVAL, "gr_tuning_memo_get: out is NULL");
  if (!memo_find(n_pol, *kernel, height, width, slot, out))
    return fail(GR_EINVAL, "gr_tuning_memo_get: no entry for this problem class");
  return GR_OK;
}

extern "C" void gr_tuning_memo_clear(void) {
  std::lock_guard<std::mutex> lock(g_memo_mu);
  g_memo.clear();
}

extern "C" gr_status gr_wslice_kernel(const gr_kernel* table, double w_first, double inv_width, int32_t slice,
                                      gr_kernel* out) {
  gr_status st = validate_kernel(table, false);
  if (st != GR_OK) return st;
  if (out == nullptr) return fail(GR_EINVAL, "gr_wslice_kernel: out is NULL");
  if (!std::isfinite(w_first) || !std::isfinite(inv_width) || inv_width <= 0)
    return fail(GR_EINVAL, "gr_wslice_kernel: w_first must be finite and inv_width finite and > 0");
  if (slice < 0 || slice > 254) return fail(GR_EINVAL, "gr_wslice_kernel: slice must be in 0..254");
  gr_kernel k = *table;
  {
#pragma clang fp contract(off)
    k.w_min = w_first + (slice + 0.5) / inv_width + table->w_min;
  }
  if (!std::isfinite(k.w_min)) return fail(GR_EINVAL, "gr_wslice_kernel: the slice's w_min is not finite");
  *out = k;
  return GR_OK;
}

// ---- gr_grid without a caller workspace: a static scratch array per device.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is passed on.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of `scratch` on it

gr_status scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GR_EDEVICE, "gr_grid_noalloc: no current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return GR_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(GR_EDEVICE, std::string("gr_grid_noalloc: hipGetSymbolAddress of the scratch array: ") +
                                hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return GR_OK;
}
}  // namespace

extern "C" size_t gr_grid_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

extern "C" gr_status gr_grid_noalloc(const double* uvw, const void* vis, int32_t vis_dtype, const float* vis_scale,
                                     const float* weights, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                                     double inv_cell_u, double inv_cell_v, void* grid, int32_t height,
                                     int32_t width, const gr_tuning* tuning, int64_t* dev_stats, void* stream) {
  gr_status st = validate_kernel(kernel, true);
  if (st != GR_OK) return st;
  // resolve a NULL tuning once, so the size check and the call agree
  gr_tuning memo_t;
  tuning = resolve_tuning(tuning, n_pol, *kernel, height, width, 0, &memo_t);
  const size_t need = gr_grid_workspace_bytes(n_vis, n_pol, kernel, height, width, tuning);
  if (need > kNoAllocScratchBytes)
    return fail(GR_ENOMEM, "gr_grid_noalloc: these arguments need " + std::to_string(need) +
                               " bytes of scratch; the static scratch holds " +
                               std::to_string(kNoAllocScratchBytes) + " (use gr_grid with a workspace)");
  void* ws = nullptr;
  if ((st = scratch_on_current_device(&ws)) != GR_OK) return st;
  return gr_grid(uvw, vis, vis_dtype, vis_scale, weights, n_vis, n_pol, kernel, inv_cell_u, inv_cell_v, grid,
                 height, width, tuning, ws, kNoAllocScratchBytes, dev_stats, stream);
}
