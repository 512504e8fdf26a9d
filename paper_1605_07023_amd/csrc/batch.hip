// Batches of independent gridding problems in one launch sequence.
//
// The paper grids one instance (one frequency slice) per launch and notes that
// sparse slices give too few work-groups to fill the device (Section 5).  Here
// a whole batch (instances of different sizes, grids, supports and
// polarisation counts) goes through one fixed chain of launches:
//   setup (instance descriptors into the workspace; arguments by value),
//   preprocess, bin count, bin scan, bin scatter (each one launch over all
//   instances: a block finds its instance from the block ranges),
//   prefix (per group: member list and the exclusive prefix of segment counts),
//   one persistent MFMA gridder per (n_pol, complex taps) group, whose blocks
//   take (instance, segment) items from an atomic counter.
// Nothing synchronises with the host and no memset is issued (counters are
// cleared by kernels), so the sequence can be captured in a HIP graph and
// replayed.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace gr {

namespace {

constexpr int kSetupChunk = 4;      // descriptors per setup launch (passed by value)
constexpr int kGroups = 4;          // (n_pol == 4) * 2 + complex taps
constexpr int kMaxBatch = 4096;
// items with at least this many visibilities are binned for their support's
// window and gridded by the single-problem wave form (one launch each); the
// persistent work list keeps the smaller ones
constexpr int64_t kWideMin = int64_t(1) << 19;

struct SetupChunk {
  int first, count;
  BatchInst d[kSetupChunk];
};

__global__ void __launch_bounds__(64) batch_setup_kernel(SetupChunk c, BatchInst* __restrict__ table) {
  // one thread copies one descriptor, as 8-byte words
  if ((int)threadIdx.x < c.count) {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(&c.d[threadIdx.x]);
    uint64_t* dst = reinterpret_cast<uint64_t*>(&table[c.first + threadIdx.x]);
    for (size_t w = 0; w < sizeof(BatchInst) / 8; ++w) dst[w] = src[w];
  }
}

// Thread g builds group g: members (instance indices in batch order), the
// exclusive prefix of their segment counts ([n + 1] entries) and a zero work
// counter.
__global__ void __launch_bounds__(64)
batch_prefix_kernel(const BatchInst* __restrict__ inst, int n_inst, int32_t* __restrict__ members,
                    int32_t* __restrict__ prefix, int32_t* __restrict__ counters, int stride) {
  const int g = threadIdx.x;
  if (g >= kGroups) return;
  int cnt = 0, acc = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (inst[i].group != g) continue;
    members[g * stride + cnt] = i;
    prefix[g * (stride + 1) + cnt] = acc;
    acc += *inst[i].n_segs;
    ++cnt;
  }
  prefix[g * (stride + 1) + cnt] = acc;
  counters[g] = 0;
}

struct Plan {
  size_t off_table, off_members, off_prefix, off_counters, bytes;
  std::vector<size_t> off_inst;      // per instance: preprocess buffers, then bins
  std::vector<BinLayout> bins;
  std::vector<size_t> lds;           // MFMA LDS bytes per instance ((Re, Im) table entries)
  std::vector<size_t> lds_tri;       // the same with triple entries
  std::vector<char> wide;            // gridded on its own by the wave form
  int64_t total_blocks;
};

int group_of(const gr_batch_item& it) {
  return (it.n_pol == 4 ? 2 : 0) + (it.kernel.taps_complex ? 1 : 0);
}

size_t pre_size(int64_t n_vis, int n_pol) {
  return align256(sizeof(Record) * (size_t)n_vis) + align256(sizeof(float2) * (size_t)n_vis * n_pol);
}

gr_status validate_item(const gr_batch_item& it, int idx, size_t* lds) {
  const std::string at = "gr_grid_batch item " + std::to_string(idx) + ": ";
  gr_status st = validate_kernel(&it.kernel, true);
  if (st != GR_OK) return fail(st, at + gr_last_error());
  if (it.kernel.kind != GR_SEPARABLE)
    return fail(GR_EUNSUPPORTED, at + "batches take separable kernels (the MFMA gridder)");
  if (it.n_pol != 1 && it.n_pol != 4) return fail(GR_EINVAL, at + "n_pol must be 1 or 4");
  if (it.kernel.support > 56) return fail(GR_EUNSUPPORTED, at + "support must be <= 56");
  if (it.height < it.kernel.support || it.width < it.kernel.support || it.height > kMaxGrid ||
      it.width > kMaxGrid)
    return fail(GR_EINVAL, at + "grid height/width must be in [support, 32768]");
  if (it.n_vis < 0 || it.n_vis > 0x7fffffffLL) return fail(GR_EINVAL, at + "n_vis must be in [0, 2^31)");
  if (it.grid == nullptr) return fail(GR_EINVAL, at + "grid is NULL");
  if (it.n_vis > 0 && (it.uvw == nullptr || it.vis == nullptr))
    return fail(GR_EINVAL, at + "uvw and vis must be non-NULL");
  if (it.vis_dtype != GR_F32 && it.vis_dtype != GR_F16)
    return fail(GR_EINVAL, at + "vis_dtype must be GR_F32 or GR_F16");
  if (it.vis_dtype == GR_F16 && it.n_vis > 0 && it.vis_scale == nullptr)
    return fail(GR_EINVAL, at + "GR_F16 visibilities need vis_scale");
  if (!std::isfinite(it.inv_cell_u) || !std::isfinite(it.inv_cell_v) || it.inv_cell_u <= 0 ||
      it.inv_cell_v <= 0)
    return fail(GR_EINVAL, at + "inv_cell_u / inv_cell_v must be finite and > 0");
  if (it.seg_len < 0) return fail(GR_EINVAL, at + "seg_len must be >= 0");
  if ((st = plan_mfma(it.kernel, it.n_pol, lds)) != GR_OK) return fail(st, at + gr_last_error());
  return GR_OK;
}

gr_status make_plan(const gr_batch_item* items, int n, Plan* p) {
  if (n < 0 || n > kMaxBatch) return fail(GR_EINVAL, "gr_grid_batch: n_items must be in [0, 4096]");
  if (n > 0 && items == nullptr) return fail(GR_EINVAL, "gr_grid_batch: items is NULL");
  size_t off = 0;
  p->off_table = off;    off += align256(sizeof(BatchInst) * (size_t)n);
  p->off_members = off;  off += align256(sizeof(int32_t) * (size_t)kGroups * n);
  p->off_prefix = off;   off += align256(sizeof(int32_t) * (size_t)kGroups * (n + 1));
  p->off_counters = off; off += 256;
  p->off_inst.resize(n);
  p->bins.resize(n);
  p->lds.resize(n);
  p->lds_tri.resize(n);
  p->wide.resize(n);
  p->total_blocks = 0;
  for (int i = 0; i < n; ++i) {
    const gr_batch_item& it = items[i];
    gr_status st = validate_item(it, i, &p->lds[i]);
    if (st != GR_OK) return st;
    p->lds_tri[i] = block_lds_bytes(it.kernel, it.n_pol, true);
    p->off_inst[i] = off;
    // the persistent block-form gridder works on 64-cell windows: tiles of 64 - S
    // keep its segments dense even in sparse instances; a wide item is binned
    // for the window of its support, as a single problem is
    p->wide[i] = it.n_vis >= kWideMin;
    p->bins[i] = bin_layout(it.n_vis, it.n_pol, it.kernel.support, it.height, it.width,
                            it.seg_len > 0 ? it.seg_len : kDefaultSegLen, p->wide[i] ? 0 : 64);
    if (p->bins[i].n_tiles > 0x7fffffff || p->bins[i].max_segs > 0x7fffffff)
      return fail(GR_EINVAL, "gr_grid_batch item " + std::to_string(i) + ": too many tiles");
    off += pre_size(it.n_vis, it.n_pol) + p->bins[i].bytes;
    p->total_blocks += (it.n_vis + 255) / 256;
  }
  if (p->total_blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_grid_batch: too many visibilities");
  p->bytes = off;
  return GR_OK;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

}  // namespace

}  // namespace gr

using namespace gr;

extern "C" size_t gr_grid_batch_workspace_bytes(const gr_batch_item* items, int32_t n_items) {
  Plan p;
  const std::string saved = gr_last_error();
  const gr_status st = make_plan(items, n_items, &p);
  set_error(saved);
  return st == GR_OK ? p.bytes : 0;
}

extern "C" gr_status gr_grid_batch(const gr_batch_item* items, int32_t n_items, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  Plan p;
  gr_status st = make_plan(items, n_items, &p);
  if (st != GR_OK) return st;
  if (n_items == 0) return GR_OK;
  if (workspace == nullptr) return fail(GR_EINVAL, "gr_grid_batch: workspace is NULL");
  if (workspace_bytes < p.bytes)
    return fail(GR_ENOMEM, "gr_grid_batch: workspace too small (see gr_grid_batch_workspace_bytes)");
  hipStream_t s = (hipStream_t)stream;
  char* ws = reinterpret_cast<char*>(workspace);
  auto* table = reinterpret_cast<BatchInst*>(ws + p.off_table);
  auto* members = reinterpret_cast<int32_t*>(ws + p.off_members);
  auto* prefix = reinterpret_cast<int32_t*>(ws + p.off_prefix);
  auto* counters = reinterpret_cast<int32_t*>(ws + p.off_counters);

  // descriptors, built on the host and copied into the table by setup kernels
  std::vector<BatchInst> desc(n_items);
  int64_t blk = 0;
  int n_members[kGroups] = {0, 0, 0, 0};
  size_t lds_group[kGroups] = {0, 0, 0, 0};
  size_t lds_tri_group[kGroups] = {0, 0, 0, 0};
  int64_t segs_group[kGroups] = {0, 0, 0, 0};
  for (int i = 0; i < n_items; ++i) {
    const gr_batch_item& it = items[i];
    const BinLayout& L = p.bins[i];
    BatchInst& I = desc[i];
    std::memset(&I, 0, sizeof(I));
    char* base = ws + p.off_inst[i];
    I.uvw = it.uvw;
    I.vis = it.vis;
    I.vis_scale = it.vis_scale;
    I.weights = it.weights;
    I.n_vis = it.n_vis;
    I.n_pol = it.n_pol;
    I.vis_dtype = it.vis_dtype;
    int lg_o = 0;
    while ((1 << lg_o) < it.kernel.oversample) ++lg_o;
    I.lg_o = lg_o;
    I.scale_u = it.inv_cell_u * (double)it.kernel.oversample;
    I.scale_v = it.inv_cell_v * (double)it.kernel.oversample;
    I.w_min = it.kernel.w_min;
    I.inv_dw = it.kernel.inv_dw;
    I.n_planes = it.kernel.n_planes;
    I.rec = reinterpret_cast<Record*>(base);
    I.wvis = reinterpret_cast<float2*>(base + align256(sizeof(Record) * (size_t)it.n_vis));
    I.stats = reinterpret_cast<unsigned long long*>(it.dev_stats);
    I.blk_begin = blk;
    blk += (it.n_vis + 255) / 256;
    char* bins = base + pre_size(it.n_vis, it.n_pol);
    I.n_tiles = (int32_t)L.n_tiles;
    I.seg_len = L.seg_len;
    I.brec = reinterpret_cast<Record*>(bins + L.off_rec);
    I.bwvis = reinterpret_cast<float2*>(bins + L.off_wvis);
    I.count = reinterpret_cast<int32_t*>(bins + L.off_count);
    I.cursor = reinterpret_cast<int32_t*>(bins + L.off_cursor);
    I.segs = reinterpret_cast<int4*>(bins + L.off_segs);
    I.n_segs = reinterpret_cast<int32_t*>(bins + L.off_nsegs);
    I.taps = it.kernel.taps;
    I.grid = reinterpret_cast<float2*>(it.grid);
    I.d.S = it.kernel.support;
    I.d.O = it.kernel.oversample;
    I.d.n_rows_tab = it.kernel.n_planes * it.kernel.oversample;
    I.d.tap_dtype = it.kernel.tap_dtype;
    I.d.tile = L.tile;
    I.d.n_tx = L.n_tx;
    I.d.H = it.height;
    I.d.W = it.width;
    I.d.n_blocks = (uint32_t)L.max_segs;
    if (p.wide[i]) {
      I.group = -1;                                   // not in any persistent work list
      continue;
    }
    const int g = group_of(it);
    I.group = g;
    ++n_members[g];
    lds_group[g] = std::max(lds_group[g], p.lds[i]);
    lds_tri_group[g] = std::max(lds_tri_group[g], p.lds_tri[i]);
    segs_group[g] += L.max_segs;
  }
  for (int first = 0; first < n_items; first += kSetupChunk) {
    SetupChunk c{};
    c.first = first;
    c.count = std::min(kSetupChunk, n_items - first);
    for (int j = 0; j < c.count; ++j) c.d[j] = desc[first + j];
    batch_setup_kernel<<<1, 64, 0, s>>>(c, table);
  }
  if ((st = check_launch("gr_grid_batch (setup)")) != GR_OK) return st;
  if ((st = launch_batch_preprocess(table, n_items, p.total_blocks, s)) != GR_OK) return st;
  if ((st = launch_batch_bin(table, n_items, p.total_blocks, s)) != GR_OK) return st;
  batch_prefix_kernel<<<1, 64, 0, s>>>(table, n_items, members, prefix, counters, n_items);
  if ((st = check_launch("gr_grid_batch (prefix)")) != GR_OK) return st;
  const int resident = 2 * device_cus();            // two 256-thread blocks per CU
  for (int g = 0; g < kGroups; ++g) {
    if (n_members[g] == 0) continue;
    const int n_blocks = (int)std::min<int64_t>(resident, std::max<int64_t>(segs_group[g], 1));
    // triple table entries when every member's table fits them
    const bool tri = lds_tri_group[g] <= 160 * 1024;
    st = launch_mfma_persistent(table, members + g * n_items, n_members[g], prefix + g * (n_items + 1),
                                counters + g, (g & 2) ? 4 : 1, (g & 1) != 0, tri,
                                tri ? lds_tri_group[g] : lds_group[g], n_blocks, s);
    if (st != GR_OK) return st;
  }
  for (int i = 0; i < n_items; ++i) {
    if (!p.wide[i]) continue;
    const gr_batch_item& it = items[i];
    char* bins = ws + p.off_inst[i] + pre_size(it.n_vis, it.n_pol);
    st = launch_mfma(bins, p.bins[i], it.n_pol, it.kernel, reinterpret_cast<float2*>(it.grid), it.height,
                     it.width, s);
    if (st != GR_OK) return st;
  }
  return GR_OK;
}

// ---- the batch as one HIP graph ----------------------------------------------

struct gr_graph {
  hipGraphExec_t exec;
  int device;
};

extern "C" gr_status gr_grid_batch_graph(const gr_batch_item* items, int32_t n_items, void* workspace,
                                         size_t workspace_bytes, gr_graph** out) {
  if (out == nullptr) return fail(GR_EINVAL, "gr_grid_batch_graph: out is NULL");
  *out = nullptr;
  Plan p;
  gr_status st = make_plan(items, n_items, &p);       // every item checked before anything is captured
  if (st != GR_OK) return st;
  if (n_items > 0 && workspace == nullptr) return fail(GR_EINVAL, "gr_grid_batch_graph: workspace is NULL");
  if (workspace_bytes < p.bytes)
    return fail(GR_ENOMEM, "gr_grid_batch_graph: workspace too small (see gr_grid_batch_workspace_bytes)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GR_EDEVICE, "gr_grid_batch_graph: no device");
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(GR_EDEVICE, "gr_grid_batch_graph: hipStreamCreateWithFlags failed");
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    hipStreamDestroy(s);
    return fail(GR_EDEVICE, std::string("gr_grid_batch_graph: hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  st = gr_grid_batch(items, n_items, workspace, workspace_bytes, s);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  hipStreamDestroy(s);
  if (st != GR_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess || graph == nullptr)
    return fail(GR_EDEVICE, std::string("gr_grid_batch_graph: hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess)
    return fail(GR_EDEVICE, std::string("gr_grid_batch_graph: hipGraphInstantiate: ") + hipGetErrorString(e));
  *out = new gr_graph{exec, dev};
  return GR_OK;
}

extern "C" gr_status gr_graph_launch(gr_graph* g, void* stream) {
  if (g == nullptr) return fail(GR_EINVAL, "gr_graph_launch: graph is NULL");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(GR_EDEVICE, std::string("gr_graph_launch: ") + hipGetErrorString(e));
  return GR_OK;
}

extern "C" gr_status gr_graph_destroy(gr_graph* g) {
  if (g == nullptr) return GR_OK;
  const hipError_t e = hipGraphExecDestroy(g->exec);
  delete g;
  if (e != hipSuccess) return fail(GR_EDEVICE, std::string("gr_graph_destroy: ") + hipGetErrorString(e));
  return GR_OK;
}
