// Internal declarations shared by the gridding library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "gridder.h"

namespace gr {

// Thread-local error message for gr_last_error().
void set_error(const std::string& msg);
gr_status fail(gr_status st, const std::string& msg);
gr_status check_launch(const char* what);
// Raise a kernel's dynamic LDS limit to at least `bytes` (once per kernel,
// device and size; never inside a later captured launch).
gr_status ensure_lds_limit(const void* fn, size_t bytes, const char* what);

// Packed per-visibility record written by the preprocess kernel.
//   x = x0 | y0 << 16            (footprint origin, cells)
//   y = sx | sy << 8 | plane << 16 | valid << 31
struct Record {
  uint32_t x, y;
};
static_assert(sizeof(Record) == 8, "record must be 8 bytes");

constexpr uint32_t kValidBit = 0x80000000u;
constexpr int kMaxGrid = 32768;   // x0, y0 fit in 16 bits
constexpr int kMaxPlanes = 32767; // 15 bits
constexpr int kMaxOversample = 128;

__host__ __device__ inline int rec_x0(Record r) { return (int)(r.x & 0xffffu); }
__host__ __device__ inline int rec_y0(Record r) { return (int)(r.x >> 16); }
__host__ __device__ inline int rec_sx(Record r) { return (int)(r.y & 0xffu); }
__host__ __device__ inline int rec_sy(Record r) { return (int)((r.y >> 8) & 0xffu); }
__host__ __device__ inline int rec_plane(Record r) { return (int)((r.y >> 16) & 0x7fffu); }
__host__ __device__ inline bool rec_valid(Record r) { return (r.y & kValidBit) != 0; }

// Host-side validation of a kernel descriptor (shared by preprocess and grid).
gr_status validate_kernel(const gr_kernel* k, bool need_taps);

// The library's tuning memo (api.hip): slot 0 is read by gr_grid, slot 1 by
// gr_grid_records, when they are called without a tuning.
void memo_store(int n_pol, const gr_kernel& k, int height, int width, int slot, const gr_tuning& t);
bool memo_find(int n_pol, const gr_kernel& k, int height, int width, int slot, gr_tuning* out);

// Preprocess launcher (preprocess.hip).
gr_status launch_preprocess(const double* uvw, const void* vis, int vis_dtype, const float* vis_scale,
                            const float* weights, int64_t n_vis, int n_pol, const gr_kernel& k,
                            double inv_cell_u, double inv_cell_v, int height, int width,
                            Record* records, float2* wvis, int64_t* dev_stats, hipStream_t stream);

// Romein / thread-coarsening VALU gridder (grid_romein.hip).
struct RomeinPlan {
  int cu, cv;          // coarsening (cells per block, per axis)
  int nu, nv;          // blocks per bin, per axis (bin = c * n >= S + c - 1)
  int wgu, wgv;        // residue order: tiles of wgu x wgv blocks take consecutive lanes
  int vis_per_wg;      // visibilities per work-item chunk (0: equal ranges)
  int threads;         // threads per block (one block per compute unit)
  int lpad, pad_off;   // padded tap row length and offset in LDS
  size_t lds_bytes;
};
gr_status plan_romein(const gr_kernel& k, int n_pol, const gr_tuning* t, RomeinPlan* plan);
// counter (device int32, or NULL): work counter for a dynamic assignment of
// the 64-lane runs to waves; NULL: a fixed assignment (stride over the launch)
gr_status launch_romein(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol,
                        const gr_kernel& k, float2* grid, int height, int width,
                        const RomeinPlan& plan, hipStream_t stream, int32_t* counter = nullptr);

// Binning of the preprocessed stream by footprint tile (bin.hip).
struct BinLayout {
  int tile, n_tx, n_ty, seg_len;
  int64_t n_tiles, max_segs;
  size_t off_rec, off_wvis, off_count, off_cursor, off_segs, off_nsegs, off_scan, off_perm, bytes;
};
// tile edge T (cells): footprints of a tile fit the MFMA gridder's window of T + S
// cells (32, 48 or 64), and always the 64-cell window of the other binned gridders
// window = 0: the single-problem gridder's window for the support (32, 48 or
// 64 cells); batches bin for the 64-cell window of their block-form gridder.
int binned_tile(int support, int window = 0);
BinLayout bin_layout(int64_t n_vis, int n_pol, int support, int height, int width, int seg_len,
                     int window = 0);
// Preprocess and bin in one pass pair straight from the raw inputs (the
// binned stream of launch_bin in `bins`; rec_tmp: n_vis unbinned records).
gr_status launch_preprocess_bin(const double* uvw, const void* vis, int vis_dtype, const float* vis_scale,
                                const float* weights, int64_t n_vis, int n_pol, const gr_kernel& k,
                                double inv_cell_u, double inv_cell_v, int height, int width, const BinLayout& L,
                                void* bins, Record* rec_tmp, int64_t* dev_stats, hipStream_t stream,
                                const int32_t* ids = nullptr, int n_ids = 0);
// Gridding with per-visibility, per-polarisation non-separable GCFs over a
// binned stream whose records carry id * n_planes + plane (aterm.hip).
gr_status launch_aterm(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k, float2* grid,
                       int height, int width, hipStream_t stream);
// the window (cells) that gr_grid_aterm bins for: 32, 48 or 64
int aterm_window(int support);
// Compression of a preprocessed stream (compress.hip): runs of consecutive kept
// visibilities with equal records summed into one; out_rec padded with invalid
// records to n_vis; the number of runs to *out_count (device, may be NULL).
size_t compress_workspace_bytes(int64_t n_vis);
gr_status launch_compress(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol, Record* out_rec,
                          float2* out_wvis, int64_t* out_count, void* workspace, hipStream_t stream);
// Exclusive scan of n int32 counts in place (total < 2^31); the total to
// *total (device int64) when it is non-NULL.  scratch: scan_i32_scratch_bytes(n)
// of device memory for the two-level form (used when n > 16384).
size_t scan_i32_scratch_bytes(int64_t n);
void launch_scan_i32(int32_t* data, int n, int64_t* total, int32_t* scratch, hipStream_t stream);
// W-stacking's split (wstack.hip): stable partition of (uvw, vis, weights) by
// w slice; slice_offsets [n_slices + 1] (device int64).
size_t wslice_workspace_bytes(int64_t n_vis, int n_slices);
gr_status launch_wslice_partition(const double* uvw, const float2* vis, const float* wts, int64_t n_vis, int n_pol,
                                  double w_first, double inv_width, int n_slices, double* uvw_out,
                                  float2* vis_out, float* wts_out, int64_t* slice_offsets, void* workspace,
                                  hipStream_t stream);
// Degridding's binning: records (rec_tmp) and tile counts from uvw, scan,
// then kept records and their input indices (int32, in the wvis slot of the
// layout) to the binned positions.
gr_status launch_degrid_bin(const double* uvw, int64_t n_vis, int n_pol, const gr_kernel& k, double inv_cell_u,
                            double inv_cell_v, int height, int width, const BinLayout& L, void* bins,
                            Record* rec_tmp, float2* vis_out, int64_t* dev_stats, hipStream_t stream);
// The degridder on such a binned stream (degrid.hip); vis_out complex64
// [n_vis][n_pol], valid entries written, the caller zeroes the rest.
gr_status plan_degrid(const gr_kernel& k, int n_pol, size_t* lds_bytes);
gr_status launch_degrid(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                        const float2* grid, int height, int width, float2* vis_out, int64_t n_vis,
                        hipStream_t stream);
gr_status launch_bin(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol,
                     const BinLayout& L, void* bins, hipStream_t stream);

// MFMA gridder over the binned stream (grid_mfma.hip).
gr_status plan_mfma(const gr_kernel& k, int n_pol, size_t* lds_bytes);
// LDS bytes of the block-form MFMA gridder: tri = (-Im, Re, Im) table entries
// (the form used where they fit), else (Re, Im) pairs (what plan_mfma checks)
size_t block_lds_bytes(const gr_kernel& k, int n_pol, bool tri);
// ng: row groups per wave of the wave form (<= 0: the default for the window)
gr_status launch_mfma(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                      float2* grid, int height, int width, hipStream_t stream, int ng = 0);

// gr_grid_binned with the wave form's row groups per wave (api.hip; ng as
// launch_mfma; ng < 0: the memo's variant-2 entry for the problem class, if any).
gr_status grid_binned(const void* bins, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel, int32_t seg_len,
                      void* grid, int32_t height, int32_t width, void* stream, int ng);
// The binned gridder for the kernel's kind (api.hip); ng as launch_mfma.
gr_status launch_binned(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                        float2* grid, int height, int width, hipStream_t stream, int ng = 0);

// Non-separable table gridder over the binned stream (aterm.hip).
gr_status launch_table2d(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                         float2* grid, int height, int width, hipStream_t stream);

// Learned-tap (network) gridder over the binned stream (mlp.hip).
gr_status launch_grid_mlp(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                          float2* grid, int height, int width, hipStream_t stream);

constexpr int kDefaultSegLen = 4096;
// largest support of the binned gridders: footprints must fit the 64-cell window
// with a tile of at least 8 cells
constexpr int kMaxBinnedSupport = 56;
size_t align256(size_t v);

// Launch parameters of the MFMA gridder (grid_mfma.hip).
struct MfmaDev {
  int S, O, n_rows_tab, tap_dtype, tile, n_tx, H, W;
  uint32_t n_blocks;
};

// ---- Batches of independent gridding problems (batch.hip) -------------------
// Device descriptor of one instance: every batched kernel reads its instance's
// pointers and sizes from a table of these in the workspace.
struct BatchInst {
  // preprocess
  const double* uvw;
  const void* vis;
  const float* vis_scale;
  const float* weights;
  int64_t n_vis;
  int32_t n_pol, vis_dtype;
  double scale_u, scale_v, w_min, inv_dw;
  int32_t lg_o, n_planes;
  Record* rec;                   // preprocess output
  float2* wvis;
  unsigned long long* stats;     // may be NULL
  int64_t blk_begin;             // first block of this instance in the batched per-visibility launches
  // binning (bin.hip layout, per instance)
  int32_t n_tiles, seg_len;
  Record* brec;
  float2* bwvis;
  int32_t* count;
  int32_t* cursor;
  int4* segs;
  int32_t* n_segs;
  // gridding
  const void* taps;
  float2* grid;
  MfmaDev d;                     // d.tile, d.n_tx are the binning tile and tiles per row
  int32_t group;                 // persistent launch group: (n_pol == 4) * 2 + complex taps
  int32_t pad_;
};
static_assert(sizeof(BatchInst) % 8 == 0, "descriptors are copied as 8-byte words");

// Instance whose block range holds block b (blk_begin ascending, first one 0).
__device__ inline int batch_find(const BatchInst* inst, int n_inst, int64_t b) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].blk_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

gr_status launch_batch_preprocess(const BatchInst* inst, int n_inst, int64_t total_blocks,
                                  hipStream_t stream);
gr_status launch_batch_bin(const BatchInst* inst, int n_inst, int64_t total_blocks,
                           hipStream_t stream);
// Persistent MFMA gridder over the segments of the instances `members`
// (group_prefix: [n_members + 1] exclusive prefix of their segment counts,
// written on the device; counter: zeroed work counter).  The gridder works on
// 64-cell windows; tri selects the triple-entry tap table (block_lds_bytes with
// tri = true must fit every member), lds_bytes is the largest member's need.
gr_status launch_mfma_persistent(const BatchInst* inst, const int32_t* members, int n_members,
                                 const int32_t* group_prefix, int32_t* counter, int n_pol,
                                 bool complex_taps, bool tri, size_t lds_bytes, int n_blocks,
                                 hipStream_t stream);

}  // namespace gr
