/*
 * gridder.h -- C ABI of the MI355X (gfx950) convolutional gridding library.
 *
 * Method: B. Merry, "Faster GPU-based convolutional gridding via thread
 * coarsening" (Astronomy and Computing, 2016; arXiv:1605.07023).
 *
 * Conventions shared by every entry point
 *   - Pointers named dev_* or described as "device" are device (HBM) pointers
 *     owned by the caller; the library keeps no reference after the call
 *     returns, allocates no device memory, and never synchronises the device.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is only enqueued on it.
 *   - Every argument is validated on the host before anything is enqueued.
 *     A non-OK status means nothing was enqueued (except GR_EDEVICE, which
 *     reports a failed launch).  gr_last_error() returns a thread-local
 *     message for the last non-OK status.  The library never aborts.
 *   - complex64 is interleaved (re, im) float32, the layout of torch.complex64.
 *   - Grid layout: complex64 [P][H][W], row-major; cell (y, x) with uv = 0 at
 *     (H/2, W/2), u along x (columns), v along y (rows).
 */
#ifndef GRIDDER_H
#define GRIDDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GR_OK = 0,
  GR_EINVAL = -1,       /* invalid argument (null pointer, bad size, ...) */
  GR_ENOMEM = -2,       /* workspace too small */
  GR_EDEVICE = -3,      /* HIP launch or runtime error */
  GR_EUNSUPPORTED = -4  /* valid but not supported by this build (e.g. table too large) */
} gr_status;

typedef enum { GR_F32 = 0, GR_F16 = 1, GR_BF16 = 2, GR_F64 = 3 } gr_dtype;

typedef enum { GR_SEPARABLE = 0, GR_TABLE2D = 1, GR_MLP = 2 } gr_kernel_kind;

/* Gridding convolution function (GCF) description (Section 2.2: precomputed
 * tables sampled at `oversample` times the grid resolution; Section 4: a
 * separable GCF, G_ij = G^u_i G^v_j, the same for every polarisation).
 *
 * A visibility at pixel position p = ix + s/O (see gr_preprocess) has footprint
 * cells ix - S/2 + 1 ... ix + S/2 on each axis; tap k of phase s multiplies
 * cell ix - S/2 + 1 + k and samples the GCF at k - S/2 + 1 - s/O.
 *
 * taps (device):
 *   GR_SEPARABLE: [n_planes][O][S] elements, used along u and along v;
 *   GR_TABLE2D:   [n_planes][O][O][S][S] indexed [plane][s_v][s_u][k_v][k_u].
 *   GR_MLP:       the FP32 weight blob of a learned tap network (see
 *                 gr_mlp_eval); tap_dtype must be GR_F32 and taps_complex 1.
 *                 The plane index p of a visibility enters the network as
 *                 x0 = blob[0] + p * blob[1], so n_planes may be a fine grid
 *                 in w (up to 32767 planes), and oversample up to 128, at no
 *                 memory cost.
 * Element type `tap_dtype` (GR_F32, GR_F16 or GR_BF16); complex taps are
 * (re, im) pairs of that type. */
typedef struct {
  int32_t kind;          /* gr_kernel_kind */
  int32_t tap_dtype;     /* gr_dtype of each tap component */
  int32_t taps_complex;  /* 1: complex taps, 0: real taps */
  int32_t support;       /* S: even, 2..64 */
  int32_t oversample;    /* O: power of two, 1..128 */
  int32_t n_planes;      /* >= 1; plane index selected from w when > 1 */
  double w_min;          /* plane = rint((w - w_min) * inv_dw) in FP64 */
  double inv_dw;
  const void* taps;      /* device */
} gr_kernel;

/* Work-decomposition parameters (Sections 3-4 and the autotuning of
 * Section 4).  Any field <= 0 selects the library default for it.
 *   cu, cv      thread-coarsening factors: each work-item owns a cu x cv block
 *               of cells (Section 3); 1, 2, 4 or 8
 *   wg_u, wg_v  VALU kernel: the bin's blocks are visited in tiles of
 *               wg_u x wg_v blocks (Section 2.2 tiles; u first, edge tiles
 *               clipped), and consecutive work-items of a visibility chunk
 *               take consecutive blocks in that order; <= 64 each (default:
 *               the whole bin, row by row).  MFMA kernel, with variant = 2
 *               given explicitly: wg_v is the number of 4-row (n_pol = 4) or
 *               16-row (n_pol = 1) groups of the window one wave accumulates
 *               (the work-group shape of the wave form: 2, 4 or 8 for the
 *               32-cell window, 2, 3, 4 or 6 for 48, 2 or 4 for 64 at
 *               n_pol = 4; 1 or 2, 1 or 3, 1, 2 or 4 at n_pol = 1); other
 *               values give GR_EUNSUPPORTED
 *   vis_per_wg  visibilities per work-item chunk (Section 4 uses 1024 per
 *               work-group; default: equal chunks, about four 64-lane runs
 *               per wave) for the VALU kernel; maximum segment length for the
 *               binned MFMA kernel
 *   variant     0 = library choice, 1 = VALU work-item kernel on the input
 *               order (gr_grid_records), 2 = MFMA kernel on the binned stream
 * A NULL tuning means the library's tuning memo (gr_tuning_memo_put), else
 * the defaults. */
typedef struct {
  int32_t cu, cv, wg_u, wg_v, vis_per_wg, variant;
} gr_tuning;

/* Preprocess (Section 4: the gridder's per-visibility inputs -- cell, phase
 * into the oversampled GCF, w plane, weighted values -- are computed in a pass
 * of their own before gridding).  Per visibility n, in FP64:
 *   fx = rint(u * (inv_cell_u * O)) + (W/2) O   (round half to even)
 *   ix = fx >> log2 O, sx = fx & (O - 1), x0 = ix - S/2 + 1   (likewise v, y)
 *   plane = rint((w - w_min) * inv_dw), or 0 when n_planes == 1.
 * A visibility is dropped (record marked invalid, counted) when any of its
 * u, v, w, visibility or weight values is not finite, its plane is outside
 * [0, n_planes), or its footprint leaves the H x W grid.
 *
 *   uvw       device f64 [n_vis][3], wavelengths
 *   vis       device [n_vis][n_pol] complex: vis_dtype GR_F32 = complex64;
 *             GR_F16 = (re, im) float16 pairs scaled by vis_scale[n / 256]
 *   vis_scale device f32 [ceil(n_vis / 256)] (GR_F16 only, else NULL)
 *   weights   device f32 [n_vis][n_pol] or NULL (all ones)
 *   records   device out, 8 bytes per visibility: two uint32,
 *             {x0 | y0 << 16} and {sx | sy << 8 | plane << 16 | valid << 31}
 *   wvis      device out, complex64 [n_vis][n_pol] weighted visibilities
 *   dev_stats device int64 [2] or NULL: {gridded, dropped} are ADDED to it */
gr_status gr_preprocess(const double* uvw, const void* vis, int32_t vis_dtype,
                        const float* vis_scale, const float* weights, int64_t n_vis,
                        int32_t n_pol, const gr_kernel* kernel, double inv_cell_u,
                        double inv_cell_v, int32_t height, int32_t width, void* records,
                        void* wvis, int64_t* dev_stats, void* stream);

/* Grid preprocessed visibilities (records/wvis from gr_preprocess, in the same
 * order as the input) onto grid, complex64 [n_pol][height][width], which is
 * ACCUMULATED into (+=).  This is the Romein work distribution with thread
 * coarsening (Sections 2.2-4): one work-item per (chunk of consecutive
 * visibilities, residue of the bin); each keeps a register block of
 * cu x cv cells per polarisation and flushes it with atomic adds when the
 * block leaves the bounding box, and at the end of the chunk.  One block per
 * compute unit stages the tap table in LDS once.  tuning may be NULL (the
 * memo's slot 1 entry for this problem class, else defaults); cu * cv * n_pol
 * <= 64. */
gr_status gr_grid_records(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                          const gr_kernel* kernel, void* grid, int32_t height, int32_t width,
                          const gr_tuning* tuning, void* stream);

/* Size in bytes of the `bins` buffer of gr_bin / gr_grid_binned (0 if the
 * arguments are invalid), including 4 bytes per visibility for the pairing
 * order that gr_grid_binned writes.  seg_len <= 0 selects the default (4096). */
size_t gr_bin_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height, int32_t width,
                    int32_t seg_len);

/* Bin preprocessed visibilities by footprint position.  The grid is cut into
 * square tiles of T = W - S cells, W = 32 for S <= 16, 48 for S <= 32, else 64;
 * each valid visibility goes to the tile that holds its footprint origin
 * (x0, y0), so every footprint of a tile lies in a W x W-cell window.  The input order (the baseline-ordered stream of
 * Section 4) is kept within each run of 64 consecutive visibilities of a
 * tile; each tile's list is cut into segments of at most seg_len entries.
 * bins (device, gr_bin_bytes) receives the reordered records, the reordered
 * weighted visibilities and the segment table.  support <= 56; n_vis < 2^31. */
gr_status gr_bin(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                 int32_t support, int32_t height, int32_t width, int32_t seg_len, void* bins,
                 size_t bins_bytes, void* stream);

/* Size in bytes of the `bins` buffer of gr_preprocess_bin: gr_bin_bytes plus
 * 8 bytes per visibility, 256-aligned (0 if the arguments are invalid). */
size_t gr_preprocess_bin_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                               int32_t width, int32_t seg_len);

/* gr_preprocess followed by gr_bin without the intermediate weighted
 * visibilities (Section 4's preprocessing, and the binning of gr_bin): a
 * first pass reads only uvw and writes the records and the per-tile counts,
 * a second pass reads each kept record with its visibilities and weights and
 * writes both, weighted, to the binned position.  The first gr_bin_bytes
 * bytes of bins then hold exactly what gr_bin would write (the input to
 * gr_grid_binned with the same n_vis, n_pol, support, height, width and
 * seg_len); the rest holds the unbinned records.  A visibility whose values
 * or weights are not finite is dropped as by gr_preprocess: it is counted as
 * dropped in dev_stats and contributes nothing, but keeps a slot of zero
 * values in its tile list.  Arguments as gr_preprocess and gr_bin;
 * bins_bytes >= gr_preprocess_bin_bytes; support <= 56; n_vis < 2^31.
 * About 112 bytes of HBM traffic per quad-polarisation visibility against
 * 184 for gr_preprocess + gr_bin. */
gr_status gr_preprocess_bin(const double* uvw, const void* vis, int32_t vis_dtype,
                            const float* vis_scale, const float* weights, int64_t n_vis,
                            int32_t n_pol, const gr_kernel* kernel, double inv_cell_u,
                            double inv_cell_v, int32_t height, int32_t width, int32_t seg_len,
                            void* bins, size_t bins_bytes, int64_t* dev_stats, void* stream);

/* Grid a binned stream (gr_bin output; the same n_vis, n_pol, support,
 * height, width and seg_len) onto grid (+=).  Per segment, the W x W-cell
 * window is accumulated in matrix-core registers: the separable tile update
 * of Section 4, in the factored form G^u_i (G^v_j V_p) of Section 6, is a
 * rank-2 product per pair of visibilities (v_mfma_f32_16x16x4_f32), and the
 * window is added to the grid once with FP32 atomic adds (Section 2.2).
 * The tap table is staged in LDS once per block: one block per compute unit
 * (1024 threads; 768 for W = 32 with n_pol = 4) whose waves take (segment,
 * row part) work from a counter in the bins workspace and stage their own
 * visibility batches, or, when the table leaves too little LDS for that, one
 * 256-thread block per segment.  The first form pairs consecutive
 * visibilities of an order that a small kernel writes into the bins
 * workspace first: each segment sorted by the D tiles its footprints touch
 * (first row group, first column group, and whether a footprint reaches one
 * more of each), so that the two visibilities of a pair mostly touch the same
 * tiles.  The call therefore writes to bins (the counter and that order);
 * calls that share one bins buffer must not overlap.  The first form keeps W - S zero entries after
 * every table row (and before the first), so that no operand address needs a
 * clamp: W - S + planes x O x W entries of 12 bytes ((-Im, Re, Im)) where that
 * fits beside the waves' staging (32 pair records each, 1.3 to 3.8 KiB),
 * else of 8 bytes ((Re, Im)).
 * The number of row groups one wave accumulates comes from the tuning memo's
 * slot 0 entry for this problem class when that entry is a variant-2 tuning
 * (its wg_v; see gr_tuning), else the default for the window.
 * support <= 56; the FP32 tap table [planes][O][S + 2] as (Re, Im) pairs plus
 * 12 KiB of staging must fit in 160 KiB.
 * With a GR_TABLE2D kernel the non-separable taps are read per visibility
 * from the [planes][O][O][S][S] table instead: one 256-work-item block per
 * segment keeps the window in registers, C x C cells per polarisation and
 * work-item (C = window / 16).  With a GR_MLP kernel
 * the block evaluates each visibility's S x S taps with the network into LDS
 * first (FP16 matrix-core layers, FP32 accumulation), then updates the window
 * the same way. */
gr_status gr_grid_binned(const void* bins, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                         int32_t seg_len, void* grid, int32_t height, int32_t width, void* stream);

/* Compression (Section 2.2, after Muscat; Section 4 applies it once, in the
 * preprocess): adjacent visibilities at the same position of the oversampled
 * grid and in the same w plane meet the same GCF samples and are added into
 * one.  Here "adjacent" is consecutive in the stream of gr_preprocess, and a
 * dropped visibility separates runs.  records / wvis: gr_preprocess output
 * (n_vis entries, input order).  out_records / out_wvis (same layouts and
 * sizes, must not overlap the inputs) receive the compressed stream first, one
 * entry per run in input order with the run's weighted visibilities summed in
 * input order (deterministic), then invalid records up to n_vis (their
 * out_wvis slots are left unwritten), so that gr_bin and gr_grid_binned take
 * them with the same n_vis and no host synchronisation; gridding them gives the grid of the input up to FP32
 * rounding.  out_count (device int64, or NULL) receives the number of runs
 * (overwritten).  workspace: gr_compress_workspace_bytes(n_vis). */
size_t gr_compress_workspace_bytes(int64_t n_vis);
gr_status gr_compress(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                      void* out_records, void* out_wvis, int64_t* out_count, void* workspace,
                      size_t workspace_bytes, void* stream);

/* W-stacking's split (Section 5 grids the data as a stack of slices by w,
 * one problem per slice, each with a GCF for the w offset from the slice's
 * centre): a stable partition of the stream by
 *   slice = floor((w - w_first) * inv_width)         (FP64)
 * into 1 <= n_slices <= 255 slices.  uvw [n_vis][3] f64, vis complex64
 * [n_vis][n_pol], weights f32 [n_vis][n_pol] or NULL (device, input order)
 * are copied to uvw_out / vis_out / weights_out (same layouts and sizes;
 * weights_out is needed exactly when weights is given; none may overlap an
 * input): slice 0's visibilities first, in input order, then slice 1's, and
 * so on, then those whose slice falls outside [0, n_slices) or whose w is not
 * finite, in input order.  The output is a permutation of the input, moved
 * bit for bit.  slice_offsets (device int64 [n_slices + 1], overwritten):
 * slice s occupies [slice_offsets[s], slice_offsets[s + 1]) for s < n_slices
 * (with slice_offsets[n_slices] the first visibility outside every slice),
 * which lets each slice be gridded as its own problem (gr_grid_batch items
 * pointing into the outputs) with the kernel's w_min moved to that slice.
 * No host synchronisation.  workspace: gr_wslice_partition_workspace_bytes. */
size_t gr_wslice_partition_workspace_bytes(int64_t n_vis, int32_t n_slices);

/* The GCF descriptor of W-stacking slice `slice` (Section 5: each slice has
 * its own GCF for the w offset from the slice's centre): *out is a copy of
 * *table, whose plane rule is relative to the centre, with w_min moved there,
 *   out->w_min = w_first + (slice + 1/2) / inv_width + table->w_min   (FP64),
 * so that plane = rint((w - out->w_min) * inv_dw) for the slice's
 * visibilities.  w_first and inv_width as gr_wslice_partition; 0 <= slice <=
 * 254.  Host-only. */
gr_status gr_wslice_kernel(const gr_kernel* table, double w_first, double inv_width, int32_t slice,
                           gr_kernel* out);
gr_status gr_wslice_partition(const double* uvw, const void* vis, const float* weights, int64_t n_vis,
                              int32_t n_pol, double w_first, double inv_width, int32_t n_slices,
                              double* uvw_out, void* vis_out, float* weights_out, int64_t* slice_offsets,
                              void* workspace, size_t workspace_bytes, void* stream);

/* Gridding with non-separable GCFs that change per visibility and per
 * polarisation, as A-projection's do (Section 6: they depend on time,
 * frequency, polarisation and possibly baseline and are not separable; the
 * paper expects their loads to dominate).  Each visibility n carries a GCF id
 * kernel_id[n] (device int32 [n_vis]; for instance its time and frequency
 * interval); with the indices of gr_preprocess,
 *   grid[p][y0+ky][x0+kx] += w[n][p] V[n][p] T[kernel_id[n]][plane][sy][sx][p][ky][kx]
 * where `kernel` is a GR_TABLE2D descriptor (complex taps, FP32/FP16/BF16,
 * support <= 56) whose table holds n_ids x n_planes x O x O x n_pol x S x S
 * complex values in that order (polarisation-dependent; each correlation
 * has its own GCF, no mixing between them), n_ids x n_planes <= 32767.  A
 * visibility whose id falls outside [0, n_ids) is dropped and counted like
 * one off the grid.  uvw, vis, vis_dtype, vis_scale, weights, dev_stats, grid
 * (accumulated, +=) as gr_grid.  The visibilities are preprocessed and binned
 * in one pass pair for windows of 32, 48 or 64 cells (S <= 16, <= 32, else),
 * then one 256-work-item block per segment keeps its window in registers
 * (C x C cells x n_pol per work-item, C = window / 16) and adds it to the grid
 * once with atomic adds.
 * workspace: gr_grid_aterm_workspace_bytes. */
size_t gr_grid_aterm_workspace_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                                     int32_t width);
gr_status gr_grid_aterm(const double* uvw, const void* vis, int32_t vis_dtype, const float* vis_scale,
                        const float* weights, const int32_t* kernel_id, int32_t n_ids, int64_t n_vis,
                        int32_t n_pol, const gr_kernel* kernel, double inv_cell_u, double inv_cell_v,
                        void* grid, int32_t height, int32_t width, void* workspace, size_t workspace_bytes,
                        int64_t* dev_stats, void* stream);

/* Degridding, the adjoint of gridding (Section 6 names degridding with thread
 * coarsening as the next step): predicts every visibility from the grid
 * through the same separable GCF,
 *   vis_out[n][p] = sum_{ky,kx} Tv[plane][sy][ky] Tu[plane][sx][kx] grid[p][y0+ky][x0+kx]
 * with the indices of gr_preprocess.  With the complex-conjugated taps it is
 * the exact adjoint of gr_grid for unit weights.  vis_out (device, complex64
 * [n_vis][n_pol]) is OVERWRITTEN; visibilities dropped by the coordinate rule
 * of gr_preprocess get 0, and dev_stats (or NULL) receives {kept, dropped}
 * (added).  The visibilities are binned as for gr_grid_binned (seg_len as
 * there, at most 4096) and each segment is put in Z (Morton) order of its
 * footprint origins; then one 1024-thread block per compute unit stages the tap table
 * once and, per segment, the grid window of all polarisations in LDS; waves
 * contract it with the G^u rows of 8 visibilities at a time on the matrix
 * cores (v_mfma_f32_16x16x4_f32) and apply the G^v taps per row.  Each
 * visibility is written once (deterministic; no atomics).  kernel: separable,
 * support <= 56, (window x window x n_pol) complex64 plus the (Re, Im) tap
 * table [planes][O][S + 2] must fit in 160 KiB of LDS (window 32 for S <= 16,
 * 48 for S <= 32, else 64).  workspace: gr_degrid_workspace_bytes. */
size_t gr_degrid_workspace_bytes(int64_t n_vis, int32_t n_pol, int32_t support, int32_t height,
                                 int32_t width, int32_t seg_len);
gr_status gr_degrid(const double* uvw, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                    double inv_cell_u, double inv_cell_v, const void* grid, int32_t height,
                    int32_t width, void* vis_out, int32_t seg_len, void* workspace,
                    size_t workspace_bytes, int64_t* dev_stats, void* stream);

/* Bytes of workspace gr_grid needs (depends on the variant gr_grid selects
 * for these arguments, a NULL tuning read from the memo as gr_grid does; 0
 * if they are invalid). */
size_t gr_grid_workspace_bytes(int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                               int32_t height, int32_t width, const gr_tuning* tuning);

/* The whole hot path: either gr_preprocess into `workspace` then the kernel
 * of gr_grid_records (variant 1; its waves take their work in turn from a
 * counter at the end of the workspace), or gr_preprocess_bin into `workspace` then
 * gr_grid_binned (variant 2; chosen by default when the kernel allows it).
 * Same semantics as those calls.  A NULL tuning takes the memo's slot 0
 * entry for this problem class (gr_tuning_memo_put), else the defaults. */
gr_status gr_grid(const double* uvw, const void* vis, int32_t vis_dtype, const float* vis_scale,
                  const float* weights, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                  double inv_cell_u, double inv_cell_v, void* grid, int32_t height,
                  int32_t width, const gr_tuning* tuning, void* workspace,
                  size_t workspace_bytes, int64_t* dev_stats, void* stream);

/* gr_grid for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments and result as gr_grid without `workspace`, which comes from
 * a static device array of gr_grid_noalloc_scratch_bytes() bytes (64 MiB)
 * that the library holds on every device it runs on until the process ends
 * (its address is looked up once per device, on the first call there).
 * Calls whose gr_grid_workspace_bytes exceeds it return GR_ENOMEM before
 * anything is enqueued: with n_pol = 4, about 1.26 million visibilities on a
 * 4096^2 grid.  Nothing is allocated and no allocating routine is called.
 * Every call on one device shares that device's array, and the kernels
 * clear what must start at zero; calls that overlap on one device (other
 * streams, other threads) race on it and must be serialised by the caller. */
size_t gr_grid_noalloc_scratch_bytes(void);
gr_status gr_grid_noalloc(const double* uvw, const void* vis, int32_t vis_dtype, const float* vis_scale,
                          const float* weights, int64_t n_vis, int32_t n_pol, const gr_kernel* kernel,
                          double inv_cell_u, double inv_cell_v, void* grid, int32_t height,
                          int32_t width, const gr_tuning* tuning, int64_t* dev_stats, void* stream);

/* Autotuning (Section 4: the work decomposition is chosen by timing a
 * synthetic problem under many coarsening and work-group settings).
 * Times each of n_candidates tunings on preprocessed records/wvis: variant 1
 * candidates with gr_grid_records, others with gr_bin (into `bins`, sized for
 * the largest seg_len = vis_per_wg among them) + gr_grid_binned, `reps` times
 * after one warm-up, accumulating into `grid` (scratch: its contents become
 * meaningless).  times_ms[c] receives the mean time (+inf when the candidate
 * is unsupported); *best the fastest index.  Unlike every other entry point
 * this one SYNCHRONISES `stream` (once per candidate).  The winner is stored
 * in the tuning memo for (n_pol, kernel, height, width): slot 0 (with its
 * variant made explicit), and the fastest variant-1 candidate in slot 1. */
gr_status gr_autotune(const void* records, const void* wvis, int64_t n_vis, int32_t n_pol,
                      const gr_kernel* kernel, void* grid, int32_t height, int32_t width,
                      void* bins, size_t bins_bytes, const gr_tuning* candidates,
                      int32_t n_candidates, int32_t reps, float* times_ms, int32_t* best,
                      void* stream);

/* The library's tuning memo (Section 4: the autotuner's choice is remembered
 * and used again).  An entry is keyed by the current device, n_pol, the
 * kernel's kind, taps_complex, tap_dtype and support, the grid's side class
 * (the power of two >= max(height, width)) and a slot: slot 0 is read by
 * gr_grid and gr_grid_workspace_bytes, slot 1 by gr_grid_records, when their
 * tuning is NULL.  gr_autotune writes both; gr_tuning_memo_put writes one
 * (slot 1 takes variant 0 or 1).  gr_tuning_memo_get copies an entry to *out
 * (GR_EINVAL when there is none).  Entries last until gr_tuning_memo_clear
 * or the end of the process; callers that keep tunings across processes
 * read them out and put them back.  Host-only (the kernel's taps pointer is
 * not used), thread-safe; a change of the memo between
 * gr_grid_workspace_bytes and gr_grid can make gr_grid report GR_ENOMEM. */
gr_status gr_tuning_memo_put(int32_t n_pol, const gr_kernel* kernel, int32_t height, int32_t width,
                             int32_t slot, const gr_tuning* tuning);
gr_status gr_tuning_memo_get(int32_t n_pol, const gr_kernel* kernel, int32_t height, int32_t width,
                             int32_t slot, gr_tuning* out);
void gr_tuning_memo_clear(void);

/* Kaiser-Bessel taps (real, one plane), evaluated in FP64 on the device and
 * stored as out_dtype (GR_F64, GR_F32, GR_F16 or GR_BF16), layout [O][S]:
 *   tap[s][k] = I0(beta sqrt(1 - (2 d / S)^2)) / I0(beta) for |d| < S/2 else 0,
 *   d = k - S/2 + 1 - s/O.
 * (Section 2.2: an anti-aliasing GCF tabulated with oversampling.) */
gr_status gr_make_kb_table(double beta, int32_t support, int32_t oversample, int32_t out_dtype,
                           void* out, void* stream);

/* Separable W-projection taps (Section 2.2 treats the w term as a
 * convolution; Section 4 uses a separable approximation), complex, evaluated
 * in FP64 on the device, layout [n_planes][O][S] of (re, im) out_dtype pairs:
 *   g(d) = c * sum_{j<M} t(nu_j) exp(-i pi w_hat nu_j^2) exp(-2 pi i d nu_j)
 * with nu_j = (j + 1/2)/M - 1/2, t the image response of a Kaiser-Bessel
 * window of width support_aa and shape beta, w_hat = w_hat_first + plane *
 * w_hat_step (w in pixel units), M = n_samples (<= 0: 4 S), c normalising the
 * w = 0, s = 0 taps to unit sum, and g = 0 where |d| >= S/2.  When the planes'
 * w_hat values are symmetric about 0 (w_hat_first + (n_planes - 1) / 2 *
 * w_hat_step within 1e-12 of their range), plane n_planes - 1 - p holds
 * exactly the complex conjugates of plane p: the lower plane of each mirror
 * pair is evaluated at the negated w_hat of its partner (the middle plane of an
 * odd count at 0), and the samples at nu and -nu are summed together.
 * gr_grid_binned recognises such tables and reads conjugates from the mirror
 * plane instead of flipping signs. */
gr_status gr_make_wkernel_table(int32_t support, int32_t oversample, int32_t n_planes,
                                double w_hat_first, double w_hat_step, int32_t support_aa,
                                double beta, int32_t n_samples, int32_t out_dtype, void* out,
                                void* stream);

/* Exact (non-paraxial) 2-D W-projection taps (the w term of Section 2.2
 * without the separable approximation of Section 4), complex, FP64 on the
 * device, layout [n_planes][O][O][S][S] of (re, im) out_dtype pairs, indexed
 * [plane][s_v][s_u][k_v][k_u]:
 *   C(du, dv) = c^2 sum_a sum_b t(nu_a) t(nu_b)
 *               exp(2 pi i (w_hat / fov^2) (sqrt(1 - fov^2 (nu_a^2 + nu_b^2)) - 1))
 *               exp(-2 pi i (du nu_a + dv nu_b))
 * with the taper t, midpoints nu, M = n_samples (<= 0: 4 S) and normaliser c of
 * gr_make_wkernel_table, fov the field of view in direction cosines
 * (0 < fov < sqrt 2), and zero where |du| or |dv| >= S/2. */
gr_status gr_make_wkernel2d_table(int32_t support, int32_t oversample, int32_t n_planes,
                                  double w_hat_first, double w_hat_step, double fov,
                                  int32_t support_aa, double beta, int32_t n_samples,
                                  int32_t out_dtype, void* out, void* stream);

/* ---- Learned tap network (GR_MLP) ------------------------------------------
 * Replaces the precomputed oversampled table of Section 2.2 by a function of
 * the table's own coordinates.  Weight blob (device, FP32, gr_mlp_blob_floats()
 * floats, 16-byte aligned):
 *   [0] x0 offset, [1] x0 step per plane, [2] out_scale, [3] unused,
 *   then W1 [64][64], b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64],
 *   W4 [64][2], b4 [2]  (W stored [in][out], row-major), then padding.
 * Inputs x (3 per sample): x0 = w_hat / w_hat_range, x1 = d_u / (S/2),
 *   x2 = d_v / (S/2), where d = k - S/2 + 1 - s/O is the GCF argument of tap
 *   k at phase s (a tap depends on k and s only through d) and w_hat_range is
 *   chosen so that |x0| <= 1/2 (the encoding has period 2).
 * Features e[12 i + 2 k] = sin(pi 2^k x_i), e[12 i + 2 k + 1] = cos(pi 2^k x_i)
 *   for i < 3, k < 6, e[36..63] = 0;  h1 = relu(e W1 + b1), h2 = relu(h1 W2 + b2),
 *   h3 = relu(h2 W3 + b3), y = h3 W4 + b4; tap = out_scale * (y0 + i y1),
 *   and 0 where |d_u| or |d_v| >= S/2 (the support rule of the tables).
 * The three 64-wide layers run on FP16 matrix cores (inputs rounded to FP16,
 * FP32 accumulation); the output layer likewise. */
int32_t gr_mlp_blob_floats(void);

/* out[2 n] (re, im) = tap network at inputs[3 n]; n >= 0; all device pointers. */
gr_status gr_mlp_eval(const float* weights, const float* inputs, int64_t n, float* out,
                      void* stream);

/* Training set from a complex FP32 GR_TABLE2D table (gr_make_wkernel2d_table
 * output): for every entry i of [n_planes][O][O][S][S], inputs[3 i] are its
 * network inputs with x0 = (w_hat_first + plane * w_hat_step) / w_hat_range,
 * and targets[2 i] = tap / out_scale.  Device pointers, sized by the caller
 * (3 and 2 floats per entry). */
gr_status gr_mlp_dataset(const void* table2d, int32_t support, int32_t oversample,
                         int32_t n_planes, double w_hat_first, double w_hat_step,
                         double w_hat_range, float out_scale, float* inputs, float* targets,
                         void* stream);

/* Gradients of the loss (1/B) sum_b |y(inputs[idx[b]]) - targets[idx[b]]|^2
 * over the batch b < batch (B = batch) with respect to every parameter of the
 * blob, written to grads (same layout as the blob; the header floats get 0).
 * Forward on FP16 matrix cores as in gr_mlp_eval; backward in FP32 on the
 * rounded activations.  *loss_sum (device, may be NULL) receives the loss.
 * idx values must index the inputs/targets arrays. */
gr_status gr_mlp_grads(const float* weights, const float* inputs, const float* targets,
                       const int32_t* idx, int32_t batch, float* grads, float* loss_sum,
                       void* stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8, step >= 1
 * counting from 1) on every parameter after gr_mlp_grads; adam_m / adam_v are
 * zero-initialised device arrays of the blob size kept by the caller; grads is
 * device scratch of the blob size.  The blob header is not changed. */
gr_status gr_mlp_train_step(float* weights, float* adam_m, float* adam_v, float* grads,
                            const float* inputs, const float* targets, const int32_t* idx,
                            int32_t batch, int32_t step, float lr, float* loss_sum, void* stream);

/* ---- Batches --------------------------------------------------------------
 * One independent gridding problem of a batch: the arguments of gr_grid for
 * it (the visibility stream, its kernel, cell sizes and grid), plus the
 * segment length of its binning (0: default).  Every pointer is device
 * memory; `kernel` is embedded by value (its taps pointer is device memory). */
typedef struct {
  const double* uvw;        /* [n_vis][3] */
  const void* vis;          /* as gr_preprocess */
  int32_t vis_dtype;        /* GR_F32 or GR_F16 */
  int32_t n_pol;            /* 1 or 4 */
  const float* vis_scale;   /* GR_F16 only */
  const float* weights;     /* may be NULL */
  int64_t n_vis;            /* >= 0, < 2^31 */
  gr_kernel kernel;         /* GR_SEPARABLE */
  double inv_cell_u, inv_cell_v;
  void* grid;               /* [n_pol][height][width] complex64, accumulated (+=) */
  int32_t height, width;
  int32_t seg_len;          /* binning segment length (gr_bin); 0: default */
  int32_t reserved;         /* must be 0 */
  int64_t* dev_stats;       /* may be NULL: as gr_preprocess */
} gr_batch_item;

/* Bytes of workspace gr_grid_batch needs for these items (0 if any is invalid). */
size_t gr_grid_batch_workspace_bytes(const gr_batch_item* items, int32_t n_items);

/* Grid a batch of independent problems (0 <= n_items <= 4096), each with the
 * result gr_grid would give it (binned MFMA path; separable kernels with
 * support <= 56).  The paper launches one problem at a time and observes that
 * sparse slices leave the device underused (Section 5); here all problems go
 * through one fixed launch sequence: per-visibility preprocess and binning
 * kernels spanning every item, then one persistent gridder per (n_pol, real or
 * complex taps) group whose work-groups take (item, segment) work from an
 * atomic counter, and one launch of the single-problem MFMA gridder for each
 * item of at least 2^19 visibilities (binned for its support's window).  The sequence issues no memset and never synchronises with
 * the host, so it can be captured into a HIP graph and replayed (the items'
 * buffers and the workspace must then stay allocated).  Items are validated
 * on the host before anything is launched; the first invalid item's index is
 * named in gr_last_error. */
gr_status gr_grid_batch(const gr_batch_item* items, int32_t n_items, void* workspace,
                        size_t workspace_bytes, void* stream);

/* The whole gr_grid_batch sequence for these items, captured once into a HIP
 * graph (on a stream of the library's own) and instantiated: *out receives an
 * opaque handle.  Items and workspace are validated on the host first, as by
 * gr_grid_batch; nothing runs until gr_graph_launch.  Every launch grids the
 * items again into their grids (+=: zero them in between to repeat a result);
 * the items' buffers and the workspace must stay allocated and unchanged in
 * size while the handle lives.  The graph holds only kernel nodes (no
 * memset).  Creating it synchronises nothing on the device. */
typedef struct gr_graph gr_graph;
gr_status gr_grid_batch_graph(const gr_batch_item* items, int32_t n_items, void* workspace,
                              size_t workspace_bytes, gr_graph** out);

/* Enqueue one replay of the captured batch on `stream`. */
gr_status gr_graph_launch(gr_graph* graph, void* stream);

/* Release the handle (NULL is accepted); the caller makes sure no launch of it
 * is still pending if its buffers are to be freed. */
gr_status gr_graph_destroy(gr_graph* graph);

/* Thread-local description of the last non-OK status ("" if none). */
const char* gr_last_error(void);

/* Library ABI version (increments on incompatible changes). */
int32_t gr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRIDDER_H */
