// Gridding with non-separable GCF tables over the binned stream.  The
// paper's speed-ups rely on a separable GCF (Section 4); without separability
// the S x S taps of every visibility must be read, so these paths are bound by
// tap loads from L2 / Infinity Cache rather than by arithmetic.  Two tables:
//  * GR_TABLE2D through gr_grid / gr_grid_binned: [planes][O][O][S][S], one
//    tap per cell shared by the polarisations (the exact 2-D W kernel, the
//    reference the learned kernel is measured against);
//  * gr_grid_aterm: GCFs that change per visibility and per polarisation, as
//    A-projection's do (Merry 2016, Section 6: such GCFs depend on time,
//    frequency, polarisation and possibly baseline, are not separable, and
//    their loads, not the arithmetic, are expected to set the speed).
//
// The caller gives every visibility a GCF id (for instance its time and
// frequency interval); the fused preprocess stores id * n_planes + plane in
// the record's plane field, so the binned stream carries it.  The table is
// complex [n_ids][n_planes][O][O][P][S][S]: one visibility reads one
// contiguous block of P * S * S taps, one tap per (polarisation, cell), each
// used once (8 flops per 8-byte tap at FP32).
//
// The window is the support's (32, 48 or 64 cells for S <= 16, 32, 56, as the
// MFMA gridders bin).  One 256-work-item block per segment; work-item t owns
// the C x C cells (C = window / 16) at rows C (t / 16) + i, columns
// C (t % 16) + j, for every polarisation, in registers (register accumulation
// with coarsening, Sections 2.2-3); a smaller window keeps more work-items
// inside each footprint.  Wave w owns block rows 4 w .. 4 w + 3 and skips, with
// one uniform branch, a visibility whose footprint misses them.  Visibilities
// are staged through LDS in batches of 256.  The work-items whose block meets
// the footprint load their taps (C consecutive complex values per row and
// polarisation, contiguous across neighbouring work-items) and accumulate
// tap x V per polarisation.  The window is added to the grid once with atomic
// adds.  (Accumulating into an LDS window with LDS atomics, every lane on one
// visibility's taps, measured slower: 378 against 301 ms for the 64-cell
// register window at S = 16.)
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <string>

#include "internal.h"

namespace gr {

namespace {

// complex tap idx of a table stored as TDT (a compile-time choice: no branch per tap)
template <int TDT>
__device__ __forceinline__ float2 load_tap2(const void* __restrict__ t, int64_t idx) {
  if constexpr (TDT == GR_F32) {
    return reinterpret_cast<const float2*>(t)[idx];
  } else if constexpr (TDT == GR_F16) {
    const __half2 h = reinterpret_cast<const __half2*>(t)[idx];
    return make_float2(__low2float(h), __high2float(h));
  } else {
    const uint32_t w = reinterpret_cast<const uint32_t*>(t)[idx];   // (re, im) bf16 pair
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
  }
}

struct AtermDev {
  int S, O, tap_dtype, tile, n_tx, H, W;
};

constexpr int kAtermBatch = 256;

template <int P, int C, bool POL, int TDT>
__global__ void __launch_bounds__(256)
grid_nonsep_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis, const int4* __restrict__ segs,
                  const int32_t* __restrict__ n_segs_p, const void* __restrict__ taps, float2* __restrict__ grid,
                  AtermDev d) {
  __shared__ Record b_rec[kAtermBatch];
  __shared__ float2 b_vis[kAtermBatch * P];
  const int seg = (int)blockIdx.x;
  if (seg >= *n_segs_p) return;
  const int4 sg = segs[seg];
  const int begin = sg.x, len = sg.y, tile_id = sg.z;
  const int win_x0 = (tile_id % d.n_tx) * d.tile;
  const int win_y0 = (tile_id / d.n_tx) * d.tile;
  const int t = threadIdx.x;
  const int wrow = 4 * C * (t >> 6);                    // the wave's first window row
  const int cy = C * (t >> 4), cx = C * (t & 15);       // the work-item's block origin
  const int S = d.S, O = d.O;
  const int64_t SS = (int64_t)S * S;

  float2 acc[C][C][P];
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int p = 0; p < P; ++p) acc[i][j][p] = make_float2(0.f, 0.f);

  for (int b0 = 0; b0 < len; b0 += kAtermBatch) {
    const int nb = min(kAtermBatch, len - b0);
    __syncthreads();
    if (t < nb) b_rec[t] = rec[begin + b0 + t];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int e = t + j * kAtermBatch;
      if (e < nb * P) b_vis[e] = wvis[(int64_t)(begin + b0) * P + e];
    }
    __syncthreads();
    for (int q = 0; q < nb; ++q) {
      const Record r = b_rec[q];
      const int oy = rec_y0(r) - win_y0, ox = rec_x0(r) - win_x0;
      if (oy >= wrow + 4 * C || oy + S <= wrow) continue;        // uniform for the wave
      if (cy + C - 1 < oy || cy >= oy + S || cx + C - 1 < ox || cx >= ox + S) continue;
      float2 v[P];
#pragma unroll
      for (int p = 0; p < P; ++p) v[p] = b_vis[q * P + p];
      const int64_t base = (((int64_t)rec_plane(r) * O + rec_sy(r)) * O + rec_sx(r)) * (POL ? P : 1) * SS;
#pragma unroll
      for (int i = 0; i < C; ++i) {
        const int ky = cy + i - oy;
        if ((unsigned)ky >= (unsigned)S) continue;
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const int kx = cx + j - ox;
          if ((unsigned)kx >= (unsigned)S) continue;
          float2 g = load_tap2<TDT>(taps, base + ky * S + kx);
#pragma unroll
          for (int p = 0; p < P; ++p) {
            if (POL && p > 0) g = load_tap2<TDT>(taps, base + p * SS + ky * S + kx);
            float2& a = acc[i][j][p];
            a.x = fmaf(g.x, v[p].x, a.x);
            a.x = fmaf(-g.y, v[p].y, a.x);
            a.y = fmaf(g.x, v[p].y, a.y);
            a.y = fmaf(g.y, v[p].x, a.y);
          }
        }
      }
    }
  }
  float* gridf = reinterpret_cast<float*>(grid);
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int row = win_y0 + cy + i;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int col = win_x0 + cx + j;
      if (row >= d.H || col >= d.W) continue;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        float* cell = gridf + (((int64_t)p * d.H + row) * d.W + col) * 2;
        if (acc[i][j][p].x != 0.f) unsafeAtomicAdd(cell, acc[i][j][p].x);
        if (acc[i][j][p].y != 0.f) unsafeAtomicAdd(cell + 1, acc[i][j][p].y);
      }
    }
  }
}

using AtermFn = void (*)(const Record*, const float2*, const int4*, const int32_t*, const void*, float2*, AtermDev);

template <int P, bool POL, int TDT>
AtermFn nonsep_fn_t(int window) {
  return window == 32 ? grid_nonsep_kernel<P, 2, POL, TDT>
                      : window == 48 ? grid_nonsep_kernel<P, 3, POL, TDT> : grid_nonsep_kernel<P, 4, POL, TDT>;
}

template <int P, bool POL>
AtermFn nonsep_fn(int window, int tap_dtype) {
  return tap_dtype == GR_F32   ? nonsep_fn_t<P, POL, GR_F32>(window)
         : tap_dtype == GR_F16 ? nonsep_fn_t<P, POL, GR_F16>(window)
                               : nonsep_fn_t<P, POL, GR_BF16>(window);
}

gr_status launch_nonsep(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k, float2* grid,
                        int height, int width, bool pol, const char* who, hipStream_t stream) {
  if (!k.taps_complex) return fail(GR_EUNSUPPORTED, std::string(who) + ": the GCF table must be complex");
  if (k.support > 56) return fail(GR_EUNSUPPORTED, std::string(who) + ": support must be <= 56");
  const int window = aterm_window(k.support);
  if (L.tile + k.support > window)
    return fail(GR_EINVAL, std::string(who) + ": binning tile does not fit the window");
  const char* base = reinterpret_cast<const char*>(bins);
  const auto* rec = reinterpret_cast<const Record*>(base + L.off_rec);
  const auto* wv = reinterpret_cast<const float2*>(base + L.off_wvis);
  const auto* segs = reinterpret_cast<const int4*>(base + L.off_segs);
  const auto* nsegs = reinterpret_cast<const int32_t*>(base + L.off_nsegs);
  AtermDev d{k.support, k.oversample, k.tap_dtype, L.tile, L.n_tx, height, width};
  if (L.max_segs > 0x7fffffff) return fail(GR_EINVAL, std::string(who) + ": too many segments");
  if (L.max_segs == 0) return check_launch(who);
  AtermFn fn;
  if (pol) fn = n_pol == 4 ? nonsep_fn<4, true>(window, k.tap_dtype) : nonsep_fn<1, true>(window, k.tap_dtype);
  else fn = n_pol == 4 ? nonsep_fn<4, false>(window, k.tap_dtype) : nonsep_fn<1, false>(window, k.tap_dtype);
  hipLaunchKernelGGL(fn, dim3((unsigned)L.max_segs), dim3(256), 0, stream, rec, wv, segs, nsegs, k.taps, grid, d);
  return check_launch(who);
}

}  // namespace

int aterm_window(int support) { return support <= 16 ? 32 : support <= 32 ? 48 : 64; }

gr_status launch_aterm(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k, float2* grid,
                       int height, int width, hipStream_t stream) {
  return launch_nonsep(bins, L, n_pol, k, grid, height, width, true, "gr_grid_aterm", stream);
}

gr_status launch_table2d(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k, float2* grid,
                         int height, int width, hipStream_t stream) {
  return launch_nonsep(bins, L, n_pol, k, grid, height, width, false, "gr_grid_binned (table2d)", stream);
}

}  // namespace gr
