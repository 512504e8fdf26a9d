// W-stacking slices (Merry 2016, Section 5): the visibilities are split by w
// into slices and each slice is gridded as its own problem, with a GCF that
// corrects only the w offset from the slice's centre.  This file holds the
// split: a stable partition of the stream (uvw, visibilities, weights) by
//     slice = floor((w - w_first) * inv_width)          (FP64, one rounding each)
// with visibilities outside [0, n_slices) (or with a non-finite w) after the
// last slice.  Within a slice the input order is kept, so the time order of
// the tracks, which compression and the gridders' locality rely on, survives.
//
// Three launches and a tiny fourth: per block of 2048 consecutive
// visibilities the count of each slice (LDS histogram) into a slice-major
// table [slice][block]; one exclusive scan over that table, which makes every
// entry the output position of its (slice, block) run; per block, in 8 rounds
// of 256, the stable rank of each visibility among the block's visibilities
// of its slice (wave ballots, per-wave counts and a running position per
// slice in LDS) and the copy; the slice offsets from the table.
#include <algorithm>

#include "internal.h"

namespace gr {

namespace {

constexpr int kSliceBlock = 256;
constexpr int kSliceRounds = 8;                      // a block takes 8 x 256 consecutive visibilities
constexpr int kSliceChunk = kSliceBlock * kSliceRounds;

__device__ __forceinline__ int slice_of(const double* __restrict__ uvw, int64_t i, double w_first,
                                        double inv_width, int n_slices) {
  const double t = (uvw[3 * i + 2] - w_first) * inv_width;
  return (t >= 0.0 && t < (double)n_slices) ? (int)floor(t) : n_slices;   // NaN fails both
}

__global__ void __launch_bounds__(kSliceBlock)
slice_count_kernel(const double* __restrict__ uvw, int64_t n, double w_first, double inv_width, int n_slices,
                   int32_t* __restrict__ counts, int n_blocks) {
  extern __shared__ int hist[];                      // [n_slices + 1]
  for (int s = threadIdx.x; s <= n_slices; s += blockDim.x) hist[s] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSliceChunk + threadIdx.x;
#pragma unroll
  for (int r = 0; r < kSliceRounds; ++r) {
    const int64_t i = base + r * kSliceBlock;
    if (i < n) atomicAdd(&hist[slice_of(uvw, i, w_first, inv_width, n_slices)], 1);
  }
  __syncthreads();
  for (int s = threadIdx.x; s <= n_slices; s += blockDim.x)
    counts[(int64_t)s * n_blocks + blockIdx.x] = hist[s];
}

template <int P, bool HAS_W>
__global__ void __launch_bounds__(kSliceBlock)
slice_scatter_kernel(const double* __restrict__ uvw, const float2* __restrict__ vis, const float* __restrict__ wts,
                     int64_t n, double w_first, double inv_width, int n_slices, const int32_t* __restrict__ offs,
                     int n_blocks, double* __restrict__ uvw_out, float2* __restrict__ vis_out,
                     float* __restrict__ wts_out) {
  // LDS: per slice the running output position of the block, then per wave the
  // slice counts of the current round
  extern __shared__ int lds[];
  const int ns1 = n_slices + 1;
  int* run = lds;                                    // [n_slices + 1]
  int* wave_cnt = lds + ns1;                         // [4 waves][n_slices + 1]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < ns1; e += blockDim.x) run[e] = offs[(int64_t)e * n_blocks + blockIdx.x];
  for (int r = 0; r < kSliceRounds; ++r) {
    for (int e = threadIdx.x; e < (kSliceBlock / 64) * ns1; e += blockDim.x) wave_cnt[e] = 0;
    __syncthreads();                                 // run[] of the previous round final, wave_cnt clear
    const int64_t i = (int64_t)blockIdx.x * kSliceChunk + r * kSliceBlock + threadIdx.x;
    const bool act = i < n;
    const int s = act ? slice_of(uvw, i, w_first, inv_width, n_slices) : -1;
    // rank among the wave's earlier lanes of the same slice, one ballot per
    // distinct slice in the wave; the lowest lane of each slice records its count
    uint64_t todo = __ballot(act);
    int rank = 0;
    while (todo != 0) {
      const int leader = __builtin_ctzll(todo);
      const int v = __shfl(s, leader);
      const uint64_t mask = __ballot(act && s == v);
      if (act && s == v) rank = __popcll(mask & ((1ull << lane) - 1ull));
      if (lane == leader) wave_cnt[wave * ns1 + v] = __popcll(mask);
      todo &= ~mask;
    }
    __syncthreads();
    if (act) {
      int before = run[s];
      for (int w = 0; w < wave; ++w) before += wave_cnt[w * ns1 + s];
      const int64_t dst = (int64_t)before + rank;
#pragma unroll
      for (int c = 0; c < 3; ++c) uvw_out[3 * dst + c] = uvw[3 * i + c];
#pragma unroll
      for (int p = 0; p < P; ++p) vis_out[dst * P + p] = vis[i * P + p];
      if constexpr (HAS_W) {
#pragma unroll
        for (int p = 0; p < P; ++p) wts_out[dst * P + p] = wts[i * P + p];
      }
    }
    __syncthreads();                                 // every lane has read run[] of this round
    for (int e = threadIdx.x; e < ns1; e += blockDim.x) {
      int add = 0;
#pragma unroll
      for (int w = 0; w < kSliceBlock / 64; ++w) add += wave_cnt[w * ns1 + e];
      run[e] += add;
    }
    __syncthreads();                                 // wave_cnt read before the next round clears it
  }
}

// slice_offsets[s] = first output position of slice s (s = n_slices: the
// first visibility outside every slice)
__global__ void __launch_bounds__(256)
slice_offsets_kernel(const int32_t* __restrict__ offs, int n_blocks, int n_slices, int64_t* __restrict__ out) {
  const int s = threadIdx.x;
  if (s <= n_slices) out[s] = n_blocks > 0 ? (int64_t)offs[(int64_t)s * n_blocks] : 0;
}

}  // namespace

size_t wslice_workspace_bytes(int64_t n_vis, int n_slices) {
  const int64_t blocks = (n_vis + kSliceChunk - 1) / kSliceChunk;
  const int64_t entries = blocks * (int64_t)(n_slices + 1);
  return align256(sizeof(int32_t) * (size_t)entries) + scan_i32_scratch_bytes(entries) + 256;
}

gr_status launch_wslice_partition(const double* uvw, const float2* vis, const float* wts, int64_t n_vis, int n_pol,
                                  double w_first, double inv_width, int n_slices, double* uvw_out,
                                  float2* vis_out, float* wts_out, int64_t* slice_offsets, void* workspace,
                                  hipStream_t stream) {
  const int64_t blocks = (n_vis + kSliceChunk - 1) / kSliceChunk;
  const int64_t entries = blocks * (int64_t)(n_slices + 1);
  if (entries > 0x7fffffffLL) return fail(GR_EINVAL, "gr_wslice_partition: n_vis x (n_slices + 1) too large");
  auto* counts = reinterpret_cast<int32_t*>(workspace);
  const size_t hist_lds = sizeof(int) * (size_t)(n_slices + 1);
  if (blocks > 0) {
    slice_count_kernel<<<(unsigned)blocks, kSliceBlock, hist_lds, stream>>>(uvw, n_vis, w_first, inv_width,
                                                                            n_slices, counts, (int)blocks);
    auto* scan_scratch = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) +
                                                   align256(sizeof(int32_t) * (size_t)entries));
    launch_scan_i32(counts, (int)entries, nullptr, scan_scratch, stream);
    using Fn = void (*)(const double*, const float2*, const float*, int64_t, double, double, int, const int32_t*,
                        int, double*, float2*, float*);
    Fn fn;
    if (n_pol == 4) fn = wts ? slice_scatter_kernel<4, true> : slice_scatter_kernel<4, false>;
    else fn = wts ? slice_scatter_kernel<1, true> : slice_scatter_kernel<1, false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kSliceBlock), (1 + kSliceBlock / 64) * hist_lds, stream, uvw,
                       vis, wts, n_vis, w_first, inv_width, n_slices, counts, (int)blocks, uvw_out, vis_out,
                       wts_out);
  }
  slice_offsets_kernel<<<1, 256, 0, stream>>>(counts, (int)blocks, n_slices, slice_offsets);
  return check_launch("gr_wslice_partition");
}

}  // namespace gr
