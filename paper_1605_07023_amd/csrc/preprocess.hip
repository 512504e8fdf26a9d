// Preprocess: uvw -> footprint origin, oversampled phase, w-plane; pre-weighted
// visibilities; drop rule.  FP64 for every coordinate computation.
//
// Merry (2016), Section 4: everything the gridder needs per visibility (cell
// position, oversampling phase, w plane, weighted values) is worked out in a
// separate pass before gridding, once per visibility.
#include <algorithm>

#include <hip/hip_fp16.h>

#include "internal.h"
#include "prep.h"

namespace gr {

namespace {

using namespace prep;

// Visibility i (< a.n): record, weighted visibilities; returns whether it is
// kept.  P = a.n_pol (1 or 4).
template <int VDT, int P>
__device__ __forceinline__ bool preprocess_one(int64_t i, const PreArgs& a) {
  float2 vw[P];
  const bool fin = weighted_vis<VDT, P>(i, a, vw);
  Record r = coord_record(i, a);
  const bool ok = rec_valid(r) && fin;
#pragma unroll
  for (int p = 0; p < P; ++p) a.wvis[i * P + p] = ok ? vw[p] : make_float2(0.f, 0.f);
  if (!ok) r = Record{0, 0};
  a.rec[i] = r;
  return ok;
}

// Block-level kept / dropped counts into stats[0], stats[1].
__device__ __forceinline__ void add_stats(bool ok, bool in, unsigned long long* stats) {
  const int n_ok = __syncthreads_count(ok ? 1 : 0);
  const int n_in = __syncthreads_count(in ? 1 : 0);
  if (stats != nullptr && threadIdx.x == 0 && n_in > 0) {
    atomicAdd(&stats[0], (unsigned long long)n_ok);
    atomicAdd(&stats[1], (unsigned long long)(n_in - n_ok));
  }
}

// Grid-stride over the visibilities (block size 256, a few blocks per CU):
// per-thread kept / dropped counts, one reduction per block.
template <int VDT, int P>
__global__ void __launch_bounds__(256)
preprocess_kernel(PreArgs a, unsigned long long* __restrict__ stats) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int n_ok = 0, n_drop = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    if (preprocess_one<VDT, P>(i, a)) ++n_ok;
    else ++n_drop;
  }
  add_block_counts(n_ok, n_drop, stats);
}

// Batched form: block b belongs to the instance whose [blk_begin, next blk_begin)
// range holds b (every instance starts on a fresh block).
__global__ void __launch_bounds__(256)
batch_preprocess_kernel(const BatchInst* __restrict__ inst, int n_inst) {
  __shared__ int s_i;
  if (threadIdx.x == 0) s_i = batch_find(inst, n_inst, (int64_t)blockIdx.x);
  __syncthreads();
  const BatchInst& I = inst[s_i];
  const PreArgs a{I.uvw, I.vis, I.vis_scale, I.weights, I.n_vis, I.n_pol, I.scale_u, I.scale_v,
                  I.lg_o, I.d.S, I.d.H, I.d.W, I.n_planes, I.w_min, I.inv_dw, I.rec, I.wvis};
  const int64_t i = ((int64_t)blockIdx.x - I.blk_begin) * blockDim.x + threadIdx.x;
  bool ok = false;
  if (i < a.n) {
    if (I.n_pol == 4)
      ok = I.vis_dtype == GR_F32 ? preprocess_one<GR_F32, 4>(i, a) : preprocess_one<GR_F16, 4>(i, a);
    else
      ok = I.vis_dtype == GR_F32 ? preprocess_one<GR_F32, 1>(i, a) : preprocess_one<GR_F16, 1>(i, a);
  }
  add_stats(ok, i < a.n, I.stats);
}

}  // namespace

gr_status launch_preprocess(const double* uvw, const void* vis, int vis_dtype, const float* vis_scale,
                            const float* weights, int64_t n_vis, int n_pol, const gr_kernel& k,
                            double inv_cell_u, double inv_cell_v, int height, int width,
                            Record* records, float2* wvis, int64_t* dev_stats, hipStream_t stream) {
  if (n_vis == 0) return GR_OK;
  const int64_t blocks = std::min<int64_t>((n_vis + 255) / 256, (int64_t)device_cu_count() * 16);
  auto* st = reinterpret_cast<unsigned long long*>(dev_stats);
  const PreArgs a = make_pre_args(uvw, vis, vis_scale, weights, n_vis, n_pol, k, inv_cell_u, inv_cell_v, height,
                                  width, records, wvis);
  using Fn = void (*)(PreArgs, unsigned long long*);
  Fn fn;
  if (n_pol == 4) fn = vis_dtype == GR_F32 ? preprocess_kernel<GR_F32, 4> : preprocess_kernel<GR_F16, 4>;
  else fn = vis_dtype == GR_F32 ? preprocess_kernel<GR_F32, 1> : preprocess_kernel<GR_F16, 1>;
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, stream, a, st);
  return check_launch("gr_preprocess");
}

gr_status launch_batch_preprocess(const BatchInst* inst, int n_inst, int64_t total_blocks,
                                  hipStream_t stream) {
  if (total_blocks == 0) return GR_OK;
  if (total_blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_grid_batch: too many visibilities");
  batch_preprocess_kernel<<<(unsigned)total_blocks, 256, 0, stream>>>(inst, n_inst);
  return check_launch("gr_grid_batch (preprocess)");
}

}  // namespace gr
