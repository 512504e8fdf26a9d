// Preprocess: uvw -> footprint origin, oversampled phase, w-plane; pre-weighted
// visibilities; drop rule.  FP64 for every coordinate computation.
//
// Merry (2016), Section 4: the gridding kernel receives, per visibility, the
// integer grid coordinates, the sub-grid coordinates used to index the GCF,
// the w-plane index and the pre-weighted visibility; this is computed once,
// ahead of gridding.
#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

constexpr double kBig = 1099511627776.0;  // 2^40: anything larger is off every grid

template <int VDT>
__device__ inline float2 load_vis(const void* __restrict__ vis, const float* __restrict__ scale,
                                  int64_t i, int p, int n_pol) {
  if constexpr (VDT == GR_F32) {
    return reinterpret_cast<const float2*>(vis)[i * n_pol + p];
  } else {
    const __half2 h = reinterpret_cast<const __half2*>(vis)[i * n_pol + p];
    const float s = scale[i >> 8];
    return make_float2(__low2float(h) * s, __high2float(h) * s);
  }
}

struct PreArgs {
  const double* uvw;
  const void* vis;
  const float* vis_scale;
  const float* weights;
  int64_t n;
  int n_pol;
  double scale_u, scale_v;
  int lg_o, S, H, W, n_planes;
  double w_min, inv_dw;
  Record* rec;
  float2* wvis;
};

// Visibility i (< a.n): record, weighted visibilities; returns whether it is kept.
template <int VDT>
__device__ __forceinline__ bool preprocess_one(int64_t i, const PreArgs& a) {
#pragma clang fp contract(off)
  const double u = a.uvw[3 * i], v = a.uvw[3 * i + 1], w = a.uvw[3 * i + 2];
  bool ok = isfinite(u) && isfinite(v) && isfinite(w);
  // one correctly rounded multiply each: scale = inv_cell * O is exact (O = 2^k)
  const double xh = u * a.scale_u;
  const double yh = v * a.scale_v;
  ok = ok && fabs(xh) < kBig && fabs(yh) < kBig;
  const int O = 1 << a.lg_o;
  const int64_t fx = (int64_t)rint(ok ? xh : 0.0) + (int64_t)(a.W / 2) * O;
  const int64_t fy = (int64_t)rint(ok ? yh : 0.0) + (int64_t)(a.H / 2) * O;
  const int64_t x0 = (fx >> a.lg_o) - a.S / 2 + 1;
  const int64_t y0 = (fy >> a.lg_o) - a.S / 2 + 1;
  int64_t plane = 0;
  if (a.n_planes > 1) {
    const double ph = (w - a.w_min) * a.inv_dw;
    ok = ok && fabs(ph) < kBig;
    plane = (int64_t)rint(ok ? ph : 0.0);
  }
  ok = ok && plane >= 0 && plane < a.n_planes && x0 >= 0 && x0 + a.S <= a.W && y0 >= 0 &&
       y0 + a.S <= a.H;
  // visibilities and weights must be finite as well
  for (int p = 0; p < a.n_pol; ++p) {
    const float2 vv = load_vis<VDT>(a.vis, a.vis_scale, i, p, a.n_pol);
    const float wt = a.weights ? a.weights[i * a.n_pol + p] : 1.0f;
    ok = ok && isfinite(vv.x) && isfinite(vv.y) && isfinite(wt);
  }
  for (int p = 0; p < a.n_pol; ++p) {
    const float2 vv = load_vis<VDT>(a.vis, a.vis_scale, i, p, a.n_pol);
    const float wt = a.weights ? a.weights[i * a.n_pol + p] : 1.0f;
    a.wvis[i * a.n_pol + p] = ok ? make_float2(vv.x * wt, vv.y * wt) : make_float2(0.f, 0.f);
  }
  Record r;
  if (ok) {
    r.x = (uint32_t)x0 | ((uint32_t)y0 << 16);
    r.y = (uint32_t)(fx & (O - 1)) | ((uint32_t)(fy & (O - 1)) << 8) | ((uint32_t)plane << 16) |
          kValidBit;
  } else {
    r.x = 0;
    r.y = 0;
  }
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

// One thread per visibility.  Block size 256.
template <int VDT>
__global__ void __launch_bounds__(256)
preprocess_kernel(PreArgs a, unsigned long long* __restrict__ stats) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < a.n ? preprocess_one<VDT>(i, a) : false;
  add_stats(ok, i < a.n, stats);
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
  if (i < a.n) ok = I.vis_dtype == GR_F32 ? preprocess_one<GR_F32>(i, a) : preprocess_one<GR_F16>(i, a);
  add_stats(ok, i < a.n, I.stats);
}

}  // namespace

gr_status launch_preprocess(const double* uvw, const void* vis, int vis_dtype, const float* vis_scale,
                            const float* weights, int64_t n_vis, int n_pol, const gr_kernel& k,
                            double inv_cell_u, double inv_cell_v, int height, int width,
                            Record* records, float2* wvis, int64_t* dev_stats, hipStream_t stream) {
  if (n_vis == 0) return GR_OK;
  int lg_o = 0;
  while ((1 << lg_o) < k.oversample) ++lg_o;
  const double su = inv_cell_u * (double)k.oversample;
  const double sv = inv_cell_v * (double)k.oversample;
  const int64_t blocks = (n_vis + 255) / 256;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_preprocess: n_vis too large");
  auto* st = reinterpret_cast<unsigned long long*>(dev_stats);
  const PreArgs a{uvw, vis, vis_scale, weights, n_vis, n_pol, su, sv, lg_o, k.support, height, width,
                  k.n_planes, k.w_min, k.inv_dw, records, wvis};
  if (vis_dtype == GR_F32)
    preprocess_kernel<GR_F32><<<(unsigned)blocks, 256, 0, stream>>>(a, st);
  else
    preprocess_kernel<GR_F16><<<(unsigned)blocks, 256, 0, stream>>>(a, st);
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
