// Preprocess: uvw -> footprint origin, oversampled phase, w-plane; pre-weighted
// visibilities; drop rule.  FP64 for every coordinate computation.
//
// Merry (2016), Section 4: the gridding kernel receives, per visibility, the
// integer grid coordinates, the sub-grid coordinates used to index the GCF,
// the w-plane index and the pre-weighted visibility; this is computed once,
// ahead of gridding.
#include <algorithm>

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

// Visibility i (< a.n): record, weighted visibilities; returns whether it is
// kept.  P = a.n_pol (1 or 4): one pass over the visibilities and weights,
// held in registers between the finiteness test and the weighted store.
template <int VDT, int P>
__device__ __forceinline__ bool preprocess_one(int64_t i, const PreArgs& a) {
#pragma clang fp contract(off)
  const double u = a.uvw[3 * i], v = a.uvw[3 * i + 1], w = a.uvw[3 * i + 2];
  float2 vv[P];
  float wt[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    vv[p] = load_vis<VDT>(a.vis, a.vis_scale, i, p, P);
    wt[p] = a.weights ? a.weights[i * P + p] : 1.0f;
  }
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
#pragma unroll
  for (int p = 0; p < P; ++p) ok = ok && isfinite(vv[p].x) && isfinite(vv[p].y) && isfinite(wt[p]);
#pragma unroll
  for (int p = 0; p < P; ++p)
    a.wvis[i * P + p] = ok ? make_float2(vv[p].x * wt[p], vv[p].y * wt[p]) : make_float2(0.f, 0.f);
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

// Sum two per-thread counts over the block and add them to stats[0], stats[1]
// (one pair of atomics per block).
__device__ __forceinline__ void add_block_counts(int n_ok, int n_drop, unsigned long long* stats) {
  __shared__ int s_ok[16], s_drop[16];
  for (int o = 32; o > 0; o >>= 1) {
    n_ok += __shfl_xor(n_ok, o);
    n_drop += __shfl_xor(n_drop, o);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    s_ok[wave] = n_ok;
    s_drop[wave] = n_drop;
  }
  __syncthreads();
  if (threadIdx.x == 0 && stats != nullptr) {
    unsigned long long ok = 0, drop = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      ok += (unsigned long long)s_ok[w];
      drop += (unsigned long long)s_drop[w];
    }
    if (ok) atomicAdd(&stats[0], ok);
    if (drop) atomicAdd(&stats[1], drop);
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
  int lg_o = 0;
  while ((1 << lg_o) < k.oversample) ++lg_o;
  const double su = inv_cell_u * (double)k.oversample;
  const double sv = inv_cell_v * (double)k.oversample;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  const int64_t blocks = std::min<int64_t>((n_vis + 255) / 256, (int64_t)cus * 16);
  auto* st = reinterpret_cast<unsigned long long*>(dev_stats);
  const PreArgs a{uvw, vis, vis_scale, weights, n_vis, n_pol, su, sv, lg_o, k.support, height, width,
                  k.n_planes, k.w_min, k.inv_dw, records, wvis};
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
