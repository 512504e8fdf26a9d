// Per-visibility preprocessing shared by the preprocess kernels and the fused
// preprocess-and-bin kernels: the record (footprint origin, oversampling
// phases, w-plane, valid bit) from the coordinates, in FP64, and the weighted
// visibilities with their finiteness (the two parts of the drop rule).
//
// Merry (2016), Section 4: the per-visibility inputs of the gridder are
// prepared ahead of it, in a pass of their own.
#pragma once

#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {
namespace prep {

constexpr double kBig = 1099511627776.0;  // 2^40: anything larger is off every grid

template <int VDT>
__device__ __forceinline__ float2 load_vis(const void* __restrict__ vis, const float* __restrict__ scale,
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
  // per-visibility GCF ids (NULL: none): the record's plane field then holds
  // id * n_planes + plane, and an id outside [0, n_ids) drops the visibility
  const int32_t* ids = nullptr;
  int n_ids = 0;
  // degridding's output (NULL: none): a dropped visibility's n_pol values are
  // zeroed by the count pass, so the output needs no separate fill
  float2* zero_dropped = nullptr;
};

// Record of visibility i (< a.n) from its coordinates alone: the drop rule's
// coordinate part (non-finite or off-grid uvw, plane out of range); the valid
// bit is set when it keeps the visibility.
__device__ __forceinline__ Record coord_record(int64_t i, const PreArgs& a) {
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
  if (a.ids != nullptr) {
    const int id = a.ids[i];
    ok = ok && id >= 0 && id < a.n_ids;
    plane += (int64_t)(ok ? id : 0) * a.n_planes;
  }
  Record r{0, 0};
  if (ok) {
    r.x = (uint32_t)x0 | ((uint32_t)y0 << 16);
    r.y = (uint32_t)(fx & (O - 1)) | ((uint32_t)(fy & (O - 1)) << 8) | ((uint32_t)plane << 16) |
          kValidBit;
  }
  return r;
}

// Visibilities and weights of visibility i, and whether all are finite (the
// drop rule's value part); vw receives the weighted values.
template <int VDT, int P>
__device__ __forceinline__ bool weighted_vis(int64_t i, const PreArgs& a, float2 (&vw)[P]) {
  float2 vv[P];
  float wt[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    vv[p] = load_vis<VDT>(a.vis, a.vis_scale, i, p, P);
    wt[p] = a.weights ? a.weights[i * P + p] : 1.0f;
  }
  bool fin = true;
#pragma unroll
  for (int p = 0; p < P; ++p) fin = fin && isfinite(vv[p].x) && isfinite(vv[p].y) && isfinite(wt[p]);
#pragma unroll
  for (int p = 0; p < P; ++p) vw[p] = fin ? make_float2(vv[p].x * wt[p], vv[p].y * wt[p]) : make_float2(0.f, 0.f);
  return fin;
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

inline PreArgs make_pre_args(const double* uvw, const void* vis, const float* vis_scale, const float* weights,
                             int64_t n_vis, int n_pol, const gr_kernel& k, double inv_cell_u, double inv_cell_v,
                             int height, int width, Record* records, float2* wvis) {
  int lg_o = 0;
  while ((1 << lg_o) < k.oversample) ++lg_o;
  return PreArgs{uvw, vis, vis_scale, weights, n_vis, n_pol, inv_cell_u * (double)k.oversample,
                 inv_cell_v * (double)k.oversample, lg_o, k.support, height, width, k.n_planes, k.w_min, k.inv_dw,
                 records, wvis};
}

inline int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  return cus;
}

}  // namespace prep
}  // namespace gr
