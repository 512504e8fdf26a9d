// GCF table generation on the device, in FP64 (Section 2.2: the GCF is
// precomputed numerically and sampled at `oversample` times the grid
// resolution; Section 4: separable, polarisation-independent).
//
// Tap k of oversampled phase s samples the kernel at d = k - S/2 + 1 - s/O;
// every table is zero where |d| >= S/2.
#include <cmath>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

// Modified Bessel function I0 from its power series sum_m ((x/2)^m / m!)^2,
// summed until the terms no longer change the FP64 result.
__device__ double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int m = 1; m < 500; ++m) {
    term *= q / ((double)m * (double)m);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

__device__ inline void store_elem(void* out, int64_t idx, int dtype, double v) {
  switch (dtype) {
    case GR_F64: reinterpret_cast<double*>(out)[idx] = v; break;
    case GR_F32: reinterpret_cast<float*>(out)[idx] = (float)v; break;
    case GR_F16: reinterpret_cast<__half*>(out)[idx] = __float2half((float)v); break;
    default: reinterpret_cast<__hip_bfloat16*>(out)[idx] = __float2bfloat16((float)v); break;
  }
}

__global__ void kb_table_kernel(double beta, int S, int O, int dtype, void* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S * O) return;
  const int s = t / S, k = t % S;
  const double d = (double)(k - S / 2 + 1) - (double)s / (double)O;
  double v = 0.0;
  if (fabs(d) < 0.5 * S) {
    const double x = 2.0 * d / (double)S;
    v = bessel_i0(beta * sqrt(1.0 - x * x)) / bessel_i0(beta);
  }
  store_elem(out, t, dtype, v);
}

// Image response of a Kaiser-Bessel window of width `aa` at image coordinate nu.
__device__ double kb_taper(double nu, int aa, double beta) {
  const double a = M_PI * (double)aa * nu;
  const double r = beta * beta - a * a;
  if (r > 0.0) {
    const double s = sqrt(r);
    return sinh(s) / s;
  }
  if (r < 0.0) {
    const double s = sqrt(-r);
    return sin(s) / s;
  }
  return 1.0;
}

// One block per (plane, s) row; blockDim 256; dynamic LDS: M doubles of taper.
__global__ void __launch_bounds__(256)
wkernel_table_kernel(int S, int O, int n_planes, double wh0, double whs, int aa, double beta, int M,
                     int dtype, void* out) {
  extern __shared__ double sh[];      // [M] taper, then [256] reduction scratch
  double* taper = sh;
  double* red = sh + M;
  const int row = blockIdx.x;         // plane * O + s
  const int plane = row / O, s = row % O;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const double nu = ((double)j + 0.5) / (double)M - 0.5;
    taper[j] = kb_taper(nu, aa, beta);
  }
  __syncthreads();
  // normalisation: real part of the w = 0, s = 0 taps, summed over the support
  double part = 0.0;
  for (int q = threadIdx.x; q < S * M; q += blockDim.x) {
    const int k = q / M, j = q % M;
    const double d = (double)(k - S / 2 + 1);
    if (fabs(d) < 0.5 * S) {
      const double nu = ((double)j + 0.5) / (double)M - 0.5;
      part += taper[j] * cospi(2.0 * d * nu);
    }
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double c = 1.0 / red[0];
  double wh = wh0 + (double)plane * whs;
  if (n_planes > 1) {
    // planes at w values symmetric about 0 get exactly conjugate taps: the lower
    // plane of a mirror pair takes the exact negative of its partner's w (the
    // middle plane of an odd count takes 0), and every rounding below commutes
    // with negating w
    const double wm = wh0 + (double)(n_planes - 1 - plane) * whs;
    if (fabs(wh + wm) <= 1e-12 * (fabs(wh0) + fabs(whs) * (double)(n_planes - 1))) {
      if (2 * plane + 1 == n_planes) wh = 0.0;
      else if (2 * plane + 1 < n_planes) wh = -wm;
    }
  }
  for (int k = threadIdx.x; k < S; k += blockDim.x) {
    const double d = (double)(k - S / 2 + 1) - (double)s / (double)O;
    double re = 0.0, im = 0.0;
    if (fabs(d) < 0.5 * S) {
      // the samples at nu and -nu summed together:
      //   exp(-i pi (w nu^2 + 2 d nu)) + exp(-i pi (w nu^2 - 2 d nu)) = 2 cos(2 pi d nu) exp(-i pi w nu^2)
      for (int j = 0; j < M / 2; ++j) {
        const double nu = ((double)j + 0.5) / (double)M - 0.5;
        const double a = wh * nu * nu;
        double sn, cs;
        sincospi(fabs(a), &sn, &cs);
        if (a < 0.0) sn = -sn;
        const double t = 2.0 * taper[j] * cospi(2.0 * d * nu);
        re += t * cs;                                       // exp(-i pi a) = cos - i sin
        im -= t * sn;
      }
      if (M & 1) re += taper[M / 2];                        // nu = 0
      re *= c;
      im *= c;
    }
    const int64_t idx = ((int64_t)row * S + k) * 2;
    store_elem(out, idx, dtype, re);
    store_elem(out, idx + 1, dtype, im);
  }
}

// Exact (non-paraxial) 2-D W kernel, one block per (plane, s_v, k_v):
//   C(du, dv) = c^2 sum_a sum_b t(nu_a) t(nu_b) exp(2 pi i (w_hat / fov^2)
//               (sqrt(1 - fov^2 (nu_a^2 + nu_b^2)) - 1)) exp(-2 pi i (du nu_a + dv nu_b)),
// zero where |du| or |dv| >= S/2, computed as a row-column transform:
// first half[a] = sum_b exp(-2 pi i dv nu_b) screen(b, a) for this block's dv,
// then every (s_u, k_u) output of the block sums over a.
// Output [plane][s_v][s_u][k_v][k_u] of (re, im).  Dynamic LDS: 4 M doubles + 256.
__global__ void __launch_bounds__(256)
wkernel2d_table_kernel(int S, int O, double wh0, double whs, double fov, int aa, double beta, int M,
                       int dtype, void* out) {
  extern __shared__ double sh2[];
  double* taper = sh2;              // [M]
  double* hre = sh2 + M;            // [M]
  double* him = sh2 + 2 * M;        // [M]
  double* red = sh2 + 3 * M;        // [256]
  const int blk = blockIdx.x;       // (plane * O + s_v) * S + k_v
  const int kv = blk % S, sv = (blk / S) % O, plane = blk / (S * O);
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const double nu = ((double)j + 0.5) / (double)M - 0.5;
    taper[j] = kb_taper(nu, aa, beta);
  }
  __syncthreads();
  double part = 0.0;                // 1-D normalisation, as in the separable table
  for (int q = threadIdx.x; q < S * M; q += blockDim.x) {
    const int k = q / M, j = q % M;
    const double d = (double)(k - S / 2 + 1);
    if (fabs(d) < 0.5 * S) {
      const double nu = ((double)j + 0.5) / (double)M - 0.5;
      part += taper[j] * cospi(2.0 * d * nu);
    }
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double c = 1.0 / red[0];
  const double wh = wh0 + (double)plane * whs;
  const double dv = (double)(kv - S / 2 + 1) - (double)sv / (double)O;
  const bool vin = fabs(dv) < 0.5 * S;
  for (int a = threadIdx.x; a < M; a += blockDim.x) {
    double re = 0.0, im = 0.0;
    if (vin) {
      const double nua = ((double)a + 0.5) / (double)M - 0.5;
      for (int b = 0; b < M; ++b) {
        const double nub = ((double)b + 0.5) / (double)M - 0.5;
        const double rho2 = nua * nua + nub * nub;
        // screen phase (turns) minus the dv term
        const double ph = (wh / (fov * fov)) * (sqrt(1.0 - fov * fov * rho2) - 1.0) - dv * nub;
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double amp = taper[a] * taper[b];
        re += amp * cs;
        im += amp * sn;
      }
    }
    hre[a] = re;
    him[a] = im;
  }
  __syncthreads();
  const double c2 = c * c;
  for (int q = threadIdx.x; q < O * S; q += blockDim.x) {
    const int su = q / S, ku = q % S;
    const double du = (double)(ku - S / 2 + 1) - (double)su / (double)O;
    double re = 0.0, im = 0.0;
    if (vin && fabs(du) < 0.5 * S) {
      for (int a = 0; a < M; ++a) {
        const double nua = ((double)a + 0.5) / (double)M - 0.5;
        double sn, cs;
        sincospi(-2.0 * du * nua, &sn, &cs);
        re += hre[a] * cs - him[a] * sn;
        im += hre[a] * sn + him[a] * cs;
      }
      re *= c2;
      im *= c2;
    }
    const int64_t idx = ((((int64_t)plane * O + sv) * O + su) * S + kv) * S + ku;
    store_elem(out, 2 * idx, dtype, re);
    store_elem(out, 2 * idx + 1, dtype, im);
  }
}

bool dtype_ok(int d) { return d == GR_F64 || d == GR_F32 || d == GR_F16 || d == GR_BF16; }
bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

}  // namespace gr

using namespace gr;

extern "C" gr_status gr_make_kb_table(double beta, int32_t support, int32_t oversample,
                                      int32_t out_dtype, void* out, void* stream) {
  if (out == nullptr) return fail(GR_EINVAL, "gr_make_kb_table: out is NULL");
  if (support < 2 || support > 64 || (support & 1))
    return fail(GR_EINVAL, "gr_make_kb_table: support must be even, 2..64");
  if (!pow2(oversample) || oversample > kMaxOversample)
    return fail(GR_EINVAL, "gr_make_kb_table: oversample must be a power of two <= 128");
  if (!dtype_ok(out_dtype)) return fail(GR_EINVAL, "gr_make_kb_table: bad out_dtype");
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(GR_EINVAL, "gr_make_kb_table: bad beta");
  const int n = support * oversample;
  kb_table_kernel<<<(n + 255) / 256, 256, 0, (hipStream_t)stream>>>(beta, support, oversample,
                                                                     out_dtype, out);
  return check_launch("gr_make_kb_table");
}

extern "C" gr_status gr_make_wkernel_table(int32_t support, int32_t oversample, int32_t n_planes,
                                           double w_hat_first, double w_hat_step,
                                           int32_t support_aa, double beta, int32_t n_samples,
                                           int32_t out_dtype, void* out, void* stream) {
  if (out == nullptr) return fail(GR_EINVAL, "gr_make_wkernel_table: out is NULL");
  if (support < 2 || support > 64 || (support & 1))
    return fail(GR_EINVAL, "gr_make_wkernel_table: support must be even, 2..64");
  if (!pow2(oversample) || oversample > kMaxOversample)
    return fail(GR_EINVAL, "gr_make_wkernel_table: oversample must be a power of two <= 128");
  if (n_planes < 1 || n_planes > kMaxPlanes)
    return fail(GR_EINVAL, "gr_make_wkernel_table: n_planes out of range");
  if (support_aa < 1 || support_aa > support)
    return fail(GR_EINVAL, "gr_make_wkernel_table: support_aa must be in 1..support");
  if (!std::isfinite(w_hat_first) || !std::isfinite(w_hat_step) || !std::isfinite(beta) || beta < 0.0)
    return fail(GR_EINVAL, "gr_make_wkernel_table: non-finite parameter");
  if (!dtype_ok(out_dtype)) return fail(GR_EINVAL, "gr_make_wkernel_table: bad out_dtype");
  const int M = n_samples > 0 ? n_samples : 4 * support;
  if (M > 8192) return fail(GR_EINVAL, "gr_make_wkernel_table: n_samples must be <= 8192");
  const size_t lds = sizeof(double) * (size_t)(M + 256);
  wkernel_table_kernel<<<n_planes * oversample, 256, lds, (hipStream_t)stream>>>(
      support, oversample, n_planes, w_hat_first, w_hat_step, support_aa, beta, M, out_dtype, out);
  return check_launch("gr_make_wkernel_table");
}

extern "C" gr_status gr_make_wkernel2d_table(int32_t support, int32_t oversample, int32_t n_planes,
                                             double w_hat_first, double w_hat_step, double fov,
                                             int32_t support_aa, double beta, int32_t n_samples,
                                             int32_t out_dtype, void* out, void* stream) {
  if (out == nullptr) return fail(GR_EINVAL, "gr_make_wkernel2d_table: out is NULL");
  if (support < 2 || support > 64 || (support & 1))
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: support must be even, 2..64");
  if (!pow2(oversample) || oversample > kMaxOversample)
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: oversample must be a power of two <= 128");
  if (n_planes < 1 || n_planes > kMaxPlanes)
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: n_planes out of range");
  if (support_aa < 1 || support_aa > support)
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: support_aa must be in 1..support");
  if (!std::isfinite(w_hat_first) || !std::isfinite(w_hat_step) || !std::isfinite(beta) || beta < 0.0)
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: non-finite parameter");
  if (!(fov > 0.0) || !(fov < 1.4142))
    return fail(GR_EINVAL, "gr_make_wkernel2d_table: fov must be in (0, sqrt 2)");
  if (!dtype_ok(out_dtype)) return fail(GR_EINVAL, "gr_make_wkernel2d_table: bad out_dtype");
  const int M = n_samples > 0 ? n_samples : 4 * support;
  if (M > 2048) return fail(GR_EINVAL, "gr_make_wkernel2d_table: n_samples must be <= 2048");
  const int64_t blocks = (int64_t)n_planes * oversample * support;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_make_wkernel2d_table: table too large");
  const size_t lds = sizeof(double) * (size_t)(3 * M + 256);
  wkernel2d_table_kernel<<<(unsigned)blocks, 256, lds, (hipStream_t)stream>>>(
      support, oversample, w_hat_first, w_hat_step, fov, support_aa, beta, M, out_dtype, out);
  return check_launch("gr_make_wkernel2d_table");
}
