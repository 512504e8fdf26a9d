// Learned W kernel: a small network that returns a tap's complex value from
// its coordinates, trained on the exact 2-D W-kernel table and evaluated
// inside the gridder in place of the table.  (The paper tabulates the GCF,
// Section 2.2; this replaces the multi-megabyte oversampled table by 12.6 K
// weights, and its w-planes and phases by continuous inputs.)
//
// Network (weights blob, FP32): inputs x0 = w_hat / w_hat_range (|x0| <= 1/2),
// x1 = d_u / (S/2), x2 = d_v / (S/2) with d = k - S/2 + 1 - s/O the GCF
// argument of the tap; features e[12 i + 2 k] = sin(pi 2^k x_i),
// e[12 i + 2 k + 1] = cos(pi 2^k x_i) (i < 3, k < 6), e[36..63] = 0; three
// hidden ReLU layers of 64; a linear layer to (Re, Im); tap = out_scale * y,
// and 0 where |d_u| or |d_v| >= S/2.
//
// gfx950 form: the 64-wide layers run on v_mfma_f32_16x16x32_f16 in
// transposed form, Z^T = W^T H^T: the weights are the A operand (register
// resident) and 16 samples the B operand.  The contraction index K is laid
// out so that a layer's D registers are exactly the next layer's B registers:
// lane group g = lane / 16, element q of K block kk holds
// K = 32 kk + 16 (q / 4) + 4 g + (q % 4), which is the D row of output tile
// 2 kk + q / 4 that the same lane holds.  The same mapping indexes the
// weights, so the product is unchanged.  Activations are rounded to FP16
// between layers, accumulation is FP32.  Training: forward as above; backward
// and weight gradients in FP32 on the VALU from LDS copies of the rounded
// activations; Adam in FP32.
#include <cmath>

#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// relu of two FP32 values rounded to FP16 (round to nearest even), as one packed
// word: max(round(x), 0) = round(max(x, 0)), since rounding is monotonic and
// keeps 0 (v_cvt_pk_f16_f32 and v_pk_max_f16, one instruction each per pair)
__device__ __forceinline__ uint32_t relu_h2(f2v v) {
  const h2v zero = {(_Float16)0.f, (_Float16)0.f};
  const h2v h = __builtin_elementwise_max(__builtin_convertvector(v, h2v), zero);
  return __builtin_bit_cast(uint32_t, h);
}

constexpr int kIn = 64, kHid = 64, kFeat = 36;

// FP32 blob layout (floats)
constexpr int kHdr = 4;                                  // x0 offset, x0 step, out_scale, unused
constexpr int kW1 = kHdr, kB1 = kW1 + kIn * kHid;
constexpr int kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid, kB3 = kW3 + kHid * kHid;
constexpr int kW4 = kB3 + kHid, kB4 = kW4 + kHid * 2;
constexpr int kParams = kB4 + 2;                         // 12,614
constexpr int kBlob = (kParams + 3) & ~3;

// K index held by lane group g, element q of K block kk (see the file header)
__device__ __forceinline__ int kidx(int kk, int g, int q) { return 32 * kk + 16 * (q >> 2) + 4 * g + (q & 3); }

__device__ __forceinline__ float feature(const float (&x)[3], int f) {
  if (f >= kFeat) return 0.f;
  const int i = f / 12, r = f % 12, k = r >> 1;
  float s, c;
  sincospif(x[i] * (float)(1 << k), &s, &c);
  return (r & 1) ? c : s;
}

// A operand of W^T for a layer W [in = 64][out = n_out], 16-row output tiles
template <int MT>
__device__ __forceinline__ void load_wfrag(const float* __restrict__ W, int n_out, h8 (&frag)[MT][2], int lane) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int m = 16 * mt + (lane & 15);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = kidx(kk, lane >> 4, q);
        frag[mt][kk][q] = (_Float16)(m < n_out ? W[k * n_out + m] : 0.f);
      }
    }
}

// biases of the D rows a lane holds: m = 16 mt + 4 (lane / 16) + i
template <int MT>
__device__ __forceinline__ void load_bias(const float* __restrict__ b, int n_out, float (&bias)[MT][4], int lane) {
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = 16 * mt + 4 * (lane >> 4) + i;
      bias[mt][i] = m < n_out ? b[m] : 0.f;
    }
}

struct Net {
  h8 w2[4][2], w3[4][2], w4[1][2];
  float b2[4][4], b3[4][4], b4[1][4];
};

__device__ __forceinline__ void load_net(const float* __restrict__ blob, Net& n, int lane) {
  load_wfrag<4>(blob + kW2, kHid, n.w2, lane);
  load_wfrag<4>(blob + kW3, kHid, n.w3, lane);
  load_wfrag<1>(blob + kW4, 2, n.w4, lane);
  load_bias<4>(blob + kB2, kHid, n.b2, lane);
  load_bias<4>(blob + kB3, kHid, n.b3, lane);
  load_bias<1>(blob + kB4, 2, n.b4, lane);
}

// One hidden layer on a 16-sample tile: h (B operand) -> relu(W^T h + b).
// keep (optional) receives the FP16-rounded outputs as FP32 per output tile.
__device__ __forceinline__ void layer(const h8 (&w)[4][2], const float (&b)[4][4], const h8 (&h)[2],
                                      h8 (&out)[2], f4* keep) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 d = {0.f, 0.f, 0.f, 0.f};
    d = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[mt][0], h[0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[mt][1], h[1], d, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const _Float16 z = (_Float16)fmaxf(d[i] + b[mt][i], 0.f);
      out[mt >> 1][4 * (mt & 1) + i] = z;
      if (keep) keep[mt][i] = (float)z;
    }
  }
}

// Output layer: lanes 0..15 return (Re, Im) of y for sample (lane & 15).
__device__ __forceinline__ float2 out_layer(const Net& n, const h8 (&h)[2]) {
  f4 d = {0.f, 0.f, 0.f, 0.f};
  d = __builtin_amdgcn_mfma_f32_16x16x32_f16(n.w4[0][0], h[0], d, 0, 0, 0);
  d = __builtin_amdgcn_mfma_f32_16x16x32_f16(n.w4[0][1], h[1], d, 0, 0, 0);
  return make_float2(d[0] + n.b4[0][0], d[1] + n.b4[0][1]);
}

// First layer on MFMA from explicit inputs (features of sample lane & 15).
// e_keep (optional, 16 floats) receives the lane's FP16-rounded features in
// (kk, q) order.
__device__ __forceinline__ void layer1(const float (&x)[3], const h8 (&w1)[4][2], const float (&b1)[4][4],
                                       h8 (&h)[2], int lane, float* e_keep, f4* keep) {
  h8 e[2];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const _Float16 v = (_Float16)feature(x, kidx(kk, lane >> 4, q));
      e[kk][q] = v;
      if (e_keep) e_keep[8 * kk + q] = (float)v;
    }
  layer(w1, b1, e, h, keep);
}

__device__ __forceinline__ bool inside_support(const float (&x)[3]) {
  return fabsf(x[1]) < 1.f && fabsf(x[2]) < 1.f;
}

// --------------------------------------------------------------------------
// evaluation: out[n] = tap at inputs[n]
__global__ void __launch_bounds__(256) mlp_eval_kernel(const float* __restrict__ blob,
                                                       const float* __restrict__ inputs, int64_t n,
                                                       float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  Net net;
  load_net(blob, net, lane);
  h8 w1[4][2];
  float b1[4][4];
  load_wfrag<4>(blob + kW1, kHid, w1, lane);
  load_bias<4>(blob + kB1, kHid, b1, lane);
  const float scale = blob[2];
  for (int tile = 0; tile < 4; ++tile) {             // 64 samples per wave
    const int64_t s = wave * 64 + tile * 16 + (lane & 15);
    float x[3] = {0.f, 0.f, 0.f};
    if (s < n)
      for (int i = 0; i < 3; ++i) x[i] = inputs[s * 3 + i];
    h8 h1[2], h2[2], h3[2];
    layer1(x, w1, b1, h1, lane, nullptr, nullptr);
    layer(net.w2, net.b2, h1, h2, nullptr);
    layer(net.w3, net.b3, h2, h3, nullptr);
    const float2 y = out_layer(net, h3);
    if (lane < 16 && s < n) {
      const bool in = inside_support(x);
      out[2 * s] = in ? scale * y.x : 0.f;
      out[2 * s + 1] = in ? scale * y.y : 0.f;
    }
  }
}

// --------------------------------------------------------------------------
// Gradients of the batch loss (1/B) sum |y - t|^2, accumulated into grads.
// One wave per block, 64 samples per wave.  LDS: E, H1, H2, H3 and two delta
// buffers ([64 samples][65] FP32: the pad keeps per-sample rows on distinct
// banks) and W2, W3, W4 (FP32).
constexpr int kLd = 65;
constexpr int kAct = 64 * kLd;
constexpr int kTrainLds = (6 * kAct + 2 * 64 * 64 + 64 * 2) * 4;

__global__ void __launch_bounds__(64)
mlp_grad_kernel(const float* __restrict__ blob, const float* __restrict__ inputs,
                const float* __restrict__ targets, const int32_t* __restrict__ idx, int batch,
                float inv_batch, float* __restrict__ grads, float* __restrict__ loss_sum) {
  extern __shared__ float sm[];
  float* E = sm;
  float* H1 = E + kAct;
  float* H2 = H1 + kAct;
  float* H3 = H2 + kAct;
  float* DA = H3 + kAct;
  float* DB = DA + kAct;
  float* W2 = DB + kAct;
  float* W3 = W2 + 4096;
  float* W4 = W3 + 4096;
  const int lane = threadIdx.x;
  for (int e = lane; e < 4096; e += 64) {
    W2[e] = blob[kW2 + e];
    W3[e] = blob[kW3 + e];
  }
  for (int e = lane; e < 128; e += 64) W4[e] = blob[kW4 + e];
  Net net;
  load_net(blob, net, lane);
  h8 w1[4][2];
  float b1[4][4];
  load_wfrag<4>(blob + kW1, kHid, w1, lane);
  load_bias<4>(blob + kB1, kHid, b1, lane);
  const int base = blockIdx.x * 64;
  const int g = lane >> 4;
  float sq = 0.f;
  // forward: 4 tiles of 16 samples; keep the FP16-rounded activations in LDS
  for (int tile = 0; tile < 4; ++tile) {
    const int sl = tile * 16 + (lane & 15);           // local sample
    const int sg = base + sl;
    const bool live = sg < batch;
    const int64_t src = live ? (int64_t)idx[sg] : 0;
    float x[3];
    for (int i = 0; i < 3; ++i) x[i] = live ? inputs[src * 3 + i] : 0.f;
    float ek[16];
    f4 k1[4], k2[4], k3[4];
    h8 h1[2], h2[2], h3[2];
    layer1(x, w1, b1, h1, lane, ek, k1);
    layer(net.w2, net.b2, h1, h2, k2);
    layer(net.w3, net.b3, h2, h3, k3);
    const float2 y = out_layer(net, h3);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int q = 0; q < 8; ++q) E[sl * kLd + kidx(kk, g, q)] = ek[8 * kk + q];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int f = 16 * mt + 4 * g + i;
        H1[sl * kLd + f] = k1[mt][i];
        H2[sl * kLd + f] = k2[mt][i];
        H3[sl * kLd + f] = k3[mt][i];
      }
    if (lane < 16) {
      const float t0 = live ? targets[2 * src] : 0.f, t1 = live ? targets[2 * src + 1] : 0.f;
      const float r0 = live ? y.x - t0 : 0.f, r1 = live ? y.y - t1 : 0.f;
      sq += r0 * r0 + r1 * r1;
      DA[sl * 2] = 2.f * r0 * inv_batch;              // dL/dy as [64][2] at the start of DA
      DA[sl * 2 + 1] = 2.f * r1 * inv_batch;
    }
  }
  __syncthreads();
  // from here the lane is sample s
  const int s = lane;
  const float dy0 = DA[2 * s], dy1 = DA[2 * s + 1];
  __syncthreads();
  // delta of layer 3: (dy W4^T) * relu'(z3)  (z3 > 0 exactly where h3 > 0)
  for (int i = 0; i < 64; ++i)
    DB[s * kLd + i] = H3[s * kLd + i] > 0.f ? dy0 * W4[2 * i] + dy1 * W4[2 * i + 1] : 0.f;
  // output layer: lane = input feature i
  {
    float g0 = 0.f, g1 = 0.f;
    for (int t = 0; t < 64; ++t) {
      const float h = H3[t * kLd + lane];
      g0 += h * __shfl(dy0, t);
      g1 += h * __shfl(dy1, t);
    }
    atomicAdd(&grads[kW4 + 2 * lane], g0);
    atomicAdd(&grads[kW4 + 2 * lane + 1], g1);
    float sb0 = dy0, sb1 = dy1;
    for (int o = 32; o > 0; o >>= 1) {
      sb0 += __shfl_xor(sb0, o);
      sb1 += __shfl_xor(sb1, o);
    }
    if (lane == 0) {
      atomicAdd(&grads[kB4], sb0);
      atomicAdd(&grads[kB4 + 1], sb1);
    }
  }
  __syncthreads();
  // hidden layers from the top; `delta` holds dL/dz of the current layer
  float* delta = DB;
  float* other = DA;
  for (int L = 0; L < 3; ++L) {
    const float* A = L == 0 ? H2 : (L == 1 ? H1 : E);   // the layer's input
    const int woff = L == 0 ? kW3 : (L == 1 ? kW2 : kW1);
    const int boff = L == 0 ? kB3 : (L == 1 ? kB2 : kB1);
    // dW[i][j] = sum_s A[s][i] delta[s][j]; lane = j (rows of always-zero features skipped)
    const int n_rows = L == 2 ? kFeat : 64;
    for (int i = 0; i < n_rows; ++i) {
      float gsum = 0.f;
      for (int t = 0; t < 64; ++t) gsum += A[t * kLd + i] * delta[t * kLd + lane];
      atomicAdd(&grads[woff + i * 64 + lane], gsum);
    }
    {
      float gb = 0.f;
      for (int t = 0; t < 64; ++t) gb += delta[t * kLd + lane];
      atomicAdd(&grads[boff + lane], gb);
    }
    if (L < 2) {
      // delta of the layer below: (delta W^T) * relu'(A); lane = sample s
      const float* Wl = L == 0 ? W3 : W2;
      for (int i = 0; i < 64; ++i) {
        float a = 0.f;
        for (int j = 0; j < 64; ++j) a += delta[s * kLd + j] * Wl[i * 64 + j];
        other[s * kLd + i] = A[s * kLd + i] > 0.f ? a : 0.f;
      }
      __syncthreads();
      float* t = delta;
      delta = other;
      other = t;
    }
  }
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
  if (lane == 0 && loss_sum) atomicAdd(loss_sum, sq * inv_batch);
}

__global__ void __launch_bounds__(256) fill_f32(float* p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Adam (Kingma & Ba 2015) on every parameter; the header floats are left alone.
__global__ void __launch_bounds__(256)
mlp_adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                const float* __restrict__ g, int step, float lr, float b1, float b2, float eps) {
  const int i = kHdr + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Training set from a 2-D table [planes][O][O][S][S] of complex f32 (indexed
// [plane][s_v][s_u][k_v][k_u]): inputs (w_hat / w_hat_range, d_u / (S/2),
// d_v / (S/2)) and targets tap / out_scale.
__global__ void __launch_bounds__(256)
mlp_dataset_kernel(const float2* __restrict__ table, int S, int O, int64_t n, double wh0,
                   double whs, double wh_range, float inv_scale, float* __restrict__ inputs,
                   float* __restrict__ targets) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ku = (int)(i % S), kv = (int)((i / S) % S);
  const int su = (int)((i / ((int64_t)S * S)) % O), sv = (int)((i / ((int64_t)S * S * O)) % O);
  const int64_t plane = i / ((int64_t)S * S * O * O);
  const double h = 0.5 * S;
  inputs[3 * i] = (float)((wh0 + (double)plane * whs) / wh_range);
  inputs[3 * i + 1] = (float)(((double)ku - h + 1.0 - (double)su / O) / h);
  inputs[3 * i + 2] = (float)(((double)kv - h + 1.0 - (double)sv / O) / h);
  const float2 t = table[i];
  targets[2 * i] = t.x * inv_scale;
  targets[2 * i + 1] = t.y * inv_scale;
}

// --------------------------------------------------------------------------
// Fused gridding with network taps over the binned stream.  Per visibility:
//  (1) the first layer splits into a per-visibility part c (features of x0,
//      plus b1) and per-tap parts U[k_u], V[k_v] (features of x1, x2), each a
//      64-vector, computed in FP32 into LDS;
//  (2) the block's 4 waves evaluate h1 = relu(c + U + V) and the remaining
//      layers for all S x S taps on matrix cores, taps into LDS;
//  (3) every work-item updates its C x C cells of the window (C = window / 16,
//      the support's window of 32, 48 or 64 cells) from LDS; the window is
//      added to the grid once at the end of the segment.
// The layer weights stay in registers as A operands and the hidden biases are
// read from LDS when used, so that two waves fit per SIMD.
struct MlpGridDev {
  int S, O, tile, n_tx, H, W;
};

// One hidden layer of the gridder on a 16-sample tile, its biases read from
// LDS (bias[m], m = 16 mt + 4 (lane / 16) + i, the D rows the lane holds) into
// the accumulator: relu(b + W^T h).
__device__ __forceinline__ void layer_lds_bias(const h8 (&w)[4][2], const float* __restrict__ bias,
                                               const h8 (&h)[2], h8 (&out)[2], int lane) {
  u4 words[2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f4 d = *reinterpret_cast<const f4*>(bias + 16 * mt + 4 * (lane >> 4));
    d = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[mt][0], h[0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[mt][1], h[1], d, 0, 0, 0);
    // element 4 (mt & 1) + i of out[mt / 2] is relu(d[i]); two elements per word
    words[mt >> 1][2 * (mt & 1)] = relu_h2(f2v{d[0], d[1]});
    words[mt >> 1][2 * (mt & 1) + 1] = relu_h2(f2v{d[2], d[3]});
  }
  out[0] = __builtin_bit_cast(h8, words[0]);
  out[1] = __builtin_bit_cast(h8, words[1]);
}

// row pitch (floats) of the layer-1 parts, [axis][k][64 units] with 4 floats
// of padding: the 16 lanes of a tap tile read 16 consecutive k at the same
// units, 272 bytes apart, so each lane's 16-byte read lands on its own 4 of
// the 64 banks
constexpr int kUVP = 68;

// layer_lds_bias on two independent tiles with the same weights, their
// products interleaved
__device__ __forceinline__ void layer_lds_bias2(const h8 (&w)[4][2], const float* __restrict__ bias,
                                                const h8 (&h)[2][2], h8 (&out)[2][2], int lane) {
  u4 words[2][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f4 b = *reinterpret_cast<const f4*>(bias + 16 * mt + 4 * (lane >> 4));
    f4 d[2] = {b, b};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int c = 0; c < 2; ++c) d[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w[mt][kk], h[c][kk], d[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      words[c][mt >> 1][2 * (mt & 1)] = relu_h2(f2v{d[c][0], d[c][1]});
      words[c][mt >> 1][2 * (mt & 1) + 1] = relu_h2(f2v{d[c][2], d[c][3]});
    }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    out[c][0] = __builtin_bit_cast(h8, words[c][0]);
    out[c][1] = __builtin_bit_cast(h8, words[c][1]);
  }
}

template <int P, int C>
__device__ __forceinline__ void grid_mlp_body(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                                              const int4* __restrict__ segs, const int32_t* __restrict__ n_segs_p,
                                              const float* __restrict__ blob, float2* __restrict__ grid,
                                              const MlpGridDev& d) {
  extern __shared__ __align__(16) float smg[];
  const int S = d.S, O = d.O;
  float* W1e = smg;                        // [12][64] rows 0..11 of W1 (w features)
  float* F = W1e + 12 * 64;                // [2][S][12] offset features, 0 = u, 1 = v
  // per-tap layer-1 parts, tap-major: UV[axis][k][unit] with row pitch kUVP, so
  // that a lane's four runs of 4 consecutive units (the K layout of kidx) are
  // four aligned 16-byte reads
  float* UV = F + 2 * S * 12;
  float* E = UV + 2 * S * kUVP;            // [64] the visibility's w features (12 used)
  float* zero = E + 64;                    // [2][S] 1 where the offset is outside the support
  float2* taps = reinterpret_cast<float2*>(zero + 2 * S);   // [S * S] (2 S is even: 8-byte aligned)
  float* bias = reinterpret_cast<float*>(taps + S * S);    // [2][64] b2, b3 (S * S * 8 bytes: 16-byte aligned)
  const int seg = (int)blockIdx.x;
  if (seg >= *n_segs_p) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // layer-1 weights of this thread's hidden unit j (every (j, k) entry it forms
  // below has j = t mod 64): w features, u features, v features, and the bias
  const int jh = t & 63;
  float w1u[12], w1v[12];
#pragma unroll
  for (int f = 0; f < 12; ++f) {
    w1u[f] = blob[kW1 + (12 + f) * kHid + jh];
    w1v[f] = blob[kW1 + (24 + f) * kHid + jh];
  }
  const float b1j = blob[kB1 + jh];
  for (int e = t; e < 12 * 64; e += 256) W1e[e] = blob[kW1 + e];
  if (t < 2 * kHid) bias[t] = t < kHid ? blob[kB2 + t] : blob[kB3 + t - kHid];
  h8 w2[4][2], w3[4][2], w4[1][2];
  float b4[1][4];
  load_wfrag<4>(blob + kW2, kHid, w2, lane);
  load_wfrag<4>(blob + kW3, kHid, w3, lane);
  load_wfrag<1>(blob + kW4, 2, w4, lane);
  load_bias<1>(blob + kB4, 2, b4, lane);
  const float x0_off = blob[0], x0_step = blob[1], out_scale = blob[2];
  const float half = 0.5f * (float)S;
  const int4 sg = segs[seg];
  const int begin = sg.x, len = sg.y, tile_id = sg.z;
  const int win_x0 = (tile_id % d.n_tx) * d.tile;
  const int win_y0 = (tile_id / d.n_tx) * d.tile;
  const int cy = C * (t >> 4), cx = C * (t & 15);
  float2 acc[C][C][P];
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
      for (int p = 0; p < P; ++p) acc[i][j][p] = make_float2(0.f, 0.f);
  const int n_taps = S * S;
  const uint32_t magic_s = (uint32_t)((0x100000000ull + (uint64_t)S - 1) / (uint64_t)S);   // ceil(2^32 / S)
  for (int q = 0; q < len; ++q) {
    const Record r = rec[begin + q];
    __syncthreads();                                    // the previous visibility's LDS is consumed
    // the features: sin and cos of pi 2^kf x for the visibility's w (items 0..5)
    // and for the offset of every (axis, k) (items 6 + 6 e + kf), one sincos each
    const float xw = x0_off + (float)rec_plane(r) * x0_step;
    for (int it = t; it < 6 + 12 * S; it += 256) {
      if (it < 6) {
        float sn, cs;
        sincospif(xw * (float)(1 << it), &sn, &cs);
        E[2 * it] = sn;
        E[2 * it + 1] = cs;
      } else {
        const int e = (it - 6) / 6, kf = (it - 6) - 6 * e, axis = e / S, k = e - axis * S;
        const int s = axis ? rec_sy(r) : rec_sx(r);
        const float dd = ((float)k - half + 1.f - (float)s / (float)O) / half;
        float sn, cs;
        sincospif(dd * (float)(1 << kf), &sn, &cs);
        F[e * 12 + 2 * kf] = sn;
        F[e * 12 + 2 * kf + 1] = cs;
        if (kf == 0) zero[e] = fabsf(dd) < 1.f ? 0.f : 1.f;
      }
    }
    __syncthreads();
    {
      // the per-visibility part of layer 1 for this thread's j, joined to the u
      // part once per (j, k) in the order (c + U) + V of the layer-1 sum
      float ef[12];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float4 v4 = reinterpret_cast<const float4*>(E)[q];
        ef[4 * q] = v4.x; ef[4 * q + 1] = v4.y; ef[4 * q + 2] = v4.z; ef[4 * q + 3] = v4.w;
      }
      float cj = b1j;
#pragma unroll
      for (int f = 0; f < 12; ++f) cj += ef[f] * W1e[f * 64 + jh];
      // the 2 S rows (axis, k) of F, four per pass of the block (one per wave):
      // c[j] + U[j][k] for the u rows, V[j][k] for the v rows
      auto row_part = [&](int row, const float (&w)[12]) -> float {
        const float4* fr = reinterpret_cast<const float4*>(F + row * 12);
        float fv[12];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float4 v4 = fr[q];
          fv[4 * q] = v4.x; fv[4 * q + 1] = v4.y; fv[4 * q + 2] = v4.z; fv[4 * q + 3] = v4.w;
        }
        float a = 0.f;
#pragma unroll
        for (int f = 0; f < 12; ++f) a += fv[f] * w[f];
        return a;
      };
      for (int k = t >> 6; k < S; k += 4) UV[k * kUVP + jh] = cj + row_part(k, w1u);
      for (int k = t >> 6; k < S; k += 4) UV[(S + k) * kUVP + jh] = row_part(S + k, w1v);
    }
    __syncthreads();
    // taps: the waves take 16-tap tiles in turn, two at a time (tiles tb and
    // tb + 64), so that each wave has two independent chains of layer products
    // in flight
    for (int tb = wave * 16; tb < n_taps; tb += 128) {
      int tap[2], ku[2], kv[2];
      bool live[2];
      h8 h1[2][2], h2[2][2], h3[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        tap[c] = tb + 64 * c + (lane & 15);
        live[c] = tap[c] < n_taps;
        const int qv = (int)__umulhi((uint32_t)tap[c], magic_s);   // tap / S (tap < 2^12)
        ku[c] = live[c] ? tap[c] - qv * S : 0;
        kv[c] = live[c] ? qv : 0;
        const float* U = UV + ku[c] * kUVP;
        const float* V = UV + (S + kv[c]) * kUVP;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          u4 words;
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            // elements 4 half .. 4 half + 3 are units kidx(kk, g, 4 half) + 0..3
            const int f0 = kidx(kk, lane >> 4, 4 * half);
            const float4 u = *reinterpret_cast<const float4*>(U + f0);
            const float4 v = *reinterpret_cast<const float4*>(V + f0);
            words[2 * half] = relu_h2(f2v{u.x + v.x, u.y + v.y});
            words[2 * half + 1] = relu_h2(f2v{u.z + v.z, u.w + v.w});
          }
          h1[c][kk] = __builtin_bit_cast(h8, words);
        }
      }
      layer_lds_bias2(w2, bias, h1, h2, lane);
      layer_lds_bias2(w3, bias + kHid, h2, h3, lane);
      f4 dy[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) dy[c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int c = 0; c < 2; ++c) dy[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(w4[0][kk], h3[c][kk], dy[c], 0, 0, 0);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float2 y = make_float2(dy[c][0] + b4[0][0], dy[c][1] + b4[0][1]);
        if (lane < 16 && live[c]) {
          const bool out = zero[ku[c]] != 0.f || zero[S + kv[c]] != 0.f;
          taps[tap[c]] = out ? make_float2(0.f, 0.f) : make_float2(out_scale * y.x, out_scale * y.y);
        }
      }
    }
    __syncthreads();
    const int oy = rec_y0(r) - win_y0, ox = rec_x0(r) - win_x0;
    if (cy + C - 1 < oy || cy >= oy + S || cx + C - 1 < ox || cx >= ox + S) continue;
    float2 vv[P];
#pragma unroll
    for (int p = 0; p < P; ++p) vv[p] = wvis[(int64_t)(begin + q) * P + p];
#pragma unroll
    for (int i = 0; i < C; ++i) {
      const int ky = cy + i - oy;
      if ((unsigned)ky >= (unsigned)S) continue;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int kx = cx + j - ox;
        if ((unsigned)kx >= (unsigned)S) continue;
        const float2 g = taps[ky * S + kx];
#pragma unroll
        for (int p = 0; p < P; ++p) {
          float2& a = acc[i][j][p];
          a.x = fmaf(g.x, vv[p].x, a.x);
          a.x = fmaf(-g.y, vv[p].y, a.x);
          a.y = fmaf(g.x, vv[p].y, a.y);
          a.y = fmaf(g.y, vv[p].x, a.y);
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

// 32- and 48-cell windows: two waves per SIMD; the 64-cell window's 4 x 4 x P
// accumulators would spill under that limit, so it runs one
template <int P, int C>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
grid_mlp_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis, const int4* __restrict__ segs,
                const int32_t* __restrict__ n_segs_p, const float* __restrict__ blob, float2* __restrict__ grid,
                MlpGridDev d) {
  grid_mlp_body<P, C>(rec, wvis, segs, n_segs_p, blob, grid, d);
}

template <int P>
__global__ void __launch_bounds__(256)
grid_mlp_kernel_w64(const Record* __restrict__ rec, const float2* __restrict__ wvis, const int4* __restrict__ segs,
                    const int32_t* __restrict__ n_segs_p, const float* __restrict__ blob, float2* __restrict__ grid,
                    MlpGridDev d) {
  grid_mlp_body<P, 4>(rec, wvis, segs, n_segs_p, blob, grid, d);
}

size_t grid_mlp_lds(int S) {
  return sizeof(float) * (12 * 64 + 2 * (size_t)S * 12 + 2 * (size_t)S * kUVP + 64 + 2 * (size_t)S) +
         sizeof(float2) * (size_t)S * S + sizeof(float) * 2 * kHid;
}

}  // namespace

gr_status launch_grid_mlp(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                          float2* grid, int height, int width, hipStream_t stream) {
  if (k.support > 56) return fail(GR_EUNSUPPORTED, "the binned gridders need support <= 56");
  if (L.max_segs > 0x7fffffff) return fail(GR_EINVAL, "too many segments");
  if (L.max_segs == 0) return GR_OK;
  const char* base = reinterpret_cast<const char*>(bins);
  const auto* rec = reinterpret_cast<const Record*>(base + L.off_rec);
  const auto* wv = reinterpret_cast<const float2*>(base + L.off_wvis);
  const auto* segs = reinterpret_cast<const int4*>(base + L.off_segs);
  const auto* nsegs = reinterpret_cast<const int32_t*>(base + L.off_nsegs);
  MlpGridDev d{k.support, k.oversample, L.tile, L.n_tx, height, width};
  const int window = L.tile + k.support;             // 32, 48 or 64: the support's window
  if (window != 32 && window != 48 && window != 64)
    return fail(GR_EINVAL, "gr_grid_binned (network taps): binning tile does not match a 32, 48 or 64-cell window");
  const size_t lds = grid_mlp_lds(k.support);
  using Fn = void (*)(const Record*, const float2*, const int4*, const int32_t*, const float*, float2*, MlpGridDev);
  Fn fn;
  if (n_pol == 4) fn = window == 32 ? grid_mlp_kernel<4, 2> : window == 48 ? grid_mlp_kernel<4, 3> : grid_mlp_kernel_w64<4>;
  else fn = window == 32 ? grid_mlp_kernel<1, 2> : window == 48 ? grid_mlp_kernel<1, 3> : grid_mlp_kernel_w64<1>;
  {
    const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds, "mlp.hip");
    if (lst != GR_OK) return lst;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)L.max_segs), dim3(256), lds, stream, rec, wv, segs, nsegs,
                     reinterpret_cast<const float*>(k.taps), grid, d);
  return check_launch("gr_grid_binned (network taps)");
}

}  // namespace gr

using namespace gr;

extern "C" int32_t gr_mlp_blob_floats(void) { return kBlob; }

extern "C" gr_status gr_mlp_eval(const float* weights, const float* inputs, int64_t n, float* out,
                                 void* stream) {
  if (n < 0) return fail(GR_EINVAL, "gr_mlp_eval: n must be >= 0");
  if (weights == nullptr || (n > 0 && (inputs == nullptr || out == nullptr)))
    return fail(GR_EINVAL, "gr_mlp_eval: NULL pointer");
  if (n == 0) return GR_OK;
  const int64_t waves = (n + 63) / 64, blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_mlp_eval: n too large");
  mlp_eval_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(weights, inputs, n, out);
  return check_launch("gr_mlp_eval");
}

extern "C" gr_status gr_mlp_grads(const float* weights, const float* inputs, const float* targets,
                                  const int32_t* idx, int32_t batch, float* grads, float* loss_sum,
                                  void* stream) {
  if (weights == nullptr || inputs == nullptr || targets == nullptr || idx == nullptr || grads == nullptr)
    return fail(GR_EINVAL, "gr_mlp_grads: NULL pointer");
  if (batch < 1) return fail(GR_EINVAL, "gr_mlp_grads: batch must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  fill_f32<<<(kBlob + 255) / 256, 256, 0, s>>>(grads, kBlob, 0.f);
  if (loss_sum) fill_f32<<<1, 64, 0, s>>>(loss_sum, 1, 0.f);
  const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(mlp_grad_kernel), kTrainLds, "gr_mlp_grads");
  if (lst != GR_OK) return lst;
  mlp_grad_kernel<<<(batch + 63) / 64, 64, kTrainLds, s>>>(weights, inputs, targets, idx, batch,
                                                            1.f / (float)batch, grads, loss_sum);
  return check_launch("gr_mlp_grads");
}

extern "C" gr_status gr_mlp_train_step(float* weights, float* adam_m, float* adam_v, float* grads,
                                       const float* inputs, const float* targets, const int32_t* idx,
                                       int32_t batch, int32_t step, float lr, float* loss_sum,
                                       void* stream) {
  if (adam_m == nullptr || adam_v == nullptr) return fail(GR_EINVAL, "gr_mlp_train_step: NULL Adam state");
  if (step < 1) return fail(GR_EINVAL, "gr_mlp_train_step: step counts from 1");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(GR_EINVAL, "gr_mlp_train_step: bad learning rate");
  gr_status st = gr_mlp_grads(weights, inputs, targets, idx, batch, grads, loss_sum, stream);
  if (st != GR_OK) return st;
  mlp_adam_kernel<<<(kParams - kHdr + 255) / 256, 256, 0, (hipStream_t)stream>>>(
      weights, adam_m, adam_v, grads, step, lr, 0.9f, 0.999f, 1e-8f);
  return check_launch("gr_mlp_train_step");
}

extern "C" gr_status gr_mlp_dataset(const void* table2d, int32_t support, int32_t oversample,
                                    int32_t n_planes, double w_hat_first, double w_hat_step,
                                    double w_hat_range, float out_scale, float* inputs, float* targets,
                                    void* stream) {
  if (table2d == nullptr || inputs == nullptr || targets == nullptr)
    return fail(GR_EINVAL, "gr_mlp_dataset: NULL pointer");
  if (support < 2 || support > 64 || oversample < 1 || oversample > kMaxOversample || n_planes < 1 ||
      n_planes > kMaxPlanes || !(w_hat_range > 0.0) || !(out_scale > 0.f) || !std::isfinite(w_hat_first) ||
      !std::isfinite(w_hat_step))
    return fail(GR_EINVAL, "gr_mlp_dataset: bad sizes or scales");
  const int64_t n = (int64_t)n_planes * oversample * oversample * support * support;
  mlp_dataset_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      reinterpret_cast<const float2*>(table2d), support, oversample, n, w_hat_first, w_hat_step,
      w_hat_range, 1.f / out_scale, inputs, targets);
  return check_launch("gr_mlp_dataset");
}
