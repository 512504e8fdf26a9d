// Romein work distribution with thread coarsening, on the VALU.
//
// Merry (2016), Sections 2.2-4:
//  * the grid is divided into bins at least as large as the GCF; a work-item
//    owns every cell at the same position modulo the bin (Section 2.2);
//  * with thread coarsening each work-item owns a block of cu x cv cells and
//    the bounding box around the footprint is aligned to block edges, so it is
//    B = c * n >= S + c - 1 cells wide; padding taps are zero (Section 3);
//  * a work-item keeps register accumulators for its current block and flushes
//    them with atomic adds when the block leaves the bounding box (Section 2.2);
//  * work-items take a fixed number of consecutive visibilities in the given
//    order (Section 4 uses 1024 per work-group), one per residue of the bin;
//  * the separable GCF: each work-item loads cu + cv taps and forms the
//    products in registers (Section 4), using the factored form
//    G^u_i (G^v_j V_p) named as future work in Section 6 (the factor shared
//    along the shorter side of the block is formed first).
//
// gfx950 mapping.  Work-items of the method are independent, so their
// grouping into waves is free: the work-items (chunk c, residue r) are ordered
// chunk-major, and each wave takes 64 consecutive ones, so no lane idles at
// the edge of a bin (a wave may straddle two or three chunks; its lanes then
// read different visibilities, each group one address).  One block per
// compute unit stages the zero-padded tap table in LDS once, as FP32, and its
// waves (16 per CU, or 8 for 64 accumulators) take 64-lane runs in turn from a
// work counter (gr_grid's workspace holds one), or with a fixed stride over
// the launch (gr_grid_records, which has no workspace).  A work-item streams its chunk with the next
// visibility's loads in flight while it updates the current one; flushes are
// FP32 global atomic adds (no-return), skipping zero values.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace gr {

namespace {

struct RomeinDev {
  int nu, nv, n_res;              // blocks per bin per axis, residues per bin
  int wgu, wgv, tiles_u;          // residue order: tiles of wgu x wgv blocks, u first
  int lpad, pad_off, n_rows_tab, S, H, W, O, tap_dtype;
  uint32_t magic_u, magic_v;      // ceil(2^32 / n): x mod n by one high multiply
  int koff_u, koff_v;             // multiples of nu, nv above any block index
  int n_vis, chunk_len;           // this launch's piece of the stream (< 2^26)
  int n_runs;                     // runs: 64 consecutive work-items (< 2^31)
  int32_t* counter;               // runs taken in turn from it, or NULL: fixed stride
};

__device__ inline float load_tap(const void* __restrict__ t, int64_t idx, int dtype) {
  switch (dtype) {
    case GR_F32: return reinterpret_cast<const float*>(t)[idx];
    case GR_F16: return __half2float(reinterpret_cast<const __half*>(t)[idx]);
    default: return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(t)[idx]);
  }
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Threads per block for a work-item holding A = cu * cv * n_pol complex
// accumulators: 4 waves per SIMD (128 registers each) up to 32, 2 above.
__host__ __device__ constexpr int romein_threads(int acc) { return acc <= 32 ? 1024 : 512; }

template <int CU, int CV, int P, bool CPLX>
__global__ void __launch_bounds__(romein_threads(CU * CV * P))
romein_valu_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                   const void* __restrict__ taps, float2* __restrict__ grid, RomeinDev d) {
  using Tap = typename std::conditional<CPLX, float2, float>::type;
  constexpr int THREADS = romein_threads(CU * CV * P);
  constexpr int WAVES = THREADS / 64;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Tap* lds = reinterpret_cast<Tap*>(lds_raw);
  // residue order: res_of[q] = ru | rv << 8 for the q-th residue
  uint16_t* res_of = reinterpret_cast<uint16_t*>(lds_raw + (size_t)d.n_rows_tab * d.lpad * sizeof(Tap));

  // ---- stage the zero-padded tap table: [plane * O + s][lpad], FP32
  const int n_elem = d.n_rows_tab * d.lpad;
  for (int e = threadIdx.x; e < n_elem; e += THREADS) {
    const int row = e / d.lpad;
    const int k = e - row * d.lpad - d.pad_off;
    Tap v;
    if constexpr (CPLX) {
      v = make_float2(0.f, 0.f);
      if (k >= 0 && k < d.S) {
        const int64_t base = ((int64_t)row * d.S + k) * 2;
        v = make_float2(load_tap(taps, base, d.tap_dtype), load_tap(taps, base + 1, d.tap_dtype));
      }
    } else {
      v = 0.f;
      if (k >= 0 && k < d.S) v = load_tap(taps, (int64_t)row * d.S + k, d.tap_dtype);
    }
    lds[e] = v;
  }
  // ---- residue order: tiles of wgu x wgv blocks (edge tiles clipped), u first
  for (int e = threadIdx.x; e < d.n_res; e += THREADS) {
    const int rv = e / d.nu, ru = e - rv * d.nu;
    const int tu = ru / d.wgu, tv = rv / d.wgv;
    const int h = min(d.wgv, d.nv - tv * d.wgv), w = min(d.wgu, d.nu - tu * d.wgu);
    const int q = tv * d.wgv * d.nu + tu * d.wgu * h + (rv - tv * d.wgv) * w + (ru - tu * d.wgu);
    res_of[q] = (uint16_t)(ru | (rv << 8));
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int stride = (int)gridDim.x * WAVES;
  const char* rec_b = reinterpret_cast<const char*>(rec);
  const char* vis_b = reinterpret_cast<const char*>(wvis);
  // the wave's next run: from the counter (wave-uniform), or the fixed stride
  auto next_run = [&](int prev) -> int {
    if (d.counter == nullptr) return prev < 0 ? (int)blockIdx.x * WAVES + wave : prev + stride;
    int r = 0;
    if (lane == 0) r = atomicAdd(d.counter, 1);
    return __builtin_amdgcn_readfirstlane(r);
  };
  for (int run = next_run(-1); run < d.n_runs; run = next_run(run)) {
    // this lane's work-item: (chunk, residue) number run * 64 + lane
    const int64_t e = (int64_t)run * 64 + lane;
    const int chunk = (int)(e / d.n_res);
    const int q = (int)(e - (int64_t)chunk * d.n_res);
    const int nbase = chunk * d.chunk_len;                    // < 2^26 + chunk_len: no overflow
    const int len = nbase < d.n_vis ? min(d.chunk_len, d.n_vis - nbase) : 0;
    const uint32_t rr = res_of[q];
    // residues offset by a multiple of n above any block index: (r - b) mod n
    // is then taken of a non-negative number
    const int ru_k = (int)(rr & 0xffu) + d.koff_u, rv_k = (int)(rr >> 8) + d.koff_v;
    // every lane of the run in one chunk: the visibility is wave-uniform and is
    // decoded on the scalar unit
    const int64_t e0 = (int64_t)run * 64;
    const bool uniform_run = e0 / d.n_res == (e0 + 63) / d.n_res;

    auto body = [&](auto uniform_tag) {
      constexpr bool UNI = decltype(uniform_tag)::value;
      float2 acc[CU][CV][P];
#pragma unroll
      for (int i = 0; i < CU; ++i)
#pragma unroll
        for (int j = 0; j < CV; ++j)
#pragma unroll
          for (int p = 0; p < P; ++p) acc[i][j][p] = make_float2(0.f, 0.f);
      int cju = -1, cjv = -1;                                 // current block (block units)

      auto flush = [&]() {
#pragma unroll
        for (int j = 0; j < CV; ++j) {
          const int row = cjv * CV + j;
#pragma unroll
          for (int i = 0; i < CU; ++i) {
            const int col = cju * CU + i;
            const bool inside = row < d.H && col < d.W;
#pragma unroll
            for (int p = 0; p < P; ++p) {
              float* cell = reinterpret_cast<float*>(grid + ((int64_t)p * d.H + row) * d.W + col);
              const float2 a = acc[i][j][p];
              if (inside && a.x != 0.f) unsafeAtomicAdd(cell, a.x);
              if (inside && a.y != 0.f) unsafeAtomicAdd(cell + 1, a.y);
              acc[i][j][p] = make_float2(0.f, 0.f);
            }
          }
        }
      };

      // the next visibility's record and values, loaded one step ahead (a lane
      // past its chunk's end re-reads the chunk's last entry, one past the
      // piece's end reads entry 0, and both ignore what they read); 32-bit
      // byte offsets (a piece holds < 2^26 visibilities)
      auto load = [&](int k, Record& r, float2 (&v)[P]) {
        const uint32_t n = len > 0 ? (uint32_t)(nbase + min(k, len - 1)) : 0u;
        r = *reinterpret_cast<const Record*>(rec_b + n * 8u);
        if constexpr (P == 4) {
          const float4* src = reinterpret_cast<const float4*>(vis_b + n * 32u);
          const float4 a = src[0], b = src[1];
          v[0] = make_float2(a.x, a.y); v[1] = make_float2(a.z, a.w);
          v[2] = make_float2(b.x, b.y); v[3] = make_float2(b.z, b.w);
        } else {
          v[0] = *reinterpret_cast<const float2*>(vis_b + n * 8u);
        }
      };
      const int len_w = UNI ? (int)uni((uint32_t)len) : len;
      // one visibility: its record r and weighted values vis, at position k
      auto step = [&](int k, Record r, const float2 (&vis_in)[P]) {
        float2 vis[P];
#pragma unroll
        for (int p = 0; p < P; ++p) vis[p] = vis_in[p];
        if constexpr (UNI) {
          r.x = uni(r.x);
          r.y = uni(r.y);
#pragma unroll
          for (int p = 0; p < P; ++p) vis[p] = make_float2(uni(vis[p].x), uni(vis[p].y));
        }
        if (k < len_w && rec_valid(r)) {
          const int x0 = rec_x0(r), y0 = rec_y0(r);
          // aligned bounding box origin (blocks); this work-item's block is the
          // one in [b, b + n) congruent to its residue: b + (r - b) mod n
          const int bu = x0 / CU, bv = y0 / CV;
          const uint32_t tu = (uint32_t)(ru_k - bu), tv = (uint32_t)(rv_k - bv);
          const int ju = bu + (int)(tu - __umulhi(tu, d.magic_u) * (uint32_t)d.nu);
          const int jv = bv + (int)(tv - __umulhi(tv, d.magic_v) * (uint32_t)d.nv);
          if (ju != cju || jv != cjv) {
            if (cju >= 0) flush();
            cju = ju;
            cjv = jv;
          }
          // taps: cu along u, cv along v, from the padded LDS rows
          const int row_u = (rec_plane(r) * d.O + rec_sx(r)) * d.lpad - x0 + d.pad_off;
          const int row_v = (rec_plane(r) * d.O + rec_sy(r)) * d.lpad - y0 + d.pad_off;
          const Tap* tu_row = lds + row_u + ju * CU;
          const Tap* tv_row = lds + row_v + jv * CV;
          Tap gu[CU], gv[CV];
#pragma unroll
          for (int i = 0; i < CU; ++i) gu[i] = tu_row[i];
#pragma unroll
          for (int j = 0; j < CV; ++j) gv[j] = tv_row[j];
          // the shorter side's taps times the visibilities first, then the
          // longer side's taps times those: acc_ijp += G^u_i (G^v_j V_p)
          constexpr bool V_FIRST = CV <= CU;
          constexpr int NS = V_FIRST ? CV : CU, NL = V_FIRST ? CU : CV;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const Tap gs = V_FIRST ? gv[s] : gu[s];
#pragma unroll
            for (int p = 0; p < P; ++p) {
              float2 t;
              if constexpr (CPLX) {
                t.x = gs.x * vis[p].x - gs.y * vis[p].y;
                t.y = gs.x * vis[p].y + gs.y * vis[p].x;
              } else {
                t.x = gs * vis[p].x;
                t.y = gs * vis[p].y;
              }
#pragma unroll
              for (int l = 0; l < NL; ++l) {
                const Tap g = V_FIRST ? gu[l] : gv[l];
                float2& a = V_FIRST ? acc[l][s][p] : acc[s][l][p];
                if constexpr (CPLX) {
                  a.x = fmaf(g.x, t.x, a.x);
                  a.x = fmaf(-g.y, t.y, a.x);
                  a.y = fmaf(g.x, t.y, a.y);
                  a.y = fmaf(g.y, t.x, a.y);
                } else {
                  a.x = fmaf(g, t.x, a.x);
                  a.y = fmaf(g, t.y, a.y);
                }
              }
            }
          }
        }
      };
      // two register sets for the loads in flight, used in turn
      Record ra, rb;
      float2 va[P], vb[P];
      load(0, ra, va);
      for (int k = 0; k < d.chunk_len; k += 2) {
        load(k + 1, rb, vb);
        step(k, ra, va);
        load(k + 2, ra, va);
        step(k + 1, rb, vb);
      }
      if (cju >= 0) flush();
    };
    if (uniform_run) body(std::true_type{});
    else body(std::false_type{});
  }
}

using KernFn = void (*)(const Record*, const float2*, const void*, float2*, RomeinDev);

template <int CU, int CV>
KernFn pick_pc(int n_pol, bool cplx) {
  if (n_pol == 1) return cplx ? romein_valu_kernel<CU, CV, 1, true> : romein_valu_kernel<CU, CV, 1, false>;
  if constexpr (CU * CV <= 16)
    return cplx ? romein_valu_kernel<CU, CV, 4, true> : romein_valu_kernel<CU, CV, 4, false>;
  return nullptr;
}

template <int CU>
KernFn pick_v(int cv, int n_pol, bool cplx) {
  switch (cv) {
    case 1: return pick_pc<CU, 1>(n_pol, cplx);
    case 2: return pick_pc<CU, 2>(n_pol, cplx);
    case 4: return pick_pc<CU, 4>(n_pol, cplx);
    case 8: return pick_pc<CU, 8>(n_pol, cplx);
    default: return nullptr;
  }
}

KernFn pick(int cu, int cv, int n_pol, bool cplx) {
  switch (cu) {
    case 1: return pick_v<1>(cv, n_pol, cplx);
    case 2: return pick_v<2>(cv, n_pol, cplx);
    case 4: return pick_v<4>(cv, n_pol, cplx);
    case 8: return pick_v<8>(cv, n_pol, cplx);
    default: return nullptr;
  }
}

bool valid_c(int c) { return c == 1 || c == 2 || c == 4 || c == 8; }

int g_cus = 0;

int device_cus() {
  if (g_cus > 0) return g_cus;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    g_cus = cus;
  return g_cus > 0 ? g_cus : 256;
}

}  // namespace

gr_status plan_romein(const gr_kernel& k, int n_pol, const gr_tuning* t, RomeinPlan* plan) {
  const int S = k.support;
  RomeinPlan p{};
  int cu = t && t->cu > 0 ? t->cu : 0;
  int cv = t && t->cv > 0 ? t->cv : 0;
  if (cu == 0 || cv == 0) {
    int du, dv;
    if (S <= 8) { du = 2; dv = 2; }
    else if (n_pol == 4) { du = 8; dv = 1; }
    else { du = 4; dv = 4; }
    if (cu == 0) cu = du;
    if (cv == 0) cv = dv;
  }
  if (!valid_c(cu) || !valid_c(cv)) return fail(GR_EINVAL, "tuning: cu and cv must be 1, 2, 4 or 8");
  if (cu * cv * n_pol > 64)
    return fail(GR_EUNSUPPORTED, "tuning: cu * cv * n_pol > 64 exceeds the register budget");
  p.cu = cu;
  p.cv = cv;
  p.nu = (S + cu - 1 + cu - 1) / cu;   // smallest n with c n >= S + c - 1
  p.nv = (S + cv - 1 + cv - 1) / cv;
  if (p.nu > 255 || p.nv > 255) return fail(GR_EUNSUPPORTED, "more than 255 blocks per bin axis");
  if (t && (t->wg_u > 64 || t->wg_v > 64)) return fail(GR_EINVAL, "tuning: wg_u and wg_v must be <= 64");
  p.wgu = std::min(t && t->wg_u > 0 ? t->wg_u : p.nu, p.nu);
  p.wgv = std::min(t && t->wg_v > 0 ? t->wg_v : p.nv, p.nv);
  p.vis_per_wg = t && t->vis_per_wg > 0 ? t->vis_per_wg : 0;
  p.threads = romein_threads(cu * cv * n_pol);
  p.pad_off = std::max(cu, cv) - 1;
  p.lpad = std::max(cu * p.nu, cv * p.nv) + p.pad_off;
  const size_t elem = k.taps_complex ? 8 : 4;
  p.lds_bytes = (size_t)k.n_planes * k.oversample * p.lpad * elem + (size_t)p.nu * p.nv * sizeof(uint16_t);
  if (p.lds_bytes > 160 * 1024)
    return fail(GR_EUNSUPPORTED, "tap table does not fit in LDS (planes * O * padded row)");
  *plan = p;
  return GR_OK;
}

__global__ void __launch_bounds__(64) zero_run_counter(int32_t* c) {
  if (threadIdx.x == 0) *c = 0;
}

gr_status launch_romein(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol,
                        const gr_kernel& k, float2* grid, int height, int width,
                        const RomeinPlan& p, hipStream_t stream, int32_t* counter) {
  if (n_vis == 0) return GR_OK;
  KernFn fn = pick(p.cu, p.cv, n_pol, k.taps_complex != 0);
  if (fn == nullptr) return fail(GR_EUNSUPPORTED, "no kernel instance for this tuning");
  RomeinDev d{};
  d.nu = p.nu; d.nv = p.nv; d.n_res = p.nu * p.nv;
  d.wgu = p.wgu; d.wgv = p.wgv; d.tiles_u = (p.nu + p.wgu - 1) / p.wgu;
  d.lpad = p.lpad; d.pad_off = p.pad_off;
  d.n_rows_tab = k.n_planes * k.oversample;
  d.S = k.support; d.H = height; d.W = width; d.O = k.oversample;
  d.tap_dtype = k.tap_dtype;
  d.magic_u = (uint32_t)((0x100000000ull + p.nu - 1) / p.nu);
  d.magic_v = (uint32_t)((0x100000000ull + p.nv - 1) / p.nv);
  // block indices are below 2^15 (x0, y0 < 32768): a multiple of n at or above that
  d.koff_u = (32768 + p.nu - 1) / p.nu * p.nu;
  d.koff_v = (32768 + p.nv - 1) / p.nv * p.nv;
  const int waves = p.threads / 64;
  const int64_t slots = (int64_t)device_cus() * waves;      // waves of one full launch
  {
    const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(fn), p.lds_bytes, "grid_romein.hip");
    if (lst != GR_OK) return lst;
  }
  // the stream in pieces of < 2^26 visibilities (32-bit offsets in the kernel),
  // each piece its own launch; chunks never straddle pieces
  constexpr int64_t kPiece = (int64_t)1 << 26;
  for (int64_t first = 0; first < n_vis; first += kPiece) {
    const int64_t n = std::min(kPiece, n_vis - first);
    int64_t len = p.vis_per_wg;
    if (len <= 0) {
      // equal chunks: about four 64-lane runs per wave of the launch (eight
      // when the waves take them in turn from the counter)
      const int64_t per_wave = counter != nullptr ? 8 : 4;
      const int64_t chunks = std::max<int64_t>(1, per_wave * slots * 64 / d.n_res);
      len = (n + chunks - 1) / chunks;
      len = std::max<int64_t>(64, (len + 63) / 64 * 64);
    }
    len = std::min<int64_t>(len, kPiece);
    d.n_vis = (int)n;
    d.chunk_len = (int)len;
    const int64_t n_chunks = (n + len - 1) / len;
    const int64_t n_runs = (n_chunks * d.n_res + 63) / 64;    // < 2^20 chunks x 2^16 residues / 64
    d.n_runs = (int)n_runs;
    d.counter = counter;
    const int64_t blocks = std::min<int64_t>(device_cus(), (n_runs + waves - 1) / waves);
    if (counter != nullptr) zero_run_counter<<<1, 64, 0, stream>>>(counter);
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(p.threads), p.lds_bytes, stream, rec + first,
                       wvis + first * n_pol, k.taps, grid, d);
    const gr_status st = check_launch("gr_grid_records (romein)");
    if (st != GR_OK) return st;
  }
  return GR_OK;
}

}  // namespace gr
