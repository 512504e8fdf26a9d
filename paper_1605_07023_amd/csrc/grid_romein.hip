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
//  * the bin is split into tiles, one per wave here, processed in parallel;
//    each work-group takes a fixed number of consecutive visibilities in the
//    given order (Section 4 uses 1024);
//  * the separable GCF: each work-item loads cu + cv taps and forms the
//    products in registers (Section 4), using the factored form
//    G^u_i (G^v_j V_p) named as future work in Section 6.
//
// gfx950 mapping: a tile is one wave64; the visibility record and the P
// visibility values are wave-uniform and are read with scalar loads; the tap
// table, zero-padded so that every block index in the bounding box is a valid
// address, is staged once per work-group in LDS as FP32; flushes are FP32
// global atomic adds (no-return), skipping zero values.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

struct RomeinDev {
  int nu, nv, wgu, wgv, tiles_u, tiles_v, n_tgroups, waves_per_block;
  int vis_per_wg, lpad, pad_off, n_rows_tab, S, H, W, O, tap_dtype;
  uint32_t magic_u, magic_v;
  int64_t n_vis;
  uint32_t n_blocks;
};

__device__ inline float load_tap(const void* __restrict__ t, int64_t idx, int dtype) {
  switch (dtype) {
    case GR_F32: return reinterpret_cast<const float*>(t)[idx];
    case GR_F16: return __half2float(reinterpret_cast<const __half*>(t)[idx]);
    default: return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(t)[idx]);
  }
}

// Blocks are dispatched round-robin over the 8 XCDs.  Map the dispatch index
// so that consecutive logical blocks (the tiles of one chunk, then the next
// chunk of the same visibility stream) run on the same XCD and share its L2.
__device__ inline uint32_t xcd_logical_block(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / 8, r = nb % 8;
  const uint32_t xcd = b % 8, slot = b / 8;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

template <int CU, int CV, int P, bool CPLX>
__global__ void __launch_bounds__(256)
romein_valu_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                   const void* __restrict__ taps, float2* __restrict__ grid, RomeinDev d) {
  using Tap = typename std::conditional<CPLX, float2, float>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Tap* lds = reinterpret_cast<Tap*>(lds_raw);

  // ---- stage the zero-padded tap table: [plane * O + s][lpad], FP32
  const int n_elem = d.n_rows_tab * d.lpad;
  for (int e = threadIdx.x; e < n_elem; e += blockDim.x) {
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
  __syncthreads();

  // ---- which chunk of visibilities and which tile of the bin
  const uint32_t logical = xcd_logical_block(blockIdx.x, d.n_blocks);
  const int chunk = (int)(logical / (uint32_t)d.n_tgroups);
  const int tgroup = (int)(logical % (uint32_t)d.n_tgroups);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = tgroup * d.waves_per_block + wave;
  if (tile >= d.tiles_u * d.tiles_v) return;                 // idle wave (no more barriers)
  const int tu = tile % d.tiles_u, tv = tile / d.tiles_u;
  const int lu = lane % d.wgu, lv = lane / d.wgu;
  const int ru = tu * d.wgu + lu;                            // block residue along u
  const int rv = tv * d.wgv + lv;
  const bool active = lane < d.wgu * d.wgv && ru < d.nu && rv < d.nv;

  const int64_t i0 = (int64_t)chunk * d.vis_per_wg;
  const int64_t i1 = min(d.n_vis, i0 + d.vis_per_wg);

  float2 acc[CU][CV][P];
#pragma unroll
  for (int i = 0; i < CU; ++i)
#pragma unroll
    for (int j = 0; j < CV; ++j)
#pragma unroll
      for (int p = 0; p < P; ++p) acc[i][j][p] = make_float2(0.f, 0.f);
  int cju = -1, cjv = -1;                                    // current block (block units)

  auto flush = [&]() {
    if (cju < 0) return;
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

  for (int64_t n = i0; n < i1; ++n) {
    const Record r = rec[n];                                 // wave-uniform
    if (!rec_valid(r)) continue;
    const int x0 = rec_x0(r), y0 = rec_y0(r);
    const int sx = rec_sx(r), sy = rec_sy(r), plane = rec_plane(r);
    // aligned bounding box origin (blocks) and its residue modulo the bin
    const int bu = x0 / CU, bv = y0 / CV;
    const int mu = bu - (int)__umulhi((uint32_t)bu, d.magic_u) * d.nu;
    const int mv = bv - (int)__umulhi((uint32_t)bv, d.magic_v) * d.nv;
    int du = ru - mu;
    du += du < 0 ? d.nu : 0;
    int dv = rv - mv;
    dv += dv < 0 ? d.nv : 0;
    const int ju = bu + du, jv = bv + dv;                    // this work-item's block
    if (!active) continue;
    if (ju != cju || jv != cjv) {
      flush();
      cju = ju;
      cjv = jv;
    }
    // taps: cu along u, cv along v, from the padded LDS rows
    const Tap* tu_row = lds + (plane * d.O + sx) * d.lpad + (ju * CU - x0 + d.pad_off);
    const Tap* tv_row = lds + (plane * d.O + sy) * d.lpad + (jv * CV - y0 + d.pad_off);
    Tap gu[CU], gv[CV];
#pragma unroll
    for (int i = 0; i < CU; ++i) gu[i] = tu_row[i];
#pragma unroll
    for (int j = 0; j < CV; ++j) gv[j] = tv_row[j];
    float2 vis[P];
#pragma unroll
    for (int p = 0; p < P; ++p) vis[p] = wvis[n * P + p];   // wave-uniform
    // t_jp = G^v_j V_p, then acc_ijp += G^u_i t_jp
#pragma unroll
    for (int j = 0; j < CV; ++j) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        float2 t;
        if constexpr (CPLX) {
          t.x = gv[j].x * vis[p].x - gv[j].y * vis[p].y;
          t.y = gv[j].x * vis[p].y + gv[j].y * vis[p].x;
        } else {
          t.x = gv[j] * vis[p].x;
          t.y = gv[j] * vis[p].y;
        }
#pragma unroll
        for (int i = 0; i < CU; ++i) {
          float2& a = acc[i][j][p];
          if constexpr (CPLX) {
            a.x = fmaf(gu[i].x, t.x, a.x);
            a.x = fmaf(-gu[i].y, t.y, a.x);
            a.y = fmaf(gu[i].x, t.y, a.y);
            a.y = fmaf(gu[i].y, t.x, a.y);
          } else {
            a.x = fmaf(gu[i], t.x, a.x);
            a.y = fmaf(gu[i], t.y, a.y);
          }
        }
      }
    }
  }
  if (active) flush();
}

using KernFn = void (*)(const Record*, const float2*, const void*, float2*, RomeinDev);

template <int CU, int CV>
KernFn pick_pc(int n_pol, bool cplx) {
  if (n_pol == 1) return cplx ? romein_valu_kernel<CU, CV, 1, true> : romein_valu_kernel<CU, CV, 1, false>;
  return cplx ? romein_valu_kernel<CU, CV, 4, true> : romein_valu_kernel<CU, CV, 4, false>;
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

}  // namespace

gr_status plan_romein(const gr_kernel& k, int n_pol, const gr_tuning* t, RomeinPlan* plan) {
  const int S = k.support;
  RomeinPlan p{};
  int cu = t && t->cu > 0 ? t->cu : 0;
  int cv = t && t->cv > 0 ? t->cv : 0;
  if (cu == 0 || cv == 0) {
    int du, dv;
    if (S <= 8) { du = 2; dv = 2; }
    else if (n_pol == 4) { du = 4; dv = 2; }
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
  int wgu = t && t->wg_u > 0 ? t->wg_u : std::min(p.nu, 16);
  int wgv = t && t->wg_v > 0 ? t->wg_v : std::min(p.nv, std::max(1, 64 / wgu));
  if (wgu * wgv > 64) return fail(GR_EINVAL, "tuning: wg_u * wg_v must be <= 64 (one wave per tile)");
  wgu = std::min(wgu, p.nu);
  wgv = std::min(wgv, p.nv);
  p.wgu = wgu;
  p.wgv = wgv;
  p.tiles_u = (p.nu + wgu - 1) / wgu;
  p.tiles_v = (p.nv + wgv - 1) / wgv;
  p.waves_per_block = std::min(p.tiles_u * p.tiles_v, 4);
  p.vis_per_wg = t && t->vis_per_wg > 0 ? t->vis_per_wg : 1024;
  p.pad_off = std::max(cu, cv) - 1;
  p.lpad = std::max(cu * p.nu, cv * p.nv) + p.pad_off;
  const size_t elem = k.taps_complex ? 8 : 4;
  p.lds_bytes = (size_t)k.n_planes * k.oversample * p.lpad * elem;
  if (p.lds_bytes > 160 * 1024)
    return fail(GR_EUNSUPPORTED, "tap table does not fit in LDS (planes * O * padded row)");
  *plan = p;
  return GR_OK;
}

gr_status launch_romein(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol,
                        const gr_kernel& k, float2* grid, int height, int width,
                        const RomeinPlan& p, hipStream_t stream) {
  if (n_vis == 0) return GR_OK;
  KernFn fn = pick(p.cu, p.cv, n_pol, k.taps_complex != 0);
  if (fn == nullptr) return fail(GR_EUNSUPPORTED, "no kernel instance for this tuning");
  RomeinDev d{};
  d.nu = p.nu; d.nv = p.nv; d.wgu = p.wgu; d.wgv = p.wgv;
  d.tiles_u = p.tiles_u; d.tiles_v = p.tiles_v;
  d.waves_per_block = p.waves_per_block;
  d.n_tgroups = (p.tiles_u * p.tiles_v + p.waves_per_block - 1) / p.waves_per_block;
  d.vis_per_wg = p.vis_per_wg;
  d.lpad = p.lpad; d.pad_off = p.pad_off;
  d.n_rows_tab = k.n_planes * k.oversample;
  d.S = k.support; d.H = height; d.W = width; d.O = k.oversample;
  d.tap_dtype = k.tap_dtype;
  d.magic_u = (uint32_t)((0x100000000ull + p.nu - 1) / p.nu);
  d.magic_v = (uint32_t)((0x100000000ull + p.nv - 1) / p.nv);
  d.n_vis = n_vis;
  const int64_t n_chunks = (n_vis + p.vis_per_wg - 1) / p.vis_per_wg;
  const int64_t nb = n_chunks * d.n_tgroups;
  if (nb > 0x7fffffff) return fail(GR_EINVAL, "too many work-groups; raise vis_per_wg");
  d.n_blocks = (uint32_t)nb;
  {
    const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(fn), p.lds_bytes, "grid_romein.hip");
    if (lst != GR_OK) return lst;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)nb), dim3(64 * p.waves_per_block), p.lds_bytes, stream, rec,
                     wvis, k.taps, grid, d);
  return check_launch("gr_grid_records (romein)");
}

}  // namespace gr
