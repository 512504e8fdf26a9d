// Gridding of the binned stream with the separable tile update recast as a
// rank-K matrix product on the MFMA units.
//
// Merry (2016): a work-item accumulates grid points in registers and adds them
// to the grid only when it must (Section 2.2); thread coarsening makes each
// work-item own a block of cells so that address, oversampling-index and
// tap-fetch work is done once per block (Section 3); with a separable GCF an
// m x n block needs only m + n tap values (Section 4), and the product is best
// formed as G^u_i (G^v_j V_p) (Section 6).
//
// gfx950 form.  A segment holds visibilities whose footprints all lie inside
// one 64 x 64-cell window.  The window's accumulators live in MFMA result
// registers for the whole segment; each of the block's 4 waves owns a 16-row
// band (P = 4: D tiles of 4 rows x 4 polarisations by 8 columns x (re, im);
// P = 1: D tiles of 16 rows by 8 columns).  As in Section 4, records and
// weighted visibilities are staged through LDS in batches, each work-item
// loading its share; the tap table is staged once per block.
// For a pair of visibilities v, the update of D tile (rows R, cols C) is
//     D[(r, p), (x, re|im)] += sum_v A[(r, p), (v, re|im)] B[(v, re|im), (x, re|im)]
// with A = G^v_v[r] V_{v,p} (the factor shared by a whole row) and B built from
// G^u_v[x] so that the real product yields the complex one:
//     B[(v,re),(x,re)] = Re g, B[(v,re),(x,im)] = Im g,
//     B[(v,im),(x,re)] = -Im g, B[(v,im),(x,im)] = Re g.
// One v_mfma_f32_16x16x4_f32 therefore applies two visibilities to 32 cells
// of P = 4 polarisations (or 128 cells of P = 1).  D tiles that neither
// footprint touches are skipped by uniform branches; each lane builds one A
// value per touched row group and one B value per touched column group.
// The window is added to the grid once per segment with FP32 atomic adds,
// skipping cells that received nothing.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline float load_tap32(const void* __restrict__ t, int64_t idx, int dtype) {
  switch (dtype) {
    case GR_F32: return reinterpret_cast<const float*>(t)[idx];
    case GR_F16: return __half2float(reinterpret_cast<const __half*>(t)[idx]);
    default: return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(t)[idx]);
  }
}

// Four waves per block share one segment.  The 64-row window is cut into row
// groups of RG rows (P = 4: RG = 4, a D tile holds 4 rows x 4 polarisations;
// P = 1: RG = 16); wave w owns row groups w, w + 4, w + 8, ... so that every
// footprint gives the four waves (and the four SIMDs) nearly equal work.
constexpr int kBatch = 256;        // visibilities staged in LDS per batch
constexpr int kWin = 64;           // window edge (cells)
constexpr int kNC = 8;             // column groups of 8 cells per window

template <bool CPLX>
using TapT = typename std::conditional<CPLX, float2, float>::type;

__device__ __forceinline__ int clamp_tap(int tap, int S) { return min(max(tap, -1), S) + 1; }

// B fragment (lane: K = (v, comp), N = (x, bcomp)) from a tap g of G^u:
//   (comp, bcomp) = (0,0): Re g, (0,1): Im g, (1,0): -Im g, (1,1): Re g.
template <bool CPLX>
__device__ __forceinline__ float b_value(const TapT<CPLX>* row, int tap, int S, bool sel_re,
                                         float sgn) {
  const int idx = clamp_tap(tap, S);                 // rows are zero-padded at 0 and S + 1
  if constexpr (CPLX) {
    const float2 t = row[idx];
    return sel_re ? t.x : sgn * t.y;
  } else {
    return sel_re ? row[idx] : 0.f;
  }
}

// Stage the tap table as FP32 rows [plane * O + s] of S + 2 entries, with one
// zero before and after the S taps.
template <bool CPLX>
__device__ __forceinline__ void stage_taps(TapT<CPLX>* __restrict__ lds, const void* __restrict__ taps,
                                           const MfmaDev& d) {
  const int S = d.S, SP = d.S + 2;
  const int n_elem = d.n_rows_tab * SP;
  for (int e = threadIdx.x; e < n_elem; e += blockDim.x) {
    const int row = e / SP, k = e - row * SP - 1;
    const bool in = k >= 0 && k < S;
    const int64_t src = (int64_t)row * S + (in ? k : 0);
    if constexpr (CPLX) {
      lds[e] = in ? make_float2(load_tap32(taps, 2 * src, d.tap_dtype),
                                load_tap32(taps, 2 * src + 1, d.tap_dtype))
                  : make_float2(0.f, 0.f);
    } else {
      lds[e] = in ? load_tap32(taps, src, d.tap_dtype) : 0.f;
    }
  }
}

// One segment sg = {begin, length, tile} of the binned stream (rec, wvis) into
// grid, with the staged table lds and the batch buffers b_rec, b_vis.  The
// first statement of every batch is a block barrier, which also orders the
// table staging before its first use.
template <int P, bool CPLX>
__device__ __forceinline__ void mfma_segment(const Record* __restrict__ rec,
                                             const float2* __restrict__ wvis, const int4 sg,
                                             const TapT<CPLX>* __restrict__ lds,
                                             Record* __restrict__ b_rec, float2* __restrict__ b_vis,
                                             float2* __restrict__ grid, const MfmaDev& d) {
  constexpr int RG = 16 / P;            // rows per row group
  constexpr int NG = kWin / RG / 4;     // row groups per wave
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int S = d.S, SP = d.S + 2;
  const int begin = sg.x, len = sg.y, tile_id = sg.z;
  const int win_x0 = (tile_id % d.n_tx) * d.tile;
  const int win_y0 = (tile_id / d.n_tx) * d.tile;
  const int row0 = win_y0 + wave * RG;                // first row of this wave's first row group
  const int srow0 = __builtin_amdgcn_readfirstlane(row0);

  // lane roles in the 16x16x4 operand layouts
  const int kk = lane >> 4;              // K index: (v, re|im)
  const int v = kk >> 1, comp = kk & 1;
  const int m = lane & 15;               // A row index / B column index
  const int ar = (P == 4) ? (m >> 2) : m;
  const int ap = (P == 4) ? (m & 3) : 0;
  const int bx = m >> 1, bcomp = m & 1;
  const bool sel_re = comp == bcomp;
  const float sgn = comp == 0 ? 1.f : -1.f;

  f4 acc[NG][kNC];
#pragma unroll
  for (int j = 0; j < NG; ++j)
#pragma unroll
    for (int c = 0; c < kNC; ++c) acc[j][c] = f4{0.f, 0.f, 0.f, 0.f};

  for (int b0 = 0; b0 < len; b0 += kBatch) {
    const int nb = min(kBatch, len - b0);
    __syncthreads();                                   // previous batch consumed (and taps staged)
    {
      // each work-item loads its share of the batch: all loads first, then the LDS writes
      const int t = threadIdx.x;
      const Record r = t < nb ? rec[begin + b0 + t] : Record{0, 0};
      float2 w[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int e = t + j * 256;
        w[j] = e < nb * P ? wvis[(int64_t)(begin + b0) * P + e] : make_float2(0.f, 0.f);
      }
      if (t < nb) b_rec[t] = r;
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (t + j * 256 < nb * P) b_vis[t + j * 256] = w[j];
    }
    __syncthreads();

    for (int q = 0; q < nb; q += 2) {
      const bool hb = q + 1 < nb;
      const Record la = b_rec[q];
      const Record lb = b_rec[hb ? q + 1 : q];
      // the pair's records are wave-uniform: move them to scalar registers
      const Record ra{(uint32_t)__builtin_amdgcn_readfirstlane(la.x),
                      (uint32_t)__builtin_amdgcn_readfirstlane(la.y)};
      const Record rb{(uint32_t)__builtin_amdgcn_readfirstlane(lb.x),
                      (uint32_t)__builtin_amdgcn_readfirstlane(lb.y)};
      const int xa = rec_x0(ra), ya = rec_y0(ra), xb = rec_x0(rb), yb = rec_y0(rb);
      const int lo = min(ya, yb), hi = max(ya, yb) + S - 1;
      const int c_lo = (min(xa, xb) - win_x0) >> 3;
      const int c_hi = (max(xa, xb) + S - 1 - win_x0) >> 3;

      // this lane's visibility of the pair (a missing second one has V = 0)
      const Record rv = v ? rb : ra;
      const int x0v = rec_x0(rv), y0v = rec_y0(rv);
      const int tabu = (rec_plane(rv) * d.O + rec_sx(rv)) * SP;
      const int tabv = (rec_plane(rv) * d.O + rec_sy(rv)) * SP;
      const float2 vv = ((v == 0) || hb) ? b_vis[(q + v) * P + ap] : make_float2(0.f, 0.f);
      // A = G^v V: component 0 is t.x vr - t.y vi, component 1 is t.x vi + t.y vr
      const float va = comp == 0 ? vv.x : vv.y;
      const float vb = comp == 0 ? -vv.y : vv.x;

      // A fragments for this wave's row groups and B fragments for every column
      // group, branch-free (all LDS reads in flight together)
      float afr[NG];
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int idx = clamp_tap(row0 + j * 4 * RG + ar - y0v, S);
        if constexpr (CPLX) {
          const float2 t = lds[tabv + idx];
          afr[j] = t.x * va + t.y * vb;                 // component of G^v V
        } else {
          afr[j] = lds[tabv + idx] * va;
        }
      }
      float bfr[kNC];
#pragma unroll
      for (int c = 0; c < kNC; ++c)
        bfr[c] = b_value<CPLX>(lds + tabu, win_x0 + c * 8 + bx - x0v, S, sel_re, sgn);
      // wave-uniform mask of the D tiles either footprint touches
      uint32_t rmask = 0;
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const int r0 = srow0 + j * 4 * RG;
        rmask |= (r0 + RG - 1 >= lo && r0 <= hi) ? (1u << j) : 0u;
      }
      const uint32_t cmask = ((2u << c_hi) - 1u) & ~((1u << c_lo) - 1u);
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        if (rmask & (1u << j)) {
#pragma unroll
          for (int c = 0; c < kNC; ++c) {
            if (cmask & (1u << c))
              acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[j], bfr[c], acc[j][c], 0, 0, 0);
          }
        }
      }
    }
  }

  // ---- add the window to the grid (D layout: lane holds rows 4*(lane>>4)+i, column lane&15)
  float* gridf = reinterpret_cast<float*>(grid);
  const int col_in = m >> 1, ccomp = m & 1;
#pragma unroll
  for (int j = 0; j < NG; ++j) {
#pragma unroll
    for (int c = 0; c < kNC; ++c) {
      const int col = win_x0 + c * 8 + col_in;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = (P == 4) ? kk : 4 * kk + i;
        const int p = (P == 4) ? i : 0;
        const int row = row0 + j * 4 * RG + r;
        const float val = acc[j][c][i];
        if (val != 0.f && row < d.H && col < d.W)
          unsafeAtomicAdd(gridf + (((int64_t)p * d.H + row) * d.W + col) * 2 + ccomp, val);
      }
    }
  }
}

template <int P, bool CPLX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
grid_mfma_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                 const int4* __restrict__ segs, const int32_t* __restrict__ n_segs_p,
                 const void* __restrict__ taps, float2* __restrict__ grid, MfmaDev d) {
  using Tap = TapT<CPLX>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Record* b_rec = reinterpret_cast<Record*>(lds_raw);                            // [kBatch]
  float2* b_vis = reinterpret_cast<float2*>(lds_raw + kBatch * sizeof(Record));  // [kBatch][P]
  Tap* lds = reinterpret_cast<Tap*>(lds_raw + kBatch * sizeof(Record) + kBatch * P * sizeof(float2));
  // Segments are listed in tile order and their count is only known on the
  // device, so blocks take segments in dispatch order: consecutive segments
  // (neighbouring tiles) land on different XCDs, which spreads the dense
  // centre of the uv plane over the whole chip.
  const int seg = (int)blockIdx.x;
  if (seg >= *n_segs_p) return;                       // uniform for the block
  stage_taps<CPLX>(lds, taps, d);
  mfma_segment<P, CPLX>(rec, wvis, segs[seg], lds, b_rec, b_vis, grid, d);
}

// Persistent form for batches: a fixed set of blocks takes (instance, segment)
// work items from an atomic counter until the group's items run out; the tap
// table is restaged only when the instance changes.  Every block exits once
// the counter passes the item total, which the prefix kernel wrote before
// this launch.
template <int P, bool CPLX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
grid_mfma_persistent(const BatchInst* __restrict__ inst, const int32_t* __restrict__ members,
                     int n_members, const int32_t* __restrict__ prefix,
                     int32_t* __restrict__ counter) {
  using Tap = TapT<CPLX>;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Record* b_rec = reinterpret_cast<Record*>(lds_raw);
  float2* b_vis = reinterpret_cast<float2*>(lds_raw + kBatch * sizeof(Record));
  Tap* lds = reinterpret_cast<Tap*>(lds_raw + kBatch * sizeof(Record) + kBatch * P * sizeof(float2));
  __shared__ int s_inst, s_seg;
  const int total = prefix[n_members];
  int staged = -1;
  for (;;) {
    if (threadIdx.x == 0) {
      const int item = atomicAdd(counter, 1);
      int mi = -1;
      if (item < total) {
        int lo = 0, hi = n_members - 1;               // last member with prefix <= item
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (prefix[mid] <= item) lo = mid;
          else hi = mid - 1;
        }
        mi = lo;
      }
      s_inst = mi >= 0 ? members[mi] : -1;
      s_seg = mi >= 0 ? item - prefix[mi] : 0;
    }
    __syncthreads();                                  // also: the previous segment is finished
    const int ii = __builtin_amdgcn_readfirstlane(s_inst);
    const int ls = __builtin_amdgcn_readfirstlane(s_seg);
    if (ii < 0) break;
    const BatchInst& I = inst[ii];
    const MfmaDev d = I.d;
    if (ii != staged) {
      stage_taps<CPLX>(lds, I.taps, d);
      staged = ii;
    }
    mfma_segment<P, CPLX>(I.brec, I.bwvis, I.segs[ls], lds, b_rec, b_vis, I.grid, d);
  }
}


using MfmaFn = void (*)(const Record*, const float2*, const int4*, const int32_t*, const void*,
                        float2*, MfmaDev);

}  // namespace

int binned_tile(int support) { return 64 - support; }

gr_status plan_mfma(const gr_kernel& k, int n_pol, size_t* lds_bytes) {
  if (k.support > 56) return fail(GR_EUNSUPPORTED, "MFMA gridder needs support <= 56");
  const size_t elem = k.taps_complex ? 8 : 4;
  const size_t lds = (size_t)k.n_planes * k.oversample * (k.support + 2) * elem +
                     (size_t)kBatch * (sizeof(Record) + (size_t)n_pol * sizeof(float2));
  if (lds > 160 * 1024) return fail(GR_EUNSUPPORTED, "tap table does not fit in LDS");
  *lds_bytes = lds;
  return GR_OK;
}

gr_status launch_mfma(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                      float2* grid, int height, int width, hipStream_t stream) {
  size_t lds = 0;
  gr_status st = plan_mfma(k, n_pol, &lds);
  if (st != GR_OK) return st;
  const char* base = reinterpret_cast<const char*>(bins);
  const auto* rec = reinterpret_cast<const Record*>(base + L.off_rec);
  const auto* wv = reinterpret_cast<const float2*>(base + L.off_wvis);
  const auto* segs = reinterpret_cast<const int4*>(base + L.off_segs);
  const auto* nsegs = reinterpret_cast<const int32_t*>(base + L.off_nsegs);
  MfmaDev d{};
  d.S = k.support; d.O = k.oversample; d.n_rows_tab = k.n_planes * k.oversample;
  d.tap_dtype = k.tap_dtype; d.tile = L.tile; d.n_tx = L.n_tx; d.H = height; d.W = width;
  const int64_t nb = L.max_segs;
  if (nb > 0x7fffffff) return fail(GR_EINVAL, "too many segments");
  if (nb == 0) return GR_OK;
  d.n_blocks = (uint32_t)nb;
  MfmaFn fn;
  if (n_pol == 4) fn = k.taps_complex ? grid_mfma_kernel<4, true> : grid_mfma_kernel<4, false>;
  else fn = k.taps_complex ? grid_mfma_kernel<1, true> : grid_mfma_kernel<1, false>;
  {
    const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds, "grid_mfma.hip");
    if (lst != GR_OK) return lst;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)nb), dim3(256), lds, stream, rec, wv, segs, nsegs, k.taps,
                     grid, d);
  return check_launch("gr_grid_binned (mfma)");
}

gr_status launch_mfma_persistent(const BatchInst* inst, const int32_t* members, int n_members,
                                 const int32_t* group_prefix, int32_t* counter, int n_pol,
                                 bool complex_taps, size_t lds_bytes, int n_blocks,
                                 hipStream_t stream) {
  if (n_members == 0 || n_blocks <= 0) return GR_OK;
  using PFn = void (*)(const BatchInst*, const int32_t*, int, const int32_t*, int32_t*);
  PFn fn;
  if (n_pol == 4) fn = complex_taps ? grid_mfma_persistent<4, true> : grid_mfma_persistent<4, false>;
  else fn = complex_taps ? grid_mfma_persistent<1, true> : grid_mfma_persistent<1, false>;
  {
    const gr_status lst = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds_bytes, "grid_mfma.hip");
    if (lst != GR_OK) return lst;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)n_blocks), dim3(256), lds_bytes, stream, inst, members, n_members,
                     group_prefix, counter);
  return check_launch("gr_grid_batch (persistent mfma)");
}

}  // namespace gr
