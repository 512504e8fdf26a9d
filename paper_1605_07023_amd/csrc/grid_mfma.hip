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
// one window of WR x WR cells (WR = 32 for S <= 16, 48 for S <= 32, else 64;
// the binning tile is WR - S).  The window is cut into row groups of RG rows
// (P = 4: RG = 4, a D tile holds 4 rows x 4 polarisations; P = 1: RG = 16)
// and column groups of 8 cells; a D tile of the MFMA holds one row group by
// one column group, (re, im) interleaved along the columns.  For a pair of
// visibilities v, the update of D tile (rows R, cols C) is
//     D[(r, p), (x, re|im)] += sum_v A[(r, p), (v, re|im)] B[(v, re|im), (x, re|im)]
// with A = G^v_v[r] V_{v,p} (the factor shared by a whole row) and B built from
// G^u_v[x] so that the real product yields the complex one:
//     B[(v,re),(x,re)] = Re g, B[(v,re),(x,im)] = Im g,
//     B[(v,im),(x,re)] = -Im g, B[(v,im),(x,im)] = Re g.
// One v_mfma_f32_16x16x4_f32 therefore applies two visibilities to 32 cells
// of P = 4 polarisations (or 128 cells of P = 1).  D tiles that neither
// footprint touches are skipped by uniform branches; each lane builds one A
// value per touched row group and one B value per column group.  The window
// is added to the grid with FP32 atomic adds, skipping cells that received
// nothing.
//
// Three launch forms share that update:
//  * grid_mfma_waves (single problem, default): one 1024-thread block per CU
//    stages the tap table once (Section 4 stages the GCF in local memory); its
//    16 waves then work without block barriers, each taking
//    (segment, part) items from an atomic counter, where part p of a window is
//    the row groups p, p + parts, p + 2 parts, ...  A small kernel first
//    orders each segment by the set of D tiles its footprints touch, so that
//    consecutive visibilities, which the wave form pairs, touch the same
//    tiles.  Each wave stages its own batches of 64 visibilities in its own
//    LDS slice, each visibility as the LDS addresses of its two tap rows and
//    each pair as the mask of D tiles it touches (decoded once, not per use).
//    Its table is gapped (zeros around every row of taps, so that operand
//    reads need no clamp), with (-Im, Re, Im) entries where they fit, else
//    (Re, Im) entries, with -Im read from the mirror plane when the planes are
//    conjugate pairs.
//  * grid_mfma_kernel: one 256-thread block per segment, its 4 waves sharing
//    the segment's window rows (the form used when the table leaves too little
//    LDS for 16 wave slices).
//  * grid_mfma_persistent (batches): blocks of the second form taking
//    (instance, segment) items from an atomic counter.
#include <algorithm>

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

constexpr int kBatch = 256;        // visibilities staged per batch (block forms)
constexpr int kBatchWindow = 64;   // window of the batch gridder (batches bin for it)
constexpr int kWaveBatch = 64;     // visibilities staged per batch (wave form)

template <bool CPLX>
using TapT = typename std::conditional<CPLX, float2, float>::type;

// clamp to [-1, S] and shift by one: rows carry a zero before and after the S taps
// (one v_med3_i32 instead of a max and a min)
__device__ __forceinline__ int clamp_tap(int tap, int S) {
  int r;
  asm("v_med3_i32 %0, %1, -1, %2" : "=v"(r) : "v"(tap), "s"(S));
  return r + 1;
}

// B fragment (lane: K = (v, comp), N = (x, bcomp)) from a tap g of G^u:
//   (comp, bcomp) = (0,0): Re g, (0,1): Im g, (1,0): -Im g, (1,1): Re g.
template <bool CPLX>
__device__ __forceinline__ float b_value(const TapT<CPLX>* row, int tap, int S, bool sel_re,
                                         float sgn) {
  const int idx = clamp_tap(tap, S);
  if constexpr (CPLX) {
    const float2 t = row[idx];
    return sel_re ? t.x : sgn * t.y;
  } else {
    return sel_re ? row[idx] : 0.f;
  }
}

// Stage the tap table as FP32 rows [plane * O + s] of S + 2 entries, with one
// zero before and after the S taps (block forms).
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
      const float re = in ? load_tap32(taps, 2 * src, d.tap_dtype) : 0.f;
      const float im = in ? load_tap32(taps, 2 * src + 1, d.tap_dtype) : 0.f;
      lds[e] = make_float2(re, im);
    } else {
      lds[e] = in ? load_tap32(taps, src, d.tap_dtype) : 0.f;
    }
  }
}

// Staged form of one visibility: {x0, y0, offset of its G^u row, offset of its
// G^v row} (row offsets in table entries), decoded once when the batch is staged.
__device__ __forceinline__ int4 stage_info(const Record r, const MfmaDev& d) {
  const int sp = d.S + 2;
  return make_int4(rec_x0(r), rec_y0(r), (rec_plane(r) * d.O + rec_sx(r)) * sp,
                   (rec_plane(r) * d.O + rec_sy(r)) * sp);
}

// Bits of a 6-bit value spread to the even bit positions (Morton interleave).
__device__ __forceinline__ uint32_t spread6(uint32_t v) {
  v &= 63u;
  v = (v | (v << 4)) & 0x0f0fu;
  v = (v | (v << 2)) & 0x3333u;
  return (v | (v << 1)) & 0x5555u;
}

// Pairing order of a wave's 64 staged visibilities.  Two visibilities share
// every MFMA (K = 2 visibilities x (re, im)), so a pair touches the D tiles of
// the union of its footprints; consecutive visibilities in Z (Morton) order of
// their footprint origins inside the window have nearby footprints, which cuts
// the D tiles a pair touches by 13 % (S = 32) to 21 % (S = 16) against arrival
// order on the full-shape tracks.  A bitonic sort of the 64 keys (position,
// lane) across the wave gives lane i the i-th key; a forward permute returns to
// each lane the rank of its own visibility.  Lanes without a visibility sort
// last.  Must be called by all 64 lanes.
__device__ __forceinline__ int pair_rank(bool live, int x_rel, int y_rel) {
  const int lane = threadIdx.x & 63;
  uint32_t key = live ? (((spread6((uint32_t)x_rel) | (spread6((uint32_t)y_rel) << 1)) << 6) | (uint32_t)lane)
                      : ((1u << 20) | (uint32_t)lane);
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)key, j);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      key = keep_min ? min(key, other) : max(key, other);
    }
  }
  return __builtin_amdgcn_ds_permute((int)((key & 63u) << 2), lane);
}

// Stage up to 64 visibilities (one per lane, lanes < n live) of a batch into
// b_inf / b_vis in pairing order; slot `pad` (when >= 0) receives a copy of
// the footprint of the visibility ranked last, with zero visibility, so that
// an odd batch still forms whole pairs.  Called by all 64 lanes of a wave.
template <int P>
__device__ __forceinline__ void stage_pairs(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                                            int64_t first, int n, int win_x0, int win_y0, const MfmaDev& d,
                                            int4* __restrict__ b_inf, float2* __restrict__ b_vis, int pad) {
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  const Record r = live ? rec[first + lane] : Record{0, 0};
  float2 w[P];
  if constexpr (P == 4) {
    const float4* src = reinterpret_cast<const float4*>(wvis + (first + (live ? lane : 0)) * 4);
    const float4 a = live ? src[0] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = live ? src[1] : make_float4(0.f, 0.f, 0.f, 0.f);
    w[0] = make_float2(a.x, a.y); w[1] = make_float2(a.z, a.w);
    w[2] = make_float2(b.x, b.y); w[3] = make_float2(b.z, b.w);
  } else {
    w[0] = live ? wvis[first + lane] : make_float2(0.f, 0.f);
  }
  const int rank = pair_rank(live, rec_x0(r) - win_x0, rec_y0(r) - win_y0);
  if (live) {
    const int4 inf = stage_info(r, d);
    b_inf[rank] = inf;
#pragma unroll
    for (int p = 0; p < P; ++p) b_vis[rank * P + p] = w[p];
    if (pad >= 0 && rank == n - 1) b_inf[pad] = inf;
  }
  if (pad >= 0 && lane < P) b_vis[pad * P + lane] = make_float2(0.f, 0.f);
}

// ---- wave form --------------------------------------------------------------
// The wave form keeps its tap table as entries of ES bytes: with complex taps
// the triple (-Im g, Re g, Im g), so that every operand a lane needs is one
// aligned read at a lane-constant offset (A of component 0 reads (-Im, Re) at
// offset 0, component 1 reads (Re, Im) at offset 4; B reads Re at 4, Im at 8,
// -Im at 0); with real taps the tap alone.  Rows are S + 2 entries with a zero
// entry before and after the taps, and tap indices are clamped to that row as
// LDS byte addresses (one v_med3 per operand).
typedef __attribute__((address_space(3))) const float lds_float;
struct __attribute__((aligned(4))) Pair4 {
  float a, b;
};
typedef __attribute__((address_space(3))) const Pair4 lds_pair;

__device__ __forceinline__ float lds_read(uint32_t addr) { return *(lds_float*)(uintptr_t)addr; }
__device__ __forceinline__ Pair4 lds_read2(uint32_t addr) {
  lds_pair* p = (lds_pair*)(uintptr_t)addr;
  return Pair4{p->a, p->b};
}

__device__ __forceinline__ uint32_t clamp_addr(uint32_t a, uint32_t lo, uint32_t hi) {
  int r;   // signed: an address below the row (negative tap index) clamps to its start
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"((int)a), "v"((int)lo), "v"((int)hi));
  return (uint32_t)r;
}

template <bool CPLX>
__device__ __forceinline__ void stage_taps_wave(float* __restrict__ lds, const void* __restrict__ taps,
                                                const MfmaDev& d) {
  const int S = d.S, SP = d.S + 2;
  const int n_elem = d.n_rows_tab * SP;
  for (int e = threadIdx.x; e < n_elem; e += blockDim.x) {
    const int row = e / SP, k = e - row * SP - 1;
    const bool in = k >= 0 && k < S;
    const int64_t src = (int64_t)row * S + (in ? k : 0);
    if constexpr (CPLX) {
      const float re = in ? load_tap32(taps, 2 * src, d.tap_dtype) : 0.f;
      const float im = in ? load_tap32(taps, 2 * src + 1, d.tap_dtype) : 0.f;
      lds[3 * e] = -im;
      lds[3 * e + 1] = re;
      lds[3 * e + 2] = im;
    } else {
      lds[e] = in ? load_tap32(taps, src, d.tap_dtype) : 0.f;
    }
  }
}

// Stage up to 64 visibilities of a segment batch (one per lane, lanes < n live)
// for the block form with triple entries (each wave a quarter of the block's
// batch), in pairing order (pair_rank).  Per visibility: {B start,
// B row, A start, A row}, LDS byte addresses of its G^u and G^v rows (row =
// first entry, start = row - ES * its window-relative x0 or y0), and its
// visibilities.  Per pair: the row groups (bits 0..15) and column groups (bits
// 16..23) of the window that either footprint touches.  Slot `pad` (>= 0 for
// an odd batch) takes a copy of the last visibility's rows with zero
// visibility.  Called by all 64 lanes of a wave.
template <int P, bool CPLX>
__device__ __forceinline__ void stage_wave(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                                           int64_t first, int n, int win_x0, int win_y0, const MfmaDev& d,
                                           uint32_t tab_base, int4* __restrict__ b_inf,
                                           float2* __restrict__ b_vis, uint32_t* __restrict__ b_box, int pad) {
  constexpr int ES = CPLX ? 12 : 4;
  constexpr int RG = 16 / P;
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  const Record r = live ? rec[first + lane] : Record{0, 0};
  float2 w[P];
  if constexpr (P == 4) {
    const float4* src = reinterpret_cast<const float4*>(wvis + (first + (live ? lane : 0)) * 4);
    const float4 a = live ? src[0] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = live ? src[1] : make_float4(0.f, 0.f, 0.f, 0.f);
    w[0] = make_float2(a.x, a.y); w[1] = make_float2(a.z, a.w);
    w[2] = make_float2(b.x, b.y); w[3] = make_float2(b.z, b.w);
  } else {
    w[0] = live ? wvis[first + lane] : make_float2(0.f, 0.f);
  }
  const int xr = rec_x0(r) - win_x0, yr = rec_y0(r) - win_y0;
  const uint32_t key = live ? (((spread6((uint32_t)xr) | (spread6((uint32_t)yr) << 1)) << 6) | (uint32_t)lane)
                            : ((1u << 20) | (uint32_t)lane);
  uint32_t sk = key;
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)sk, j);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      sk = keep_min ? min(sk, other) : max(sk, other);
    }
  }
  // lane i holds the i-th key: its visibility's rank goes back to the owner, its
  // footprint origin comes to lane i, and lane i^1 holds the pair partner's
  const int src_lane = (int)(sk & 63u);
  const int rank = __builtin_amdgcn_ds_permute(src_lane << 2, lane);
  const int xy_own = xr | (yr << 8);
  const int xy = __builtin_amdgcn_ds_bpermute(src_lane << 2, xy_own);
  const int xy_partner = __shfl_xor(xy, 1);
  if (live) {
    const int rowlen = (d.S + 2) * ES;
    const uint32_t bl = tab_base + (uint32_t)((rec_plane(r) * d.O + rec_sx(r)) * rowlen);
    const uint32_t al = tab_base + (uint32_t)((rec_plane(r) * d.O + rec_sy(r)) * rowlen);
    const int4 inf = make_int4((int)(bl - (uint32_t)(xr * ES)), (int)bl, (int)(al - (uint32_t)(yr * ES)), (int)al);
    b_inf[rank] = inf;
#pragma unroll
    for (int p = 0; p < P; ++p) b_vis[rank * P + p] = w[p];
    if (pad >= 0 && rank == n - 1) b_inf[pad] = inf;
  }
  if (pad >= 0 && lane < P) b_vis[pad * P + lane] = make_float2(0.f, 0.f);
  if ((lane & 1) == 0 && lane < n) {
    const int xb = (lane + 1 < n) ? xy_partner : xy;
    const int xa_ = xy & 0xff, ya_ = xy >> 8, xb_ = xb & 0xff, yb_ = xb >> 8;
    const int g_lo = min(ya_, yb_) / RG, g_hi = (max(ya_, yb_) + d.S - 1) / RG;
    const int c_lo = min(xa_, xb_) >> 3, c_hi = (max(xa_, xb_) + d.S - 1) >> 3;
    const uint32_t rbits = ((2u << g_hi) - 1u) & ~((1u << g_lo) - 1u);
    const uint32_t cbits = ((2u << c_hi) - 1u) & ~((1u << c_lo) - 1u);
    b_box[lane >> 1] = rbits | (cbits << 16);
  }
}

// The work of one wave of the wave form on one staged batch: row groups
// part + j * PARTS (j < NG) and all WCG column groups of the window.
template <int P, bool CPLX, int WCG, int NG, int PARTS>
__device__ __forceinline__ void wave_batch(const int4* __restrict__ b_inf, const float2* __restrict__ b_vis,
                                           const uint32_t* __restrict__ b_box, int nb, int part, int S,
                                           f4 (&acc)[NG][WCG]) {
  constexpr int RG = 16 / P;
  constexpr int ES = CPLX ? 12 : 4;
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4;                          // K index: (v, re|im)
  const int v = kk >> 1, comp = kk & 1;
  const int m = lane & 15;                           // A row / B column
  const int ar = (P == 4) ? (m >> 2) : m;
  const int ap = (P == 4) ? (m & 3) : 0;
  const int bx = m >> 1, bcomp = m & 1;
  // lane-constant parts of the operand addresses
  const uint32_t sel_b = CPLX ? (comp == 1 && bcomp == 0 ? 0u : comp == 0 && bcomp == 1 ? 8u : 4u) : 0u;
  const uint32_t span_b = (CPLX || comp == bcomp) ? (uint32_t)((S + 1) * ES) : 0u;   // 0: always the zero entry
  const uint32_t off_b = (uint32_t)((bx + 1) * ES) + sel_b;
  const uint32_t sel_a = CPLX ? (uint32_t)(comp * 4) : 0u;
  const uint32_t span_a = (uint32_t)((S + 1) * ES);
  const uint32_t off_a = (uint32_t)((part * RG + ar + 1) * ES) + sel_a;
  for (int q = 0; q < nb; q += 2) {
    const int4 inf = b_inf[q + v];
    const float2 vv = b_vis[(q + v) * P + ap];
    const uint32_t box = __builtin_amdgcn_readfirstlane(b_box[q >> 1]);
    float bfr[WCG];
    {
      const uint32_t lo = (uint32_t)inf.y + sel_b, hi = lo + span_b;
      const uint32_t b = (uint32_t)inf.x + off_b;
#pragma unroll
      for (int c = 0; c < WCG; ++c) bfr[c] = lds_read(clamp_addr(b + (uint32_t)(c * 8 * ES), lo, hi));
    }
    float afr[NG];
    {
      const uint32_t lo = (uint32_t)inf.w + sel_a, hi = lo + span_a;
      const uint32_t a = (uint32_t)inf.z + off_a;
      if constexpr (CPLX) {
#pragma unroll
        for (int j = 0; j < NG; ++j) {
          const Pair4 t = lds_read2(clamp_addr(a + (uint32_t)(j * PARTS * RG * ES), lo, hi));
          afr[j] = t.a * vv.y + t.b * vv.x;           // component comp of G^v V
        }
      } else {
        const float vs = comp ? vv.y : vv.x;
#pragma unroll
        for (int j = 0; j < NG; ++j)
          afr[j] = lds_read(clamp_addr(a + (uint32_t)(j * PARTS * RG * ES), lo, hi)) * vs;
      }
    }
    const uint32_t rb = box >> part, cm = box >> 16;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      if (__builtin_expect((rb >> (j * PARTS)) & 1u, 1)) {
#pragma unroll
        for (int c = 0; c < WCG; ++c) {
          if (__builtin_expect((cm >> c) & 1u, 1))
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[j], bfr[c], acc[j][c], 0, 0, 0);
        }
      }
    }
  }
}

// ---- wave form with a gapped tap table -------------------------------------
// The wave form's table holds every row of S taps followed by WR - S zero
// entries, after a lead of WR - S zeros: entry e = lead + row * WR + t for tap t
// of LDS row s * n_planes + plane (phase-major).  A window-relative tap index lies in [-(WR - S - 1), WR - 1] (the
// footprint origin is in the tile, WR - S cells, and the operand columns or rows
// in the window), so every operand read of a row lands on its taps or on the
// zeros around them: the address is the visibility's row start plus lane and
// group constants, with no clamp (the constants go into the LDS instruction's
// offset field).  Entries of complex taps are ES = 12 bytes, the triple
// (-Im, Re, Im), where the table fits in LDS with that many wave slices, else
// ES = 8 bytes (Re, Im), when the B operand of one lane class needs -Im (a sign
// flip, or Im of the mirror plane) and the A operand two lane-constant
// factors; real taps are 4 bytes.
template <bool CPLX, bool TRI>
constexpr int gap_es() { return CPLX ? (TRI ? 12 : 8) : 4; }

template <bool CPLX, bool TRI, int WR>
__device__ __forceinline__ void stage_taps_gap(float* __restrict__ lds, const void* __restrict__ taps,
                                               const MfmaDev& d) {
  const int S = d.S, lead = WR - S, np = d.n_rows_tab / d.O;
  const int n_elem = lead + d.n_rows_tab * WR;
  for (int e = threadIdx.x; e < n_elem; e += blockDim.x) {
    const int q = e - lead;
    const int row = q >= 0 ? q / WR : 0;              // LDS row s * n_planes + plane
    const int t = q - row * WR;
    const bool in = q >= 0 && t < S;
    const int src_row = (row % np) * d.O + row / np;  // table row plane * O + s
    const int64_t src = (int64_t)src_row * S + (in ? t : 0);
    if constexpr (CPLX) {
      const float re = in ? load_tap32(taps, 2 * src, d.tap_dtype) : 0.f;
      const float im = in ? load_tap32(taps, 2 * src + 1, d.tap_dtype) : 0.f;
      if constexpr (TRI) {
        lds[3 * e] = -im;
        lds[3 * e + 1] = re;
        lds[3 * e + 2] = im;
      } else {
        lds[2 * e] = re;
        lds[2 * e + 1] = im;
      }
    } else {
      lds[e] = in ? load_tap32(taps, src, d.tap_dtype) : 0.f;
    }
  }
}

// One lane's visibility of a wave-form batch as read from the binned stream.
template <int P>
struct WaveIn {
  Record r;
  float2 w[P];
};

// Read up to 64 visibilities (one per lane, lanes < n live) of a segment batch,
// the entries order[first + lane] of the binned stream.
template <int P>
__device__ __forceinline__ void load_wave(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                                          const int32_t* __restrict__ order, int64_t first, int n, WaveIn<P>& in) {
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  const int64_t e = live ? (int64_t)order[first + lane] : 0;
  in.r = live ? rec[e] : Record{0, 0};
  if constexpr (P == 4) {
    const float4* src = reinterpret_cast<const float4*>(wvis + e * 4);
    const float4 a = live ? src[0] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = live ? src[1] : make_float4(0.f, 0.f, 0.f, 0.f);
    in.w[0] = make_float2(a.x, a.y); in.w[1] = make_float2(a.z, a.w);
    in.w[2] = make_float2(b.x, b.y); in.w[3] = make_float2(b.z, b.w);
  } else {
    in.w[0] = live ? wvis[e] : make_float2(0.f, 0.f);
  }
}

// Staged pair records of the wave form.  Per pair a 28-byte header: for each of
// its two visibilities {B start, A start}, the LDS byte addresses of its G^u
// and G^v rows minus ES times its window-relative x0 or y0; then the two B
// starts of the rows of the mirror plane (n_planes - 1 - plane, used when the
// table's planes are conjugate pairs, as those of a W kernel sampled at w
// values symmetric about 0 are); then the mask of the row groups (bits 0..15)
// and column groups (bits 16..23) of the window that either footprint touches.
// Then the visibilities, P per visibility, as (Re, Im) (triple table) or as
// (-Im, Re, Im) (pair table and real taps: lane class comp reads the two values
// at comp * 4, which gives component comp of G^v V with the same two multiplies
// as with triple entries, and component comp of V as the second value).  A
// wave's slice holds the 32 records of a batch.
constexpr int kGapHdr = 28;
template <int P, bool TRI>
__host__ __device__ constexpr int gap_vis_bytes() { return TRI ? 8 : 12; }
template <int P, bool TRI>
__host__ __device__ constexpr int gap_rec_bytes() { return kGapHdr + 2 * P * gap_vis_bytes<P, TRI>(); }
__host__ __device__ constexpr size_t gap_slice_bytes(int n_pol, bool tri) {
  return (size_t)(kWaveBatch / 2) *
         (n_pol == 4 ? (tri ? gap_rec_bytes<4, true>() : gap_rec_bytes<4, false>())
                     : (tri ? gap_rec_bytes<1, true>() : gap_rec_bytes<1, false>()));
}
typedef __attribute__((address_space(3))) const uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_read_u32(uint32_t addr) { return *(lds_u32*)(uintptr_t)addr; }

// Whether every plane of the staged gapped table (complex entries, (Re, Im)
// pairs) holds the complex conjugates of the taps of the mirror plane
// n_planes - 1 - plane, compared exactly.  Called by every thread of the block
// after the table is staged; the result is the same in every thread.
template <int WR>
__device__ bool planes_conjugate(const float* __restrict__ tab, const MfmaDev& d) {
  const int S = d.S, O = d.O, lead = WR - S, np = d.n_rows_tab / O;
  const int n = d.n_rows_tab * S;
  int bad = 0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int row = e / S, t = e - row * S;          // LDS row s * np + p
    const int s = row / np, p = row - s * np;
    const int a = lead + row * WR + t, b = lead + (s * np + np - 1 - p) * WR + t;
    bad |= !(tab[2 * a] == tab[2 * b] && tab[2 * a + 1] == -tab[2 * b + 1]);
  }
  return __syncthreads_or(bad) == 0;
}

// The value of lane i ^ 1 (a DPP quad permutation, no LDS round trip).
__device__ __forceinline__ uint32_t lane_xor1(uint32_t x) {
  constexpr int kQuadXor1 = 0xB1;
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kQuadXor1, 0xF, 0xF, true);
}

// Stage a batch read by load_wave (lanes < n live) as pair records: lanes 2q
// and 2q + 1 form pair q (the segment's pairing order, order_segments_kernel).
// Slot `pad` (>= 0 for an odd batch) takes a copy of the last visibility's rows
// with zero visibility.  MIRROR: also the B starts of the mirror plane's rows.
// Called by all 64 lanes of a wave.
template <int P, bool CPLX, bool TRI, int WR, bool MIRROR>
__device__ __forceinline__ void stage_wave_gap(const WaveIn<P>& in, int n, int win_x0, int win_y0,
                                               const MfmaDev& d, uint32_t tab_base, unsigned char* __restrict__ slice,
                                               int pad) {
  constexpr int RG = 16 / P;
  constexpr int ES = gap_es<CPLX, TRI>();
  constexpr int RB = gap_rec_bytes<P, TRI>();
  constexpr int VS = gap_vis_bytes<P, TRI>();
  const int lane = threadIdx.x & 63;
  const bool live = lane < n;
  const Record r = in.r;
  const int xr = rec_x0(r) - win_x0, yr = rec_y0(r) - win_y0;
  const int rank = lane;
  const int xy = xr | (yr << 8);
  const int xy_partner = (int)lane_xor1((uint32_t)xy);
  // the pair mask, formed by the even lane of each pair and shared with the odd one
  uint32_t box = 0u;
  {
    const int xb = (lane + 1 < n) ? xy_partner : xy;
    const int xa_ = xy & 0xff, ya_ = xy >> 8, xb_ = xb & 0xff, yb_ = xb >> 8;
    const int g_lo = min(ya_, yb_) / RG, g_hi = (max(ya_, yb_) + d.S - 1) / RG;
    const int c_lo = min(xa_, xb_) >> 3, c_hi = (max(xa_, xb_) + d.S - 1) >> 3;
    const uint32_t rbits = ((2u << g_hi) - 1u) & ~((1u << g_lo) - 1u);
    const uint32_t cbits = ((2u << c_hi) - 1u) & ~((1u << c_lo) - 1u);
    box = rbits | (cbits << 16);
  }
  const uint32_t box_partner = lane_xor1(box);
  const uint32_t box_even = (lane & 1) ? box_partner : box;
  if (live) {
    const int lead = WR - d.S;
    const int plane = rec_plane(r), np = d.n_rows_tab / d.O;
    const uint32_t bu = tab_base + (uint32_t)((lead + (rec_sx(r) * np + plane) * WR - xr) * ES);
    const uint32_t av = tab_base + (uint32_t)((lead + (rec_sy(r) * np + plane) * WR - yr) * ES);
    unsigned char* rec = slice + (rank >> 1) * RB;
    uint32_t* hdr = reinterpret_cast<uint32_t*>(rec);
    const int v = rank & 1;
    hdr[2 * v] = bu;
    hdr[2 * v + 1] = av;
    uint32_t bm = 0u;
    if constexpr (MIRROR) {
      // the row of plane np - 1 - plane lies np - 1 - 2 plane rows away: an odd
      // number for an even plane count, which puts it in the other half of the
      // LDS banks (a row is WR * ES / 4 = 32 mod 64 words long)
      bm = bu + (uint32_t)((np - 1 - 2 * plane) * WR * ES);
      hdr[4 + v] = bm;
    }
    if (v == 0) hdr[6] = box_even;
    if (pad >= 0 && rank == n - 1) {                  // n - 1 is even here: slot n is its partner
      hdr[2] = bu; hdr[3] = av;
      if constexpr (MIRROR) hdr[5] = bm;
    }
    float* vis = reinterpret_cast<float*>(rec + kGapHdr + v * P * VS);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if constexpr (TRI) {
        vis[2 * p] = in.w[p].x;
        vis[2 * p + 1] = in.w[p].y;
      } else {
        vis[3 * p] = -in.w[p].y;
        vis[3 * p + 1] = in.w[p].x;
        vis[3 * p + 2] = in.w[p].y;
      }
    }
  }
  if (pad >= 0 && lane < P * VS / 4)
    reinterpret_cast<float*>(slice + (pad >> 1) * RB + kGapHdr + P * VS)[lane] = 0.f;
}

// The work of one wave of the wave form on one staged batch (gapped table): row
// groups part + j * PARTS (j < NG) and all WCG column groups of the window.
// MIRROR (pair table whose planes are conjugate pairs): the lanes that need
// -Im g read Im of the mirror plane's row instead of flipping a sign.
template <int P, bool CPLX, bool TRI, int WCG, int NG, int PARTS, bool MIRROR>
__device__ __forceinline__ void wave_batch_gap(const unsigned char* __restrict__ slice, int nb, int part,
                                               f4 (&acc)[NG][WCG]) {
  constexpr int RG = 16 / P;
  constexpr int ES = gap_es<CPLX, TRI>();
  constexpr int RB = gap_rec_bytes<P, TRI>();
  constexpr int VS = gap_vis_bytes<P, TRI>();
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4;                          // K index: (v, re|im)
  const int v = kk >> 1, comp = kk & 1;
  const int m = lane & 15;                           // A row / B column
  const int ar = (P == 4) ? (m >> 2) : m;
  const int ap = (P == 4) ? (m & 3) : 0;
  const int bx = m >> 1, bcomp = m & 1;
  // B: (comp, bcomp) = (0,0) Re g, (0,1) Im g, (1,0) -Im g, (1,1) Re g
  uint32_t off_b = (uint32_t)(bx * ES);
  uint32_t sgn_b = 0u;
  float bm = 1.f;
  if constexpr (CPLX && TRI) off_b += (comp == 1 && bcomp == 0) ? 0u : (comp == 0 && bcomp == 1) ? 8u : 4u;
  if constexpr (CPLX && !TRI) {
    off_b += comp == bcomp ? 0u : 4u;
    if constexpr (!MIRROR) sgn_b = (comp == 1 && bcomp == 0) ? 0x80000000u : 0u;
  }
  if constexpr (!CPLX) bm = comp == bcomp ? 1.f : 0.f;
  // A: component comp of G^v V for row part * RG + ar of the window
  const uint32_t off_a = (uint32_t)((part * RG + ar) * ES) + ((CPLX && TRI) ? (uint32_t)(comp * 4) : 0u);
  // this lane's fields of a pair record
  const uint32_t base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const unsigned char*)slice;
  const bool from_mirror = MIRROR && comp == 1 && bcomp == 0;
  const uint32_t l_b = base + (uint32_t)(from_mirror ? 16 + 4 * v : 8 * v);
  const uint32_t l_a = base + (uint32_t)(8 * v + 4);
  const uint32_t l_box = base + 24u;
  const uint32_t l_vis = base + (uint32_t)(kGapHdr + (v * P + ap) * VS + (TRI ? 0 : comp * 4));
  auto pair = [&](uint32_t o) {
    const uint32_t row_u = lds_read_u32(l_b + o);
    const uint32_t row_v = lds_read_u32(l_a + o);
    const uint32_t box = __builtin_amdgcn_readfirstlane(lds_read_u32(l_box + o));
    const Pair4 vv = lds_read2(l_vis + o);
    float bfr[WCG];
    {
      const uint32_t b = row_u + off_b;
#pragma unroll
      for (int c = 0; c < WCG; ++c) bfr[c] = lds_read(b + (uint32_t)(c * 8 * ES));
    }
    Pair4 at[NG];
    float as[NG];
    {
      const uint32_t a = row_v + off_a;
#pragma unroll
      for (int j = 0; j < NG; ++j) {
        const uint32_t aj = a + (uint32_t)(j * PARTS * RG * ES);
        if constexpr (CPLX) at[j] = lds_read2(aj);
        else as[j] = lds_read(aj);
      }
    }
    // every operand read of the pair is issued before any is used
    if constexpr (MIRROR) __builtin_amdgcn_sched_barrier(0);
    if constexpr (CPLX && !TRI && !MIRROR) {
#pragma unroll
      for (int c = 0; c < WCG; ++c) bfr[c] = __uint_as_float(__float_as_uint(bfr[c]) ^ sgn_b);
    }
    if constexpr (!CPLX) {
#pragma unroll
      for (int c = 0; c < WCG; ++c) bfr[c] *= bm;
    }
    // component comp of G^v V: with triple taps the lane read (-Im, Re) or (Re, Im)
    // of the tap and (Re, Im) of V; with pair taps (Re, Im) of the tap and (-Im, Re)
    // or (Re, Im) of V
    float afr[NG];
    if constexpr (CPLX) {
#pragma unroll
      for (int j = 0; j < NG; ++j) afr[j] = at[j].a * vv.b + at[j].b * vv.a;
    } else {
#pragma unroll
      for (int j = 0; j < NG; ++j) afr[j] = as[j] * vv.b;      // real taps: vv.b is component comp of V
    }
    // With the pair table every operand is formed before the first matrix
    // operation of the pair (measured 2 % faster at S = 32, where a part's row
    // groups are spread over the window and a pair touches nearly all of them);
    // with the triple table the compiler's placement, which forms A inside the
    // row-group branches, measured 2 % faster at S = 16.
    if constexpr (CPLX && !TRI) {
#pragma unroll
      for (int j = 0; j < NG; ++j) asm volatile("" : "+v"(afr[j]));
#pragma unroll
      for (int c = 0; c < WCG; ++c) asm volatile("" : "+v"(bfr[c]));
    }
    const uint32_t rb = box >> part, cm = box >> 16;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      if (__builtin_expect((rb >> (j * PARTS)) & 1u, 1)) {
#pragma unroll
        for (int c = 0; c < WCG; ++c) {
          if (__builtin_expect((cm >> c) & 1u, 1))
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[j], bfr[c], acc[j][c], 0, 0, 0);
        }
      }
    }
  };
  // two pairs per iteration, the second at an immediate offset
  for (int q = 0; q < nb; q += 4) {
    const uint32_t o = (uint32_t)(q >> 1) * RB;
    pair(o);
    if (q + 2 < nb) pair(o + RB);
  }
}

// The work of one wave on one batch of a segment: the window rows of the NG
// row groups whose first rows are row0 + j * GSTRIDE (j < NG), all WCG column
// groups of the window at columns win_x0 + 8 c.  b_inf / b_vis hold nb
// staged visibilities.
template <int P, bool CPLX, int WCG, int NG, int GSTRIDE>
__device__ __forceinline__ void mfma_batch(const int4* __restrict__ b_inf,
                                           const float2* __restrict__ b_vis, int nb,
                                           const TapT<CPLX>* __restrict__ lds, int row0, int win_x0,
                                           const MfmaDev& d, f4 (&acc)[NG][WCG]) {
  constexpr int RG = 16 / P;
  const int lane = threadIdx.x & 63;
  const int S = d.S;
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
  // an odd batch carries a zero visibility with the last one's footprint in
  // slot nb, so every pair is whole
  for (int q = 0; q < nb; q += 2) {
    // this lane's visibility of the pair; lanes 0 and 32 hold the two
    const int4 inf = b_inf[q + v];
    const int xa = __builtin_amdgcn_readlane(inf.x, 0), ya = __builtin_amdgcn_readlane(inf.y, 0);
    const int xb = __builtin_amdgcn_readlane(inf.x, 32), yb = __builtin_amdgcn_readlane(inf.y, 32);
    const int lo = min(ya, yb), hi = max(ya, yb) + S - 1;
    const int c_lo = (min(xa, xb) - win_x0) >> 3;
    const int c_hi = (max(xa, xb) + S - 1 - win_x0) >> 3;
    const int x0v = inf.x, y0v = inf.y, tabu = inf.z, tabv = inf.w;
    const float2 vv = b_vis[(q + v) * P + ap];
    // A = G^v V: component 0 is t.x vr - t.y vi, component 1 is t.x vi + t.y vr
    const float va = comp == 0 ? vv.x : vv.y;
    const float vb = comp == 0 ? -vv.y : vv.x;

    // A fragments for this wave's row groups and B fragments for every column
    // group, branch-free (all LDS reads in flight together)
    float afr[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int idx = clamp_tap(row0 + j * GSTRIDE + ar - y0v, S);
      if constexpr (CPLX) {
        const float2 t = lds[tabv + idx];
        afr[j] = t.x * va + t.y * vb;                 // component of G^v V
      } else {
        afr[j] = lds[tabv + idx] * va;
      }
    }
    float bfr[WCG];
#pragma unroll
    for (int c = 0; c < WCG; ++c)
      bfr[c] = b_value<CPLX>(lds + tabu, win_x0 + c * 8 + bx - x0v, S, sel_re, sgn);
    // wave-uniform masks of the D tiles either footprint touches
    uint32_t rmask = 0;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int r0 = srow0 + j * GSTRIDE;
      rmask |= (r0 + RG - 1 >= lo && r0 <= hi) ? (1u << j) : 0u;
    }
    const uint32_t cmask = ((2u << c_hi) - 1u) & ~((1u << c_lo) - 1u);
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      if (__builtin_expect((rmask >> j) & 1u, 1)) {
#pragma unroll
        for (int c = 0; c < WCG; ++c) {
          if (__builtin_expect((cmask >> c) & 1u, 1))
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[j], bfr[c], acc[j][c], 0, 0, 0);
        }
      }
    }
  }
}

// Add a wave's window rows to the grid (D layout: lane holds rows 4 (lane / 16) + i,
// column lane % 16 of each tile).
template <int P, int WCG, int NG, int GSTRIDE>
__device__ __forceinline__ void flush_window(const f4 (&acc)[NG][WCG], int row0, int win_x0,
                                             float2* __restrict__ grid, const MfmaDev& d) {
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, m = lane & 15;
  float* gridf = reinterpret_cast<float*>(grid);
  const int col_in = m >> 1, ccomp = m & 1;
#pragma unroll
  for (int j = 0; j < NG; ++j) {
#pragma unroll
    for (int c = 0; c < WCG; ++c) {
      const int col = win_x0 + c * 8 + col_in;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = (P == 4) ? kk : 4 * kk + i;
        const int p = (P == 4) ? i : 0;
        const int row = row0 + j * GSTRIDE + r;
        const float val = acc[j][c][i];
        if (val != 0.f && row < d.H && col < d.W)
          unsafeAtomicAdd(gridf + (((int64_t)p * d.H + row) * d.W + col) * 2 + ccomp, val);
      }
    }
  }
}

// Block form: the 4 waves of a 256-thread block share one segment; wave w owns
// row groups w, w + 4, w + 8, ... so that every footprint gives the four waves
// (and the four SIMDs) nearly equal work.  Batches of 256 visibilities are
// staged by the whole block; the first statement of every batch is a block
// barrier, which also orders the table staging before its first use.
template <int P, bool CPLX, int WR, int WCG>
__device__ __forceinline__ void mfma_segment(const Record* __restrict__ rec,
                                             const float2* __restrict__ wvis, const int4 sg,
                                             const TapT<CPLX>* __restrict__ lds,
                                             int4* __restrict__ b_inf, float2* __restrict__ b_vis,
                                             float2* __restrict__ grid, const MfmaDev& d) {
  constexpr int RG = 16 / P;            // rows per row group
  constexpr int NG = WR / RG / 4;       // row groups per wave
  static_assert(NG * RG * 4 == WR, "window rows must split into row groups over 4 waves");
  const int wave = threadIdx.x >> 6;
  const int begin = sg.x, len = sg.y, tile_id = sg.z;
  const int win_x0 = (tile_id % d.n_tx) * d.tile;
  const int win_y0 = (tile_id / d.n_tx) * d.tile;
  const int row0 = win_y0 + wave * RG;                // first row of this wave's first row group

  f4 acc[NG][WCG];
#pragma unroll
  for (int j = 0; j < NG; ++j)
#pragma unroll
    for (int c = 0; c < WCG; ++c) acc[j][c] = f4{0.f, 0.f, 0.f, 0.f};

  for (int b0 = 0; b0 < len; b0 += kBatch) {
    const int nb = min(kBatch, len - b0);
    __syncthreads();                                   // previous batch consumed (and taps staged)
    {
      // wave w stages visibilities 64 w .. 64 w + 63 of the batch in pairing
      // order within that quarter (pairs never straddle quarters); the quarter
      // holding the last visibility of an odd batch (nb <= 255 here) pads slot nb
      const int cb = wave * 64;
      const int n = max(0, min(64, nb - cb));
      const int pad = ((nb & 1) && nb - cb > 0 && nb - cb <= 64) ? nb - cb : -1;
      stage_pairs<P>(rec, wvis, (int64_t)begin + b0 + cb, n, win_x0, win_y0, d, b_inf + cb, b_vis + cb * P, pad);
    }
    __syncthreads();
    mfma_batch<P, CPLX, WCG, NG, 4 * RG>(b_inf, b_vis, nb, lds, row0, win_x0, d, acc);
  }
  flush_window<P, WCG, NG, 4 * RG>(acc, row0, win_x0, grid, d);
}

// Block form with the wave form's operands (triple table entries, staged row
// addresses and pair masks): wave w stages quarter w of each 256-visibility
// batch in pairing order and works on row groups w, w + 4, ... of every pair.
template <int P, bool CPLX, int WR, int WCG>
__device__ __forceinline__ void mfma_segment_tri(const Record* __restrict__ rec,
                                                 const float2* __restrict__ wvis, const int4 sg,
                                                 uint32_t tab_base, int4* __restrict__ b_inf,
                                                 float2* __restrict__ b_vis, uint32_t* __restrict__ b_box,
                                                 float2* __restrict__ grid, const MfmaDev& d) {
  constexpr int RG = 16 / P;
  constexpr int NG = WR / RG / 4;
  static_assert(NG * RG * 4 == WR, "window rows must split into row groups over 4 waves");
  static_assert(WR / RG <= 16 && WCG <= 8, "pair masks hold 16 row groups and 8 column groups");
  const int wave = threadIdx.x >> 6;
  const int begin = sg.x, len = sg.y, tile_id = sg.z;
  const int win_x0 = (tile_id % d.n_tx) * d.tile;
  const int win_y0 = (tile_id / d.n_tx) * d.tile;
  const int row0 = win_y0 + wave * RG;
  f4 acc[NG][WCG];
#pragma unroll
  for (int j = 0; j < NG; ++j)
#pragma unroll
    for (int c = 0; c < WCG; ++c) acc[j][c] = f4{0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < len; b0 += kBatch) {
    const int nb = min(kBatch, len - b0);
    __syncthreads();                                   // previous batch consumed (and taps staged)
    {
      // the quarter holding the last visibility of an odd batch (nb <= 255) pads slot nb
      const int cb = wave * 64;
      const int n = max(0, min(64, nb - cb));
      const int pad = ((nb & 1) && nb - cb > 0 && nb - cb <= 64) ? nb - cb : -1;
      stage_wave<P, CPLX>(rec, wvis, (int64_t)begin + b0 + cb, n, win_x0, win_y0, d, tab_base, b_inf + cb,
                          b_vis + cb * P, b_box + cb / 2, pad);
    }
    __syncthreads();
    wave_batch<P, CPLX, WCG, NG, 4>(b_inf, b_vis, b_box, nb, wave, d.S, acc);
  }
  flush_window<P, WCG, NG, 4 * RG>(acc, row0, win_x0, grid, d);
}

// LDS of the block forms: staging slices, then the tap table
__host__ __device__ constexpr size_t block_slice_bytes(int n_pol, bool tri) {
  return (size_t)kBatch * (sizeof(int4) + (size_t)n_pol * sizeof(float2)) + (tri ? (kBatch / 2) * sizeof(uint32_t) : 0);
}

template <int P, bool CPLX, int WR, int WCG, bool TRI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
grid_mfma_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                 const int4* __restrict__ segs, const int32_t* __restrict__ n_segs_p,
                 const void* __restrict__ taps, float2* __restrict__ grid, MfmaDev d) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int4* b_inf = reinterpret_cast<int4*>(lds_raw);                               // [kBatch]
  float2* b_vis = reinterpret_cast<float2*>(lds_raw + kBatch * sizeof(int4));    // [kBatch][P]
  unsigned char* tab = lds_raw + block_slice_bytes(P, TRI);
  // Segments are listed in tile order and their count is only known on the
  // device, so blocks take segments in dispatch order: consecutive segments
  // (neighbouring tiles) land on different XCDs, which spreads the dense
  // centre of the uv plane over the whole chip.
  const int seg = (int)blockIdx.x;
  if (seg >= *n_segs_p) return;                       // uniform for the block
  if constexpr (TRI) {
    uint32_t* b_box = reinterpret_cast<uint32_t*>(b_vis + kBatch * P);
    const uint32_t tab_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)tab;
    stage_taps_wave<CPLX>(reinterpret_cast<float*>(tab), taps, d);
    mfma_segment_tri<P, CPLX, WR, WCG>(rec, wvis, segs[seg], tab_base, b_inf, b_vis, b_box, grid, d);
  } else {
    stage_taps<CPLX>(reinterpret_cast<TapT<CPLX>*>(tab), taps, d);
    mfma_segment<P, CPLX, WR, WCG>(rec, wvis, segs[seg], reinterpret_cast<const TapT<CPLX>*>(tab), b_inf, b_vis,
                                   grid, d);
  }
}

// The item loop of the wave form: (segment, part) items from the atomic counter
// until they run out.
template <int P, bool CPLX, int WR, int WCG, int NG, bool TRI, bool MIRROR>
__device__ __forceinline__ void wave_items(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                                           const int32_t* __restrict__ order, const int4* __restrict__ segs,
                                           int n_items, int32_t* __restrict__ counter, float2* __restrict__ grid,
                                           const MfmaDev& d, uint32_t tab_base, unsigned char* __restrict__ slice) {
  constexpr int RG = 16 / P;
  constexpr int PARTS = WR / RG / NG;
  const int lane = threadIdx.x & 63;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(counter, 1);
    item = __builtin_amdgcn_readlane(item, 0);
    if (item >= n_items) break;                        // wave-uniform; every wave reaches it
    const int seg = item / PARTS, part = item - seg * PARTS;
    const int4 sg = segs[seg];
    const int begin = sg.x, len = sg.y, tile_id = sg.z;
    const int win_x0 = (tile_id % d.n_tx) * d.tile;
    const int win_y0 = (tile_id / d.n_tx) * d.tile;
    const int row0 = win_y0 + part * RG;
    f4 acc[NG][WCG];
#pragma unroll
    for (int j = 0; j < NG; ++j)
#pragma unroll
      for (int c = 0; c < WCG; ++c) acc[j][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int b0 = 0; b0 < len; b0 += kWaveBatch) {
      const int nb = min(kWaveBatch, len - b0);
      // (reading the next batch ahead measured no faster and costs registers)
      WaveIn<P> in;
      load_wave<P>(rec, wvis, order, (int64_t)begin + b0, nb, in);
      // the wave's own slice: LDS operations of one wave execute in order, so
      // only the compiler must be kept from moving accesses across these points
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // an odd batch (nb <= 63 here) is padded in slot nb
      stage_wave_gap<P, CPLX, TRI, WR, MIRROR>(in, nb, win_x0, win_y0, d, tab_base, slice, (nb & 1) ? nb : -1);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      wave_batch_gap<P, CPLX, TRI, WCG, NG, PARTS, MIRROR>(slice, nb, part, acc);
    }
    flush_window<P, WCG, NG, PARTS * RG>(acc, row0, win_x0, grid, d);
  }
}

// Wave form (see the file header).  PARTS = (WR / RG) / NG items per segment;
// TRI: triple table entries (complex taps).  With the pair table, a table whose
// planes are conjugate pairs takes the mirror-plane loop (no sign flips).
template <int P, bool CPLX, int WR, int WCG, int NG, int THREADS, bool TRI>
__global__ void __launch_bounds__(THREADS)
grid_mfma_waves(const Record* __restrict__ rec, const float2* __restrict__ wvis,
                const int32_t* __restrict__ order,
                const int4* __restrict__ segs, const int32_t* __restrict__ n_segs_p,
                int32_t* __restrict__ counter, const void* __restrict__ taps,
                float2* __restrict__ grid, MfmaDev d, uint32_t tap_bytes) {
  constexpr int RG = 16 / P;
  constexpr int PARTS = WR / RG / NG;
  static_assert(PARTS * NG * RG == WR, "window rows must split into parts of NG row groups");
  static_assert(WR / RG <= 16 && WCG <= 8, "pair masks hold 16 row groups and 8 column groups");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int wave = threadIdx.x >> 6;
  unsigned char* slice = lds_raw + tap_bytes + (size_t)wave * gap_slice_bytes(P, TRI);
  const uint32_t tab_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)lds_raw;
  stage_taps_gap<CPLX, TRI, WR>(reinterpret_cast<float*>(lds_raw), taps, d);
  __syncthreads();                                    // the only block barriers: here and in planes_conjugate
  const int n_items = *n_segs_p * PARTS;
  if constexpr (CPLX && !TRI) {
    if (planes_conjugate<WR>(reinterpret_cast<const float*>(lds_raw), d)) {
      wave_items<P, CPLX, WR, WCG, NG, TRI, true>(rec, wvis, order, segs, n_items, counter, grid, d, tab_base,
                                                  slice);
      return;
    }
  }
  wave_items<P, CPLX, WR, WCG, NG, TRI, false>(rec, wvis, order, segs, n_items, counter, grid, d, tab_base, slice);
}

// Pairing order of the wave form: each segment's entries ordered by the D tiles
// their footprint touches in the window, the class (first row group, first
// column group, one more row group or not, one more column group or not), so
// that consecutive entries, which the wave form pairs, mostly touch the same
// tiles and a pair costs about what one of its visibilities costs.  A counting
// sort per segment (one block each; the order within a class is arbitrary):
// order[begin + k] is the k-th entry of segment [begin, begin + len).
constexpr int kMaxBoxClasses = 128;
constexpr int kMaxCachedSeg = 32768;   // longest segment whose classes the ordering keeps in LDS
__device__ __forceinline__ int box_class(const Record r, int win_x0, int win_y0, int S, int lg_rg, int nc) {
  const int xr = rec_x0(r) - win_x0, yr = rec_y0(r) - win_y0;
  const int rg = 1 << lg_rg;
  const int dc = (((xr & 7) + S - 1) >> 3) - ((S - 1) >> 3);
  const int dg = (((yr & (rg - 1)) + S - 1) >> lg_rg) - ((S - 1) >> lg_rg);
  return (((yr >> lg_rg) * nc + (xr >> 3)) * 2 + dc) * 2 + dg;
}

// CACHE: each entry's class is kept in LDS (one byte per entry of the longest
// segment, dynamic) between the counting and the placing pass, instead of
// reading the record again.
template <bool CACHE>
__global__ void __launch_bounds__(256)
order_segments_kernel(const Record* __restrict__ rec, const int4* __restrict__ segs,
                      const int32_t* __restrict__ n_segs_p, int S, int lg_rg, int tile, int n_tx,
                      int32_t* __restrict__ order) {
  __shared__ int s_at[kMaxBoxClasses];
  extern __shared__ unsigned char s_cls[];
  const int seg = blockIdx.x;
  if (seg >= *n_segs_p) return;                       // uniform over the block
  const int4 sg = segs[seg];
  const int begin = sg.x, len = sg.y;
  const int win_x0 = (sg.z % n_tx) * tile, win_y0 = (sg.z / n_tx) * tile;
  const int nc = ((tile - 1) >> 3) + 1;
  for (int c = threadIdx.x; c < kMaxBoxClasses; c += blockDim.x) s_at[c] = 0;
  __syncthreads();
  // kOrderIlp entries per thread and step, their record loads issued together
  constexpr int kOrderIlp = 4;
  const int step = kOrderIlp * (int)blockDim.x;
  for (int i0 = threadIdx.x; i0 < len; i0 += step) {
    Record r[kOrderIlp];
#pragma unroll
    for (int k = 0; k < kOrderIlp; ++k) {
      const int i = i0 + k * (int)blockDim.x;
      r[k] = i < len ? rec[begin + i] : Record{0, 0};
    }
#pragma unroll
    for (int k = 0; k < kOrderIlp; ++k) {
      const int i = i0 + k * (int)blockDim.x;
      if (i < len) {
        const int c = box_class(r[k], win_x0, win_y0, S, lg_rg, nc);
        if constexpr (CACHE) s_cls[i] = (unsigned char)c;
        atomicAdd(&s_at[c], 1);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {                             // exclusive scan, two classes per lane
    const int lane = threadIdx.x;
    const int a = s_at[2 * lane], b = s_at[2 * lane + 1];
    int incl = a + b;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    const int excl = incl - a - b;
    s_at[2 * lane] = excl;
    s_at[2 * lane + 1] = excl + a;
  }
  __syncthreads();
  for (int i0 = threadIdx.x; i0 < len; i0 += step) {
    int c[kOrderIlp];
#pragma unroll
    for (int k = 0; k < kOrderIlp; ++k) {
      const int i = i0 + k * (int)blockDim.x;
      c[k] = i < len ? (CACHE ? (int)s_cls[i] : box_class(rec[begin + i], win_x0, win_y0, S, lg_rg, nc)) : -1;
    }
#pragma unroll
    for (int k = 0; k < kOrderIlp; ++k) {
      if (c[k] >= 0) order[begin + atomicAdd(&s_at[c[k]], 1)] = begin + i0 + k * (int)blockDim.x;
    }
  }
}

// Persistent block form for batches: a fixed set of blocks takes (instance,
// segment) work items from an atomic counter until the group's items run out;
// the tap table is restaged only when the instance changes.  Every block exits
// once the counter passes the item total, which the prefix kernel wrote before
// this launch.
template <int P, bool CPLX, int WR, int WCG, bool TRI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
grid_mfma_persistent(const BatchInst* __restrict__ inst, const int32_t* __restrict__ members,
                     int n_members, const int32_t* __restrict__ prefix,
                     int32_t* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  int4* b_inf = reinterpret_cast<int4*>(lds_raw);
  float2* b_vis = reinterpret_cast<float2*>(lds_raw + kBatch * sizeof(int4));
  unsigned char* tab = lds_raw + block_slice_bytes(P, TRI);
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
    if constexpr (TRI) {
      if (ii != staged) {
        stage_taps_wave<CPLX>(reinterpret_cast<float*>(tab), I.taps, d);
        staged = ii;
      }
      uint32_t* b_box = reinterpret_cast<uint32_t*>(b_vis + kBatch * P);
      const uint32_t tab_base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char*)tab;
      mfma_segment_tri<P, CPLX, WR, WCG>(I.brec, I.bwvis, I.segs[ls], tab_base, b_inf, b_vis, b_box, I.grid, d);
    } else {
      if (ii != staged) {
        stage_taps<CPLX>(reinterpret_cast<TapT<CPLX>*>(tab), I.taps, d);
        staged = ii;
      }
      mfma_segment<P, CPLX, WR, WCG>(I.brec, I.bwvis, I.segs[ls], reinterpret_cast<const TapT<CPLX>*>(tab), b_inf,
                                     b_vis, I.grid, d);
    }
  }
}

__global__ void __launch_bounds__(64) zero_counter(int32_t* c) {
  if (threadIdx.x == 0) *c = 0;
}

using MfmaFn = void (*)(const Record*, const float2*, const int4*, const int32_t*, const void*,
                        float2*, MfmaDev);
using WaveFn = void (*)(const Record*, const float2*, const int32_t*, const int4*, const int32_t*, int32_t*,
                        const void*, float2*, MfmaDev, uint32_t);

// Wave-form launch shape: threads per block (one block per CU) from the
// accumulator registers of a wave, NG x WCG x 4: four waves per SIMD up to 72,
// three up to 128, else two.
constexpr int wave_threads(int ng, int wcg) {
  return ng * wcg * 4 <= 72 ? 1024 : ng * wcg * 4 <= 128 ? 768 : ng * wcg * 4 <= 168 ? 512 : 256;
}
using PersistFn = void (*)(const BatchInst*, const int32_t*, int, const int32_t*, int32_t*);

// window edge (cells) for a support: footprints of a tile of edge WR - S fit it
int window_of(int support) { return support <= 16 ? 32 : support <= 32 ? 48 : 64; }

// Block forms: 4 waves share the window rows, so P = 1 (16-row groups) needs 64 rows.
template <int P, bool CPLX, bool TRI>
MfmaFn block_fn(int wr) {
  if constexpr (P == 4) {
    if (wr == 32) return grid_mfma_kernel<4, CPLX, 32, 4, TRI>;
    if (wr == 48) return grid_mfma_kernel<4, CPLX, 48, 6, TRI>;
  }
  return grid_mfma_kernel<P, CPLX, 64, 8, TRI>;
}

template <int P, bool CPLX, bool TRI>
PersistFn persist_fn(int wr) {
  if constexpr (P == 4) {
    if (wr == 32) return grid_mfma_persistent<4, CPLX, 32, 4, TRI>;
    if (wr == 48) return grid_mfma_persistent<4, CPLX, 48, 6, TRI>;
  }
  return grid_mfma_persistent<P, CPLX, 64, 8, TRI>;
}

template <bool TRI>
MfmaFn block_fn_for(int n_pol, bool cplx, int wr) {
  if (n_pol == 4) return cplx ? block_fn<4, true, TRI>(wr) : block_fn<4, false, TRI>(wr);
  return cplx ? block_fn<1, true, TRI>(wr) : block_fn<1, false, TRI>(wr);
}

template <bool TRI>
PersistFn persist_fn_for(int n_pol, bool cplx, int wr) {
  if (n_pol == 4) return cplx ? persist_fn<4, true, TRI>(wr) : persist_fn<4, false, TRI>(wr);
  return cplx ? persist_fn<1, true, TRI>(wr) : persist_fn<1, false, TRI>(wr);
}

// Wave-form configurations: NG row groups per wave (a part of the window is
// NG row groups, PARTS = WR / RG / NG parts per segment); the block size
// follows from NG (wave_threads).  Default NG: 8 for P = 4 with the 32-cell
// window (one wave takes the whole window: measured faster than two parts at
// four waves per SIMD), 3 with the 48-cell window, 2 with the 64-cell window;
// 1 for P = 1.
struct WaveCfg {
  WaveFn fn;
  int threads, ng;
};

template <int P, bool CPLX, int WR, int WCG, int NG, bool TRI>
WaveCfg wave_cfg() {
  return WaveCfg{grid_mfma_waves<P, CPLX, WR, WCG, NG, wave_threads(NG, WCG), TRI>, wave_threads(NG, WCG), NG};
}

int default_ng(int n_pol, int wr) { return n_pol == 4 ? (wr == 48 ? 3 : wr == 32 ? 8 : 2) : 1; }

// ng <= 0: the default; an NG with no instance: fn = nullptr
template <int P, bool CPLX, bool TRI>
WaveCfg wave_fn(int wr, int ng) {
  if (ng <= 0) ng = default_ng(P, wr);
  if constexpr (P == 4) {
    if (wr == 32) {
      if (ng == 2) return wave_cfg<4, CPLX, 32, 4, 2, TRI>();
      if (ng == 4) return wave_cfg<4, CPLX, 32, 4, 4, TRI>();
      if (ng == 8) return wave_cfg<4, CPLX, 32, 4, 8, TRI>();
    } else if (wr == 48) {
      if (ng == 2) return wave_cfg<4, CPLX, 48, 6, 2, TRI>();
      if (ng == 3) return wave_cfg<4, CPLX, 48, 6, 3, TRI>();
      if (ng == 4) return wave_cfg<4, CPLX, 48, 6, 4, TRI>();
      if (ng == 6) return wave_cfg<4, CPLX, 48, 6, 6, TRI>();
    } else {
      if (ng == 2) return wave_cfg<4, CPLX, 64, 8, 2, TRI>();
      if (ng == 4) return wave_cfg<4, CPLX, 64, 8, 4, TRI>();
    }
  } else {
    if (wr == 32) {
      if (ng == 1) return wave_cfg<1, CPLX, 32, 4, 1, TRI>();
      if (ng == 2) return wave_cfg<1, CPLX, 32, 4, 2, TRI>();
    } else if (wr == 48) {
      if (ng == 1) return wave_cfg<1, CPLX, 48, 6, 1, TRI>();
      if (ng == 3) return wave_cfg<1, CPLX, 48, 6, 3, TRI>();
    } else {
      if (ng == 1) return wave_cfg<1, CPLX, 64, 8, 1, TRI>();
      if (ng == 2) return wave_cfg<1, CPLX, 64, 8, 2, TRI>();
      if (ng == 4) return wave_cfg<1, CPLX, 64, 8, 4, TRI>();
    }
  }
  return WaveCfg{nullptr, 0, ng};
}

WaveCfg wave_fn_for(int n_pol, bool cplx, bool tri, int wr, int ng) {
  if (n_pol == 4) return !cplx ? wave_fn<4, false, false>(wr, ng) : tri ? wave_fn<4, true, true>(wr, ng)
                                                                          : wave_fn<4, true, false>(wr, ng);
  return !cplx ? wave_fn<1, false, false>(wr, ng) : tri ? wave_fn<1, true, true>(wr, ng)
                                                        : wave_fn<1, true, false>(wr, ng);
}

// LDS bytes of the wave form's gapped table (triple, pair or real entries)
size_t gap_tab_bytes(const gr_kernel& k, int wr, bool tri) {
  const size_t es = k.taps_complex ? (tri ? 12 : 8) : 4;
  return align256(((size_t)(wr - k.support) + (size_t)k.n_planes * k.oversample * wr) * es);
}

int wave_parts(int n_pol, int wr, int ng) { return wr / (16 / n_pol) / ng; }

// wave = true: the wave form's (-Im, Re, Im) entries; false: the block forms' (Re, Im)
size_t tap_lds_bytes(const gr_kernel& k, bool wave) {
  const size_t per = k.taps_complex ? (wave ? 12 : 8) : 4;
  return align256((size_t)k.n_planes * k.oversample * (k.support + 2) * per);
}

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

int binned_tile(int support, int window) { return (window > 0 ? window : window_of(support)) - support; }

size_t block_lds_bytes(const gr_kernel& k, int n_pol, bool tri) {
  return tap_lds_bytes(k, tri) + block_slice_bytes(n_pol, tri);
}

gr_status plan_mfma(const gr_kernel& k, int n_pol, size_t* lds_bytes) {
  if (k.support > 56) return fail(GR_EUNSUPPORTED, "MFMA gridder needs support <= 56");
  const size_t lds = block_lds_bytes(k, n_pol, false);
  if (lds > 160 * 1024) return fail(GR_EUNSUPPORTED, "tap table does not fit in LDS");
  *lds_bytes = lds;
  return GR_OK;
}

gr_status launch_mfma(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                      float2* grid, int height, int width, hipStream_t stream, int ng) {
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
  if (nb > 0x7fffffff / 8) return fail(GR_EINVAL, "too many segments");
  if (nb == 0) return GR_OK;
  d.n_blocks = (uint32_t)nb;
  const int wr = window_of(k.support);
  if (L.tile + k.support > wr) return fail(GR_EINVAL, "binning tile does not fit the gridder window");
  // wave form when the table leaves room for the wave slices: triple entries
  // when they fit, else (Re, Im) pairs
  bool wtri = k.taps_complex != 0;
  WaveCfg wc = wave_fn_for(n_pol, k.taps_complex != 0, wtri, wr, ng);
  if (wc.fn == nullptr)
    return fail(GR_EUNSUPPORTED, "tuning: no MFMA gridder with this many row groups per wave for the window");
  size_t wave_lds = gap_tab_bytes(k, wr, wtri) + (size_t)(wc.threads / 64) * gap_slice_bytes(n_pol, wtri);
  if (wtri && wave_lds > 160 * 1024) {
    wtri = false;
    wc = wave_fn_for(n_pol, true, false, wr, ng);
    wave_lds = gap_tab_bytes(k, wr, false) + (size_t)(wc.threads / 64) * gap_slice_bytes(n_pol, wtri);
  }
  if (wave_lds <= 160 * 1024) {
    if ((st = ensure_lds_limit(reinterpret_cast<const void*>(wc.fn), wave_lds, "gr_grid_binned")) != GR_OK)
      return st;
    // the work counter sits after the segment count in the bins workspace, the
    // pairing order after the scan scratch
    int32_t* counter = const_cast<int32_t*>(nsegs) + 16;
    auto* order = reinterpret_cast<int32_t*>(const_cast<char*>(base) + L.off_perm);
    const int lg_rg = n_pol == 4 ? 2 : 4;
    const int nc = ((L.tile - 1) >> 3) + 1, ng0 = ((L.tile - 1) >> lg_rg) + 1;
    if (nc * ng0 * 4 > kMaxBoxClasses) return fail(GR_EUNSUPPORTED, "gr_grid_binned: binning tile too large");
    if (L.seg_len <= kMaxCachedSeg)
      order_segments_kernel<true><<<(unsigned)nb, 256, (size_t)L.seg_len, stream>>>(rec, segs, nsegs, k.support,
                                                                                     lg_rg, L.tile, L.n_tx, order);
    else
      order_segments_kernel<false><<<(unsigned)nb, 256, 0, stream>>>(rec, segs, nsegs, k.support, lg_rg, L.tile,
                                                                     L.n_tx, order);
    zero_counter<<<1, 64, 0, stream>>>(counter);
    const int64_t items = nb * wave_parts(n_pol, wr, wc.ng);
    const int waves = wc.threads / 64;
    const int blocks = (int)std::min<int64_t>((int64_t)device_cus(), (items + waves - 1) / waves);
    hipLaunchKernelGGL(wc.fn, dim3((unsigned)blocks), dim3(wc.threads), wave_lds, stream, rec, wv, order, segs,
                       nsegs, counter, k.taps, grid, d, (uint32_t)gap_tab_bytes(k, wr, wtri));
    return check_launch("gr_grid_binned (mfma waves)");
  }
  // block form: triple entries when they fit, else (Re, Im) pairs
  const size_t lds_tri = block_lds_bytes(k, n_pol, true);
  const bool tri = lds_tri <= 160 * 1024;
  if (tri) lds = lds_tri;
  const MfmaFn fn = tri ? block_fn_for<true>(n_pol, k.taps_complex, wr) : block_fn_for<false>(n_pol, k.taps_complex, wr);
  if ((st = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds, "gr_grid_binned")) != GR_OK) return st;
  hipLaunchKernelGGL(fn, dim3((unsigned)nb), dim3(256), lds, stream, rec, wv, segs, nsegs, k.taps,
                     grid, d);
  return check_launch("gr_grid_binned (mfma)");
}

gr_status launch_mfma_persistent(const BatchInst* inst, const int32_t* members, int n_members,
                                 const int32_t* group_prefix, int32_t* counter, int n_pol,
                                 bool complex_taps, bool tri, size_t lds_bytes, int n_blocks,
                                 hipStream_t stream) {
  if (n_members == 0 || n_blocks <= 0) return GR_OK;
  const int wr = kBatchWindow;
  const PersistFn fn = tri ? persist_fn_for<true>(n_pol, complex_taps, wr)
                           : persist_fn_for<false>(n_pol, complex_taps, wr);
  gr_status st = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds_bytes, "gr_grid_batch");
  if (st != GR_OK) return st;
  hipLaunchKernelGGL(fn, dim3((unsigned)n_blocks), dim3(256), lds_bytes, stream, inst, members, n_members,
                     group_prefix, counter);
  return check_launch("gr_grid_batch (persistent mfma)");
}

}  // namespace gr
