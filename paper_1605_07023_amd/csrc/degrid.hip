// Degridding: the adjoint of gridding.  Merry (2016) names degridding with
// thread coarsening as the next step (Section 6); the operation predicts each
// visibility from the grid through the same separable GCF:
//     V[n, p] = sum_{ky, kx} Tv[plane][sy][ky] Tu[plane][sx][kx] G[p][y0 + ky][x0 + kx]
// (complex products; with the conjugated taps it is the exact adjoint of the
// gridding of unit-weight visibilities).
//
// gfx950 form, on the binned stream of gridding (one window of W x W cells
// per segment, W = T + S):
//  * One 1024-thread block per compute unit stages the tap table once, then
//    takes segments from an atomic counter; per segment the block stages the
//    grid window (all polarisations) in LDS, once, and its 16 waves share it.
//  * A wave takes batches of 8 visibilities.  Stage 1 contracts the window
//    with each visibility's G^u row on the matrix cores: for a row group (4
//    rows x 4 polarisations, or 16 rows at P = 1) and a column group of 8
//    cells, Z[(r, p), (v, re|im)] += sum_{(x, re|im)} G[(r, p), (x, re|im)]
//    B[(x, re|im), (v, re|im)], four v_mfma_f32_16x16x4_f32 per column group
//    (K = 2 cells x (re, im)), with B the sign pattern that makes the real
//    product the complex G . G^u.  Only the row groups and the cell pairs
//    (one MFMA each) that the batch's footprints touch are issued.  The A operand is one LDS read at a
//    lane-constant address plus an immediate offset; the window lines are
//    padded so that those reads are free of bank conflicts.
//  * Stage 2, per row group: each lane multiplies its Z values by its
//    visibility's G^v tap of that row (the complex product needs the partner
//    component, one lane swap) and accumulates; at the end the partial sums
//    of the 4 row lanes are added across the wave and each visibility is
//    written once to its input position (no atomics: the result is
//    deterministic).
#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace gr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kVisPerBatch = 8;     // N = 8 visibilities x (re, im)
constexpr int kDegridThreads = 1024;

__device__ inline float tap_value(const void* __restrict__ t, int64_t idx, int dtype) {
  switch (dtype) {
    case GR_F32: return reinterpret_cast<const float*>(t)[idx];
    case GR_F16: return __half2float(reinterpret_cast<const __half*>(t)[idx]);
    default: return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(t)[idx]);
  }
}

// window lines: 2 W + 2 floats per (row, polarisation).  A wave's LDS read is
// served 32 lanes at a time over 32 banks; the A reads of lanes 0..31 (16
// (row, polarisation) lines x K values 0, 1) then fall in 32 different banks,
// as do lanes 32..63 (measured: 2 W + 4, conflict-free for 64 banks, spent 6x
// more cycles in bank conflicts)
__host__ __device__ constexpr int degrid_line(int wr) { return 2 * wr + 2; }

// clamp a tap index to the padded row (-1 and S read the zero entries)
__device__ __forceinline__ int tap_slot(int t, int S) {
  int r;
  asm("v_med3_i32 %0, %1, -1, %2" : "=v"(r) : "v"(t), "s"(S));
  return r + 1;
}

template <int P, int WR>
__global__ void __launch_bounds__(kDegridThreads)
degrid_kernel(const Record* __restrict__ rec, const int32_t* __restrict__ idx, const int4* __restrict__ segs,
              const int32_t* __restrict__ n_segs_p, int32_t* __restrict__ counter, const void* __restrict__ taps,
              int taps_complex, const float2* __restrict__ grid, float2* __restrict__ vis_out, MfmaDev d) {
  constexpr int RG = 16 / P;
  constexpr int NRG = WR / RG;
  constexpr int WCG = WR / 8;
  constexpr int LS = degrid_line(WR);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float* win = reinterpret_cast<float*>(lds_raw);                                   // [WR][P][LS]
  float2* tab = reinterpret_cast<float2*>(lds_raw + (size_t)WR * P * LS * sizeof(float));   // [rows][S + 2]
  __shared__ int s_seg;

  // tap table: rows [plane * O + s] of S + 2 (re, im) entries, zero at both ends,
  // and one row of zeros after them for the lanes of a batch's missing visibilities
  {
    const int S = d.S, SP = d.S + 2;
    const int n_elem = (d.n_rows_tab + 1) * SP;
    for (int e = threadIdx.x; e < n_elem; e += blockDim.x) {
      const int row = e / SP, kk = e - row * SP - 1;
      const bool in = kk >= 0 && kk < S && row < d.n_rows_tab;
      const int64_t src = (int64_t)row * S + (in ? kk : 0);
      float re = 0.f, im = 0.f;
      if (in) {
        if (taps_complex) {
          re = tap_value(taps, 2 * src, d.tap_dtype);
          im = tap_value(taps, 2 * src + 1, d.tap_dtype);
        } else {
          re = tap_value(taps, src, d.tap_dtype);
        }
      }
      tab[e] = make_float2(re, im);
    }
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
  const int m = lane & 15, k = lane >> 4;
  const int ar = (P == 4) ? (m >> 2) : m, ap = (P == 4) ? (m & 3) : 0;   // A row: (row, polarisation)
  const int v = m >> 1, comp = m & 1;                                     // B and D column: (visibility, re|im)
  const int xk = k >> 1, bcomp = k & 1;                                   // B row: (cell of the K slice, re|im)
  const int a_lane = (ar * P + ap) * LS + 2 * xk + bcomp;
  const int S = d.S;
  const int n_items = *n_segs_p;

  // The next segment's window is read from HBM into registers while the current
  // one is degridded (each thread its share, issued after its wave's last record
  // read of the segment, so that no record read waits for it); the 64-cell window
  // at P = 4 would need 32 more registers and loads its window after the barrier.
  constexpr int WE = WR * P * WR;                                        // window values
  constexpr int PER = (WE + kDegridThreads - 1) / kDegridThreads;        // per thread
  constexpr bool PF = PER <= 9;
  float2 nxt[PF ? PER : 1];
  auto fetch = [&](int sgi) {
    const int4 q = segs[sgi];
    const int wx0 = (q.z % d.n_tx) * d.tile, wy0 = (q.z / d.n_tx) * d.tile;
#pragma unroll
    for (int u = 0; u < (PF ? PER : 1); ++u) {
      const int e = threadIdx.x + u * kDegridThreads;
      const int x = e % WR, t = e / WR, p = t % P, row = t / P;
      const int gy = wy0 + row, gx = wx0 + x;
      nxt[u] = (e < WE && gy < d.H && gx < d.W) ? grid[((int64_t)p * d.H + gy) * d.W + gx] : make_float2(0.f, 0.f);
    }
  };
  __syncthreads();                                   // the table is staged
  if (threadIdx.x == 0) s_seg = atomicAdd(counter, 1);
  __syncthreads();
  int seg = s_seg;
  if (PF && seg < n_items) fetch(seg);
  for (;;) {
    if (seg >= n_items) break;                       // uniform for the block
    __syncthreads();                                 // previous window consumed
    const int4 sg = segs[seg];
    const int begin = sg.x, len = sg.y, tile_id = sg.z;
    const int win_x0 = (tile_id % d.n_tx) * d.tile;
    const int win_y0 = (tile_id / d.n_tx) * d.tile;
    // the window, all polarisations; cells past the grid edge read as zero
    if constexpr (PF) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = threadIdx.x + u * kDegridThreads;
        if (e < WE) {
          const int x = e % WR, t = e / WR, p = t % P, row = t / P;
          *reinterpret_cast<float2*>(win + (row * P + p) * LS + 2 * x) = nxt[u];
        }
      }
    } else {
      for (int e = threadIdx.x; e < WE; e += blockDim.x) {
        const int x = e % WR, t = e / WR, p = t % P, row = t / P;
        const int gy = win_y0 + row, gx = win_x0 + x;
        float2 g = make_float2(0.f, 0.f);
        if (gy < d.H && gx < d.W) g = grid[((int64_t)p * d.H + gy) * d.W + gx];
        *reinterpret_cast<float2*>(win + (row * P + p) * LS + 2 * x) = g;
      }
    }
    if (threadIdx.x == 0) s_seg = atomicAdd(counter, 1);
    __syncthreads();                                 // window complete, next segment claimed
    const int seg_next = s_seg;
    bool fetched = !PF || seg_next >= n_items;

    for (int b0 = wave * kVisPerBatch; b0 < len; b0 += n_waves * kVisPerBatch) {
      const int nb = min(kVisPerBatch, len - b0);
      const bool live = v < nb;
      const Record r = rec[begin + b0 + (live ? v : 0)];
      const int64_t n_out = idx[begin + b0 + (live ? v : 0)];
      if (!fetched && b0 + n_waves * kVisPerBatch >= len) {   // this wave's last batch of the segment
        fetch(seg_next);
        fetched = true;
      }
      const int xr = rec_x0(r) - win_x0, yr = rec_y0(r) - win_y0;
      // a missing visibility reads the zero row: its B values and G^v taps are 0
      const int zero_row = d.n_rows_tab * (S + 2);
      const int rowu = live ? (rec_plane(r) * d.O + rec_sx(r)) * (S + 2) : zero_row;
      const int rowv = live ? (rec_plane(r) * d.O + rec_sy(r)) * (S + 2) : zero_row;
      // row and column groups that the batch's footprints touch (lane 2q holds visibility q)
      int xlo = 1 << 30, xhi = -(1 << 30), ylo = 1 << 30, yhi = -(1 << 30);
      for (int q = 0; q < nb; ++q) {
        const int xq = __builtin_amdgcn_readlane(xr, 2 * q), yq = __builtin_amdgcn_readlane(yr, 2 * q);
        xlo = min(xlo, xq);
        xhi = max(xhi, xq);
        ylo = min(ylo, yq);
        yhi = max(yhi, yq);
      }
      const int g_lo = __builtin_amdgcn_readfirstlane(ylo / RG);
      const int g_hi = __builtin_amdgcn_readfirstlane((yhi + S - 1) / RG);
      // cell pairs (one MFMA's K slice) that the footprints touch
      const int c_lo = __builtin_amdgcn_readfirstlane(xlo >> 1);
      const int c_hi = __builtin_amdgcn_readfirstlane((xhi + S - 1) >> 1);
      const uint64_t cmask = ((2ull << c_hi) - 1ull) & ~((1ull << c_lo) - 1ull);
      // B: visibility v's G^u tap at cell 8c + 2s + xk, as the (bcomp, comp) entry of the complex product
      // (bcomp, comp) = (0,0) and (1,1): Re t; (0,1): Im t; (1,0): -Im t, one read of the
      // entry's component and a lane-constant sign
      const float* tabf = reinterpret_cast<const float*>(tab);
      const int bsel = bcomp == comp ? 0 : 1;
      const uint32_t bsgn = (bcomp == 1 && comp == 0) ? 0x80000000u : 0u;
      float bfr[WCG][4];
#pragma unroll
      for (int c = 0; c < WCG; ++c) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (!((cmask >> (4 * c + s)) & 1ull)) continue;   // uniform; the value is not used
          const float t = tabf[2 * (rowu + tap_slot(8 * c + 2 * s + xk - xr, S)) + bsel];
          bfr[c][s] = __uint_as_float(__float_as_uint(t) ^ bsgn);
        }
      }
      // stage 2 sums, per lane: pr = sum Re(t) Z_own, pi = sum Im(t) Z_own over its rows; the
      // complex product takes the partner lane's pi once, after the last row group
      constexpr int NA = P == 4 ? 4 : 1;
      float pr[NA], pi[NA];
#pragma unroll
      for (int i = 0; i < NA; ++i) pr[i] = pi[i] = 0.f;
      // wave-uniform mask of the row groups in the batch's footprints
      const uint32_t rmask = ((2u << g_hi) - 1u) & ~((1u << g_lo) - 1u);
#pragma unroll
      for (int j = 0; j < NRG; ++j) {
        if (!((rmask >> j) & 1u)) continue;          // uniform
        // the row group's A operands first (every column group: reads stay in the
        // window), so that the wave waits for LDS once per row group
        float av[WCG][4];
        const float* a = win + a_lane + j * RG * P * LS;
#pragma unroll
        for (int c = 0; c < WCG; ++c)
#pragma unroll
          for (int s = 0; s < 4; ++s) av[c][s] = a[16 * c + 4 * s];
        f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < WCG; ++c) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if ((cmask >> (4 * c + s)) & 1ull)           // uniform
              z = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c][s], bfr[c][s], z, 0, 0, 0);
          }
        }
        // stage 2: D row 4k + i of this lane is (row k, pol i) at P = 4, row 4k + i at P = 1
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = j * RG + ((P == 4) ? k : 4 * k + i);
          const float2 tv = tab[rowv + tap_slot(row - yr, S)];
          pr[(P == 4) ? i : 0] = fmaf(tv.x, z[i], pr[(P == 4) ? i : 0]);
          pi[(P == 4) ? i : 0] = fmaf(tv.y, z[i], pi[(P == 4) ? i : 0]);
        }
      }
      // the complex product: component 0 is sum Re(t) Z_re - Im(t) Z_im, component 1 is
      // sum Re(t) Z_im + Im(t) Z_re; Z's other component sits in the neighbouring lane
      // (DPP quad permutation (1, 0, 3, 2)).  Then the partial sums of the 4 row lanes are
      // added; lanes 0..15 write (visibility, component).
      float vacc[NA];
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const float pi_partner =
            __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(pi[i]), 0xB1, 0xF, 0xF, true));
        vacc[i] = comp ? pr[i] + pi_partner : pr[i] - pi_partner;
        vacc[i] += __shfl_xor(vacc[i], 16);
        vacc[i] += __shfl_xor(vacc[i], 32);
      }
      if (k == 0 && live) {
        float* out = reinterpret_cast<float*>(vis_out) + n_out * P * 2 + comp;
#pragma unroll
        for (int i = 0; i < (P == 4 ? 4 : 1); ++i) out[2 * i] = vacc[i];
      }
    }
    if (!fetched) fetch(seg_next);                   // a wave with no batch in this segment
    seg = seg_next;
  }
}

// Per segment: reorder its (record, input index) entries into the Z (Morton)
// order of their footprint origins inside the tile, so that the 8 visibilities
// of a batch are neighbours and their footprints' union stays small (about
// 24 % fewer MFMAs at S = 32, 36 % at S = 16 than in arrival order on the
// full-shape tracks).  One 256-thread block per segment in turn: a counting
// sort over the tile's cells (side^2 buckets, side the power of two >= the
// tile edge) with LDS histograms, then the entries gathered through LDS and
// written back in place.  Entries of one cell keep no particular order.
constexpr int kSortMax = 4096;       // entries per segment (seg_len <= 4096)
constexpr int kSortThreads = 256;

__device__ __forceinline__ int spread6i(int v) {
  v &= 63;
  v = (v | (v << 4)) & 0x0f0f;
  v = (v | (v << 2)) & 0x3333;
  return (v | (v << 1)) & 0x5555;
}

__global__ void __launch_bounds__(kSortThreads)
sort_segments_kernel(Record* __restrict__ rec, int32_t* __restrict__ idx, const int4* __restrict__ segs,
                     const int32_t* __restrict__ n_segs_p, int tile, int n_tx, int buckets) {
  __shared__ int slot[kSortMax];         // cell, then destination, of entry i
  __shared__ int offs[kSortMax];         // per cell: count, then running offset
  __shared__ uint2 tmp[kSortMax];
  const int n_segs = *n_segs_p;
  const int t = threadIdx.x;
  for (int seg = blockIdx.x; seg < n_segs; seg += gridDim.x) {
    const int4 sg = segs[seg];
    const int begin = sg.x, len = sg.y;
    if (len <= 1) continue;                          // uniform for the block
    const int wx0 = (sg.z % n_tx) * tile, wy0 = (sg.z / n_tx) * tile;
    for (int b = t; b < buckets; b += kSortThreads) offs[b] = 0;
    __syncthreads();
    for (int i = t; i < len; i += kSortThreads) {
      const Record r = rec[begin + i];
      const int c = spread6i(rec_x0(r) - wx0) | (spread6i(rec_y0(r) - wy0) << 1);
      slot[i] = c;
      atomicAdd(&offs[c], 1);
    }
    __syncthreads();
    // exclusive scan of the bucket counts: each thread a contiguous run
    {
      const int per = (buckets + kSortThreads - 1) / kSortThreads;
      const int a = min(buckets, t * per), b = min(buckets, a + per);
      int sum = 0;
      for (int q = a; q < b; ++q) sum += offs[q];
      __shared__ int s_part[kSortThreads];
      s_part[t] = sum;
      __syncthreads();
      for (int o = 1; o < kSortThreads; o <<= 1) {   // Hillis-Steele inclusive scan
        const int x = t >= o ? s_part[t - o] : 0;
        __syncthreads();
        s_part[t] += x;
        __syncthreads();
      }
      int run = s_part[t] - sum;
      for (int q = a; q < b; ++q) {
        const int v = offs[q];
        offs[q] = run;
        run += v;
      }
    }
    __syncthreads();
    for (int i = t; i < len; i += kSortThreads) slot[i] = atomicAdd(&offs[slot[i]], 1);
    __syncthreads();
    // gather through LDS, then write back in place (all reads before any write)
    for (int i = t; i < len; i += kSortThreads) {
      const Record r = rec[begin + i];
      tmp[slot[i]] = make_uint2(r.x, r.y);
    }
    __syncthreads();
    for (int i = t; i < len; i += kSortThreads) rec[begin + i] = Record{tmp[i].x, tmp[i].y};
    __syncthreads();
    for (int i = t; i < len; i += kSortThreads) tmp[slot[i]].x = (uint32_t)idx[begin + i];
    __syncthreads();
    for (int i = t; i < len; i += kSortThreads) idx[begin + i] = (int32_t)tmp[i].x;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(64) zero_i32(int32_t* c) {
  if (threadIdx.x == 0) *c = 0;
}

int window_for(int support) { return support <= 16 ? 32 : support <= 32 ? 48 : 64; }

size_t degrid_lds(const gr_kernel& k, int n_pol) {
  const int wr = window_for(k.support);
  return align256((size_t)wr * n_pol * degrid_line(wr) * sizeof(float)) +
         ((size_t)k.n_planes * k.oversample + 1) * (k.support + 2) * sizeof(float2);
}

using DegridFn = void (*)(const Record*, const int32_t*, const int4*, const int32_t*, int32_t*, const void*, int,
                          const float2*, float2*, MfmaDev);

DegridFn degrid_fn(int n_pol, int wr) {
  if (n_pol == 4) return wr == 32 ? degrid_kernel<4, 32> : wr == 48 ? degrid_kernel<4, 48> : degrid_kernel<4, 64>;
  return wr == 32 ? degrid_kernel<1, 32> : wr == 48 ? degrid_kernel<1, 48> : degrid_kernel<1, 64>;
}

}  // namespace

gr_status plan_degrid(const gr_kernel& k, int n_pol, size_t* lds_bytes) {
  if (k.kind != GR_SEPARABLE) return fail(GR_EUNSUPPORTED, "gr_degrid takes separable kernels");
  if (k.support > 56) return fail(GR_EUNSUPPORTED, "gr_degrid needs support <= 56");
  const size_t lds = degrid_lds(k, n_pol);
  if (lds > 160 * 1024)
    return fail(GR_EUNSUPPORTED, "gr_degrid: grid window and tap table do not fit in LDS (160 KiB)");
  *lds_bytes = lds;
  return GR_OK;
}

gr_status launch_degrid(const void* bins, const BinLayout& L, int n_pol, const gr_kernel& k,
                        const float2* grid, int height, int width, float2* vis_out, int64_t n_vis,
                        hipStream_t stream) {
  size_t lds = 0;
  gr_status st = plan_degrid(k, n_pol, &lds);
  if (st != GR_OK) return st;
  const int wr = window_for(k.support);
  if (L.tile + k.support > wr) return fail(GR_EINVAL, "gr_degrid: binning tile does not fit the window");
  // dropped visibilities were zeroed by the binning's count pass; every kept one is written below
  if (L.max_segs == 0 || n_vis == 0) return check_launch("gr_degrid");
  const char* base = reinterpret_cast<const char*>(bins);
  const auto* rec = reinterpret_cast<const Record*>(base + L.off_rec);
  const auto* idx = reinterpret_cast<const int32_t*>(base + L.off_wvis);
  const auto* segs = reinterpret_cast<const int4*>(base + L.off_segs);
  auto* nsegs = const_cast<int32_t*>(reinterpret_cast<const int32_t*>(base + L.off_nsegs));
  int32_t* counter = nsegs + 16;                     // after the segment count, in the same 256 bytes
  MfmaDev d{};
  d.S = k.support; d.O = k.oversample; d.n_rows_tab = k.n_planes * k.oversample;
  d.tap_dtype = k.tap_dtype; d.tile = L.tile; d.n_tx = L.n_tx; d.H = height; d.W = width;
  const DegridFn fn = degrid_fn(n_pol, wr);
  if ((st = ensure_lds_limit(reinterpret_cast<const void*>(fn), lds, "gr_degrid")) != GR_OK) return st;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  if (L.seg_len > kSortMax) return fail(GR_EINVAL, "gr_degrid: seg_len must be <= 4096");
  {
    const int sblocks = (int)std::min<int64_t>((int64_t)cus * 8, L.max_segs);
    int side = 1;
    while (side < L.tile) side <<= 1;
    sort_segments_kernel<<<sblocks, kSortThreads, 0, stream>>>(const_cast<Record*>(rec), const_cast<int32_t*>(idx),
                                                             segs, nsegs, L.tile, L.n_tx, side * side);
  }
  zero_i32<<<1, 64, 0, stream>>>(counter);
  const int blocks = (int)std::min<int64_t>(cus, L.max_segs);
  hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kDegridThreads), lds, stream, rec, idx, segs, nsegs, counter,
                     k.taps, k.taps_complex ? 1 : 0, grid, vis_out, d);
  return check_launch("gr_degrid");
}

}  // namespace gr
