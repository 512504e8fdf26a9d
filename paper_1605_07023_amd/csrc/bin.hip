// Binning of the preprocessed visibility stream by footprint position.
//
// The grid is cut into square tiles of T cells; each valid visibility goes to
// the tile that holds its footprint origin (x0, y0), so its whole footprint
// lies inside the tile's (T + S - 1)-cell window.  Within a tile the input
// order is kept for every run of 64 consecutive visibilities (in practice runs
// of one baseline's track), so that neighbouring entries of a tile's list are
// neighbours on the sky as they are in the paper's baseline-ordered stream
// (Section 4).  Each tile's list is cut into segments of at most L entries;
// one segment is the unit of work of the MFMA gridder.
//
// Kernels: count (wave-aggregated atomics per tile), scan (one block:
// offsets, segment table), scatter (wave-aggregated reservation, stable
// within each wave's 64 entries).
#include <algorithm>

#include "internal.h"
#include "prep.h"

namespace gr {

namespace {

__device__ inline int tile_of(Record r, int tile, int n_tx) {
  return (rec_y0(r) / tile) * n_tx + rec_x0(r) / tile;
}

__global__ void __launch_bounds__(256) fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// One visibility per lane; lanes of a wave with the same tile add once.
__device__ __forceinline__ void bin_count_one(const Record* __restrict__ rec, int64_t n, int64_t i,
                                              int tile, int n_tx, int32_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  int key = -1;
  if (i < n) {
    const Record r = rec[i];
    if (rec_valid(r)) key = tile_of(r, tile, n_tx);
  }
  uint64_t todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int k = __shfl(key, leader);
    const uint64_t same = __ballot(key == k);
    if (lane == leader) atomicAdd(&count[k], (int32_t)__popcll(same));
    todo &= ~same;
  }
}

__global__ void __launch_bounds__(256)
bin_count_kernel(const Record* __restrict__ rec, int64_t n, int tile, int n_tx,
                 int32_t* __restrict__ count) {
  bin_count_one(rec, n, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, tile, n_tx, count);
}

// One block of 1024 threads: exclusive scan of counts -> cursor (list
// offsets), and the segment table {begin, length, tile, 0}.
__device__ __forceinline__ void bin_scan_block(const int32_t* __restrict__ count, int n_tiles,
                                               int seg_len, int32_t* __restrict__ cursor,
                                               int4* __restrict__ segs,
                                               int32_t* __restrict__ n_segs_out) {
  __shared__ int64_t s_vis[1024];
  __shared__ int64_t s_seg[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (n_tiles + T - 1) / T;
  const int a = min(n_tiles, t * per), b = min(n_tiles, a + per);
  int64_t v = 0, g = 0;
  for (int i = a; i < b; ++i) {
    v += count[i];
    g += (count[i] + seg_len - 1) / seg_len;
  }
  s_vis[t] = v;
  s_seg[t] = g;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {          // Hillis-Steele inclusive scan
    int64_t xv = 0, xg = 0;
    if (t >= off) {
      xv = s_vis[t - off];
      xg = s_seg[t - off];
    }
    __syncthreads();
    s_vis[t] += xv;
    s_seg[t] += xg;
    __syncthreads();
  }
  int64_t base = s_vis[t] - v, sbase = s_seg[t] - g;
  for (int i = a; i < b; ++i) {
    const int c = count[i];
    cursor[i] = (int32_t)base;
    for (int s0 = 0; s0 < c; s0 += seg_len) {
      segs[sbase++] = make_int4((int)(base + s0), min(seg_len, c - s0), i, 0);
    }
    base += c;
  }
  if (t == T - 1) *n_segs_out = (int32_t)s_seg[T - 1];
}

// ---- parallel scan of the tile counts (single-problem paths) ----------------
// Three launches: per-block sums of 256 tiles' counts and segment counts, one
// block scanning those sums, then per block the tile offsets (cursor) and the
// segment table entries.  Visibility and segment totals fit int32 (n_vis < 2^31).
constexpr int kScanTiles = 256;

// exclusive block-wide prefix of (a, b) over a 256-thread block; totals in ta, tb
__device__ __forceinline__ void block_exclusive_scan2(int a, int b, int& pa, int& pb, int& ta, int& tb) {
  __shared__ int s_a[4], s_b[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int ia = a, ib = b;                                // inclusive scan within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xa = __shfl_up(ia, o), xb = __shfl_up(ib, o);
    if (lane >= o) {
      ia += xa;
      ib += xb;
    }
  }
  if (lane == 63) {
    s_a[wave] = ia;
    s_b[wave] = ib;
  }
  __syncthreads();
  int oa = 0, ob = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (w < wave) {
      oa += s_a[w];
      ob += s_b[w];
    }
    ta += s_a[w];
    tb += s_b[w];
  }
  pa = oa + ia - a;
  pb = ob + ib - b;
}

__global__ void __launch_bounds__(kScanTiles)
scan_sums_kernel(const int32_t* __restrict__ count, int n_tiles, int seg_len, int32_t* __restrict__ sums) {
  const int i = blockIdx.x * kScanTiles + threadIdx.x;
  const int v = i < n_tiles ? count[i] : 0;
  const int g = (v + seg_len - 1) / seg_len;
  int pa, pb, ta, tb;
  block_exclusive_scan2(v, g, pa, pb, ta, tb);
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = ta;
    sums[2 * blockIdx.x + 1] = tb;
  }
}

// one 1024-thread block: exclusive prefix of the n_blocks (count, segments)
// sums in place; the segment total to n_segs_out
__global__ void __launch_bounds__(1024)
scan_blocks_kernel(int32_t* __restrict__ sums, int n_blocks, int32_t* __restrict__ n_segs_out) {
  __shared__ int s_v[1024], s_g[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (n_blocks + T - 1) / T;
  const int a = min(n_blocks, t * per), b = min(n_blocks, a + per);
  int v = 0, g = 0;
  for (int i = a; i < b; ++i) {
    v += sums[2 * i];
    g += sums[2 * i + 1];
  }
  s_v[t] = v;
  s_g[t] = g;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {            // Hillis-Steele inclusive scan
    int xv = 0, xg = 0;
    if (t >= off) {
      xv = s_v[t - off];
      xg = s_g[t - off];
    }
    __syncthreads();
    s_v[t] += xv;
    s_g[t] += xg;
    __syncthreads();
  }
  int bv = s_v[t] - v, bg = s_g[t] - g;
  for (int i = a; i < b; ++i) {
    const int cv = sums[2 * i], cg = sums[2 * i + 1];
    sums[2 * i] = bv;
    sums[2 * i + 1] = bg;
    bv += cv;
    bg += cg;
  }
  if (t == T - 1) *n_segs_out = s_g[T - 1];
}

__global__ void __launch_bounds__(kScanTiles)
scan_write_kernel(const int32_t* __restrict__ count, int n_tiles, int seg_len,
                  const int32_t* __restrict__ sums, int32_t* __restrict__ cursor, int4* __restrict__ segs) {
  const int i = blockIdx.x * kScanTiles + threadIdx.x;
  const int v = i < n_tiles ? count[i] : 0;
  const int g = (v + seg_len - 1) / seg_len;
  int pa, pb, ta, tb;
  block_exclusive_scan2(v, g, pa, pb, ta, tb);
  if (i >= n_tiles) return;
  const int base = sums[2 * blockIdx.x] + pa;
  int sbase = sums[2 * blockIdx.x + 1] + pb;
  cursor[i] = base;
  for (int s0 = 0; s0 < v; s0 += seg_len) segs[sbase++] = make_int4(base + s0, min(seg_len, v - s0), i, 0);
}

// List position of each lane's entry (lanes with key >= 0): the wave's lanes
// are grouped by tile, each lane learning its group's first lane, its rank in
// the group and (for the first lane) the group size; then all groups reserve
// their list space with one atomic instruction.  Keeps lane order within a
// group.  Called by all 64 lanes.
__device__ __forceinline__ int reserve_grouped(int key, int32_t* __restrict__ cursor) {
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int leader = lane, rank = 0, count = 0;
  uint64_t todo = __ballot(key >= 0);
  while (todo) {
    const int l = __ffsll((unsigned long long)todo) - 1;
    const int k = __shfl(key, l);
    const uint64_t same = __ballot(key == k);
    if (key == k) {
      leader = l;
      rank = (int)__popcll(same & below);
      count = (int)__popcll(same);
    }
    todo &= ~same;
  }
  int base = 0;
  if (key >= 0 && lane == leader) base = atomicAdd(&cursor[key], count);
  base = __shfl(base, leader);
  return base + rank;
}

__device__ __forceinline__ void bin_scatter_one(const Record* __restrict__ rec,
                                                const float2* __restrict__ wvis, int64_t n,
                                                int64_t i, int n_pol, int tile, int n_tx,
                                                int32_t* __restrict__ cursor,
                                                Record* __restrict__ out_rec,
                                                float2* __restrict__ out_wvis) {
  int key = -1;
  Record r{0, 0};
  if (i < n) {
    r = rec[i];
    if (rec_valid(r)) key = tile_of(r, tile, n_tx);
  }
  const int pos = reserve_grouped(key, cursor);
  if (key >= 0) {
    out_rec[pos] = r;
    for (int p = 0; p < n_pol; ++p) out_wvis[(int64_t)pos * n_pol + p] = wvis[i * n_pol + p];
  }
}

__global__ void __launch_bounds__(256)
bin_scatter_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis, int64_t n,
                   int n_pol, int tile, int n_tx, int32_t* __restrict__ cursor,
                   Record* __restrict__ out_rec, float2* __restrict__ out_wvis) {
  bin_scatter_one(rec, wvis, n, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, n_pol, tile, n_tx,
                  cursor, out_rec, out_wvis);
}

// ---- preprocess and bin in one pass over the visibilities -------------------
// Pass 1 reads only uvw: the record from the coordinates (into an unbinned
// record array) and the per-tile counts.  Pass 2, after the scan, reads the
// record, the visibilities and the weights, applies the weights and writes
// both to the binned position.  A visibility whose values are not finite
// stays in its list with zero values and moves from the kept to the dropped
// count, so the grid and the statistics are those of gr_preprocess + gr_bin.

// Count a wave's keys over R visibilities per lane (chunks of 64 consecutive
// visibilities): one atomic per distinct tile, issued by the first lane that
// holds it.  On the full-shape tracks 64 consecutive visibilities touch about 8
// tiles and 256 about 14, so four chunks need 2.4 times fewer atomics.
template <int R>
__device__ __forceinline__ void count_grouped(const int (&key)[R], int32_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  uint64_t todo[R];
#pragma unroll
  for (int q = 0; q < R; ++q) todo[q] = __ballot(key[q] >= 0);
  for (;;) {
    int k = -1, leader = -1;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (leader < 0 && todo[q]) {
        leader = __ffsll((unsigned long long)todo[q]) - 1;
        k = __shfl(key[q], leader);
      }
    }
    if (leader < 0) break;                            // uniform
    int total = 0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const uint64_t same = __ballot(key[q] == k);
      total += (int)__popcll(same);
      todo[q] &= ~same;
    }
    if (lane == leader) atomicAdd(&count[k], total);
  }
}

constexpr int kCountChunks = 4;   // visibilities per lane and step of prebin_count_kernel

__global__ void __launch_bounds__(256)
prebin_count_kernel(prep::PreArgs a, int tile, int n_tx, int32_t* __restrict__ count,
                    unsigned long long* __restrict__ stats) {
  constexpr int R = kCountChunks;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  int n_ok = 0, n_drop = 0;
  // a wave takes 64 R consecutive visibilities per step (grid-stride by whole
  // waves, so the wave-wide votes see every lane)
  for (int64_t i0 = wave * 64 * R; i0 < a.n; i0 += n_waves * 64 * R) {
    int key[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = i0 + q * 64 + lane;
      key[q] = -1;
      if (i < a.n) {
        const Record r = prep::coord_record(i, a);
        a.rec[i] = r;
        if (rec_valid(r)) {
          key[q] = tile_of(r, tile, n_tx);
          ++n_ok;
        } else {
          ++n_drop;
          if (a.zero_dropped != nullptr)
            for (int p = 0; p < a.n_pol; ++p) a.zero_dropped[i * a.n_pol + p] = make_float2(0.f, 0.f);
        }
      }
    }
    count_grouped<R>(key, count);
  }
  prep::add_block_counts(n_ok, n_drop, stats);
}

// Pass 2 of the fused binning, by blocks of kScatterBlock consecutive
// visibilities: the block groups its entries by tile (a table of its distinct
// tiles in LDS), reserves each tile's run in the list with one atomic, stages
// the entries in LDS run by run, and then writes them so that consecutive
// lanes write consecutive list slots.  Within a run, the entries of one wave
// (64 consecutive visibilities) keep their input order.
constexpr int kScatterBlock = 512;
template <int VDT, int P>
__global__ void __launch_bounds__(kScatterBlock)
prebin_scatter_kernel(prep::PreArgs a, int tile, int n_tx, int32_t* __restrict__ cursor,
                      Record* __restrict__ out_rec, float2* __restrict__ out_wvis,
                      unsigned long long* __restrict__ stats) {
  constexpr int T = kScatterBlock, HS = kScatterBlock;     // at most T distinct tiles per block
  __shared__ int s_key[HS], s_len[HS], s_start[HS], s_base[HS];
  __shared__ Record s_rec[T];
  __shared__ float2 s_vis[T * P];
  __shared__ short s_slot[T];
  __shared__ int s_wave_tot[T / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t i = (int64_t)blockIdx.x * T + t;
  for (int h = t; h < HS; h += T) { s_key[h] = -1; s_len[h] = 0; }
  int key = -1;
  Record r{0, 0};
  if (i < a.n) {
    r = a.rec[i];
    if (rec_valid(r)) key = tile_of(r, tile, n_tx);
  }
  float2 vw[P];
  bool bad = false;
  if (key >= 0) bad = !prep::weighted_vis<VDT, P>(i, a, vw);
  // the wave's lanes grouped by tile: group leader, rank in the group, group size
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int leader = lane, rank = 0, count = 0;
  {
    uint64_t todo = __ballot(key >= 0);
    while (todo) {
      const int l = __ffsll((unsigned long long)todo) - 1;
      const int k = __shfl(key, l);
      const uint64_t same = __ballot(key == k);
      if (key == k) {
        leader = l;
        rank = (int)__popcll(same & below);
        count = (int)__popcll(same);
      }
      todo &= ~same;
    }
  }
  __syncthreads();                                   // the table is cleared
  // each group's leader finds (or claims) its tile's slot and takes the group's
  // offset in the block's run of that tile
  int slot = 0, off = 0;
  if (key >= 0 && lane == leader) {
    int h = (int)(((uint32_t)key * 2654435761u) >> 23) & (HS - 1);
    for (;;) {
      const int prev = atomicCAS(&s_key[h], -1, key);
      if (prev == -1 || prev == key) break;
      h = (h + 1) & (HS - 1);
    }
    slot = h;
    off = atomicAdd(&s_len[h], count);
  }
  slot = __shfl(slot, leader);
  off = __shfl(off, leader) + rank;
  __syncthreads();                                   // every run length is final
  // block-local run starts (exclusive scan of the run lengths over the slots,
  // HS / T slots per thread) and one reservation per run in the tile's list
  {
    const int len = s_len[t];
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63) s_wave_tot[w] = incl;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < w; ++q) before += s_wave_tot[q];
    s_start[t] = before + incl - len;
    if (len > 0) s_base[t] = atomicAdd(&cursor[s_key[t]], len);
  }
  __syncthreads();
  int n_kept = 0;
  for (int q = 0; q < T / 64; ++q) n_kept += s_wave_tot[q];
  if (key >= 0) {
    const int local = s_start[slot] + off;
    s_rec[local] = r;
#pragma unroll
    for (int p = 0; p < P; ++p) s_vis[local * P + p] = vw[p];
    s_slot[local] = (short)slot;
  }
  __syncthreads();
  if (t < n_kept) {
    const int h = s_slot[t];
    const int64_t pos = (int64_t)s_base[h] + (t - s_start[h]);
    out_rec[pos] = s_rec[t];
#pragma unroll
    for (int p = 0; p < P; ++p) out_wvis[pos * P + p] = s_vis[t * P + p];
  }
  const uint64_t n_bad = __ballot(bad);
  if (n_bad != 0 && lane == 0 && stats != nullptr) {
    const unsigned long long nb = (unsigned long long)__popcll(n_bad);
    atomicAdd(&stats[0], 0ull - nb);                // modular: subtracts nb
    atomicAdd(&stats[1], nb);
  }
}

// Degridding's binning: records from uvw and tile counts as above, then each
// kept record and its input index (int32) to the binned slot.
__global__ void __launch_bounds__(256)
index_scatter_kernel(const Record* __restrict__ rec, int64_t n, int tile, int n_tx, int32_t* __restrict__ cursor,
                     Record* __restrict__ out_rec, int32_t* __restrict__ out_idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int key = -1;
  Record r{0, 0};
  if (i < n) {
    r = rec[i];
    if (rec_valid(r)) key = tile_of(r, tile, n_tx);
  }
  const int pos = reserve_grouped(key, cursor);
  if (key >= 0) {
    out_rec[pos] = r;
    out_idx[pos] = (int32_t)i;
  }
}

// ---- batched forms (one launch for all instances of a batch) ----------------

// zero every instance's tile counts and segment count (block per instance)
__global__ void __launch_bounds__(256) batch_bin_zero_kernel(const BatchInst* __restrict__ inst) {
  const BatchInst& I = inst[blockIdx.x];
  for (int t = threadIdx.x; t < I.n_tiles; t += blockDim.x) I.count[t] = 0;
  if (threadIdx.x == 0) *I.n_segs = 0;
}

__global__ void __launch_bounds__(256)
batch_bin_count_kernel(const BatchInst* __restrict__ inst, int n_inst) {
  __shared__ int s_i;
  if (threadIdx.x == 0) s_i = batch_find(inst, n_inst, (int64_t)blockIdx.x);
  __syncthreads();
  const BatchInst& I = inst[s_i];
  bin_count_one(I.rec, I.n_vis, ((int64_t)blockIdx.x - I.blk_begin) * blockDim.x + threadIdx.x,
                I.d.tile, I.d.n_tx, I.count);
}

__global__ void __launch_bounds__(1024) batch_bin_scan_kernel(const BatchInst* __restrict__ inst) {
  const BatchInst& I = inst[blockIdx.x];
  bin_scan_block(I.count, I.n_tiles, I.seg_len, I.cursor, I.segs, I.n_segs);
}

__global__ void __launch_bounds__(256)
batch_bin_scatter_kernel(const BatchInst* __restrict__ inst, int n_inst) {
  __shared__ int s_i;
  if (threadIdx.x == 0) s_i = batch_find(inst, n_inst, (int64_t)blockIdx.x);
  __syncthreads();
  const BatchInst& I = inst[s_i];
  bin_scatter_one(I.rec, I.wvis, I.n_vis, ((int64_t)blockIdx.x - I.blk_begin) * blockDim.x + threadIdx.x,
                  I.n_pol, I.d.tile, I.d.n_tx, I.cursor, I.brec, I.bwvis);
}

}  // namespace

BinLayout bin_layout(int64_t n_vis, int n_pol, int support, int height, int width, int seg_len,
                     int window) {
  BinLayout L{};
  L.tile = binned_tile(support, window);
  if (L.tile <= 0 || seg_len <= 0) return L;   // no window holds such footprints: bytes = 0
  L.n_tx = (width + L.tile - 1) / L.tile;
  L.n_ty = (height + L.tile - 1) / L.tile;
  L.n_tiles = (int64_t)L.n_tx * L.n_ty;
  L.seg_len = seg_len;
  L.max_segs = L.n_tiles + (n_vis + seg_len - 1) / seg_len;
  size_t off = 0;
  L.off_rec = off;     off += align256(sizeof(Record) * (size_t)n_vis);
  L.off_wvis = off;    off += align256(sizeof(float2) * (size_t)n_vis * n_pol);
  L.off_count = off;   off += align256(sizeof(int32_t) * (size_t)L.n_tiles);
  L.off_cursor = off;  off += align256(sizeof(int32_t) * (size_t)L.n_tiles);
  L.off_segs = off;    off += align256(sizeof(int4) * (size_t)L.max_segs);
  L.off_nsegs = off;   off += 256;
  L.off_scan = off;    off += align256(2 * sizeof(int32_t) * (size_t)((L.n_tiles + kScanTiles - 1) / kScanTiles));
  L.off_perm = off;    off += align256(sizeof(int32_t) * (size_t)n_vis);   // the MFMA gridder's pairing order
  L.bytes = off;
  return L;
}

// tile offsets, segment table and segment count from the tile counts
void launch_scan(const int32_t* count, const BinLayout& L, char* base, hipStream_t stream) {
  auto* cursor = reinterpret_cast<int32_t*>(base + L.off_cursor);
  auto* segs = reinterpret_cast<int4*>(base + L.off_segs);
  auto* nsegs = reinterpret_cast<int32_t*>(base + L.off_nsegs);
  auto* sums = reinterpret_cast<int32_t*>(base + L.off_scan);
  const int nb = (int)((L.n_tiles + kScanTiles - 1) / kScanTiles);
  scan_sums_kernel<<<nb, kScanTiles, 0, stream>>>(count, (int)L.n_tiles, L.seg_len, sums);
  scan_blocks_kernel<<<1, 1024, 0, stream>>>(sums, nb, nsegs);
  scan_write_kernel<<<nb, kScanTiles, 0, stream>>>(count, (int)L.n_tiles, L.seg_len, sums, cursor, segs);
}

gr_status launch_preprocess_bin(const double* uvw, const void* vis, int vis_dtype, const float* vis_scale,
                                const float* weights, int64_t n_vis, int n_pol, const gr_kernel& k,
                                double inv_cell_u, double inv_cell_v, int height, int width, const BinLayout& L,
                                void* bins, Record* rec_tmp, int64_t* dev_stats, hipStream_t stream,
                                const int32_t* ids, int n_ids) {
  char* base = reinterpret_cast<char*>(bins);
  auto* count = reinterpret_cast<int32_t*>(base + L.off_count);
  auto* cursor = reinterpret_cast<int32_t*>(base + L.off_cursor);
  auto* nsegs = reinterpret_cast<int32_t*>(base + L.off_nsegs);
  auto* orec = reinterpret_cast<Record*>(base + L.off_rec);
  auto* owv = reinterpret_cast<float2*>(base + L.off_wvis);
  if (L.n_tiles > 0x7fffffff) return fail(GR_EINVAL, "gr_preprocess_bin: too many tiles");
  const int64_t blocks = (n_vis + 255) / 256;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_preprocess_bin: n_vis too large");
  fill_i32<<<(unsigned)((L.n_tiles + 255) / 256), 256, 0, stream>>>(count, L.n_tiles, 0);
  fill_i32<<<1, 256, 0, stream>>>(nsegs, 1, 0);
  auto* st = reinterpret_cast<unsigned long long*>(dev_stats);
  prep::PreArgs a = prep::make_pre_args(uvw, vis, vis_scale, weights, n_vis, n_pol, k, inv_cell_u, inv_cell_v,
                                        height, width, rec_tmp, nullptr);
  a.ids = ids;
  a.n_ids = n_ids;
  if (n_vis > 0) {
    const int64_t cblocks = std::min<int64_t>(blocks, (int64_t)prep::device_cu_count() * 16);
    prebin_count_kernel<<<(unsigned)cblocks, 256, 0, stream>>>(a, L.tile, L.n_tx, count, st);
  }
  launch_scan(count, L, base, stream);
  if (n_vis > 0) {
    using Fn = void (*)(prep::PreArgs, int, int, int32_t*, Record*, float2*, unsigned long long*);
    Fn fn;
    if (n_pol == 4) fn = vis_dtype == GR_F32 ? prebin_scatter_kernel<GR_F32, 4> : prebin_scatter_kernel<GR_F16, 4>;
    else fn = vis_dtype == GR_F32 ? prebin_scatter_kernel<GR_F32, 1> : prebin_scatter_kernel<GR_F16, 1>;
    hipLaunchKernelGGL(fn, dim3((unsigned)((n_vis + kScatterBlock - 1) / kScatterBlock)), dim3(kScatterBlock), 0,
                       stream, a, L.tile, L.n_tx, cursor, orec, owv, st);
  }
  return check_launch("gr_preprocess_bin");
}

gr_status launch_degrid_bin(const double* uvw, int64_t n_vis, int n_pol, const gr_kernel& k, double inv_cell_u,
                            double inv_cell_v, int height, int width, const BinLayout& L, void* bins,
                            Record* rec_tmp, float2* vis_out, int64_t* dev_stats, hipStream_t stream) {
  char* base = reinterpret_cast<char*>(bins);
  auto* count = reinterpret_cast<int32_t*>(base + L.off_count);
  auto* cursor = reinterpret_cast<int32_t*>(base + L.off_cursor);
  auto* nsegs = reinterpret_cast<int32_t*>(base + L.off_nsegs);
  auto* orec = reinterpret_cast<Record*>(base + L.off_rec);
  auto* oidx = reinterpret_cast<int32_t*>(base + L.off_wvis);
  if (L.n_tiles > 0x7fffffff) return fail(GR_EINVAL, "gr_degrid: too many tiles");
  const int64_t blocks = (n_vis + 255) / 256;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_degrid: n_vis too large");
  fill_i32<<<(unsigned)((L.n_tiles + 255) / 256), 256, 0, stream>>>(count, L.n_tiles, 0);
  fill_i32<<<1, 256, 0, stream>>>(nsegs, 1, 0);
  auto* st = reinterpret_cast<unsigned long long*>(dev_stats);
  prep::PreArgs a = prep::make_pre_args(uvw, nullptr, nullptr, nullptr, n_vis, n_pol, k, inv_cell_u, inv_cell_v,
                                        height, width, rec_tmp, nullptr);
  a.zero_dropped = vis_out;
  if (n_vis > 0) {
    const int64_t cblocks = std::min<int64_t>(blocks, (int64_t)prep::device_cu_count() * 16);
    prebin_count_kernel<<<(unsigned)cblocks, 256, 0, stream>>>(a, L.tile, L.n_tx, count, st);
  }
  launch_scan(count, L, base, stream);
  if (n_vis > 0)
    index_scatter_kernel<<<(unsigned)blocks, 256, 0, stream>>>(rec_tmp, n_vis, L.tile, L.n_tx, cursor, orec, oidx);
  return check_launch("gr_degrid (bin)");
}

gr_status launch_bin(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol,
                     const BinLayout& L, void* bins, hipStream_t stream) {
  char* base = reinterpret_cast<char*>(bins);
  auto* count = reinterpret_cast<int32_t*>(base + L.off_count);
  auto* cursor = reinterpret_cast<int32_t*>(base + L.off_cursor);
  auto* nsegs = reinterpret_cast<int32_t*>(base + L.off_nsegs);
  auto* orec = reinterpret_cast<Record*>(base + L.off_rec);
  auto* owv = reinterpret_cast<float2*>(base + L.off_wvis);
  if (L.n_tiles > 0x7fffffff) return fail(GR_EINVAL, "gr_bin: too many tiles");
  fill_i32<<<(unsigned)((L.n_tiles + 255) / 256), 256, 0, stream>>>(count, L.n_tiles, 0);
  fill_i32<<<1, 256, 0, stream>>>(nsegs, 1, 0);
  const int64_t blocks = (n_vis + 255) / 256;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_bin: n_vis too large");
  if (n_vis > 0)
    bin_count_kernel<<<(unsigned)blocks, 256, 0, stream>>>(rec, n_vis, L.tile, L.n_tx, count);
  launch_scan(count, L, base, stream);
  if (n_vis > 0)
    bin_scatter_kernel<<<(unsigned)blocks, 256, 0, stream>>>(rec, wvis, n_vis, n_pol, L.tile, L.n_tx,
                                                            cursor, orec, owv);
  return check_launch("gr_bin");
}

gr_status launch_batch_bin(const BatchInst* inst, int n_inst, int64_t total_blocks, hipStream_t stream) {
  if (n_inst == 0) return GR_OK;
  if (total_blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_grid_batch: too many visibilities");
  batch_bin_zero_kernel<<<(unsigned)n_inst, 256, 0, stream>>>(inst);
  if (total_blocks > 0) batch_bin_count_kernel<<<(unsigned)total_blocks, 256, 0, stream>>>(inst, n_inst);
  batch_bin_scan_kernel<<<(unsigned)n_inst, 1024, 0, stream>>>(inst);
  if (total_blocks > 0) batch_bin_scatter_kernel<<<(unsigned)total_blocks, 256, 0, stream>>>(inst, n_inst);
  return check_launch("gr_grid_batch (bin)");
}

}  // namespace gr
