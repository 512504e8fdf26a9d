// Compression (Merry 2016, Section 2.2, after Muscat; applied once in the
// preprocess, Section 4): adjacent visibilities at the same position of the
// oversampled grid and in the same w plane meet the same GCF samples, so they
// are added into one visibility.  "Adjacent" is consecutive in the stream;
// a dropped visibility (invalid record) separates runs.
//
// Input: the records and weighted visibilities of gr_preprocess (input
// order).  Output: the same layout with the compressed stream first (run
// heads in input order, each run's visibilities summed in input order, one
// thread per run, so the result is deterministic) and invalid records after
// it, so that gr_bin / gr_grid_binned take the output with the input's n_vis
// and no host synchronisation.
//
// Three steps: per block of 256 positions the number of run heads; the scan of
// those counts (one block, or two levels for long streams), which also writes
// the total; per block the heads' output slots and the runs' sums.
#include <algorithm>

#include "internal.h"

namespace gr {

namespace {

constexpr int kCompressBlock = 256;

__device__ __forceinline__ bool same_key(Record a, Record b) { return a.x == b.x && a.y == b.y; }

// position i starts a run: kept, and the previous position is dropped or holds another key
__device__ __forceinline__ bool is_head(const Record* __restrict__ rec, int64_t i) {
  const Record r = rec[i];
  if (!rec_valid(r)) return false;
  return i == 0 || !same_key(rec[i - 1], r);
}

// exclusive prefix over the 256 threads of a block; total in *total
__device__ __forceinline__ int block_prefix(int v, int* total) {
  __shared__ int s_w[kCompressBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(inc, o);
    if (lane >= o) inc += x;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kCompressBlock / 64; ++w) {
    if (w < wave) off += s_w[w];
    tot += s_w[w];
  }
  *total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(kCompressBlock)
head_count_kernel(const Record* __restrict__ rec, int64_t n, int32_t* __restrict__ block_heads) {
  const int64_t i = (int64_t)blockIdx.x * kCompressBlock + threadIdx.x;
  const int h = (i < n && is_head(rec, i)) ? 1 : 0;
  int total;
  block_prefix(h, &total);
  if (threadIdx.x == 0) block_heads[blockIdx.x] = total;
}

template <int P>
__global__ void __launch_bounds__(kCompressBlock)
compress_write_kernel(const Record* __restrict__ rec, const float2* __restrict__ wvis, int64_t n,
                      const int32_t* __restrict__ block_offset, Record* __restrict__ out_rec,
                      float2* __restrict__ out_wvis) {
  const int64_t i = (int64_t)blockIdx.x * kCompressBlock + threadIdx.x;
  const bool h = i < n && is_head(rec, i);
  int total;
  const int slot = block_offset[blockIdx.x] + block_prefix(h ? 1 : 0, &total);
  if (!h) return;
  const Record r = rec[i];
  float2 acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = wvis[i * P + p];
  for (int64_t j = i + 1; j < n && same_key(rec[j], r); ++j) {   // the run, in input order
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const float2 v = wvis[j * P + p];
      acc[p].x += v.x;
      acc[p].y += v.y;
    }
  }
  out_rec[slot] = r;
#pragma unroll
  for (int p = 0; p < P; ++p) out_wvis[(int64_t)slot * P + p] = acc[p];
}

__global__ void __launch_bounds__(256) zero_records(Record* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = Record{0, 0};
}

}  // namespace

namespace {

// one 1024-thread block: exclusive prefix of n int32 counts in place (their
// total below 2^31); the total to *total (int64) when it is non-NULL
__global__ void __launch_bounds__(1024)
scan_i32_kernel(int32_t* __restrict__ data, int n, int64_t* __restrict__ total) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (n + T - 1) / T;
  const int a = min(n, t * per), b = min(n, a + per);
  int64_t v = 0;
  for (int i = a; i < b; ++i) v += data[i];
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {            // Hillis-Steele inclusive scan
    const int64_t x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int64_t run = s[t] - v;
  for (int i = a; i < b; ++i) {
    const int c = data[i];
    data[i] = (int32_t)run;
    run += c;
  }
  if (t == T - 1 && total != nullptr) *total = s[T - 1];
}

constexpr int kScanChunk = 4096;     // elements per block of the two-level scan (1024 threads x 4)

// first level: each block scans its chunk of 4096 in place (exclusive) and
// writes the chunk's total to sums[block]
__global__ void __launch_bounds__(1024)
scan_chunk_kernel(int32_t* __restrict__ data, int n, int32_t* __restrict__ sums) {
  __shared__ int s_w[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + 4 * t;
  int v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = base + j < n ? data[base + j] : 0;
  const int mine = v[0] + v[1] + v[2] + v[3];
  int inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int x = __shfl_up(inc, o);
    if (lane >= o) inc += x;
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    if (w < wave) off += s_w[w];
    tot += s_w[w];
  }
  int run = off + inc - mine;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) data[base + j] = run;
    run += v[j];
  }
  if (t == 0) sums[blockIdx.x] = tot;
}

// second level done by scan_i32_kernel on sums; then each chunk adds its offset
__global__ void __launch_bounds__(1024)
scan_add_kernel(int32_t* __restrict__ data, int n, const int32_t* __restrict__ sums) {
  const int32_t add = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + 4 * threadIdx.x;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (base + j < n) data[base + j] += add;
}

}  // namespace

size_t scan_i32_scratch_bytes(int64_t n) {
  return align256(sizeof(int32_t) * (size_t)((n + kScanChunk - 1) / kScanChunk + 1));
}

// one block when the counts are few; else chunks of 4096 scanned in parallel,
// their totals scanned by one block, and the chunk offsets added back
void launch_scan_i32(int32_t* data, int n, int64_t* total, int32_t* scratch, hipStream_t stream) {
  if (n <= 4 * kScanChunk) {
    scan_i32_kernel<<<1, 1024, 0, stream>>>(data, n, total);
    return;
  }
  const int chunks = (n + kScanChunk - 1) / kScanChunk;
  scan_chunk_kernel<<<chunks, 1024, 0, stream>>>(data, n, scratch);
  scan_i32_kernel<<<1, 1024, 0, stream>>>(scratch, chunks, total);
  scan_add_kernel<<<chunks, 1024, 0, stream>>>(data, n, scratch);
}

size_t compress_workspace_bytes(int64_t n_vis) {
  const int64_t blocks = (n_vis + kCompressBlock - 1) / kCompressBlock;
  return align256(sizeof(int32_t) * (size_t)blocks) + scan_i32_scratch_bytes(blocks) + 256;
}

gr_status launch_compress(const Record* rec, const float2* wvis, int64_t n_vis, int n_pol, Record* out_rec,
                          float2* out_wvis, int64_t* out_count, void* workspace, hipStream_t stream) {
  const int64_t blocks = (n_vis + kCompressBlock - 1) / kCompressBlock;
  if (blocks > 0x7fffffff) return fail(GR_EINVAL, "gr_compress: n_vis too large");
  auto* block_heads = reinterpret_cast<int32_t*>(workspace);
  if (n_vis > 0) {
    zero_records<<<(unsigned)((n_vis + 255) / 256), 256, 0, stream>>>(out_rec, n_vis);
    head_count_kernel<<<(unsigned)blocks, kCompressBlock, 0, stream>>>(rec, n_vis, block_heads);
  }
  auto* scan_scratch = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) +
                                                 align256(sizeof(int32_t) * (size_t)blocks));
  launch_scan_i32(block_heads, (int)blocks, out_count, scan_scratch, stream);
  if (n_vis > 0) {
    using Fn = void (*)(const Record*, const float2*, int64_t, const int32_t*, Record*, float2*);
    const Fn fn = n_pol == 4 ? compress_write_kernel<4> : compress_write_kernel<1>;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kCompressBlock), 0, stream, rec, wvis, n_vis, block_heads,
                       out_rec, out_wvis);
  }
  return check_launch("gr_compress");
}

}  // namespace gr
