// Segmented, stable LSD radix sort of (uint32 key, uint32 value) pairs.
//
// Segments are contiguous ranges sorted independently (frames when building
// the voxel structure, edges when binning source points per iteration); they
// are known on the host, so the tile -> segment table is static and every
// launch has a fixed shape.  Each 8-bit digit takes three kernels:
//   hist    per tile, a 256-bin digit histogram (LDS atomics)
//   scan    per segment, exclusive offsets over (digit, tile) in digit-major
//           order, i.e. the destination of each tile's first key of each digit
//   scatter per tile, stable ranks: within a wavefront from 8 ballots (lanes
//           sharing a digit), across the 4 wavefronts and the 8 rounds of a
//           tile from LDS counters; keys and values written to their slots.
#include "rkhsba_internal.h"

namespace rkhsba {
namespace {

__global__ __launch_bounds__(kSortThreads) void k_hist(const uint32_t* __restrict__ keys,
                                                       const SortTile* __restrict__ tiles, int shift,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const SortTile t = tiles[blockIdx.x];
  for (int r = 0; r < kSortItems; ++r) {
    const int k = r * kSortThreads + tid;
    if (k < t.count) atomicAdd(&h[(keys[t.start + k] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  hist[(int64_t)blockIdx.x * 256 + tid] = h[tid];
}

__global__ __launch_bounds__(256) void k_scan(uint32_t* __restrict__ hist, const SortSeg* __restrict__ segs) {
  __shared__ uint32_t tot[256];
  const int d = threadIdx.x;
  const SortSeg s = segs[blockIdx.x];
  uint32_t run = 0;
  for (int t = 0; t < s.n_tiles; ++t) {
    uint32_t* h = hist + (int64_t)(s.tile0 + t) * 256 + d;
    const uint32_t c = *h;
    *h = run;  // offset of this tile's first key of digit d among the segment's digit-d keys
    run += c;
  }
  tot[d] = run;
  __syncthreads();
  // exclusive scan of the 256 digit totals (Hillis-Steele on LDS)
  uint32_t v = tot[d];
  for (int o = 1; o < 256; o <<= 1) {
    __syncthreads();
    const uint32_t add = d >= o ? tot[d - o] : 0u;
    __syncthreads();
    tot[d] += add;
  }
  __syncthreads();
  const uint32_t base = tot[d] - v;
  for (int t = 0; t < s.n_tiles; ++t) hist[(int64_t)(s.tile0 + t) * 256 + d] += base;
}

__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const SortTile* __restrict__ tiles,
                                                          const SortSeg* __restrict__ segs,
                                                          const uint32_t* __restrict__ offs, int shift) {
  constexpr int W = kSortThreads / 64;
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[W][256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const SortTile t = tiles[blockIdx.x];
  const int64_t seg_start = segs[t.seg].start;
  base[tid] = offs[(int64_t)blockIdx.x * 256 + tid];
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int r = 0; r < kSortItems; ++r) {
    for (int i = tid; i < W * 256; i += kSortThreads) wcnt[i / 256][i % 256] = 0;
    __syncthreads();
    const int k = r * kSortThreads + tid;
    const bool valid = k < t.count;
    uint32_t key = 0, val = 0, d = 0;
    if (valid) {
      key = kin[t.start + k];
      val = vin[t.start + k];
      d = (key >> shift) & 0xffu;
    }
    uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool b = ((d >> bit) & 1u) != 0u;
      const uint64_t bl = __builtin_amdgcn_ballot_w64(b);
      peers &= b ? bl : ~bl;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int v = 0; v < w; ++v) pos += wcnt[v][d];
      kout[seg_start + pos] = key;
      vout[seg_start + pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int v = 0; v < W; ++v) add += wcnt[v][tid];
    base[tid] += add;
    __syncthreads();
  }
}

}  // namespace

// Sorts bits [0, bits) of every segment; the result ends in (keys, vals) or,
// for an odd number of digit passes, in (keys_tmp, vals_tmp) (*result_in_tmp).
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, uint32_t* hist,
                             const SortTile* d_tiles, int n_tiles, const SortSeg* d_segs, int n_segs, int bits,
                             hipStream_t st, bool* result_in_tmp) {
  uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += 8, ++passes) {
    if (n_tiles > 0) {
      k_hist<<<n_tiles, kSortThreads, 0, st>>>(ki, d_tiles, shift, hist);
      k_scan<<<n_segs, 256, 0, st>>>(hist, d_segs);
      k_scatter<<<n_tiles, kSortThreads, 0, st>>>(ki, vi, ko, vo, d_tiles, d_segs, hist, shift);
    }
    uint32_t* tk = ki; ki = ko; ko = tk;
    uint32_t* tv = vi; vi = vo; vo = tv;
  }
  *result_in_tmp = (passes & 1) != 0;
  return hipGetLastError();
}

}  // namespace rkhsba

// ---------------------------------------------------------------- exclusive scan (uint32)

namespace rkhsba {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const uint32_t add = tid >= o ? sh[tid - o] : 0u;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const uint32_t incl = sh[tid];
  if (total) *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

// Per tile: sum of the tile.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                              uint32_t* __restrict__ tile_sums) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the tile sums (sequential over chunks of 256).
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t* __restrict__ tile_sums, int n_tiles,
                                                             uint64_t* __restrict__ total) {
  __shared__ uint32_t sh[kScanThreads];
  uint64_t carry = 0;
  for (int c = 0; c < n_tiles; c += kScanThreads) {
    const int i = c + threadIdx.x;
    const uint32_t v = i < n_tiles ? tile_sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < n_tiles) tile_sums[i] = (uint32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t* __restrict__ in, int64_t n,
                                                             const uint32_t* __restrict__ tile_sums,
                                                             uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    v[r] = i < n ? in[i] : 0u;
    s += v[r];
  }
  uint32_t run = block_exclusive_scan(s, sh, nullptr) + tile_sums[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + r;
    if (i < n) out[i] = run;
    run += v[r];
  }
}

}  // namespace

// out[i] = sum_{k<i} in[i] (may alias in); *d_total (device, nullable) = sum of all.
// tmp: at least ceil(n / 2048) uint32.
hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint64_t* d_total,
                                 hipStream_t st) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles > 0) {
    k_scan_reduce<<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, tmp);
    k_scan_tiles<<<1, kScanThreads, 0, st>>>(tmp, (int)tiles, d_total);
    k_scan_apply<<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, tmp, out);
  } else if (d_total) {
    hipMemsetAsync(d_total, 0, sizeof(uint64_t), st);
  }
  return hipGetLastError();
}

}  // namespace rkhsba
