// Voxel-structure build: cell coordinates, cell keys, gather into key order,
// and the per-row cell tables used by the candidate sweeps.  Runs once per
// set of frames; each frame is hashed in its own local coordinates, so the
// structure does not depend on the poses.
#include <algorithm>
#include <cfloat>
#include <climits>

#include "rkhsba_device.h"

namespace rkhsba {
namespace {

constexpr int kThreads = 256;

__device__ inline void frame_of(const int64_t* __restrict__ off, int K, int64_t i, int& f, int64_t& local) {
  f = upper_segment(off, K, i);
  local = i - off[f];
}

// k = floor(x * inv_cell) per axis (FP64), and per-frame min/max (and, with
// class ids, the largest id).
// minmax layout: [f*6 + 0..2] min, [f*6 + 3..5] max; [K*6] error flag.
// A block takes kCoordItems consecutive points per thread-column (threads
// read consecutive points); the bounds of the block's first frame are reduced
// in the block (wavefront shuffles, then LDS) and written with one atomic per
// value, so a frame's few bound words see a handful of atomics per block
// instead of one per wavefront.  Points of any later frame in the block (at
// most a frame boundary or a few small frames) use per-point atomics.
constexpr int kCoordItems = 16;
constexpr int kXtabItems = 4;  // points per thread of the x-table fill

__global__ __launch_bounds__(kThreads) void k_cell_coords(const float* const* __restrict__ xyz,
                                                          const int64_t* __restrict__ off, int K, int64_t n_total,
                                                          double inv_cell, const void* const* __restrict__ cls,
                                                          int32_t* __restrict__ cell, int32_t* __restrict__ minmax,
                                                          int32_t* __restrict__ label_max) {
  // min x, y, z, max x, y, z and largest id of the block's first frame (sb[0][.]) and of the next one
  // (sb[1][.]: a block that straddles a frame boundary)
  __shared__ int32_t sb[2][7];
  const int t = threadIdx.x;
  if (t < 2) {
    for (int a = 0; a < 3; ++a) {
      sb[t][a] = INT_MAX;
      sb[t][3 + a] = INT_MIN;
    }
    sb[t][6] = -1;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kThreads * kCoordItems;
  const int f0 = upper_segment(off, K, base);
  int mn[2][3], mx[2][3], lb[2] = {-1, -1};
  for (int h = 0; h < 2; ++h)
    for (int a = 0; a < 3; ++a) {
      mn[h][a] = INT_MAX;
      mx[h][a] = INT_MIN;
    }
  bool bad = false;
  for (int it = 0; it < kCoordItems; ++it) {
    const int64_t i = base + (int64_t)it * kThreads + t;
    if (i >= n_total) break;
    int f;
    int64_t l;
    frame_of(off, K, i, f, l);
    const float* p = xyz[f] + 3 * l;
    int k[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      const double sv = (double)p[a] * inv_cell;
      if (!(fabs(sv) < 1.0e9)) bad = true;  // NaN, Inf or beyond the int32 cell range
      else k[a] = (int)floor(sv);
      cell[3 * i + a] = k[a];
    }
    const int lab = label_max ? (int)static_cast<const uint16_t*>(cls[f])[l] : -1;
    if (f <= f0 + 1) {
      const int h = f - f0;
      for (int a = 0; a < 3; ++a) {
        mn[h][a] = min(mn[h][a], k[a]);
        mx[h][a] = max(mx[h][a], k[a]);
      }
      lb[h] = max(lb[h], lab);
    } else {  // a third frame inside this block (frames of fewer points than a block)
      for (int a = 0; a < 3; ++a) {
        atomicMin(&minmax[f * 6 + a], k[a]);
        atomicMax(&minmax[f * 6 + 3 + a], k[a]);
      }
      if (label_max) atomicMax(&label_max[f], lab);
    }
  }
  if (__ballot(bad)) {
    if (bad) atomicOr(&minmax[K * 6], 1);
  }
  for (int h = 0; h < 2; ++h) {
    for (int o = 32; o > 0; o >>= 1) {
      for (int a = 0; a < 3; ++a) {
        mn[h][a] = min(mn[h][a], __shfl_xor(mn[h][a], o, 64));
        mx[h][a] = max(mx[h][a], __shfl_xor(mx[h][a], o, 64));
      }
      lb[h] = max(lb[h], __shfl_xor(lb[h], o, 64));
    }
    if ((t & 63) == 0) {
      for (int a = 0; a < 3; ++a) {
        atomicMin(&sb[h][a], mn[h][a]);
        atomicMax(&sb[h][3 + a], mx[h][a]);
      }
      atomicMax(&sb[h][6], lb[h]);
    }
  }
  __syncthreads();
  // one atomic per bound, frame and block: every block of a frame updates the same few bound words, where
  // per-point atomics (as a straddling block's second frame once had) serialise
  if (t < 14) {
    const int h = t / 7, a = t % 7, f = f0 + h;
    const int32_t v = sb[h][a];
    if (f < K) {
      if (a < 3) {
        if (v != INT_MAX) atomicMin(&minmax[f * 6 + a], v);
      } else if (a < 6) {
        if (v != INT_MIN) atomicMax(&minmax[f * 6 + a], v);
      } else if (label_max && v >= 0) {
        atomicMax(&label_max[f], v);
      }
    }
  }
}

// Cell key of every point; in a label-stacked frame the class id selects the
// layer of NZ cells that the point's z cell lies in (kz' = id * NZ + kz).
__global__ __launch_bounds__(kThreads) void k_cell_keys(const int32_t* __restrict__ cell,
                                                        const int64_t* __restrict__ off,
                                                        const FrameInfo* __restrict__ frames, int K, int64_t n_total,
                                                        const void* const* __restrict__ cls,
                                                        uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_total) return;
  int f;
  int64_t l;
  frame_of(off, K, i, f, l);
  const FrameInfo& F = frames[f];
  const uint32_t kx = (uint32_t)(cell[3 * i] - F.org[0]);
  const uint32_t ky = (uint32_t)(cell[3 * i + 1] - F.org[1]);
  uint32_t kz = (uint32_t)(cell[3 * i + 2] - F.org[2]);
  if (F.n_lab > 0) kz += (uint32_t)static_cast<const uint16_t*>(cls[f])[l] * (uint32_t)F.dim[2];
  keys[i] = (kz * (uint32_t)F.dim[1] + ky) * (uint32_t)F.dim[0] + kx;
  vals[i] = (uint32_t)l;
}

// One block per frame: the first point (frame-local sorted index) of each
// label layer of a label-stacked frame, by binary search over its sorted keys.
__global__ __launch_bounds__(kThreads) void k_label_starts(const uint32_t* __restrict__ keys,
                                                           const FrameInfo* __restrict__ frames,
                                                           const int64_t* __restrict__ lab_off,
                                                           int32_t* __restrict__ out) {
  const FrameInfo F = frames[blockIdx.x];
  if (F.n_lab <= 0) return;
  const uint32_t* k = keys + F.pt_off;
  const uint64_t layer = (uint64_t)F.dim[0] * F.dim[1] * F.dim[2];
  for (int L = threadIdx.x; L <= F.n_lab; L += kThreads) {
    const uint64_t first = (uint64_t)L * layer;  // smallest key of layer L
    int lo = 0, hi = F.n;                        // first index with key >= first
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((uint64_t)k[mid] < first) lo = mid + 1; else hi = mid;
    }
    out[lab_off[blockIdx.x] + L] = lo;
  }
}

// Round to nearest even: float32 -> bfloat16 (finite inputs).
__device__ inline uint16_t f32_to_bf16(float v) {
  const uint32_t u = __float_as_uint(v);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Round to nearest even: float32 -> OCP fp8 e4m3 (bias 7, 3 mantissa bits,
// subnormal step 2^-9), saturating at the largest finite value 448.
__device__ inline uint8_t f32_to_e4m3(float v) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t sign = (u >> 24) & 0x80u;
  const uint32_t a = u & 0x7fffffffu;
  uint32_t code;
  if (a >= 0x43e00000u) {          // |v| >= 448
    code = 0x7eu;
  } else if (a < 0x3c800000u) {    // |v| < 2^-6: multiples of 2^-9
    code = (uint32_t)rintf(__uint_as_float(a) * 512.0f);  // 0..8; 8 is the smallest normal, 2^-6
  } else {
    const uint32_t r = (a + 0x7ffffu + ((a >> 20) & 1u)) >> 20;  // biased exponent and 3 mantissa bits, rounded
    code = r - (120u << 3);                                       // exponent bias 127 -> 7
    if (code > 0x7eu) code = 0x7eu;
  }
  return (uint8_t)(sign | code);
}

// Gathers points into key order.  pts.w carries the class id bits for one-hot
// features.
__global__ __launch_bounds__(kThreads) void k_gather(const float* const* __restrict__ xyz,
                                                     const void* const* __restrict__ feats, int feat_kind,
                                                     const int64_t* __restrict__ off, int K, int64_t n_total,
                                                     const uint32_t* __restrict__ sorted_vals,
                                                     float4* __restrict__ pts, int32_t* __restrict__ perm) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n_total) return;
  int f;
  int64_t s;
  frame_of(off, K, p, f, s);
  const int64_t o = sorted_vals[p];
  const float* x = xyz[f] + 3 * o;
  float w = 0.0f;
  if (feat_kind == 0) w = __uint_as_float((uint32_t)((const uint16_t*)feats[f])[o]);
  pts[p] = make_float4(x[0], x[1], x[2], w);
  perm[p] = (int32_t)o;
}

// Gathers dense feature rows into key order, stored in the feature path's
// element type and zero padded to Dp.  One thread per stored element, in
// storage order: consecutive threads read consecutive elements of a point's
// input row and write consecutive stored elements (one thread per point would
// touch 64 scattered rows with every load and store).  IDX: the element index
// type (32 bits whenever n_total * Dp fits).
template <typename IDX>
__global__ __launch_bounds__(kThreads) void k_gather_feat(const void* const* __restrict__ feats, int feat_kind, int D,
                                                          int Dp, const int64_t* __restrict__ off, int K,
                                                          int64_t n_total, const uint32_t* __restrict__ sorted_vals,
                                                          void* __restrict__ feat, int32_t* __restrict__ neg_flag) {
  const IDX i = (IDX)blockIdx.x * kThreads + threadIdx.x;
  bool neg = false;
  if ((int64_t)i < n_total * Dp) {
    const IDX p = i / (IDX)Dp;
    const int k = (int)(i - p * (IDX)Dp);
    int f;
    int64_t s;
    frame_of(off, K, (int64_t)p, f, s);
    const int64_t o = sorted_vals[p];
    const float v = k < D ? static_cast<const float*>(feats[f])[o * D + k] : 0.0f;
    neg = v < 0.0f;
    if (feat_kind == 1) static_cast<float*>(feat)[i] = v;
    else if (feat_kind == 2) static_cast<uint16_t*>(feat)[i] = f32_to_bf16(v);
    else static_cast<uint8_t*>(feat)[i] = f32_to_e4m3(v);
  }
  // some inner products may be negative: one atomic per wavefront with such an element, none once the flag is
  // set (a per-element atomic on the one flag word serialises)
  const unsigned long long negs = __ballot(neg);
  if (negs && (int)(threadIdx.x & 63) == __builtin_ctzll(negs) && __atomic_load_n(neg_flag, __ATOMIC_RELAXED) == 0)
    atomicOr(neg_flag, 1);
}

__device__ inline void decode(uint32_t key, const FrameInfo& F, int& kx, int& ky, int& kz) {
  const uint32_t nx = (uint32_t)F.dim[0], ny = (uint32_t)F.dim[1];
  kx = (int)(key % nx);
  const uint32_t r = key / nx;
  ky = (int)(r % ny);
  kz = (int)(r / ny);
}

// Smallest value of each feature dimension over n rows of Dp FP32 values: the
// block size and the grid stride are multiples of Dp, so every thread sees
// one dimension (threadIdx.x % Dp) and reads the rows' values coalesced.
// out[d] (bit patterns of non-negative floats, ordered as integers) must hold
// +inf or a larger earlier minimum; negative values count as 0.
__global__ __launch_bounds__(kThreads) void k_feature_min(const float* __restrict__ feat, int64_t total, int Dp,
                                                          uint32_t* __restrict__ out) {
  __shared__ uint32_t sm[64];
  const int t = threadIdx.x;
  if (t < Dp) sm[t] = 0x7f800000u;
  __syncthreads();
  float m = FLT_MAX;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + t; e < total; e += (int64_t)gridDim.x * blockDim.x)
    m = fminf(m, feat[e]);
  atomicMin(&sm[t % Dp], __float_as_uint(fmaxf(m, 0.0f)));
  __syncthreads();
  if (t < Dp) atomicMin(&out[t], sm[t]);
}

__global__ __launch_bounds__(kThreads) void k_row_init(int4* __restrict__ rows, int64_t n_rows) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r < n_rows) rows[r] = make_int4(INT_MAX, INT_MIN, 0, 0);
}

// The x extent of every occupied row: a frame's points are sorted by key, so
// the points of one row are contiguous, and its first and last points give
// x_lo and x_hi (plain stores, no atomics).
__global__ __launch_bounds__(kThreads) void k_row_extent(const uint32_t* __restrict__ keys,
                                                         const FrameInfo* __restrict__ frames,
                                                         const int64_t* __restrict__ off, int K, int64_t n_total,
                                                         int4* __restrict__ rows) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n_total) return;
  int f;
  int64_t s;
  frame_of(off, K, p, f, s);
  const FrameInfo& F = frames[f];
  const uint32_t nx = (uint32_t)F.dim[0];
  const uint32_t key = keys[p];
  const uint32_t row = key / nx;
  const bool head = s == 0 || keys[p - 1] / nx != row;
  const bool tail = s + 1 == F.n || keys[p + 1] / nx != row;
  int4* R = rows + F.row_off + (int64_t)row;
  if (head) R->x = (int)(key - row * nx);
  if (tail) R->y = (int)(key - row * nx);
}

__global__ __launch_bounds__(kThreads) void k_row_sizes(const int4* __restrict__ rows, int64_t n_rows,
                                                        uint32_t* __restrict__ sizes) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n_rows) return;
  const int4 v = rows[r];
  sizes[r] = v.y >= v.x ? (uint32_t)(v.y - v.x + 2) : 0u;
}

__global__ __launch_bounds__(kThreads) void k_row_store_offsets(const uint32_t* __restrict__ offs, int64_t n_rows,
                                                                int4* __restrict__ rows) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r < n_rows) rows[r].z = (int)offs[r];
}

// xtab[row][x - x_lo] = first point (frame-local sorted index) of cell x or,
// for an empty cell, of the next occupied cell in the row; the entry after
// x_hi is the end of the row.  Every entry is written by exactly one thread:
// the head of each occupied cell fills the entries from the previous occupied
// cell of the row (exclusive) up to its own; the row's last point writes the
// end entry.
__device__ __forceinline__ void xtab_point(const uint32_t* __restrict__ keys, const FrameInfo* __restrict__ frames,
                                           const int64_t* __restrict__ off, int K, int64_t p,
                                           const int4* __restrict__ rows, uint32_t* __restrict__ xtab,
                                           uint32_t* heads_sh) {
  int f;
  int64_t s;
  frame_of(off, K, p, f, s);
  const FrameInfo& F = frames[f];
  const uint32_t key = keys[p];
  int kx, ky, kz;
  decode(key, F, kx, ky, kz);
  const int64_t row = (int64_t)kz * F.dim[1] + ky;
  const int4 R = rows[F.row_off + row];
  uint32_t* xt = xtab + F.xt_off + (uint32_t)R.z;
  const bool has_prev = s > 0;
  const bool has_next = s + 1 < F.n;
  const uint32_t kprev = has_prev ? keys[p - 1] : 0u;
  const bool head = !has_prev || kprev != key;
  {  // occupied cells: the wavefront's heads into the block's count
    const unsigned long long heads = __ballot(head), live = __ballot(1);
    if ((int)(threadIdx.x & 63) == __builtin_ctzll(live)) atomicAdd(heads_sh, (uint32_t)__popcll(heads));
  }
  if (head) {  // head of an occupied cell
    int x0 = R.x;
    if (has_prev) {
      int px, py, pz;
      decode(kprev, F, px, py, pz);
      if ((int64_t)pz * F.dim[1] + py == row) x0 = px + 1;
    }
    for (int x = x0; x <= kx; ++x) xt[x - R.x] = (uint32_t)s;
  }
  bool row_end = !has_next;
  if (has_next) {
    int nx, ny, nz;
    decode(keys[p + 1], F, nx, ny, nz);
    row_end = (int64_t)nz * F.dim[1] + ny != row;
  }
  if (row_end) xt[R.y + 1 - R.x] = (uint32_t)(s + 1);
}

__global__ __launch_bounds__(kThreads) void k_xtab_fill(const uint32_t* __restrict__ keys,
                                                        const FrameInfo* __restrict__ frames,
                                                        const int64_t* __restrict__ off, int K, int64_t n_total,
                                                        const int4* __restrict__ rows, uint32_t* __restrict__ xtab,
                                                        uint32_t* __restrict__ n_cells) {
  __shared__ uint32_t heads_sh;  // occupied cells among the block's points
  if (threadIdx.x == 0) heads_sh = 0u;
  __syncthreads();
  for (int it = 0; it < kXtabItems; ++it) {
    const int64_t p = ((int64_t)blockIdx.x * kXtabItems + it) * kThreads + threadIdx.x;
    if (p < n_total) xtab_point(keys, frames, off, K, p, rows, xtab, &heads_sh);
  }
  __syncthreads();
  // one atomic per block on the single counter (one per wavefront serialised there)
  if (threadIdx.x == 0 && heads_sh) atomicAdd(n_cells, heads_sh);
}

// Centroid of one frame: each thread sums a strided subset in FP64, then the
// partial sums are added in thread order.
__global__ __launch_bounds__(kThreads) void k_frame_centroid(const float4* __restrict__ pts, int n,
                                                             double* __restrict__ out) {
  __shared__ double sh[3][kThreads];
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const float4 p = pts[i];
    s[0] += p.x;
    s[1] += p.y;
    s[2] += p.z;
  }
  for (int a = 0; a < 3; ++a) sh[a][threadIdx.x] = s[a];
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int k = 0; k < kThreads; ++k) t += sh[threadIdx.x][k];
    out[threadIdx.x] = n > 0 ? t / n : 0.0;
  }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_frame_centroid(const float4* d_pts, int n, double* d_out, hipStream_t st) {
  k_frame_centroid<<<1, kThreads, 0, st>>>(d_pts, n, d_out);
  return hipGetLastError();
}

hipError_t launch_cell_coords(const float* const* d_xyz_ptrs, const int64_t* d_in_off, int K, int64_t n_total,
                              double inv_cell, const void* const* d_class_ptrs, int32_t* d_cell, int32_t* d_minmax,
                              int32_t* d_label_max, hipStream_t st) {
  if (d_label_max && !d_class_ptrs) return hipErrorInvalidValue;
  if (n_total > 0)
    k_cell_coords<<<(unsigned)((n_total + (int64_t)kThreads * kCoordItems - 1) / ((int64_t)kThreads * kCoordItems)),
                    kThreads, 0, st>>>(d_xyz_ptrs, d_in_off, K, n_total, inv_cell, d_class_ptrs, d_cell, d_minmax,
                                       d_label_max);
  return hipGetLastError();
}

hipError_t launch_cell_keys(const int32_t* d_cell, const int64_t* d_in_off, const FrameInfo* d_frames, int K,
                            int64_t n_total, const void* const* d_class_ptrs, uint32_t* d_keys, uint32_t* d_vals,
                            hipStream_t st) {
  if (n_total > 0)
    k_cell_keys<<<blocks(n_total), kThreads, 0, st>>>(d_cell, d_in_off, d_frames, K, n_total, d_class_ptrs, d_keys,
                                                      d_vals);
  return hipGetLastError();
}

hipError_t launch_label_starts(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_lab_off, int K,
                               int32_t* d_out, hipStream_t st) {
  if (K > 0) k_label_starts<<<K, kThreads, 0, st>>>(d_keys, d_frames, d_lab_off, d_out);
  return hipGetLastError();
}

hipError_t launch_gather(const float* const* d_xyz_ptrs, const void* const* d_feat_ptrs, int feat_kind, int D, int Dp,
                         const FrameInfo* d_frames, const int64_t* d_in_off, int K, int64_t n_total,
                         const uint32_t* d_sorted_vals, float4* d_pts, void* d_feat, int32_t* d_perm,
                         int32_t* d_neg_flag, hipStream_t st) {
  (void)d_frames;
  if (n_total <= 0) return hipSuccess;
  k_gather<<<blocks(n_total), kThreads, 0, st>>>(d_xyz_ptrs, d_feat_ptrs, feat_kind, d_in_off, K, n_total,
                                                 d_sorted_vals, d_pts, d_perm);
  if (feat_kind != 0) {
    const int64_t total = n_total * Dp;
    if (total <= (int64_t)UINT32_MAX - kThreads)
      k_gather_feat<uint32_t><<<blocks(total), kThreads, 0, st>>>(d_feat_ptrs, feat_kind, D, Dp, d_in_off, K, n_total,
                                                                  d_sorted_vals, d_feat, d_neg_flag);
    else
      k_gather_feat<uint64_t><<<blocks(total), kThreads, 0, st>>>(d_feat_ptrs, feat_kind, D, Dp, d_in_off, K, n_total,
                                                                  d_sorted_vals, d_feat, d_neg_flag);
  }
  return hipGetLastError();
}

hipError_t launch_feature_min(const float* d_feat, int64_t n, int Dp, uint32_t* d_min, hipStream_t st) {
  if (Dp <= 0 || Dp > 64 || n <= 0) return Dp > 64 ? hipErrorInvalidValue : hipSuccess;
  const int threads = Dp * (kThreads / Dp);
  const int64_t total = n * Dp;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (total + threads - 1) / threads);
  k_feature_min<<<blocks, threads, 0, st>>>(d_feat, total, Dp, d_min);
  return hipGetLastError();
}

hipError_t launch_rows(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_in_off, int K,
                       int64_t n_total, int4* d_rows, int64_t n_rows, uint32_t* d_sizes, uint32_t* d_scan_tmp,
                       uint64_t* d_total, hipStream_t st) {
  if (n_rows > 0) k_row_init<<<blocks(n_rows), kThreads, 0, st>>>(d_rows, n_rows);
  if (n_total > 0) k_row_extent<<<blocks(n_total), kThreads, 0, st>>>(d_keys, d_frames, d_in_off, K, n_total, d_rows);
  if (n_rows > 0) {
    k_row_sizes<<<blocks(n_rows), kThreads, 0, st>>>(d_rows, n_rows, d_sizes);
    hipError_t e = launch_exclusive_scan(d_sizes, d_sizes, n_rows, d_scan_tmp, d_total, st);
    if (e != hipSuccess) return e;
    k_row_store_offsets<<<blocks(n_rows), kThreads, 0, st>>>(d_sizes, n_rows, d_rows);
  }
  return hipGetLastError();
}

hipError_t launch_xtab(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_in_off, int K,
                       int64_t n_total, const int4* d_rows, uint32_t* d_xtab, uint32_t* d_n_cells, hipStream_t st) {
  if (n_total > 0)
    k_xtab_fill<<<(unsigned)((n_total + (int64_t)kThreads * kXtabItems - 1) / ((int64_t)kThreads * kXtabItems)),
                  kThreads, 0, st>>>(d_keys, d_frames, d_in_off, K, n_total, d_rows, d_xtab,
                                                      d_n_cells);
  return hipGetLastError();
}

}  // namespace rkhsba
