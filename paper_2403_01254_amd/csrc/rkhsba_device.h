// Device helpers shared by the rkhsba kernels: the FP32 membership rule, cell
// arithmetic and wavefront reductions.
#pragma once

#include "rkhsba_internal.h"

namespace rkhsba {

// Relative transform T_nm = T_n^-1 T_m of the documented membership rule, in
// FP64 with a fixed fma order (R_n^T R_m, R_n^T (t_m - t_n)).  Poses are
// [R row-major | t].
__device__ inline void rule_relative(const double* __restrict__ Tm, const double* __restrict__ Tn, double* R,
                                     double* t) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R[3 * a + b] = fma(Tn[6 + a], Tm[6 + b], fma(Tn[3 + a], Tm[3 + b], Tn[a] * Tm[b]));
  const double d0 = Tm[9] - Tn[9], d1 = Tm[10] - Tn[10], d2 = Tm[11] - Tn[11];
  for (int a = 0; a < 3; ++a) t[a] = fma(Tn[6 + a], d2, fma(Tn[3 + a], d1, Tn[a] * d0));
}

// T_nm x in FP64: the source point in the target frame before rounding.
__device__ inline double3 rule_q64(const EdgeXf& xf, float x0, float x1, float x2) {
#pragma clang fp contract(off)
  const double a = x0, b = x1, c = x2;
  double3 q;
  q.x = fma(xf.R[2], c, fma(xf.R[1], b, fma(xf.R[0], a, xf.t[0])));
  q.y = fma(xf.R[5], c, fma(xf.R[4], b, fma(xf.R[3], a, xf.t[1])));
  q.z = fma(xf.R[8], c, fma(xf.R[7], b, fma(xf.R[6], a, xf.t[2])));
  return q;
}

// q32 = float(T_nm x): the source point in the target frame, computed in FP64
// and rounded once.
__device__ inline float3 rule_q32(const EdgeXf& xf, float x0, float x1, float x2) {
  const double3 q = rule_q64(xf, x0, x1, x2);
  return make_float3((float)q.x, (float)q.y, (float)q.z);
}

// Whether a transformed source point lies in the target frame's cell grid extended by the reach on every
// side, with cell coordinates as the build's (floor of q / cell in FP64).  A source outside has no candidate:
// the binning sorts it to the grid's edge, the sweeps leave it out of their boxes and store zero moments.
__device__ inline bool source_in_grid(float3 q, const FrameInfo& F, const KConst& kc) {
  const double u[3] = {(double)q.x * kc.inv_cell - F.org[0], (double)q.y * kc.inv_cell - F.org[1],
                       (double)q.z * kc.inv_cell - F.org[2]};
  const double lim = (double)(1 << 30);
  const int r = kc.reach_cells;
  bool in = true;
  for (int a = 0; a < 3; ++a) {
    const int c = (int)fmin(fmax(floor(u[a]), -lim), lim) + r;
    in = in && c >= 0 && c <= F.dim[a] + 2 * r - 1;
  }
  return in;
}

// Zero moments for an entry whose source has no candidate (the finaliser sums every entry).
template <int MODE>
__device__ inline void store_zero_moments(const PairArgs& a, int64_t entry) {
  a.mom[entry] = 0.f;
  if constexpr (MODE == MODE_NORMAL)
    for (int k = 1; k < 10; ++k) a.mom[k * a.n_entries + entry] = 0.f;
}

// Exact widening of the stored low-precision feature formats.
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// OCP e4m3 (bias 7; no infinities; the one NaN code is never stored).
__device__ inline float fp8_to_f32(uint8_t b) {
  const uint32_t e = (b >> 3) & 15u, m = b & 7u;
  const float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0.001953125f;  // m * 2^-9
  return (b & 0x80u) ? -v : v;
}

// Feature row `row` (DP elements of the feature path's type) widened to FP32.
template <int FEAT, int DP>
__device__ inline void load_feature_row(const void* __restrict__ base, int64_t row, float (&out)[DP]) {
  if constexpr (FEAT == FEAT_DENSE) {
    const float4* f4 = reinterpret_cast<const float4*>(static_cast<const float*>(base) + row * DP);
#pragma unroll
    for (int k = 0; k < DP / 4; ++k) {
      const float4 v = f4[k];
      out[4 * k] = v.x; out[4 * k + 1] = v.y; out[4 * k + 2] = v.z; out[4 * k + 3] = v.w;
    }
  } else if constexpr (FEAT == FEAT_BF16) {
    const uint4* u4 = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + row * DP);
#pragma unroll
    for (int k = 0; k < DP / 8; ++k) {
      const uint4 v = u4[k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        out[8 * k + 2 * i] = bf16_to_f32((uint16_t)(w[i] & 0xffffu));
        out[8 * k + 2 * i + 1] = bf16_to_f32((uint16_t)(w[i] >> 16));
      }
    }
  } else {
    const uint4* u4 = reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(base) + row * DP);
#pragma unroll
    for (int k = 0; k < DP / 16; ++k) {
      const uint4 v = u4[k];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int b = 0; b < 4; ++b) out[16 * k + 4 * i + b] = fp8_to_f32((uint8_t)(w[i] >> (8 * b)));
    }
  }
}

// <f_src, f_row> with FP32 fused multiply-adds in element order.
template <int FEAT, int DP>
__device__ inline float dot_feature_row(const void* __restrict__ base, int64_t row, const float (&fs)[DP]) {
  float z[DP];
  load_feature_row<FEAT, DP>(base, row, z);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < DP; ++k) acc = fmaf(fs[k], z[k], acc);
  return acc;
}

// The K best pairs of one source point: larger ranking key c exp(-s2 / 2 ell^2)
// (FP64), then smaller FP32 squared distance s2, then smaller original index j.
// Entries are kept best first; unused entries hold a sentinel (key -1) that
// every real pair (key > 0) beats.  All indexing is static (registers).
template <int K>
struct TopK {
  double key[K];
  float s2[K], w[K], dx[K], dy[K], dz[K];
  int32_t jo[K];
  __device__ void clear() {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      key[t] = -1.0;
      s2[t] = 3.0e38f;
      jo[t] = 0x7fffffff;
      w[t] = dx[t] = dy[t] = dz[t] = 0.f;
    }
  }
  __device__ static bool better(double k1, float a1, int32_t j1, double k2, float a2, int32_t j2) {
    return k1 > k2 || (k1 == k2 && (a1 < a2 || (a1 == a2 && j1 < j2)));
  }
  // Could (key, s2) enter a list of the first k entries?  (The index tie-break is decided in insert.)
  __device__ bool may_enter(int k, double kk, float ss) const {
    double lk = -1.0;
    float ls = 3.0e38f;
#pragma unroll
    for (int t = 0; t < K; ++t)
      if (t == k - 1) {
        lk = key[t];
        ls = s2[t];
      }
    return kk > lk || (kk == lk && ss <= ls);
  }
  __device__ void insert(int k, double kk, float ss, int32_t j, float ww, float ax, float ay, float az) {
    bool placed = false;
#pragma unroll
    for (int t = K - 1; t >= 0; --t) {
      if (t >= k || placed) continue;
      if (t == k - 1 && !better(kk, ss, j, key[t], s2[t], jo[t])) {  // not better than the last kept pair
        placed = true;
        continue;
      }
      if (t > 0 && better(kk, ss, j, key[t - 1], s2[t - 1], jo[t - 1])) {
        key[t] = key[t - 1]; s2[t] = s2[t - 1]; jo[t] = jo[t - 1];
        w[t] = w[t - 1]; dx[t] = dx[t - 1]; dy[t] = dy[t - 1]; dz[t] = dz[t - 1];
      } else {
        key[t] = kk; s2[t] = ss; jo[t] = j; w[t] = ww; dx[t] = ax; dy[t] = ay; dz[t] = az;
        placed = true;
      }
    }
  }
};

// The FP32 squared distance of the membership rule.
__device__ inline float rule_s2(float3 q, float zx, float zy, float zz, float& dx, float& dy, float& dz) {
#pragma clang fp contract(off)
  dx = q.x - zx;
  dy = q.y - zy;
  dz = q.z - zz;
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

__device__ inline int cell_of(float v, double inv_cell) { return (int)floor((double)v * inv_cell); }

// 10-bit-per-axis Morton interleave.
__device__ inline uint32_t spread10(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread10(x) | (spread10(y) << 1) | (spread10(z) << 2);
}

// Wavefront (64-lane) reductions; every lane receives the result.
__device__ inline float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Index of the segment containing `pos` in an ascending offset table
// off[0..n) (off[0] == 0): the largest s with off[s] <= pos.
template <typename T>
__device__ inline int upper_segment(const T* off, int n, int64_t pos) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= pos) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace rkhsba
