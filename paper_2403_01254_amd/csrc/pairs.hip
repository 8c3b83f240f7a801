// Per-iteration hot path: relative transforms, source-point binning, the
// candidate sweep that accumulates per-point moments, and the per-point
// finalisation into per-edge Gauss-Newton blocks.
//
// Sweep (one wavefront per pass of P source points of one edge):
//   * the P source points were binned by the Morton code of their cell in the
//     target frame, so a pass is spatially compact;
//   * the pass's bounding box (of the transformed points q = T_nm x) is
//     grown by the reach (>= r_c) and walked row by row over the target
//     frame's cell rows; each row trims its x-range to the part of the ball
//     around the box that it can touch and yields one contiguous range of
//     target points (the frame is stored in cell-key order);
//   * G = 64/P lanes share a source point and split each range by stride G;
//     each lane applies the FP32 membership rule to its candidates and, for
//     pairs inside, accumulates the moments of the target-frame residual
//     d = q - z with weight w = c exp(-|d|^2 / 2 ell^2)  (Eq. (eq:irls_weight)):
//         A = sum w,  B = sum w d,  C = sum w d d^T         (10 floats)
//   * the G partial moments are summed with cross-lane shuffles and stored
//     per source point.
// Finalisation turns each point's moments into its exact contribution to the
// edge's F, b and H blocks (world-frame residual u = T_m x - T_n z, right
// perturbations, Sec. V-A) in FP64, and reduces them per block of 256 points.
#include <cfloat>

#include "rkhsba_device.h"

namespace rkhsba {
namespace {

constexpr int kThreads = 256;

__device__ inline int clamp_floor(double v, int lo, int hi) {
  v = floor(v);
  v = fmin(fmax(v, (double)lo), (double)hi);
  return (int)v;
}

// Walks the target frame's cell rows that a ball of radius `reach` around the
// box [lo, hi] can touch and calls fn(j0, j1) with each contiguous range of
// target points (frame-local sorted indices).  Every target point whose
// distance to some point of the box is <= reach lies in one of the ranges.
// lrow: the first row of the label layer walked (label_rows; < 0: no rows).
template <typename Fn>
__device__ inline void for_each_range(const FrameInfo& T, const int4* __restrict__ rows,
                                      const uint32_t* __restrict__ xtab, const KConst& kc, float3 lo, float3 hi,
                                      int64_t lrow, Fn&& fn) {
  if (lrow < 0) return;
  const double inv = kc.inv_cell, cell = kc.cell, reach = kc.reach;
  const int z0 = clamp_floor(((double)lo.z - reach) * inv - T.org[2], -1, T.dim[2]);
  const int z1 = clamp_floor(((double)hi.z + reach) * inv - T.org[2], -1, T.dim[2]);
  const int y0 = clamp_floor(((double)lo.y - reach) * inv - T.org[1], -1, T.dim[1]);
  const int y1 = clamp_floor(((double)hi.y + reach) * inv - T.org[1], -1, T.dim[1]);
  for (int kz = max(z0, 0); kz <= min(z1, T.dim[2] - 1); ++kz) {
    const double cz = (double)(kz + T.org[2]) * cell;
    const double bz = fmax(0.0, fmax(cz - (double)hi.z, (double)lo.z - (cz + cell)));
    for (int ky = max(y0, 0); ky <= min(y1, T.dim[1] - 1); ++ky) {
      const double cy = (double)(ky + T.org[1]) * cell;
      const double by = fmax(0.0, fmax(cy - (double)hi.y, (double)lo.y - (cy + cell)));
      const double r2 = kc.reach2 - by * by - bz * bz;
      if (r2 < 0.0) continue;
      const double h = sqrt(r2);
      const int4 R = rows[T.row_off + lrow + (int64_t)kz * T.dim[1] + ky];
      if (R.y < R.x) continue;
      const int xa = max(clamp_floor(((double)lo.x - h) * inv - T.org[0], -1, T.dim[0]), R.x);
      const int xb = min(clamp_floor(((double)hi.x + h) * inv - T.org[0], -1, T.dim[0]), R.y);
      if (xa > xb) continue;
      const uint32_t* xt = xtab + T.xt_off + (uint32_t)R.z;
      fn(xt[xa - R.x], xt[xb + 1 - R.x]);
    }
  }
}

// ---------------------------------------------------------------- transforms and binning

__global__ void k_edge_setup(const double* __restrict__ poses, const EdgeInfo* __restrict__ edges, int E,
                             EdgeXf* __restrict__ xf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  EdgeXf o;
  rule_relative(poses + 12 * edges[e].m, poses + 12 * edges[e].n, o.R, o.t);
  xf[e] = o;
}

// One block per sort tile (kSortTile consecutive entries of one edge): the
// Morton code of each source point's target-frame cell, clamped to the grid
// and its margin of reach cells, with kInvalidBit set when the point lies
// beyond them (it has no pair).  SORTED: the entries already hold sorted
// source indices (an earlier binning of the same set); only keys are written.
template <bool SORTED>
__global__ __launch_bounds__(kSortThreads) void k_bin(const float4* __restrict__ pts,
                                                      const FrameInfo* __restrict__ frames,
                                                      const EdgeInfo* __restrict__ edges,
                                                      const SortTile* __restrict__ tiles,
                                                      const EdgeXf* __restrict__ xf, const KConst* __restrict__ kcs,
                                                      uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const SortTile t = tiles[blockIdx.x];
  const int e = t.edge;
  const EdgeInfo ed = edges[e];
  const KConst kc = kcs[ed.prob];
  const FrameInfo Fm = frames[ed.m];
  const FrameInfo Fn = frames[ed.n];
  const EdgeXf X = xf[e];
  const int r = kc.reach_cells;
  const int lim = 1 << 30;
  for (int k = threadIdx.x; k < t.count; k += kSortThreads) {
    const int64_t i = t.start + k;
    const uint32_t src = SORTED ? vals[i] : (uint32_t)(i - ed.ent_off);
    const float4 x = pts[Fm.pt_off + src];
    const float3 q = rule_q32(X, x.x, x.y, x.z);
    // cell coordinates (validity) and sub-cell coordinates (the key): scaling by 2^key_sub is exact, so a
    // sub-cell coordinate shifted right by key_sub is its cell coordinate
    const double u[3] = {(double)q.x * kc.inv_cell - Fn.org[0], (double)q.y * kc.inv_cell - Fn.org[1],
                         (double)q.z * kc.inv_cell - Fn.org[2]};
    const int sub = Fn.key_sub;
    const uint32_t invalid = source_in_grid(q, Fn, kc) ? 0u : kInvalidBit;
    uint32_t kk[3];
    for (int a = 0; a < 3; ++a) {
      const int top = Fn.dim[a] + 2 * r - 1;
      const int cf = clamp_floor(u[a] * (double)(1 << sub), -lim, lim) + (r << sub);
      kk[a] = (uint32_t)min(max(cf, 0), ((top + 1) << sub) - 1) >> Fn.mort_shift;
    }
    keys[i] = invalid | morton3(kk[0], kk[1], kk[2]);
    if constexpr (!SORTED) vals[i] = src;
  }
}

// ---------------------------------------------------------------- pass table

// One block per edge: the edge's passes, segment after segment, each
// segment's in entry order.
__global__ __launch_bounds__(256) void k_fill_passes(const EdgeInfo* __restrict__ edges,
                                                     const FrameInfo* __restrict__ frames,
                                                     const SortSeg* __restrict__ segs,
                                                     PassInfo* __restrict__ passes) {
  const int e = blockIdx.x;
  const EdgeInfo ed = edges[e];
  const int P = ed.pass_size == 1 ? 64 : ed.pass_size;  // per-point walks: one source per lane
  const int64_t src_off = frames[ed.m].pt_off;
  int64_t base = ed.pass0;
  for (int sg = 0; sg < ed.n_seg; ++sg) {  // uniform
    const SortSeg S = segs[ed.seg0 + sg];
    const int n_pass = (int)((S.count + P - 1) / P);
    for (int k = threadIdx.x; k < n_pass; k += blockDim.x) {
      PassInfo Q;
      Q.entry0 = S.start + (int64_t)k * P;
      Q.src_off = src_off;
      Q.e = e;
      Q.count = (int)min((int64_t)P, S.count - (int64_t)k * P);
      Q.tgt = ed.n;
      Q.prob = ed.prob;
      passes[base + k] = Q;
    }
    base += n_pass;
  }
}

// ---------------------------------------------------------------- candidate sweep

// Passes of 64/G source points.  SHARED: the pass's G candidate streams walk
// the cells around the box of all its transformed source points, and every
// source tests every candidate of the walk.  LOCAL (G = 1): each lane walks
// the cells around its own transformed point only (for sparse frames, where
// a shared box would be much larger than one point's neighbourhood).
// TOPK > 0 (with LOCAL): each source point keeps only its kc.topk (<= TOPK)
// pairs with the largest kernel values c exp(-|d|^2 / 2 ell^2) (ranked in
// FP64; ties: smaller squared distance, then smaller original index); the
// moments and the pair count come from those pairs only.
template <int MODE, int FEAT, int G, int DP, bool LOCAL, int TOPK>
__global__ __launch_bounds__(kThreads) void k_pairs(PairArgs a) {
  constexpr int P = 64 / G;
  const int lane = threadIdx.x & 63;
  const int pass = (int)blockIdx.x * (kThreads / 64) + (int)(threadIdx.x >> 6);
  if (pass >= a.n_pass) return;  // whole wavefront leaves; no block barrier below
  const PassInfo pi = a.passes[a.pass0 + pass];
  const EdgeXf X = a.xf[pi.e];
  const FrameInfo Fn = a.frames[pi.tgt];
  const KConst kc = a.kcs[pi.prob];
  const int s = lane % P, g = lane / P;
  const int64_t entry = pi.entry0 + s;
  const bool in_range = s < pi.count;
  bool valid = in_range;
  uint32_t src = 0;
  if (valid) {
    valid = !(a.keys[entry] & kInvalidBit);
    src = a.vals[entry];
  }
  float3 q = make_float3(0.f, 0.f, 0.f);
  uint32_t lbl = 0;
  float fs[DP > 0 ? DP : 1];
  if (valid) {
    const float4 x = a.pts[pi.src_off + src];
    q = rule_q32(X, x.x, x.y, x.z);
    lbl = __float_as_uint(x.w);
    if constexpr (FEAT != FEAT_CLASS) load_feature_row<FEAT, DP>(a.feat, pi.src_off + src, fs);
  }
  float3 lo = q, hi = q;
  if constexpr (!LOCAL) {
    lo.x = wave_min(valid ? q.x : FLT_MAX);
    lo.y = wave_min(valid ? q.y : FLT_MAX);
    lo.z = wave_min(valid ? q.z : FLT_MAX);
    hi.x = wave_max(valid ? q.x : -FLT_MAX);
    hi.y = wave_max(valid ? q.y : -FLT_MAX);
    hi.z = wave_max(valid ? q.z : -FLT_MAX);
    if (lo.x > hi.x) {  // no valid source point in the pass (uniform)
      if (g == 0 && in_range) {
        a.cnt[entry] = 0u;
        store_zero_moments<MODE>(a, entry);
      }
      return;
    }
  }

  const float rc2 = kc.rc2, alpha = kc.alpha;
  const bool clamp = a.kc.clamp != 0;
  float A = 0.f, Bx = 0.f, By = 0.f, Bz = 0.f;
  float Cxx = 0.f, Cxy = 0.f, Cxz = 0.f, Cyy = 0.f, Cyz = 0.f, Wr2 = 0.f;  // Wr2 = sum w |d|^2 (in place of C_zz)
  uint32_t cnt = 0;
  const float4* __restrict__ tp = a.pts + Fn.pt_off;

  if (LOCAL && !valid) {  // empty walk for this lane
    lo = make_float3(FLT_MAX, FLT_MAX, FLT_MAX);
    hi = make_float3(-FLT_MAX, -FLT_MAX, -FLT_MAX);
  }
  // the label layer walked in a label-stacked target frame: each lane's own (LOCAL), or the pass's (its
  // sources share one class id: passes never straddle a class id of a stacked source frame)
  uint32_t wl = lbl;
  if constexpr (!LOCAL) wl = (uint32_t)__shfl((int)lbl, __builtin_ctzll(__ballot(valid)), 64);
  const int64_t lrow = label_rows(Fn, wl);
  TopK<(TOPK > 0 ? TOPK : 1)> best;
  if constexpr (TOPK > 0) best.clear();
  const int topk = kc.topk;
  for_each_range(Fn, a.rows, a.xtab, kc, lo, hi, lrow, [&](uint32_t j0, uint32_t j1) {
    for (uint32_t j = j0 + g; j < j1; j += G) {
      const float4 z = tp[j];
      float dx, dy, dz;
      const float s2 = rule_s2(q, z.x, z.y, z.z, dx, dy, dz);
      bool in = valid && s2 <= rc2;
      if constexpr (FEAT == FEAT_CLASS) in = in && (__float_as_uint(z.w) == lbl);
      if (in) {
        float c = 1.0f;
        if constexpr (FEAT != FEAT_CLASS) {
          const float acc = dot_feature_row<FEAT, DP>(a.feat, Fn.pt_off + j, fs);
          c = clamp ? fmaxf(acc, 0.f) : acc;
        }
        const float w = c * __builtin_amdgcn_exp2f(-alpha * s2);
        if constexpr (TOPK > 0) {
          if (c > 0.f) {
            const double key = (double)c * exp(-(double)s2 * kc.inv2l2);
            if (best.may_enter(topk, key, s2)) best.insert(topk, key, s2, a.perm[Fn.pt_off + j], w, dx, dy, dz);
          }
          continue;
        }
        A += w;
        cnt += (c != 0.f) ? 1u : 0u;
        if constexpr (MODE == MODE_NORMAL) {
          const float wx = w * dx, wy = w * dy;
          Bx += wx; By += wy; Bz = fmaf(w, dz, Bz);
          Cxx = fmaf(wx, dx, Cxx); Cxy = fmaf(wx, dy, Cxy); Cxz = fmaf(wx, dz, Cxz);
          Cyy = fmaf(wy, dy, Cyy); Cyz = fmaf(wy, dz, Cyz); Wr2 = fmaf(w, s2, Wr2);
        }
      }
    }
  });

  if constexpr (TOPK > 0) {  // moments of the kept pairs
#pragma unroll
    for (int t = 0; t < TOPK; ++t) {
      if (!(best.key[t] > 0.0)) continue;
      const float w = best.w[t], dx = best.dx[t], dy = best.dy[t], dz = best.dz[t];
      A += w;
      cnt += 1u;
      if constexpr (MODE == MODE_NORMAL) {
        const float wx = w * dx, wy = w * dy;
        Bx += wx; By += wy; Bz = fmaf(w, dz, Bz);
        Cxx = fmaf(wx, dx, Cxx); Cxy = fmaf(wx, dy, Cxy); Cxz = fmaf(wx, dz, Cxz);
        Cyy = fmaf(wy, dy, Cyy); Cyz = fmaf(wy, dz, Cyz); Wr2 = fmaf(w, best.s2[t], Wr2);
      }
    }
  }
  // Sum the G lanes that share a source point (lanes s, s+P, s+2P, ...).
#pragma unroll
  for (int o = P; o < 64; o <<= 1) {
    A += __shfl_xor(A, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
    if constexpr (MODE == MODE_NORMAL) {
      Bx += __shfl_xor(Bx, o, 64); By += __shfl_xor(By, o, 64); Bz += __shfl_xor(Bz, o, 64);
      Cxx += __shfl_xor(Cxx, o, 64); Cxy += __shfl_xor(Cxy, o, 64); Cxz += __shfl_xor(Cxz, o, 64);
      Cyy += __shfl_xor(Cyy, o, 64); Cyz += __shfl_xor(Cyz, o, 64); Wr2 += __shfl_xor(Wr2, o, 64);
    }
  }
  if (g == 0 && in_range) a.cnt[entry] = valid ? cnt : 0u;
  if (g == 0 && in_range) {  // zero moments for a source outside the target grid (the finaliser sums every entry)
    const int64_t N = a.n_entries;
    auto v = [&](float m) { return valid ? m : 0.f; };
    a.mom[entry] = v(A);
    if constexpr (MODE == MODE_NORMAL) {
      a.mom[1 * N + entry] = v(Bx); a.mom[2 * N + entry] = v(By); a.mom[3 * N + entry] = v(Bz);
      a.mom[4 * N + entry] = v(Cxx); a.mom[5 * N + entry] = v(Cxy); a.mom[6 * N + entry] = v(Cxz);
      a.mom[7 * N + entry] = v(Cyy); a.mom[8 * N + entry] = v(Cyz); a.mom[9 * N + entry] = v(Wr2);
    }
  }
}

// ---------------------------------------------------------------- per-point finalisation
//
// The normal-equation blocks of an edge are linear in a few per-point
// products of the moments (A, B, C), the source point x (frame m) and
// q = T_nm x (frame n).  With R_mn = R_nm^T, Bm = R_mn B, S = A q - B and
// Szz = A q q^T - q B^T - B q^T + C (S and Szz are the weighted sums of the
// target points z and z z^T in frame n), the per-point terms are (world
// residual u = T_m x - T_n z, right perturbations):
//   F = A,  b_m = [Bm; x cross Bm],  b_n = -[B; q cross B]
//   H_mm = [[A I, -[A x]], [[A x], tr(A x x^T) I - A x x^T]]
//   H_nn = [[A I, -[S]], [[S], tr(Szz) I - Szz]]
//   H_mn = -[I; [x]] R_mn [A I, -[S]]
//        = [[-A R_mn, R_mn [S]], [-[A x] R_mn, [x] R_mn [S]]]
// so it suffices to sum, per edge, the 37 products
//   A, B, x cross Bm, q cross B, A x, A x x^T (6), A q, Szz (6), x S^T (9)
// (plus tr C = sum w |d|^2, the lengthscale derivative's term, F and the
// pair count) and to expand the sums into the 91 values once per edge.
//
// The sweeps form d = q32 - z from q rounded to FP32 (the membership rule's
// value).  Far from a frame's origin that rounding, up to half an FP32 ulp of
// |q|, is no longer small next to d, and it is the same for every pair of one
// source point.  The per-point terms therefore use q in FP64 and moments
// moved to d + dl (dl = q64 - q32) to first order in dl, which needs only the
// moments at hand; F itself is left as the plain sum of the kernel values, so
// that it is the same number the loss-only evaluation gives.
//
// Sums run in FP64: per thread over its entries, then per block in a
// fixed order, then per edge over the blocks in order; the split into
// blocks depends only on the edge's source count, so an edge's sums do not
// depend on what else is evaluated with it.
constexpr int kStA = 0, kStB = 1, kStXBm = 4, kStQB = 7, kStAx = 10, kStAxx = 13, kStAq = 19, kStSzz = 22,
              kStXS = 28, kStWr2 = 37, kStF = 38, kStCnt = 39;

// Running sums: FP64, or FP32 with Kahan compensation (option).
template <typename T>
struct Acc;
template <>
struct Acc<double> {
  double s = 0.0;
  __device__ void add(double v) { s += v; }
  __device__ double value() const { return s; }
};
template <>
struct Acc<float> {
  float s = 0.f, c = 0.f;
  __device__ void add(float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ float value() const { return s; }
};

template <int MODE, typename T>
__global__ __launch_bounds__(kFinThreads) void k_finalize(FinArgs a, const int32_t* __restrict__ fin_off) {
  constexpr int NS = MODE == MODE_LOSS ? 2 : kFinStats;
  __shared__ T sh[(kFinThreads / 64) * kFinStats];
  const int blk = blockIdx.x;
  const int e = upper_segment(fin_off, a.E, blk);
  const EdgeInfo ed = a.edges[e];
  const EdgeXf X = a.xf[e];
  const KConst& kc = a.kcs[ed.prob];
  const float4* __restrict__ src_pts = a.pts + a.frames[ed.m].pt_off;
  const int64_t end = ed.ent_off + ed.n_src;
  const int64_t base = ed.ent_off + (int64_t)(blk - ed.fin_off) * kFinThreads * ed.fin_pt;
  const int64_t N = a.n_entries;
  Acc<T> st[NS];
  double cnt_sum = 0.0;  // pair counts: integers, exact in FP64
  // The next entry's count, key, source index and moments are read while the current one is processed
  // (three waves per SIMD at this register count hide little of the reads' latency otherwise).
  constexpr int NM = MODE == MODE_LOSS ? 1 : 10;
  struct In {
    uint32_t cnt, val;
    float m[NM];
  };
  auto load = [&](int64_t entry, In& in) __attribute__((always_inline)) {
    in.cnt = a.cnt[entry];
    if constexpr (MODE != MODE_LOSS) in.val = a.vals[entry];
#pragma unroll
    for (int k = 0; k < NM; ++k) in.m[k] = a.mom[k * N + entry];
  };
  In cur, nxt;
  int64_t entry = base + threadIdx.x;
  bool have = entry < end;
  if (have) load(entry, cur);
  for (int j = 0; j < ed.fin_pt && have; ++j) {
    const int64_t nentry = entry + kFinThreads;
    const bool nhave = j + 1 < ed.fin_pt && nentry < end;
    if (nhave) load(nentry, nxt);
    const In in = cur;
    cur = nxt;
    entry = nentry;
    have = nhave;
    cnt_sum += (double)in.cnt;  // per-entry or per-pass pair counts
    // a source outside the target grid has zero moments (the sweeps store them), so every entry is summed
    if constexpr (MODE == MODE_LOSS) {
      st[0].add((T)in.m[0]);
    } else {
      const T A = in.m[0];
      T B[3], C[6], x[3], q[3];
      for (int k = 0; k < 3; ++k) B[k] = in.m[1 + k];
      for (int k = 0; k < 5; ++k) C[k] = in.m[4 + k];
      T Wr2 = in.m[9];  // the sweeps store sum w |d|^2 in place of C_zz
      C[5] = Wr2 - C[0] - C[3];
      const float4 p = src_pts[in.val];
      const double3 q64 = rule_q64(X, p.x, p.y, p.z);
      x[0] = p.x; x[1] = p.y; x[2] = p.z;
      q[0] = (T)q64.x; q[1] = (T)q64.y; q[2] = (T)q64.z;
      // The sweeps formed d = q32 - z from the rounded q32; every pair of this
      // point has d64 = d + dl.  First-order update of the moments in dl:
      // w64 = w (1 - d.g), g = dl / ell^2 (third moments dropped).
      const T dl[3] = {(T)(q64.x - (double)(float)q64.x), (T)(q64.y - (double)(float)q64.y),
                       (T)(q64.z - (double)(float)q64.z)};
      const T two_a = (T)(2.0 * kc.inv2l2);
      const T g[3] = {dl[0] * two_a, dl[1] * two_a, dl[2] * two_a};
      const T Bg = B[0] * g[0] + B[1] * g[1] + B[2] * g[2];
      const T Bdl = B[0] * dl[0] + B[1] * dl[1] + B[2] * dl[2];
      const T Cg[3] = {C[0] * g[0] + C[1] * g[1] + C[2] * g[2], C[1] * g[0] + C[3] * g[1] + C[4] * g[2],
                       C[2] * g[0] + C[4] * g[1] + C[5] * g[2]};
      {
        const int ri[6] = {0, 0, 0, 1, 1, 2}, ci[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int k = 0; k < 6; ++k) C[k] += B[ri[k]] * dl[ci[k]] + dl[ri[k]] * B[ci[k]];
      }
      for (int k = 0; k < 3; ++k) B[k] += A * dl[k] - Cg[k] - Bg * dl[k];
      Wr2 += (T)2 * Bdl;
      const T A1 = A - Bg;
      T R[9];
      for (int k = 0; k < 9; ++k) R[k] = (T)X.R[k];
      T Bm[3];
      for (int r = 0; r < 3; ++r) Bm[r] = R[r] * B[0] + R[3 + r] * B[1] + R[6 + r] * B[2];
      st[kStF].add(A);  // F as the loss-only evaluation forms it
      st[kStA].add(A1);
      for (int k = 0; k < 3; ++k) st[kStB + k].add(B[k]);
      st[kStXBm + 0].add(x[1] * Bm[2] - x[2] * Bm[1]);
      st[kStXBm + 1].add(x[2] * Bm[0] - x[0] * Bm[2]);
      st[kStXBm + 2].add(x[0] * Bm[1] - x[1] * Bm[0]);
      st[kStQB + 0].add(q[1] * B[2] - q[2] * B[1]);
      st[kStQB + 1].add(q[2] * B[0] - q[0] * B[2]);
      st[kStQB + 2].add(q[0] * B[1] - q[1] * B[0]);
      T Ax[3], S[3];
      for (int k = 0; k < 3; ++k) {
        Ax[k] = A1 * x[k];
        st[kStAx + k].add(Ax[k]);
        st[kStAq + k].add(A1 * q[k]);
        S[k] = A1 * q[k] - B[k];
      }
      st[kStAxx + 0].add(Ax[0] * x[0]); st[kStAxx + 1].add(Ax[0] * x[1]); st[kStAxx + 2].add(Ax[0] * x[2]);
      st[kStAxx + 3].add(Ax[1] * x[1]); st[kStAxx + 4].add(Ax[1] * x[2]); st[kStAxx + 5].add(Ax[2] * x[2]);
      // Szz (upper triangle xx, xy, xz, yy, yz, zz), C in the same order
      const int ri[6] = {0, 0, 0, 1, 1, 2}, ci[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int r = ri[k], c = ci[k];
        st[kStSzz + k].add(A1 * q[r] * q[c] - q[r] * B[c] - B[r] * q[c] + C[k]);
      }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) st[kStXS + 3 * r + c].add(x[r] * S[c]);
      st[kStWr2].add(Wr2);
    }
  }
  // block sum in a fixed order: wavefront shuffles, then the four waves
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int KC = MODE == MODE_LOSS ? 1 : kStCnt;  // slot of the pair count (summed in FP64 below)
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const T t = wave_sum(st[k].value());
    if (lane == 0) sh[w * NS + k] = t;
  }
  __shared__ double shc[kFinThreads / 64];
  const double wc = wave_sum(cnt_sum);  // all lanes take part in the shuffles
  if (lane == 0) shc[w] = wc;
  __syncthreads();
  if (threadIdx.x < NS) {
    Acc<T> t;
    for (int ww = 0; ww < kFinThreads / 64; ++ww) t.add(sh[ww * NS + threadIdx.x]);
    double v = (double)t.value();
    if ((int)threadIdx.x == KC) {
      v = 0.0;
      for (int ww = 0; ww < kFinThreads / 64; ++ww) v += shc[ww];
    }
    a.partial[(int64_t)blk * kFinStats + threadIdx.x] = v;
  }
}

__device__ inline int sym_index(int r, int c) {  // upper triangle of a 6x6, row-major, r <= c
  if (r > c) { const int t = r; r = c; c = t; }
  return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

// One block per edge: deterministic sum of the edge's finalisation blocks,
// then the expansion of the 37 sums into F, b_m, b_n, H_mm, H_nn, H_mn.
template <typename TT>
__global__ __launch_bounds__(64) void k_edge_reduce(const double* __restrict__ partial,
                                                    const EdgeInfo* __restrict__ edges,
                                                    const EdgeXf* __restrict__ xf, int mode,
                                                    double* __restrict__ edge_out) {
  __shared__ TT T[kFinStats];
  __shared__ double n_pairs;
  const EdgeInfo ed = edges[blockIdx.x];
  const int ns = mode == MODE_LOSS ? 2 : kFinStats;
  const int kc = ns - 1;  // pair-count slot
  for (int t = threadIdx.x; t < kFinStats; t += blockDim.x) {
    if (t == kc) {
      double c = 0.0;
      for (int b = 0; b < ed.n_fin; ++b) c += partial[(int64_t)(ed.fin_off + b) * kFinStats + t];
      n_pairs = c;
      T[t] = (TT)0;
      continue;
    }
    Acc<TT> s;
    if (t < ns)
      for (int b = 0; b < ed.n_fin; ++b) s.add((TT)partial[(int64_t)(ed.fin_off + b) * kFinStats + t]);
    T[t] = s.value();
  }
  __syncthreads();
  double* out = edge_out + (int64_t)blockIdx.x * kEdgeVals;
  if (mode == MODE_LOSS) {
    for (int k = threadIdx.x; k < kEdgeVals; k += blockDim.x)
      out[k] = k == 0 ? (double)T[0] : k == 91 ? n_pairs : 0.0;  // (sum w r^2 needs the moments)
    return;
  }
  if (threadIdx.x != 0) return;
  const EdgeXf X = xf[blockIdx.x];
  TT Rmn[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Rmn[r][c] = X.R[3 * c + r];
  const TT A = T[kStA];
  const TT* B = T + kStB;
  TT v[kEdgeVals];
  for (int k = 0; k < kEdgeVals; ++k) v[k] = 0.0;
  v[0] = T[kStF];
  for (int r = 0; r < 3; ++r) {
    v[1 + r] = Rmn[r][0] * B[0] + Rmn[r][1] * B[1] + Rmn[r][2] * B[2];
    v[4 + r] = T[kStXBm + r];
    v[7 + r] = -B[r];
    v[10 + r] = -T[kStQB + r];
  }
  auto skew = [](const TT* a, TT (&M)[3][3]) {
    M[0][0] = 0.0;   M[0][1] = -a[2]; M[0][2] = a[1];
    M[1][0] = a[2];  M[1][1] = 0.0;   M[1][2] = -a[0];
    M[2][0] = -a[1]; M[2][1] = a[0];  M[2][2] = 0.0;
  };
  const int ri[6] = {0, 0, 0, 1, 1, 2}, ci[6] = {0, 1, 2, 1, 2, 2};
  TT Axx[3][3], Szz[3][3];
  for (int k = 0; k < 6; ++k) {
    Axx[ri[k]][ci[k]] = Axx[ci[k]][ri[k]] = T[kStAxx + k];
    Szz[ri[k]][ci[k]] = Szz[ci[k]][ri[k]] = T[kStSzz + k];
  }
  TT S[3];
  for (int k = 0; k < 3; ++k) S[k] = T[kStAq + k] - B[k];
  TT Hmm[6][6], Hnn[6][6], Hmn[6][6];
  TT Kx[3][3], Ks[3][3];
  skew(T + kStAx, Kx);
  skew(S, Ks);
  const TT trx = Axx[0][0] + Axx[1][1] + Axx[2][2];
  const TT trs = Szz[0][0] + Szz[1][1] + Szz[2][2];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const TT I = r == c ? 1.0 : 0.0;
      Hmm[r][c] = A * I;
      Hmm[r][3 + c] = -Kx[r][c];
      Hmm[3 + r][c] = Kx[r][c];
      Hmm[3 + r][3 + c] = trx * I - Axx[r][c];
      Hnn[r][c] = A * I;
      Hnn[r][3 + c] = -Ks[r][c];
      Hnn[3 + r][c] = Ks[r][c];
      Hnn[3 + r][3 + c] = trs * I - Szz[r][c];
    }
  // H_mn: [[-A R_mn, R_mn [S]], [-[A x] R_mn, sum [x] R_mn [S]]]
  TT RKs[3][3], KxR[3][3], XRS[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      RKs[r][c] = Rmn[r][0] * Ks[0][c] + Rmn[r][1] * Ks[1][c] + Rmn[r][2] * Ks[2][c];
      KxR[r][c] = Kx[r][0] * Rmn[0][c] + Kx[r][1] * Rmn[1][c] + Kx[r][2] * Rmn[2][c];
      XRS[r][c] = 0.0;
    }
  // sum_p [x_p] R_mn [S_p] = sum_{i,j} (sum_p x_i S_j) [e_i] R_mn [e_j]
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const TT mij = T[kStXS + 3 * i + j];
      TT ei[3] = {0, 0, 0}, ej[3] = {0, 0, 0};
      ei[i] = 1.0;
      ej[j] = 1.0;
      TT Ki[3][3], Kj[3][3];
      skew(ei, Ki);
      skew(ej, Kj);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          TT t = 0.0;
          for (int a0 = 0; a0 < 3; ++a0)
            for (int b0 = 0; b0 < 3; ++b0) t += Ki[r][a0] * Rmn[a0][b0] * Kj[b0][c];
          XRS[r][c] += mij * t;
        }
    }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      Hmn[r][c] = -A * Rmn[r][c];
      Hmn[r][3 + c] = RKs[r][c];
      Hmn[3 + r][c] = -KxR[r][c];
      Hmn[3 + r][3 + c] = XRS[r][c];
    }
  for (int r = 0; r < 6; ++r)
    for (int c = r; c < 6; ++c) {
      v[13 + sym_index(r, c)] = Hmm[r][c];
      v[34 + sym_index(r, c)] = Hnn[r][c];
    }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) v[55 + 6 * r + c] = Hmn[r][c];
  v[91] = (TT)0;
  v[92] = T[kStWr2];
  for (int k = 0; k < kEdgeVals; ++k) out[k] = (double)v[k];
  out[91] = n_pairs;
}

// ---------------------------------------------------------------- pair export (parity)

template <int FEAT, int DP, bool TOPK>
__global__ __launch_bounds__(kThreads) void k_export_pairs(const float4* __restrict__ pts, const int4* __restrict__ rows,
                                                           const uint32_t* __restrict__ xtab,
                                                           const FrameInfo* __restrict__ frames,
                                                           const int32_t* __restrict__ perm,
                                                           const void* __restrict__ feat,
                                                           const EdgeXf* __restrict__ xf, int m, int n, KConst kc,
                                                           int64_t cap, int32_t* __restrict__ out,
                                                           unsigned long long* __restrict__ count) {
  const FrameInfo Fm = frames[m];
  const FrameInfo Fn = frames[n];
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= Fm.n) return;
  const float4 x = pts[Fm.pt_off + i];
  const float3 q = rule_q32(xf[0], x.x, x.y, x.z);
  const uint32_t lbl = __float_as_uint(x.w);
  const int32_t oi = perm[Fm.pt_off + i];
  float fs[DP > 0 ? DP : 1];
  if constexpr (TOPK && FEAT != FEAT_CLASS) load_feature_row<FEAT, DP>(feat, Fm.pt_off + i, fs);
  TopK<kMaxTopK> best;
  if constexpr (TOPK) best.clear();
  for_each_range(Fn, rows, xtab, kc, q, q, label_rows(Fn, lbl), [&](uint32_t j0, uint32_t j1) {
    for (uint32_t j = j0; j < j1; ++j) {
      const float4 z = pts[Fn.pt_off + j];
      float dx, dy, dz;
      const float s2 = rule_s2(q, z.x, z.y, z.z, dx, dy, dz);
      bool in = s2 <= kc.rc2;
      if constexpr (FEAT == FEAT_CLASS) in = in && __float_as_uint(z.w) == lbl;
      if (!in) continue;
      if constexpr (TOPK) {
        float c = 1.0f;
        if constexpr (FEAT != FEAT_CLASS) {
          const float acc = dot_feature_row<FEAT, DP>(feat, Fn.pt_off + j, fs);
          c = kc.clamp ? fmaxf(acc, 0.f) : acc;
        }
        if (c > 0.f) {
          const double key = (double)c * exp(-(double)s2 * kc.inv2l2);
          if (best.may_enter(kc.topk, key, s2)) best.insert(kc.topk, key, s2, perm[Fn.pt_off + j], 0.f, dx, dy, dz);
        }
      } else {
        const unsigned long long k = atomicAdd(count, 1ull);
        if ((int64_t)k < cap) {
          out[2 * k] = oi;
          out[2 * k + 1] = perm[Fn.pt_off + j];
        }
      }
    }
  });
  if constexpr (TOPK) {
#pragma unroll
    for (int t = 0; t < kMaxTopK; ++t) {
      if (!(best.key[t] > 0.0)) continue;
      const unsigned long long k = atomicAdd(count, 1ull);
      if ((int64_t)k < cap) {
        out[2 * k] = oi;
        out[2 * k + 1] = best.jo[t];
      }
    }
  }
}

template <int MODE, int FEAT>
hipError_t dispatch_pairs(const PairArgs& a, int G, bool local, bool topk, int DP, hipStream_t st) {
  const unsigned nb = (unsigned)((a.n_pass + 3) / 4);
  if (nb == 0) return hipSuccess;
#define RKHSBA_LAUNCH(GG, DD, LL, TK) k_pairs<MODE, FEAT, GG, DD, LL, TK><<<nb, kThreads, 0, st>>>(a)
#define RKHSBA_ANY(DD)                                                           \
  if (topk) {                                                                    \
    if constexpr (FEAT == FEAT_CLASS || FEAT == FEAT_DENSE) RKHSBA_LAUNCH(1, DD, true, kMaxTopK); \
  } else if (local) RKHSBA_LAUNCH(1, DD, true, 0);                               \
  else if (G == 1) RKHSBA_LAUNCH(1, DD, false, 0);                               \
  else if (G == 2) RKHSBA_LAUNCH(2, DD, false, 0);                               \
  else RKHSBA_LAUNCH(4, DD, false, 0);
  if constexpr (FEAT == FEAT_CLASS) {
    RKHSBA_ANY(0)
  } else if constexpr (feat_low_precision(FEAT)) {
    if (DP <= 32) { RKHSBA_ANY(32) }
    else { RKHSBA_ANY(64) }
  } else {
    if (DP <= 8) { RKHSBA_ANY(8) }
    else if (DP <= 16) { RKHSBA_ANY(16) }
    else if (DP <= 24) { RKHSBA_ANY(24) }
    else if (DP <= 32) { RKHSBA_ANY(32) }
    else { RKHSBA_ANY(64) }
  }
#undef RKHSBA_ANY
#undef RKHSBA_LAUNCH
  return hipGetLastError();
}

}  // namespace

int dense_pad(int D, int feat_path) {
  if (feat_low_precision(feat_path)) return D <= 32 ? 32 : 64;
  return D <= 8 ? 8 : D <= 16 ? 16 : D <= 24 ? 24 : D <= 32 ? 32 : 64;
}

hipError_t launch_fill_passes(const EdgeInfo* d_edges, int E, const FrameInfo* d_frames, const SortSeg* d_segs,
                              PassInfo* d_passes, hipStream_t st) {
  if (E > 0) k_fill_passes<<<E, 256, 0, st>>>(d_edges, d_frames, d_segs, d_passes);
  return hipGetLastError();
}

hipError_t launch_edge_setup(const double* d_poses, const EdgeInfo* d_edges, int E, EdgeXf* d_xf, hipStream_t st) {
  if (E > 0) k_edge_setup<<<(E + 63) / 64, 64, 0, st>>>(d_poses, d_edges, E, d_xf);
  return hipGetLastError();
}

hipError_t launch_bin(const float4* d_pts, const FrameInfo* d_frames, const EdgeInfo* d_edges,
                      const SortTile* d_tiles, int n_tiles, const EdgeXf* d_xf, const KConst* d_kcs, uint32_t* d_keys,
                      uint32_t* d_vals, bool rebin_sorted, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (rebin_sorted)
    k_bin<true><<<(unsigned)n_tiles, kSortThreads, 0, st>>>(d_pts, d_frames, d_edges, d_tiles, d_xf, d_kcs, d_keys,
                                                            d_vals);
  else
    k_bin<false><<<(unsigned)n_tiles, kSortThreads, 0, st>>>(d_pts, d_frames, d_edges, d_tiles, d_xf, d_kcs, d_keys,
                                                             d_vals);
  return hipGetLastError();
}

hipError_t launch_pairs(const PairArgs& a, int mode, int feat_path, int pass_points, bool topk, hipStream_t st) {
  const bool local = pass_points == 1;
  const int G = local ? 1 : 64 / pass_points;
  const int DP = a.kc.Dp;
#define RKHSBA_FEATS(MM)                                                                 \
  switch (feat_path) {                                                                   \
    case FEAT_CLASS: return dispatch_pairs<MM, FEAT_CLASS>(a, G, local, topk, DP, st);   \
    case FEAT_DENSE: return dispatch_pairs<MM, FEAT_DENSE>(a, G, local, topk, DP, st);   \
    case FEAT_BF16: return dispatch_pairs<MM, FEAT_BF16>(a, G, local, false, DP, st);    \
    default: return dispatch_pairs<MM, FEAT_FP8>(a, G, local, false, DP, st);            \
  }
  if (mode == MODE_LOSS) { RKHSBA_FEATS(MODE_LOSS) }
  RKHSBA_FEATS(MODE_NORMAL)
#undef RKHSBA_FEATS
}

hipError_t launch_finalize(const FinArgs& a, const int32_t* d_fin_off, int mode, bool fp32_sums, hipStream_t st) {
  if (a.n_fin_total <= 0) return hipSuccess;
  const unsigned nb = (unsigned)a.n_fin_total;
  if (fp32_sums) {
    if (mode == MODE_LOSS) k_finalize<MODE_LOSS, float><<<nb, kFinThreads, 0, st>>>(a, d_fin_off);
    else k_finalize<MODE_NORMAL, float><<<nb, kFinThreads, 0, st>>>(a, d_fin_off);
  } else {
    if (mode == MODE_LOSS) k_finalize<MODE_LOSS, double><<<nb, kFinThreads, 0, st>>>(a, d_fin_off);
    else k_finalize<MODE_NORMAL, double><<<nb, kFinThreads, 0, st>>>(a, d_fin_off);
  }
  return hipGetLastError();
}

hipError_t launch_edge_reduce(const double* d_partial, const EdgeInfo* d_edges, const EdgeXf* d_xf, int E, int mode,
                              bool fp32_sums, double* d_edge_out, hipStream_t st) {
  if (E <= 0) return hipSuccess;
  if (fp32_sums) k_edge_reduce<float><<<E, 64, 0, st>>>(d_partial, d_edges, d_xf, mode, d_edge_out);
  else k_edge_reduce<double><<<E, 64, 0, st>>>(d_partial, d_edges, d_xf, mode, d_edge_out);
  return hipGetLastError();
}

// Sum over edges, in edge order, of each edge's F and pair count (one thread: the same order as a host
// loop over the per-edge values).
__global__ void k_edge_totals(const double* __restrict__ edge_out, int E, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double F = 0.0, np = 0.0;
  for (int e = 0; e < E; ++e) {
    F += edge_out[(int64_t)e * kEdgeVals];
    np += edge_out[(int64_t)e * kEdgeVals + 91];
  }
  out[0] = F;
  out[1] = np;
}

hipError_t launch_edge_totals(const double* d_edge_out, int E, double* d_out, hipStream_t st) {
  k_edge_totals<<<1, 64, 0, st>>>(d_edge_out, E, d_out);
  return hipGetLastError();
}

hipError_t launch_export_pairs(const float4* d_pts, const int4* d_rows, const uint32_t* d_xtab,
                               const FrameInfo* d_frames, int n_src, const int32_t* d_perm, const void* d_feat,
                               const EdgeXf* d_xf, int m, int n, int feat_path, KConst kc, int64_t cap, int32_t* d_out,
                               unsigned long long* d_count, hipStream_t st) {
  if (n_src <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n_src + kThreads - 1) / kThreads);
#define RKHSBA_EXPORT(FF, DD, TK)                                                                               \
  k_export_pairs<FF, DD, TK><<<nb, kThreads, 0, st>>>(d_pts, d_rows, d_xtab, d_frames, d_perm, d_feat, d_xf, m, n, kc, \
                                                      cap, d_out, d_count)
  if (kc.topk > 0) {
    if (feat_path == FEAT_CLASS) RKHSBA_EXPORT(FEAT_CLASS, 0, true);
    else if (kc.Dp <= 8) RKHSBA_EXPORT(FEAT_DENSE, 8, true);
    else if (kc.Dp <= 16) RKHSBA_EXPORT(FEAT_DENSE, 16, true);
    else if (kc.Dp <= 24) RKHSBA_EXPORT(FEAT_DENSE, 24, true);
    else if (kc.Dp <= 32) RKHSBA_EXPORT(FEAT_DENSE, 32, true);
    else RKHSBA_EXPORT(FEAT_DENSE, 64, true);
  } else {
    if (feat_path == FEAT_CLASS) RKHSBA_EXPORT(FEAT_CLASS, 0, false);
    else RKHSBA_EXPORT(FEAT_DENSE, 0, false);
  }
#undef RKHSBA_EXPORT
  return hipGetLastError();
}

}  // namespace rkhsba
