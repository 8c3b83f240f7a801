// Tiled candidate sweep (16 source points per wavefront, 64-candidate tiles).
//
// One wavefront (= one workgroup of 64 lanes) handles a pass of P = 16
// Morton-adjacent source points of one edge.  Lane l works for source point
// s = l % 16 and candidate stream g = l / 16.
//   1. The pass's box of transformed points q = T_nm x is grown by the reach
//      (>= r_c).  The target cell rows the ball around the box can touch are
//      evaluated 64 at a time, one row per lane (x-range trimmed to the ball,
//      contiguous target-point range from the row table), and concatenated by
//      a wavefront prefix sum into one virtual candidate list.
//   2. The list is consumed in tiles of 64 candidates: each lane fetches one
//      candidate (position, label and, for dense features, its feature row)
//      into LDS; the fetch of the next tile is issued before the current one
//      is processed.
//   3. Each 16-candidate sub-tile is processed by all lanes: lane (s, g)
//      takes candidates 4g..4g+3, so 64 (source, candidate) pairs per step.
//      Dense feature inner products c = <f_x, f_z> come from one
//      16x16x4 FP32 MFMA per 4 feature dimensions; its accumulator layout
//      (row 4(l/16)+r, column l%16) is exactly candidate 4g+r for source s.
//   4. Inside the FP32 membership rule the pair adds w = c exp(-|d|^2/2l^2)
//      to the moments A, B = sum w d, C = sum w d d^T (d = q - z) and
//      W = sum w |d|^2; C_zz is not summed (the finaliser takes it from the
//      trace, C_zz = W - C_xx - C_yy), which saves w d_z.  The four streams of
//      each source are summed with cross-lane shuffles at the end.
//   5. Spread passes (class ids): a pass whose box is wider than a few r_c
//      (isolated outliers, jumps of the Morton order) skips steps 1-3: each
//      source walks the rows of its own ball, its lanes splitting the rows.
#include <cfloat>

#include "rkhsba_device.h"

namespace rkhsba {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kLanes = 64;
constexpr int kTile = 64;

__device__ inline int clamp_floor_d(double v, int lo, int hi) {
  v = floor(v);
  v = fmin(fmax(v, (double)lo), (double)hi);
  return (int)v;
}

__device__ inline float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Cross-lane moves within rows of 16 lanes (DPP: no LDS round trip).
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
constexpr int kDppXor1 = 0xb1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4e;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within each half row
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within each row
constexpr int kDppRor8 = 0x128;        // lane i <- lane (i + 8) mod 16 within each row, i.e. i ^ 8

// Minimum / maximum over the P consecutive lanes of each lane group (P = 8, 16 or 32): the quad, then the
// other quad of the half row, then the other half row, then the other row of the 32.
template <int P>
__device__ inline float group_min(float v) {
  static_assert(P == 8 || P == 16 || P == 32, "groups of 8, 16 or 32 lanes");
  v = fminf(v, dpp_f<kDppXor1>(v));
  v = fminf(v, dpp_f<kDppXor2>(v));
  v = fminf(v, dpp_f<kDppHalfMirror>(v));
  if constexpr (P >= 16) v = fminf(v, dpp_f<kDppMirror>(v));
  if constexpr (P == 32) v = fminf(v, __shfl_xor(v, 16, 64));
  return v;
}
template <int P>
__device__ inline float group_max(float v) {
  static_assert(P == 8 || P == 16 || P == 32, "groups of 8, 16 or 32 lanes");
  v = fmaxf(v, dpp_f<kDppXor1>(v));
  v = fmaxf(v, dpp_f<kDppXor2>(v));
  v = fmaxf(v, dpp_f<kDppHalfMirror>(v));
  if constexpr (P >= 16) v = fmaxf(v, dpp_f<kDppMirror>(v));
  if constexpr (P == 32) v = fmaxf(v, __shfl_xor(v, 16, 64));
  return v;
}

// v + (v of lane ^ O), the same sum in both lanes (addition is commutative): a DPP row rotation for O = 8,
// a cross-lane read through the LDS crossbar for 16 and 32.
template <int O, typename T>
__device__ inline T xor_add(T v) {
  static_assert(O == 8 || O == 16 || O == 32, "lane distance");
  if constexpr (O == 8) {
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    return v + __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppRor8, 0xf, 0xf, false));
  } else {
    return v + __shfl_xor(v, O, 64);
  }
}

// Inclusive add-scan of unsigned values over the wavefront's 64 lanes, in the same DPP steps as the max-scan
// below (row shifts, then the last lane of a row added to the rows after it).
__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  int m = (int)v;
  m += __builtin_amdgcn_update_dpp(0, m, 0x111, 0xf, 0xf, true);   // row_shr:1
  m += __builtin_amdgcn_update_dpp(0, m, 0x112, 0xf, 0xf, true);   // row_shr:2
  m += __builtin_amdgcn_update_dpp(0, m, 0x114, 0xf, 0xf, true);   // row_shr:4
  m += __builtin_amdgcn_update_dpp(0, m, 0x118, 0xf, 0xf, true);   // row_shr:8
  m += __builtin_amdgcn_update_dpp(0, m, 0x142, 0xa, 0xf, false);  // row_bcast:15
  m += __builtin_amdgcn_update_dpp(0, m, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)m;
}

// Inclusive max-scan of unsigned values over the wavefront's 64 lanes: four
// row shifts within each row of 16 lanes, then the last lane of a row
// broadcast to the rows after it.  Lanes a shift leaves without a source read
// the identity 0.
__device__ inline uint32_t wave_inclusive_max(uint32_t v) {
  const int x = (int)v;
  int m = x;
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x111, 0xf, 0xf, true));  // row_shr:1
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x112, 0xf, 0xf, true));  // row_shr:2
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x114, 0xf, 0xf, true));  // row_shr:4
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x118, 0xf, 0xf, true));  // row_shr:8
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x142, 0xa, 0xf, false));  // row_bcast:15
  m = (int)max((uint32_t)m, (uint32_t)__builtin_amdgcn_update_dpp(0, m, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (uint32_t)m;
}

// Feature inner products of one 16-candidate sub-tile with the pass's 16
// source points: D[cand 4(l/16)+r][source l%16] += F_cand[., 4k + l/16] *
// F_src[4k + l/16][.], accumulated over the DP/4 slices of 4 dimensions.
template <int DP, int FS>
__device__ inline floatx4 tile_products(const float* __restrict__ tfeat, int s, int g, int sub,
                                        const float (&fsrc)[DP / 4]) {
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const float* arow = tfeat + (16 * sub + s) * FS + g;
  // every A element read before the first product: one LDS round trip per sub-tile, not one per pair of slices
  float av[DP / 4];
#pragma unroll
  for (int k = 0; k < DP / 4; ++k) av[k] = arow[4 * k];
  __builtin_amdgcn_sched_barrier(0);  // (the scheduler would otherwise interleave reads and products again)
#pragma unroll
  for (int k = 0; k < DP / 4; ++k) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], fsrc[k], acc, 0, 0, 0);
  return acc;
}

// Orders LDS accesses between the lanes of the workgroup, which is one
// wavefront: its LDS operations are carried out in issue order, so only the
// compiler must not move them across this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same products for feature rows stored in bfloat16 or fp8 e4m3: one
// 16x16x32 MFMA (FP32 accumulation) per 32 feature dimensions.  Lane (s, g)
// supplies elements 8g..8g+7 of the slice, of candidate 16 sub + s (A, from
// the LDS tile, RB bytes per row) and of its own source point (B, registers).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));

template <int FEAT, int DP, int RB>
__device__ inline floatx4 tile_products_lp(const uint8_t* __restrict__ tl, int s, int g, int sub,
                                           const uint64_t (&src)[FEAT == FEAT_BF16 ? DP / 16 : DP / 32]) {
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const uint8_t* row = tl + (16 * sub + s) * RB;
#pragma unroll
  for (int k = 0; k < DP / 32; ++k) {
    if constexpr (FEAT == FEAT_BF16) {
      const uint4 av = *reinterpret_cast<const uint4*>(row + 64 * k + 16 * g);
      const uint4 bv = make_uint4((uint32_t)src[2 * k], (uint32_t)(src[2 * k] >> 32), (uint32_t)src[2 * k + 1],
                                  (uint32_t)(src[2 * k + 1] >> 32));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc,
                                                    0, 0, 0);
    } else {
      const uint2 av = *reinterpret_cast<const uint2*>(row + 32 * k + 8 * g);
      const long al = (long)(((uint64_t)av.y << 32) | av.x);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(al, (long)src[k], acc, 0, 0, 0);
    }
  }
  return acc;
}

// Squared distance of candidate z to the box [lo, hi], rounded like the membership rule: each axis term
// max(lo - z, z - hi, 0) and the fused sum in rule_s2's order.  Rounding is monotone, so for every point q of
// the box this is at most rule_s2(q, z): a candidate above rc2 here fails the rule for every source in the box.
__device__ inline float box_s2(float3 lo, float3 hi, float4 z) {
#pragma clang fp contract(off)
  const float bx = fmaxf(fmaxf(lo.x - z.x, z.x - hi.x), 0.f);
  const float by = fmaxf(fmaxf(lo.y - z.y, z.y - hi.y), 0.f);
  const float bz = fmaxf(fmaxf(lo.z - z.z, z.z - hi.z), 0.f);
  return fmaf(bz, bz, fmaf(by, by, bx * bx));
}

// MM: the moments are accumulated on the matrix core.  With u = z - ref (ref =
// centre of the pass's box) and Phi(u) = [1, u, u u^T] (10 of 16 columns), the
// sums M[s][f] = sum_j w_sj Phi_f(u_j) over all candidates are one MFMA chain
// (A operand = the weights the lanes just computed, B = Phi of the same
// candidates), and A, B, C follow exactly from M and v = q - ref:
//   A = M_1, B = A v - M_u, C = A v v^T - v M_u^T - M_u v^T + M_uu.
// CM: the inner products as computed (0), negative ones clamped to 0 (1), or
// known to be positive (2: the pair count then needs no c != 0 test).
// SC: every source point's own pair count goes to its entry of a.cnt (one more
// VALU add per candidate; for parity checks of the pair set), instead of the
// pass's count on its first entry (the per-edge totals are the same).
// LS (class ids, every frame label-stacked): the pass walks the layer of its
// sources' class id, whose candidates all carry that id, so the id test is
// skipped.
template <int MODE, int FEAT, int DP, int CM, bool MM, int P, bool SC = false, bool LS = false>
__global__ __launch_bounds__(kLanes) void k_sweep(PairArgs a) {
  // P source points per pass (16; 8 or 32 for class ids); lane (s, g) takes CPL candidates of every
  // 16-candidate sub-tile
  static_assert(P == 16 || ((P == 8 || P == 32) && FEAT == FEAT_CLASS && !MM), "8 or 32-point passes: class ids only");
  static_assert(!LS || FEAT == FEAT_CLASS, "label layers: class ids only");
  // CF (class ids): the candidates of each fetched tile that lie beyond the reach of the pass's box are
  // dropped and the rest compacted into full blocks of 64 before any source tests them
  constexpr bool CF = FEAT == FEAT_CLASS;
  constexpr int CPL = P / 4;
  constexpr bool LP = feat_low_precision(FEAT);
  constexpr int FS = FEAT == FEAT_DENSE ? DP + 1 : 1;  // LDS FP32 feature row stride (odd: conflict-free column reads)
  // LDS low-precision row: DP elements + 16 (bfloat16) or 8 (fp8) bytes, so that the 16 rows one MFMA
  // operand read touches fall on disjoint banks
  constexpr int RB = !LP ? 1 : FEAT == FEAT_BF16 ? 2 * DP + 16 : DP + 8;
  constexpr int ROWB = !LP ? 1 : FEAT == FEAT_BF16 ? 2 * DP : DP;  // bytes of one stored row
  constexpr int NSRC = !LP ? 1 : FEAT == FEAT_BF16 ? DP / 16 : DP / 32;
  constexpr int PHS = 20;                  // LDS Phi row stride (conflict-free B-operand reads)
  __shared__ uint32_t row_j0[kLanes];
  __shared__ uint32_t row_off[kLanes];
  __shared__ uint32_t marker[kLanes];
  __shared__ float4 tpos[CF ? 2 * kTile : kTile];  // CF: a ring of two blocks
  __shared__ float tfeat[FEAT == FEAT_DENSE ? kTile * FS : 1];
  __shared__ __align__(16) uint8_t tlp[LP ? kTile * RB : 16];
  __shared__ float tphi[MM ? (CF ? 2 : 1) * kTile * PHS : 1];  // Phi rows of the candidates in tpos
  __shared__ float mt[MM ? 16 * 17 : 1];

  const int lane = threadIdx.x;
  const int pass = blockIdx.x;
  // every per-pass index comes from one table entry, so the loads below do not wait on each other
  const PassInfo pi = a.passes[a.pass0 + pass];
  const EdgeXf X = a.xf[pi.e];
  const FrameInfo Fn = a.frames[pi.tgt];
  const KConst kc = a.kcs[pi.prob];
  const int s = lane & (P - 1), g = lane / P;
  const int64_t entry = pi.entry0 + s;
  const bool in_range = s < pi.count;
  bool valid = in_range;
  const uint32_t src = in_range ? a.vals[entry] : 0u;
  float3 q = make_float3(0.f, 0.f, 0.f);
  uint32_t lbl = 0;
  float fsrc[FEAT == FEAT_DENSE ? DP / 4 : 1] = {};
  uint64_t slp[NSRC] = {};
  if (valid) {
    const float4 x = a.pts[pi.src_off + src];
    q = rule_q32(X, x.x, x.y, x.z);
    valid = source_in_grid(q, Fn, kc);  // (the features below are read for any entry of the pass)
    lbl = __float_as_uint(x.w);
    if constexpr (FEAT == FEAT_DENSE) {
      // B operand of the MFMA: feature 4k + g of this lane's source point
      const float* f = static_cast<const float*>(a.feat) + (pi.src_off + src) * DP;
#pragma unroll
      for (int k = 0; k < DP / 4; ++k) fsrc[k] = f[4 * k + g];
    } else if constexpr (LP) {
      // B operand: elements 32k + 8g .. 32k + 8g + 7 of this lane's source row
      const uint8_t* f = static_cast<const uint8_t*>(a.feat) + (pi.src_off + src) * (int64_t)ROWB;
#pragma unroll
      for (int k = 0; k < DP / 32; ++k) {
        if constexpr (FEAT == FEAT_BF16) {
          const uint4 v = *reinterpret_cast<const uint4*>(f + 64 * k + 16 * g);
          slp[2 * k] = ((uint64_t)v.y << 32) | v.x;
          slp[2 * k + 1] = ((uint64_t)v.w << 32) | v.z;
        } else {
          const uint2 v = *reinterpret_cast<const uint2*>(f + 32 * k + 8 * g);
          slp[k] = ((uint64_t)v.y << 32) | v.x;
        }
      }
    }
  }
  // box of the pass's transformed points: every group of P lanes holds all P sources, so the
  // reduction runs over the P lanes of a group only
  float3 lo, hi;
  lo.x = uniform_f(group_min<P>(valid ? q.x : FLT_MAX));
  lo.y = uniform_f(group_min<P>(valid ? q.y : FLT_MAX));
  lo.z = uniform_f(group_min<P>(valid ? q.z : FLT_MAX));
  hi.x = uniform_f(group_max<P>(valid ? q.x : -FLT_MAX));
  hi.y = uniform_f(group_max<P>(valid ? q.y : -FLT_MAX));
  hi.z = uniform_f(group_max<P>(valid ? q.z : -FLT_MAX));
  if (!(lo.x <= hi.x)) {  // no valid source point in this pass (uniform)
    if (g == 0 && in_range) {
      a.cnt[entry] = 0u;
      store_zero_moments<MODE>(a, entry);
    }
    return;
  }
  const float3 ref = make_float3(0.5f * (lo.x + hi.x), 0.5f * (lo.y + hi.y), 0.5f * (lo.z + hi.z));
  // A lane without a valid source point gets q at -1e18 (padding candidates sit at +1e18): its squared
  // distance to every candidate is at least ~1e36, still finite (so w * |d|^2 = 0 * s2 stays 0), and fails
  // the membership test.
  if (!valid) q = make_float3(-1.0e18f, -1.0e18f, -1.0e18f);
  floatx4 macc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  if constexpr (MM) {
#pragma unroll
    for (int k = 10; k < 16; ++k) {  // unused Phi columns stay zero
      tphi[lane * PHS + k] = 0.f;
      if constexpr (CF) tphi[(kTile + lane) * PHS + k] = 0.f;
    }
  }
  // Phi of candidate position p (zero for padding)
  auto write_phi = [&](float* ph, float4 p, bool pad) __attribute__((always_inline)) {
    const float ux = pad ? 0.f : p.x - ref.x;
    const float uy = pad ? 0.f : p.y - ref.y;
    const float uz = pad ? 0.f : p.z - ref.z;
    ph[0] = pad ? 0.f : 1.f;
    ph[1] = ux; ph[2] = uy; ph[3] = uz;
    ph[4] = ux * ux; ph[5] = ux * uy; ph[6] = ux * uz;
    ph[7] = uy * uy; ph[8] = uy * uz; ph[9] = uz * uz;
  };

  const double inv = kc.inv_cell, cell = kc.cell, reach = kc.reach;
  const int z0 = max(clamp_floor_d(((double)lo.z - reach) * inv - Fn.org[2], -1, Fn.dim[2]), 0);
  const int z1 = min(clamp_floor_d(((double)hi.z + reach) * inv - Fn.org[2], -1, Fn.dim[2]), Fn.dim[2] - 1);
  const int y0 = max(clamp_floor_d(((double)lo.y - reach) * inv - Fn.org[1], -1, Fn.dim[1]), 0);
  const int y1 = min(clamp_floor_d(((double)hi.y + reach) * inv - Fn.org[1], -1, Fn.dim[1]), Fn.dim[1] - 1);
  const int ny = y1 - y0 + 1;
  int n_rows = (z1 >= z0 && y1 >= y0) ? (z1 - z0 + 1) * ny : 0;
  // rows of the label layer the pass walks in a label-stacked target frame: the sources of a pass share
  // one class id (passes never straddle a class id of a stacked source frame)
  const int64_t lrow = label_rows(Fn, (uint32_t)__builtin_amdgcn_readlane((int)lbl, __builtin_ctzll(__ballot(valid))));
  if (lrow < 0) n_rows = 0;  // no point of the target frame carries the id
  const int4* __restrict__ trows = a.rows + Fn.row_off + (lrow < 0 ? 0 : lrow);

  const float rc2 = kc.rc2, alpha = kc.alpha;
  float A = 0.f, Bx = 0.f, By = 0.f, Bz = 0.f;
  float Cxx = 0.f, Cxy = 0.f, Cxz = 0.f, Cyy = 0.f, Cyz = 0.f, Wr2 = 0.f;
  uint32_t cnt = 0;
  uint32_t own = 0;  // this lane's pairs (SC, spread passes)
  const float4* __restrict__ tp = a.pts + Fn.pt_off;

  // Spread passes (class ids): when the pass's sources lie far apart (isolated outliers, a jump of the
  // Morton order), the ball around their common box holds mostly candidates of no source.  Each source
  // then walks the cell rows of its own ball only (the box shrunk to its point, the same row and x-range
  // trimming), its G lanes taking every G-th row, and reads the candidates straight from the frame.
  bool spread = false;
  if constexpr (FEAT == FEAT_CLASS) {
    spread = fmaxf(hi.x - lo.x, fmaxf(hi.y - lo.y, hi.z - lo.z)) > kc.spread_limit;  // uniform
    if (spread) {
      n_rows = 0;  // no shared walk
      constexpr int G = 64 / P;
      int zs0 = 0, zs1 = -1, ys0 = 0, ys1 = -1;
      if (valid) {
        zs0 = max(clamp_floor_d(((double)q.z - reach) * inv - Fn.org[2], -1, Fn.dim[2]), 0);
        zs1 = min(clamp_floor_d(((double)q.z + reach) * inv - Fn.org[2], -1, Fn.dim[2]), Fn.dim[2] - 1);
        ys0 = max(clamp_floor_d(((double)q.y - reach) * inv - Fn.org[1], -1, Fn.dim[1]), 0);
        ys1 = min(clamp_floor_d(((double)q.y + reach) * inv - Fn.org[1], -1, Fn.dim[1]), Fn.dim[1] - 1);
      }
      const int nys = ys1 - ys0 + 1;
      const int nr = (zs1 >= zs0 && ys1 >= ys0 && lrow >= 0) ? (zs1 - zs0 + 1) * nys : 0;
      // Rows g, g + G, ... of the ball, kR at a time: the row descriptors of a batch are read together, then
      // their x ranges' table entries, then the candidates kU at a time, so that the reads of a lane do not
      // wait on each other.
      constexpr int kR = 2, kU = 4;
      // this lane's rows r = g, g + G, ... as (z, y) offsets r = oz * nys + oy, stepped without a division
      int oz = 0, oy = 0, gz = 0, gy = 0;
      if (nr > 0) {
        oz = g / nys; oy = g - oz * nys;
        gz = G / nys; gy = G - gz * nys;
      }
      for (int r0 = g; r0 < nr; r0 += G * kR) {
        int4 R[kR];
        double r2s[kR];
        int64_t ri[kR];
#pragma unroll
        for (int t = 0; t < kR; ++t) {
          const int kz = zs0 + oz, ky = ys0 + oy;
          oy += gy; oz += gz;
          if (oy >= nys) { oy -= nys; ++oz; }
          r2s[t] = -1.0;
          ri[t] = 0;  // rows outside the ball read the layer's first row, which exists, and drop it below
          if (r0 + G * t < nr) {
            const double cz = (double)(kz + Fn.org[2]) * cell;
            const double cy = (double)(ky + Fn.org[1]) * cell;
            const double bz = fmax(0.0, fmax(cz - (double)q.z, (double)q.z - (cz + cell)));
            const double by = fmax(0.0, fmax(cy - (double)q.y, (double)q.y - (cy + cell)));
            r2s[t] = kc.reach2 - by * by - bz * bz;
            if (r2s[t] >= 0.0) ri[t] = (int64_t)kz * Fn.dim[1] + ky;
          }
        }
        // the batch's descriptor reads are issued together, then the rows outside the ball emptied
#pragma unroll
        for (int t = 0; t < kR; ++t) R[t] = trows[ri[t]];
#pragma unroll
        for (int t = 0; t < kR; ++t)
          if (!(r2s[t] >= 0.0)) R[t] = make_int4(1, 0, 0, 0);
        uint32_t j0[kR], j1[kR];
#pragma unroll
        for (int t = 0; t < kR; ++t) {
          j0[t] = j1[t] = 0u;
          if (r2s[t] >= 0.0 && R[t].y >= R[t].x) {
            // half-width of the ball's chord in x: the hardware FP32 root (within an ulp) widened by 2^-16,
            // which exceeds the root's and the conversion's rounding, so no cell of the chord is lost
            const double h = (double)__builtin_amdgcn_sqrtf((float)r2s[t]) * (1.0 + 0x1p-16);
            const int xa = max(clamp_floor_d(((double)q.x - h) * inv - Fn.org[0], -1, Fn.dim[0]), R[t].x);
            const int xb = min(clamp_floor_d(((double)q.x + h) * inv - Fn.org[0], -1, Fn.dim[0]), R[t].y);
            if (xa <= xb) {
              const uint32_t* xt = a.xtab + Fn.xt_off + (uint32_t)R[t].z;
              j0[t] = xt[xa - R[t].x];
              j1[t] = xt[xb + 1 - R[t].x];
            }
          }
        }
#pragma unroll
        for (int t = 0; t < kR; ++t) {
          for (uint32_t jb = j0[t]; jb < j1[t]; jb += kU) {
            float4 zu[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) zu[u] = tp[jb + u < j1[t] ? jb + u : jb];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
              const float4 z = zu[u];
              float dx, dy, dz;
              const float s2 = rule_s2(q, z.x, z.y, z.z, dx, dy, dz);
              if (!(jb + u < j1[t] && s2 <= rc2 && (LS || __float_as_uint(z.w) == lbl))) continue;
              const float w = __builtin_amdgcn_exp2f(-alpha * s2);
              own += 1u;
              A += w;
              if constexpr (MODE == MODE_NORMAL) {
                const float wx = w * dx, wy = w * dy;
                Bx += wx; By += wy; Bz = fmaf(w, dz, Bz);
                Cxx = fmaf(wx, dx, Cxx); Cxy = fmaf(wx, dy, Cxy); Cxz = fmaf(wx, dz, Cxz);
                Cyy = fmaf(wy, dy, Cyy); Cyz = fmaf(wy, dz, Cyz); Wr2 = fmaf(w, s2, Wr2);
              }
            }
          }
        }
      }
    }
  }
  const float* __restrict__ tf = static_cast<const float*>(a.feat) + Fn.pt_off * (FEAT == FEAT_DENSE ? DP : 0);
  const uint8_t* __restrict__ tl = static_cast<const uint8_t*>(a.feat) + Fn.pt_off * (int64_t)(LP ? ROWB : 0);
  const float far_ = 1.0e18f;

  // The sub-tiles of one block of 64 candidates (blk: their positions in LDS; dense features, products and
  // Phi from the tile buffers) against the pass's sources: the moments and pair counts above.
  auto process = [&](const float4* __restrict__ blk, const float* __restrict__ bphi, int n_sub)
                     __attribute__((always_inline)) {
    floatx4 cv = {1.f, 1.f, 1.f, 1.f};
    if constexpr (FEAT == FEAT_DENSE) cv = tile_products<DP, FS>(tfeat, s, g, 0, fsrc);
    if constexpr (LP) cv = tile_products_lp<FEAT, DP, RB>(tlp, s, g, 0, slp);
    // unrolled over the four sub-tiles: the products and the LDS offsets of each sub-tile get registers
    // and immediates of their own (no register copies or address updates between sub-tiles)
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      if (sub >= n_sub) break;  // uniform
      // this lane's four candidates of the sub-tile, read before any use
      const float4* zp = blk + 16 * sub + CPL * g;
      float4 z4[CPL];
#pragma unroll
      for (int rr = 0; rr < CPL; ++rr) z4[rr] = zp[rr];
      float phi4[4] = {0.f, 0.f, 0.f, 0.f};
      if constexpr (MM) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) phi4[rr] = bphi[(16 * sub + 4 * g + rr) * PHS + s];
      }
      floatx4 cur = cv;
      if constexpr (FEAT == FEAT_DENSE) {
        // issue the next sub-tile's products now: the matrix core works while the VALU runs below
        if (sub + 1 < n_sub) cv = tile_products<DP, FS>(tfeat, s, g, sub + 1, fsrc);
      } else if constexpr (LP) {
        if (sub + 1 < n_sub) cv = tile_products_lp<FEAT, DP, RB>(tlp, s, g, sub + 1, slp);
      }
#pragma unroll
      for (int rr = 0; rr < CPL; ++rr) {
        const float4 z = z4[rr];
        float dx, dy, dz;
        const float s2 = rule_s2(q, z.x, z.y, z.z, dx, dy, dz);
        const bool near = s2 <= rc2;
        bool in = near;
        float c = 1.f;
        if constexpr (FEAT == FEAT_CLASS) {
          if constexpr (!LS) in = in && (__float_as_uint(z.w) == lbl);
        } else {
          c = CM == 1 ? fmaxf(cur[rr], 0.f) : cur[rr];
        }
        const float k = __builtin_amdgcn_exp2f(-alpha * s2);
        const float w = in ? c * k : 0.f;
        // pairs counted per pass from the wavefront's lane masks (scalar unit), or per lane (SC)
        if constexpr (SC) {
          if constexpr (FEAT == FEAT_CLASS || CM == 2) own += in ? 1u : 0u;
          else own += (in && c != 0.f) ? 1u : 0u;
        } else if constexpr (LS) {
          cnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(near));
        } else if constexpr (FEAT == FEAT_CLASS) {
          // the two compares' lane masks, combined on the scalar unit (a ballot of the combined
          // condition would first turn it into a vector value and back)
          cnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(near) &
                                    __builtin_amdgcn_ballot_w64(__float_as_uint(z.w) == lbl));
        } else if constexpr (CM == 2) {
          cnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in));
        } else {
          cnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in) & __builtin_amdgcn_ballot_w64(c != 0.f));
        }
        if constexpr (MM) {
          macc[rr & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(w, phi4[rr], macc[rr & 1], 0, 0, 0);
        } else {
          A += w;
        }
        if constexpr (MODE == MODE_NORMAL && !MM) {
          const float wx = w * dx, wy = w * dy;
          Bx += wx; By += wy; Bz = fmaf(w, dz, Bz);
          Cxx = fmaf(wx, dx, Cxx); Cxy = fmaf(wx, dy, Cxy); Cxz = fmaf(wx, dz, Cxz);
          Cyy = fmaf(wy, dy, Cyy); Cyz = fmaf(wy, dz, Cyz); Wr2 = fmaf(w, s2, Wr2);
        }
      }
    }
  };

  uint32_t head = 0, tail = 0;  // CF: the ring holds the kept candidates head .. tail - 1 (uniform)
  for (int rb = 0; rb < n_rows; rb += kLanes) {
    // ---- one row per lane: its contiguous candidate range
    uint32_t j0 = 0, cntr = 0;
    const int r = rb + lane;
    if (r < n_rows) {
      const int kz = z0 + r / ny, ky = y0 + r % ny;
      const double cz = (double)(kz + Fn.org[2]) * cell;
      const double cy = (double)(ky + Fn.org[1]) * cell;
      const double bz = fmax(0.0, fmax(cz - (double)hi.z, (double)lo.z - (cz + cell)));
      const double by = fmax(0.0, fmax(cy - (double)hi.y, (double)lo.y - (cy + cell)));
      const double r2 = kc.reach2 - by * by - bz * bz;
      if (r2 >= 0.0) {
        const int4 R = trows[(int64_t)kz * Fn.dim[1] + ky];
        if (R.y >= R.x) {
          const double h = (double)__builtin_amdgcn_sqrtf((float)r2) * (1.0 + 0x1p-16);  // widened as above
          const int xa = max(clamp_floor_d(((double)lo.x - h) * inv - Fn.org[0], -1, Fn.dim[0]), R.x);
          const int xb = min(clamp_floor_d(((double)hi.x + h) * inv - Fn.org[0], -1, Fn.dim[0]), R.y);
          if (xa <= xb) {
            const uint32_t* xt = a.xtab + Fn.xt_off + (uint32_t)R.z;
            j0 = xt[xa - R.x];
            cntr = xt[xb + 1 - R.x] - j0;
          }
        }
      }
    }
    const uint32_t incl = wave_inclusive_scan(cntr);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    wave_sync();  // previous users of row_j0/row_off are done
    row_j0[lane] = j0;
    row_off[lane] = incl - cntr;
    wave_sync();
    if (total == 0) continue;

    // ---- tiles of 64 candidates, next tile fetched while the current one is processed
    // The row of every candidate of a tile: each non-empty row marks the first tile position it
    // covers, and the candidate at position p belongs to the last row marked at or before p.
    const uint32_t my_off = incl - cntr;
    auto tile_rows = [&](uint32_t base) __attribute__((always_inline)) -> int {
      marker[lane] = 0u;  // 0: no row starts here; row r is marked r + 1
      wave_sync();
      if (cntr > 0 && my_off < base + (uint32_t)kTile && my_off + cntr > base)
        marker[my_off > base ? my_off - base : 0u] = (uint32_t)lane + 1u;
      wave_sync();
      const uint32_t r = wave_inclusive_max(marker[lane]);
      wave_sync();  // markers are rewritten by the next call
      return (int)min(max(r, 1u), (uint32_t)kLanes) - 1;
    };
    auto fetch = [&](uint32_t c, float4& pos, float* fr, u32x4* lr, bool& pad) __attribute__((always_inline)) {
      const int rid = tile_rows(c - (uint32_t)lane);
      const uint32_t jc = row_j0[rid] + (c - row_off[rid]);
      pad = c >= total || jc >= (uint32_t)Fn.n;  // the second test only bounds the reads below
      // padding lanes read the frame's first point (always present when there are candidates); the consumer
      // moves it far away, where it fails every membership test and its products stay finite (replacing
      // the loaded value here would wait for the read and stall the prefetch)
      const uint32_t j = pad ? 0u : jc;
      pos = tp[j];
      if constexpr (FEAT == FEAT_DENSE) {
        const float4* f4 = reinterpret_cast<const float4*>(tf + (int64_t)j * DP);
#pragma unroll
        for (int k = 0; k < DP / 4; ++k) {
          const float4 v = f4[k];
          fr[4 * k] = v.x; fr[4 * k + 1] = v.y; fr[4 * k + 2] = v.z; fr[4 * k + 3] = v.w;
        }
      } else if constexpr (LP) {
        const u32x4* r4 = reinterpret_cast<const u32x4*>(tl + (int64_t)j * ROWB);
#pragma unroll
        for (int k = 0; k < ROWB / 16; ++k) lr[k] = r4[k];
      }
    };
    float4 npos;
    bool npad;
    float nfeat[FEAT == FEAT_DENSE ? DP : 1];
    u32x4 nlp[LP ? ROWB / 16 : 1];
    fetch((uint32_t)lane, npos, nfeat, nlp, npad);
    for (uint32_t cb = 0; cb < total; cb += kTile) {
      if constexpr (CF) {
        // keep the candidates within reach of the pass's box, appended to the ring in list order
        const bool keep = !npad && box_s2(lo, hi, npos) <= rc2;
        const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
        if (keep) {
          const uint32_t slot =
              (tail + __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u))) &
              (2 * kTile - 1);
          tpos[slot] = npos;
          if constexpr (MM) write_phi(tphi + slot * PHS, npos, false);
        }
        tail += (uint32_t)__popcll(km);
        wave_sync();
        if (cb + kTile < total) fetch(cb + kTile + lane, npos, nfeat, nlp, npad);
        if (tail - head >= (uint32_t)kTile) {  // a full block (at most one per fetched tile)
          process(tpos + (head & (2 * kTile - 1)), tphi + (head & (2 * kTile - 1)) * PHS, 4);
          head += kTile;
          wave_sync();  // the block's slots are refilled next
        }
        continue;
      }
      tpos[lane] = npad ? make_float4(far_, far_, far_, 0.f) : npos;
      if constexpr (MM) write_phi(tphi + lane * PHS, npos, npad);
      if constexpr (FEAT == FEAT_DENSE) {
#pragma unroll
        for (int k = 0; k < DP; ++k) tfeat[lane * FS + k] = nfeat[k];
      } else if constexpr (FEAT == FEAT_BF16) {
#pragma unroll
        for (int k = 0; k < ROWB / 16; ++k) *reinterpret_cast<u32x4*>(tlp + lane * RB + 16 * k) = nlp[k];
      } else if constexpr (FEAT == FEAT_FP8) {
#pragma unroll
        for (int k = 0; k < ROWB / 16; ++k) {  // RB is a multiple of 8 only: 8-byte stores
          *reinterpret_cast<u32x2*>(tlp + lane * RB + 16 * k) = nlp[k].xy;
          *reinterpret_cast<u32x2*>(tlp + lane * RB + 16 * k + 8) = nlp[k].zw;
        }
      }
      wave_sync();
      if (cb + kTile < total) fetch(cb + kTile + lane, npos, nfeat, nlp, npad);
      const uint32_t left = total - cb;
      process(tpos, tphi, left >= (uint32_t)kTile ? 4 : (int)((left + 15) / 16));
      wave_sync();  // the tile buffer is rewritten next
    }
  }
  if constexpr (CF) {
    if (tail > head) {  // the last, partial block; its empty slots hold far padding candidates
      const uint32_t rem = tail - head;
      if ((uint32_t)lane >= rem) {
        const uint32_t slot = (head + lane) & (2 * kTile - 1);
        tpos[slot] = make_float4(far_, far_, far_, 0.f);
        if constexpr (MM) write_phi(tphi + slot * PHS, tpos[slot], true);
      }
      wave_sync();
      process(tpos + (head & (2 * kTile - 1)), tphi + (head & (2 * kTile - 1)) * PHS, (int)((rem + 15) / 16));
    }
  }

  if constexpr (MM) {
    if (!spread) {  // (uniform; spread passes summed their moments on the VALU)
      // lane (s, g) holds M[source 4g + r][column s]; regroup per source through LDS
      wave_sync();
#pragma unroll
      for (int r = 0; r < 4; ++r) mt[(4 * g + r) * 17 + s] = macc[0][r] + macc[1][r];
      wave_sync();
      if (g == 0) {
        const float* m = mt + s * 17;
        const float vx = q.x - ref.x, vy = q.y - ref.y, vz = q.z - ref.z;
        A = m[0];
        const float mx = m[1], my = m[2], mz = m[3];
        Bx = A * vx - mx; By = A * vy - my; Bz = A * vz - mz;
        Cxx = A * vx * vx - 2.f * vx * mx + m[4];
        Cxy = A * vx * vy - vx * my - mx * vy + m[5];
        Cxz = A * vx * vz - vx * mz - mx * vz + m[6];
        Cyy = A * vy * vy - 2.f * vy * my + m[7];
        Cyz = A * vy * vz - vy * mz - my * vz + m[8];
        Wr2 = Cxx + Cyy + (A * vz * vz - 2.f * vz * mz + m[9]);
      }
    }
  }

  // sum the four candidate streams of each source point
  auto sum_streams = [&](auto xa) __attribute__((always_inline)) {
    A = xa(A);
    if constexpr (MODE == MODE_NORMAL) {
      Bx = xa(Bx); By = xa(By); Bz = xa(Bz);
      Cxx = xa(Cxx); Cxy = xa(Cxy); Cxz = xa(Cxz);
      Cyy = xa(Cyy); Cyz = xa(Cyz); Wr2 = xa(Wr2);
    }
  };
  if (!MM || spread) {
    if constexpr (P == 8) sum_streams([](float v) { return xor_add<8>(v); });
    if constexpr (P <= 16) sum_streams([](float v) { return xor_add<16>(v); });
    sum_streams([](float v) { return xor_add<32>(v); });
  }
  if (SC || spread) {  // every source point's own count
    if constexpr (P == 8) own = xor_add<8>(own);
    if constexpr (P <= 16) own = xor_add<16>(own);
    own = xor_add<32>(own);
    if (g == 0 && in_range) a.cnt[entry] = valid ? own : 0u;
  } else {
    // the pass's pair count goes to its first entry, zeros to the others
    if (g == 0 && in_range) a.cnt[entry] = s == 0 ? cnt : 0u;
  }
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

template <int MODE, int FEAT, int CM, bool MM, bool SC>
hipError_t dispatch(const PairArgs& a, int DP, hipStream_t st) {
  const unsigned nb = (unsigned)a.n_pass;
  if (nb == 0) return hipSuccess;
  if constexpr (FEAT == FEAT_CLASS) {
    if (a.stacked) k_sweep<MODE, FEAT, 0, 0, MM, 16, SC, true><<<nb, kLanes, 0, st>>>(a);
    else k_sweep<MODE, FEAT, 0, 0, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
  } else if constexpr (feat_low_precision(FEAT)) {
    if (DP <= 32) k_sweep<MODE, FEAT, 32, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
    else k_sweep<MODE, FEAT, 64, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
  } else {
    if (DP <= 8) k_sweep<MODE, FEAT, 8, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
    else if (DP <= 16) k_sweep<MODE, FEAT, 16, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
    else if (DP <= 24) k_sweep<MODE, FEAT, 24, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
    else if (DP <= 32) k_sweep<MODE, FEAT, 32, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
    else k_sweep<MODE, FEAT, 64, CM, MM, 16, SC><<<nb, kLanes, 0, st>>>(a);
  }
  return hipGetLastError();
}

// clamped, known-positive (FP32 features, VALU moments) or plain inner products
template <int MODE, int FEAT, bool MM, bool SC>
hipError_t dispatch_clamp(const PairArgs& a, hipStream_t st) {
  if (a.kc.clamp) return dispatch<MODE, FEAT, 1, MM, SC>(a, a.kc.Dp, st);
  if constexpr (FEAT == FEAT_DENSE && !MM)
    if (a.kc.c_positive) return dispatch<MODE, FEAT, 2, MM, SC>(a, a.kc.Dp, st);
  return dispatch<MODE, FEAT, 0, MM, SC>(a, a.kc.Dp, st);
}

template <int MODE, bool MM, bool SC>
hipError_t dispatch_mode(const PairArgs& a, int feat_path, hipStream_t st) {
  switch (feat_path) {
    case FEAT_CLASS: return dispatch<MODE, FEAT_CLASS, 0, MM, SC>(a, 0, st);
    case FEAT_DENSE: return dispatch_clamp<MODE, FEAT_DENSE, MM, SC>(a, st);
    case FEAT_BF16: return dispatch_clamp<MODE, FEAT_BF16, MM, SC>(a, st);
    default: return dispatch_clamp<MODE, FEAT_FP8, MM, SC>(a, st);
  }
}

// Class ids in passes of P = 8 or 32 source points (moments on the VALU).
template <int P>
hipError_t dispatch_class(const PairArgs& a, int mode, bool source_counts, hipStream_t st) {
  const unsigned nb = (unsigned)a.n_pass;
  if (a.stacked) {
    if (source_counts) k_sweep<MODE_NORMAL, FEAT_CLASS, 0, 0, false, P, true, true><<<nb, kLanes, 0, st>>>(a);
    else if (mode == MODE_LOSS) k_sweep<MODE_LOSS, FEAT_CLASS, 0, 0, false, P, false, true><<<nb, kLanes, 0, st>>>(a);
    else k_sweep<MODE_NORMAL, FEAT_CLASS, 0, 0, false, P, false, true><<<nb, kLanes, 0, st>>>(a);
  } else {
    if (source_counts) k_sweep<MODE_NORMAL, FEAT_CLASS, 0, 0, false, P, true><<<nb, kLanes, 0, st>>>(a);
    else if (mode == MODE_LOSS) k_sweep<MODE_LOSS, FEAT_CLASS, 0, 0, false, P><<<nb, kLanes, 0, st>>>(a);
    else k_sweep<MODE_NORMAL, FEAT_CLASS, 0, 0, false, P><<<nb, kLanes, 0, st>>>(a);
  }
  return hipGetLastError();
}

}  // namespace

// Tiled sweep for passes of 16 source points (8 or 32 for class ids on request).
// Loss-only sums stay on the VALU; Gauss-Newton moments on the VALU or the matrix cores.
hipError_t launch_sweep(const PairArgs& a, int mode, int feat_path, int pass_points, bool matrix_moments,
                        bool source_counts, hipStream_t st) {
  if (source_counts && (mode != MODE_NORMAL || matrix_moments)) return hipErrorInvalidValue;
  if (pass_points == 8 || pass_points == 32) {
    if (feat_path != FEAT_CLASS || a.n_pass == 0) return feat_path != FEAT_CLASS ? hipErrorInvalidValue : hipSuccess;
    return pass_points == 8 ? dispatch_class<8>(a, mode, source_counts, st)
                            : dispatch_class<32>(a, mode, source_counts, st);
  }
  if (source_counts) return dispatch_mode<MODE_NORMAL, false, true>(a, feat_path, st);
  if (mode == MODE_LOSS) return dispatch_mode<MODE_LOSS, false, false>(a, feat_path, st);
  return matrix_moments ? dispatch_mode<MODE_NORMAL, true, false>(a, feat_path, st)
                        : dispatch_mode<MODE_NORMAL, false, false>(a, feat_path, st);
}

}  // namespace rkhsba
