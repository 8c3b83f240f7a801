// Normal-equation assembly, FP64 Cholesky solve and SE(3) pose update of one
// Gauss-Newton / IRLS step (Sec. V-A): with the weights frozen, the step
// solves (H_red + mu I) delta = -b_red over every frame except the fixed one
// and moves T_m <- T_m exp(delta_m^) (right perturbation, eps = [rho; phi]).
//
// Assembly is one thread per entry of the system, summing that entry's
// contributing edge blocks in edge order (host-built lists, deterministic).
// The solve is one workgroup per problem: systems up to 128 unknowns are
// eliminated in LDS (one barrier per column, no square roots) and solved in
// one wavefront; larger ones run a blocked right-looking Cholesky with
// 32-wide panels, the panel kept in LDS for the trailing update.
#include "rkhsba_device.h"

namespace rkhsba {
namespace {


__device__ inline int sym_index(int r, int c) {
  if (r > c) { const int t = r; r = c; c = t; }
  return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

// reduced index <-> frame when frame `fixed` is removed (fixed < 0: none)
__device__ inline int frame_of_reduced(int k, int fixed) { return (fixed >= 0 && k >= fixed) ? k + 1 : k; }

// One thread per entry of a problem's system (grid.y = problem).
__global__ __launch_bounds__(256) void k_assemble(SolveArgs a) {
  const ProbSys S = a.sys[blockIdx.y];
  const int n = S.n;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int32_t* blk_start = a.blk_start + S.blk0;
  const int32_t* vec_start = a.vec_start + S.vec0;
  if (idx < (int64_t)n * n) {
    const int row = (int)(idx / n), col = (int)(idx % n);
    const int fa = frame_of_reduced(row / 6, S.fixed), fc = frame_of_reduced(col / 6, S.fixed);
    const int r = row % 6, s = col % 6;
    const int blk = fa * S.K + fc;
    double v = 0.0;
    for (int k = blk_start[blk]; k < blk_start[blk + 1]; ++k) {
      const int code = a.blk_list[k];
      const double* eo = a.edge_out + (int64_t)(code >> 2) * kEdgeVals;
      switch (code & 3) {
        case 0: v += eo[13 + sym_index(r, s)]; break;
        case 1: v += eo[34 + sym_index(r, s)]; break;
        case 2: v += eo[55 + 6 * r + s]; break;
        default: v += eo[55 + 6 * s + r]; break;
      }
    }
    a.H[S.h_off + idx] = v;
  } else if (idx < (int64_t)n * n + n) {
    const int row = (int)(idx - (int64_t)n * n);
    const int fa = frame_of_reduced(row / 6, S.fixed), r = row % 6;
    double v = 0.0;
    for (int k = vec_start[fa]; k < vec_start[fa + 1]; ++k) {
      const int code = a.vec_list[k];
      v += a.edge_out[(int64_t)(code >> 1) * kEdgeVals + ((code & 1) ? 7 : 1) + r];
    }
    a.b[S.v_off + row] = v;
  }
}

// F (times sigma^2) and the pair count of the current evaluation of each
// problem (one wavefront per problem, fixed summation order).
__global__ __launch_bounds__(64) void k_loss_only(SolveArgs a) {
  const ProbSys S = a.sys[blockIdx.x];
  double F = 0.0, np = 0.0;
  for (int e = S.e0 + (int)threadIdx.x; e < S.e0 + S.E; e += 64) {
    F += a.edge_out[(int64_t)e * kEdgeVals];
    np += a.edge_out[(int64_t)e * kEdgeVals + 91];
  }
  F = wave_sum(F);
  np = wave_sum(np);
  const int iter = a.state[S.state_off];
  if (threadIdx.x == 0 && iter >= 0 && iter <= S.n_iter) {
    a.loss_hist[S.hist_off + iter] = S.sigma2 * F;
    a.pairs_hist[S.hist_off + iter] = np;
  }
}

// T <- T exp(xi^): closed-form SE(3) exponential (Rodrigues for the rotation,
// V = I + B K + C K^2 for the translation), series for small angles.
__device__ __noinline__ void right_update(double* T, const double* xi) {
  const double* rho = xi;
  const double* phi = xi + 3;
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    double s, c;
    sincos(th, &s, &c);
    A = s / th;
    B = (1.0 - c) / th2;
    C = (th - s) / (th2 * th);
  }
  const double K[3][3] = {{0.0, -phi[2], phi[1]}, {phi[2], 0.0, -phi[0]}, {-phi[1], phi[0], 0.0}};
  double K2[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K2[r][c] = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
  double Re[3][3], V[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double I = r == c ? 1.0 : 0.0;
      Re[r][c] = I + A * K[r][c] + B * K2[r][c];
      V[r][c] = I + B * K[r][c] + C * K2[r][c];
    }
  double te[3];
  for (int r = 0; r < 3; ++r) te[r] = V[r][0] * rho[0] + V[r][1] * rho[1] + V[r][2] * rho[2];
  double R[3][3], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R[r][c] = T[3 * r + c];
    t[r] = T[9 + r];
  }
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) T[3 * r + c] = R[r][0] * Re[0][c] + R[r][1] * Re[1][c] + R[r][2] * Re[2][c];
    T[9 + r] = R[r][0] * te[0] + R[r][1] * te[1] + R[r][2] * te[2] + t[r];
  }
}

__device__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  __syncthreads();
  return t;
}

// A double read from one lane of the wavefront (lane index uniform).
__device__ inline double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Right-looking elimination of an n x n symmetric block held in LDS (row
// stride ld, lower triangle used), without square roots: step j subtracts
// a_ij a_kj / d_j from every trailing entry (j < k <= i), d_j the pivot of
// step j.  Afterwards the block holds M (unit-free lower factor: A = M D^-1 M^T
// with D = diag(d)), and rd[j] = 1 / d_j.  One barrier per step; threads form a
// 32 x 32 grid over the trailing rows and columns.  Returns false (in every
// thread) when a pivot is not positive.
__device__ bool eliminate_lds(double* A, int n, int ld, double* rd) {
  const int t = threadIdx.x, tx = t & 31, ty = t >> 5;
  for (int j = 0; j < n; ++j) {
    const double d = A[j * ld + j];
    if (!(d > 0.0)) return false;  // every thread read the same pivot
    const double inv = 1.0 / d;
    if (t == 0) rd[j] = inv;
    for (int i = j + 1 + ty; i < n; i += 32) {
      const double aij = A[i * ld + j] * inv;
      for (int k = j + 1 + tx; k <= i; k += 32) A[i * ld + k] -= aij * A[k * ld + j];
    }
    __syncthreads();
  }
  return true;
}

// ---- systems that fit in LDS (n <= kLdsSystem)
//
// (H + mu I) delta = -b as M D^-1 M^T delta = -b: forward M u = -b, then
// M^T delta = D u, both in wavefront 0 with two rows per lane.
constexpr int kSolveThreads = 1024;
constexpr int kLdsSystem = 128;
constexpr int kLdsDoubles = kLdsSystem * (kLdsSystem + 1);  // shared buffer of both paths

__device__ void solve_lds(const ProbSys& S, const SolveArgs& a, double mu, double* A, double* rd, int32_t* status) {
  const int n = S.n, ld = n + 1;  // odd stride: column reads spread over the banks
  const int t = threadIdx.x;
  const double* H = a.H + S.h_off;
  for (int idx = t; idx < n * n; idx += kSolveThreads) {
    const int i = idx / n, k = idx - i * n;
    if (k <= i) A[i * ld + k] = H[idx] + (i == k ? mu : 0.0);
  }
  __syncthreads();
  const bool ok = eliminate_lds(A, n, ld, rd);
  if (!ok) {
    if (t == 0) *status = -4;
    return;
  }
  if (t < 64) {
    const double* b = a.b + S.v_off;
    double u0 = t < n ? -b[t] : 0.0, u1 = t + 64 < n ? -b[t + 64] : 0.0;
    // forward: u_j = (r_j - sum_{k<j} M_jk u_k) / d_j
    for (int j = 0; j < n; ++j) {
      const double uj = lane_value(j < 64 ? u0 : u1, j & 63) * rd[j];
      if (t == (j & 63)) {
        if (j < 64) u0 = uj; else u1 = uj;
      }
      if (t > j && t < n) u0 -= A[t * ld + j] * uj;
      if (t + 64 > j && t + 64 < n) u1 -= A[(t + 64) * ld + j] * uj;
    }
    // backward: x_j = u_j - (1/d_j) sum_{k>j} M_kj x_k, columns from the last
    for (int j = n - 1; j >= 0; --j) {
      const double xj = lane_value(j < 64 ? u0 : u1, j & 63);
      if (t < j) u0 -= rd[t] * A[j * ld + t] * xj;
      if (t + 64 < j) u1 -= rd[t + 64] * A[j * ld + t + 64] * xj;
    }
    double* y = a.delta + S.v_off;
    if (t < n) y[t] = u0;
    if (t + 64 < n) y[t + 64] = u1;
  }
  __syncthreads();
}

// ---- larger systems: blocked right-looking Cholesky in global memory
//
// Panels of NB columns: the diagonal block is eliminated in LDS and scaled to
// L11; the rows below solve L21 = A21 L11^-T and are kept in LDS for the
// trailing update A22 -= L21 L21^T.  While the panel has at most kPanelCols
// rows (every system up to ~500 unknowns), each row is solved in registers
// (one row per thread, the 32 steps unrolled) and the panel is stored column
// by column, so that the trailing update's 4 x 4 register tiles, whose rows
// and columns are 32 apart, read it without bank conflicts and write A22 with
// consecutive threads on consecutive columns.  Larger panels are solved and
// read in place in global memory, with contiguous tiles.  Then L y = -b and
// L^T delta = y, panel by panel.
constexpr int NB = 32;
constexpr int kPanelCols = (kLdsDoubles - NB * (NB + 1) - 2 * NB) / NB;  // rows of a column-major panel

// Zero rows of L21: many systems are block-sparse (each frame has a few neighbours in the pose graph), and
// the factor keeps the profile of the matrix.  For systems whose panels all fit in LDS, flags[p * W + w] (W =
// ceil(n / 32) words per panel) records, bit b, whether row 32 w + b of the factor has a nonzero entry in panel
// p's columns; the row solve, the trailing update and both triangular solves skip what a zero row would
// contribute (exact zeros: the factor and the solution are the same bit for bit).  flags == nullptr: every row
// counts as nonzero.
constexpr int kFlagRows = NB + kPanelCols;  // the largest system every panel of which is solved in LDS
constexpr int kFlagWords = ((kFlagRows + 31) / 32) * ((kFlagRows + 31) / 32);

__device__ void solve_blocked(const ProbSys& S, const SolveArgs& a, double mu, double* buf, int32_t* status,
                              uint32_t* flags) {
  const int n = S.n, t = threadIdx.x, tx = t & 31, ty = t >> 5;
  const int W = (n + 31) / 32;
  if (n > kFlagRows) flags = nullptr;
  static_assert(NB == 32, "one flag word per panel row chunk");
  __shared__ int32_t live_chunks[(kFlagRows + 31) / 32];
  __shared__ int32_t n_live;
  __shared__ uint32_t chunk_mask;  // bit c: rows m0 + 32 c .. m0 + 32 c + 31 hold a nonzero row of L21
  double* H = a.H + S.h_off;
  double* Dg = buf;                       // NB x (NB + 1) diagonal block
  double* rd = buf + NB * (NB + 1);       // NB reciprocal pivots / diagonal
  double* yb = rd + NB;                   // NB solution entries of a panel
  double* P = yb + NB;                    // the panel L21, column-major (P[j * m + r])
  for (int i = t; i < n; i += kSolveThreads) H[(int64_t)i * n + i] += mu;
  __syncthreads();
  for (int kb = 0; kb < n; kb += NB) {
    const int nb = min(NB, n - kb), m0 = kb + nb, m = n - m0;
    for (int idx = t; idx < nb * nb; idx += kSolveThreads) {
      const int i = idx / nb, k = idx - i * nb;
      if (k <= i) Dg[i * (NB + 1) + k] = H[(int64_t)(kb + i) * n + kb + k];
    }
    __syncthreads();
    if (!eliminate_lds(Dg, nb, NB + 1, rd)) {
      if (t == 0) *status = -4;
      return;
    }
    // scale to L11: L_jj = sqrt(d_j), L_ij = M_ij / sqrt(d_j); rd <- 1 / L_jj
    for (int idx = t; idx < nb * nb; idx += kSolveThreads) {
      const int i = idx / nb, k = idx - i * nb;
      if (k <= i) {
        const double sk = sqrt(rd[k]);  // 1 / sqrt(d_k)
        const double v = (i == k) ? 1.0 / sk : Dg[i * (NB + 1) + k] * sk;
        Dg[i * (NB + 1) + k] = v;
        H[(int64_t)(kb + i) * n + kb + k] = v;
      }
    }
    __syncthreads();
    if (t < nb) rd[t] = 1.0 / Dg[t * (NB + 1) + t];
    __syncthreads();
    if (m <= kPanelCols) {
      // panel rows in registers, stored column-major: P[j * m + r] = L21[r][j]; a zero row of A21 stays zero
      const int pw = kb / 32;  // this panel's flag words start at pw * W
      for (int r0 = 0; r0 < m; r0 += kSolveThreads) {  // uniform trip count (the ballot below)
        const int r = r0 + t;
        bool nz = false;
        if (r < m) {
          double* row = H + (int64_t)(m0 + r) * n + kb;
          double x[NB];
#pragma unroll
          for (int j = 0; j < NB; ++j) x[j] = j < nb ? row[j] : 0.0;
#pragma unroll
          for (int j = 0; j < NB; ++j) nz = nz || x[j] != 0.0;
          if (nz) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              if (j < nb) {
                const double* Lj = Dg + j * (NB + 1);
                double s0 = x[j], s1 = 0.0;
#pragma unroll
                for (int k = 0; k + 1 < j; k += 2) {
                  s0 -= Lj[k] * x[k];
                  s1 -= Lj[k + 1] * x[k + 1];
                }
                if (j & 1) s0 -= Lj[j - 1] * x[j - 1];
                x[j] = (s0 + s1) * rd[j];
              }
            }
          }
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (j < nb) {
              if (nz) row[j] = x[j];
              P[j * m + r] = x[j];
            }
        }
        if (flags) {  // rows m0 + r0 + 64 w' + lane: two whole words per wavefront (m0 and r0 are multiples of 32)
          const uint64_t bits = __ballot(nz);
          const int wd = (m0 + r0 + (t & ~63)) / 32;
          if ((t & 63) == 0 && wd < W) flags[pw * W + wd] = (uint32_t)bits;
          if ((t & 63) == 32 && wd + 1 < W) flags[pw * W + wd + 1] = (uint32_t)(bits >> 32);
        }
      }
      __syncthreads();
      // the 32-row chunks of A22 with a nonzero row of L21 in this panel
      if (t == 0) {  // (m == 0, the last panel, has no chunk; otherwise m0 is a multiple of 32)
        int c = 0;
        uint32_t mask = 0;
        for (int w = m0 / 32; m > 0 && w < W; ++w)
          if (!flags || flags[pw * W + w]) {
            live_chunks[c++] = w * 32 - m0;
            mask |= 1u << (w - m0 / 32);
          }
        n_live = c;
        chunk_mask = mask;
      }
      __syncthreads();
      const int nl = n_live, nc = (m + 31) / 32;
      if (2 * nl <= nc) {
        // few live chunks: one 32 x 32 tile per pair of them, one entry per thread, the NB products summed in
        // the same order as below
        for (int u = 0; u < nl; ++u)
          for (int v = 0; v <= u; ++v) {
            const int i = live_chunks[u] + ty, k = live_chunks[v] + tx;
            if (i < m && k <= i) {
              double acc = 0.0;
              for (int j = 0; j < nb; ++j) acc = fma(P[j * m + i], P[j * m + k], acc);
              H[(int64_t)(m0 + i) * n + m0 + k] -= acc;
            }
          }
        __syncthreads();
        continue;
      }
      // A22 -= L21 L21^T over 128 x 128 blocks on or below the diagonal (those with a nonzero row of L21 on
      // both sides); thread (tx, ty) takes rows a0 + ty + 32p and columns b0 + tx + 32q
      const uint32_t cm = chunk_mask;
      for (int a0 = 0; a0 < m; a0 += 128)
        for (int b0 = 0; b0 <= a0; b0 += 128) {
          if (!((cm >> (a0 / 32)) & 0xFu) || !((cm >> (b0 / 32)) & 0xFu)) continue;
          double acc[4][4];
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
          for (int j = 0; j < nb; ++j) {
            const double* Pj = P + j * m;
            double li[4], lk[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const int i = a0 + ty + 32 * p, k = b0 + tx + 32 * p;
              li[p] = i < m ? Pj[i] : 0.0;
              lk[p] = k < m ? Pj[k] : 0.0;
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[p][q] = fma(li[p], lk[q], acc[p][q]);
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int i = a0 + ty + 32 * p, k = b0 + tx + 32 * q;
              if (i < m && k <= i) H[(int64_t)(m0 + i) * n + m0 + k] -= acc[p][q];
            }
        }
      __syncthreads();
      continue;
    }
    // larger panels: rows solved and read in place in global memory
    for (int r = t; r < m; r += kSolveThreads) {
      double* x = H + (int64_t)(m0 + r) * n + kb;
      for (int j = 0; j < nb; ++j) {
        const double* Lj = Dg + j * (NB + 1);
        double s0 = x[j], s1 = 0.0;
        int k = 0;
        for (; k + 1 < j; k += 2) {
          s0 -= Lj[k] * x[k];
          s1 -= Lj[k + 1] * x[k + 1];
        }
        if (k < j) s0 -= Lj[k] * x[k];
        x[j] = (s0 + s1) * rd[j];
      }
    }
    __syncthreads();
    // trailing update of the lower triangle of A22
    const int tiles = (m + 3) / 4;
    for (int ti = ty; ti < tiles; ti += 32) {
      for (int tk = tx; tk <= ti; tk += 32) {
        double acc[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
        for (int j = 0; j < nb; ++j) {
          double li[4], lk[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const int ri = 4 * ti + p, rk = 4 * tk + p;
            li[p] = ri < m ? H[(int64_t)(m0 + ri) * n + kb + j] : 0.0;
            lk[p] = rk < m ? H[(int64_t)(m0 + rk) * n + kb + j] : 0.0;
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] = fma(li[p], lk[q], acc[p][q]);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = 4 * ti + p, k = 4 * tk + q;
            if (i < m && k <= i) H[(int64_t)(m0 + i) * n + m0 + k] -= acc[p][q];
          }
      }
    }
    __syncthreads();
  }

  double* y = a.delta + S.v_off;
  const double* b = a.b + S.v_off;
  for (int i = t; i < n; i += kSolveThreads) y[i] = -b[i];
  __syncthreads();
  // L y = -b: each diagonal block staged in LDS (with the reciprocals of its diagonal) and solved in
  // wavefront 0, then the rows below updated by all threads
  auto stage_diag = [&](int kb, int nb) {
    for (int idx = t; idx < nb * nb; idx += kSolveThreads) {
      const int i = idx / nb, k = idx - i * nb;
      if (k <= i) Dg[i * (NB + 1) + k] = H[(int64_t)(kb + i) * n + kb + k];
    }
    if (t < nb) rd[t] = 1.0 / H[(int64_t)(kb + t) * n + kb + t];
    __syncthreads();
  };
  for (int kb = 0; kb < n; kb += NB) {
    const int nb = min(NB, n - kb);
    stage_diag(kb, nb);
    if (t < 64) {
      double v = t < nb ? y[kb + t] : 0.0;
      for (int j = 0; j < nb; ++j) {
        const double yj = lane_value(v, j) * rd[j];
        if (t == j) v = yj;
        else if (t > j && t < nb) v -= Dg[t * (NB + 1) + j] * yj;
      }
      if (t < nb) {
        y[kb + t] = v;
        yb[t] = v;
      }
    }
    __syncthreads();
    for (int i = kb + nb + t; i < n; i += kSolveThreads) {
      if (flags && !((flags[(kb / 32) * W + i / 32] >> (i & 31)) & 1u)) continue;  // zero row of this panel
      const double* row = H + (int64_t)i * n + kb;
      double v = y[i];
      for (int j = 0; j < nb; ++j) v -= row[j] * yb[j];
      y[i] = v;
    }
    __syncthreads();
  }
  // L^T delta = y
  for (int kb = ((n - 1) / NB) * NB; kb >= 0; kb -= NB) {
    const int nb = min(NB, n - kb);
    stage_diag(kb, nb);
    if (t < 64) {
      double v = t < nb ? y[kb + t] : 0.0;
      for (int j = nb - 1; j >= 0; --j) {
        const double xj = lane_value(v, j) * rd[j];
        if (t == j) v = xj;
        else if (t < j) v -= Dg[j * (NB + 1) + t] * xj;
      }
      if (t < nb) {
        y[kb + t] = v;
        yb[t] = v;
      }
    }
    __syncthreads();
    for (int i = t; i < kb; i += kSolveThreads) {
      if (flags && !flags[(i / 32) * W + kb / 32]) continue;  // rows kb .. kb + nb - 1 are zero in i's panel
      double v = y[i];
      for (int j = 0; j < nb; ++j) v -= H[(int64_t)(kb + j) * n + i] * yb[j];
      y[i] = v;
    }
    __syncthreads();
  }
}

// One workgroup per problem: damped solve and pose update.  A problem whose
// iteration count has reached n_iter (its last evaluation gave the final
// loss) is left unchanged.  Every branch below is block-uniform.
__global__ __launch_bounds__(kSolveThreads) void k_solve_update(SolveArgs a) {
  __shared__ double buf[kLdsDoubles];
  __shared__ uint32_t zflags[kFlagWords];
  __shared__ double rd[kLdsSystem];
  __shared__ double sh[kSolveThreads / 64];
  const ProbSys S = a.sys[blockIdx.x];
  int32_t* st = a.state + S.state_off;
  const int iter = st[0];
  const bool run = iter < S.n_iter && st[1] == 0 && S.n > 0;
  __syncthreads();
  if (run) {
    const int n = S.n;
    const double* H = a.H + S.h_off;
    double tr = 0.0;
    for (int i = threadIdx.x; i < n; i += kSolveThreads) tr += H[(int64_t)i * n + i];
    tr = block_sum(tr, sh);
    if (tr > 0.0) {  // otherwise no pair touches a free frame: nothing moves
      const double mu = S.damping_rel * tr / n;
      if (n <= kLdsSystem) solve_lds(S, a, mu, buf, rd, st + 1);
      else solve_blocked(S, a, mu, buf, st + 1, zflags);
      __syncthreads();
      if (st[1] == 0) {
        const double* y = a.delta + S.v_off;
        for (int k = threadIdx.x; k < n / 6; k += kSolveThreads)
          right_update(a.poses + 12 * (S.slot0 + frame_of_reduced(k, S.fixed)), y + 6 * k);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && iter <= S.n_iter) st[0] = iter + 1;
}

}  // namespace

hipError_t launch_assemble(const SolveArgs& a, hipStream_t st) {
  if (a.n_prob <= 0) return hipSuccess;
  const int64_t n = a.n_max;
  const int64_t work = n * n + n;
  if (work > 0) k_assemble<<<dim3((unsigned)((work + 255) / 256), (unsigned)a.n_prob), 256, 0, st>>>(a);
  k_loss_only<<<a.n_prob, 64, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_solve_update(const SolveArgs& a, hipStream_t st) {
  if (a.n_prob > 0) k_solve_update<<<a.n_prob, kSolveThreads, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_loss_only(const SolveArgs& a, hipStream_t st) {
  if (a.n_prob > 0) k_loss_only<<<a.n_prob, 64, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rkhsba
