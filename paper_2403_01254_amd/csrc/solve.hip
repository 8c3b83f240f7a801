// Normal-equation assembly, FP64 Cholesky solve and SE(3) pose update of one
// Gauss-Newton / IRLS step (Sec. V-A): with the weights frozen, the step
// solves (H_red + mu I) delta = -b_red over every frame except the fixed one
// and moves T_m <- T_m exp(delta_m^) (right perturbation, eps = [rho; phi]).
//
// Assembly is one thread per entry of the system, summing that entry's
// contributing edge blocks in edge order (host-built lists, deterministic).
// The solve is one workgroup: blocked right-looking Cholesky with 16-wide
// panels, each diagonal block factored in one wavefront's registers, panel
// rows solved one per thread, and the trailing update in 4x4 register tiles.
#include "rkhsba_device.h"

namespace rkhsba {
namespace {

constexpr int kSolveThreads = 1024;
constexpr int NB = 16;

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

// Factors the nb x nb diagonal block at (kb, kb) of the n x n matrix H in
// wavefront 0: lane i holds row i in registers; column j's pivot and entries
// are broadcast with shuffles.  Writes L11 to H and to Ld.  Returns false (in
// every lane of wave 0) on a non-positive pivot.
__device__ __noinline__ bool factor_diag(double* H, int n, int kb, int nb, double (*Ld)[NB + 1]) {
  const int i = threadIdx.x;  // wave 0 only
  double r[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) r[k] = (i < nb && k <= i) ? H[(int64_t)(kb + i) * n + kb + k] : 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    if (j < nb) {
      const double d = __shfl(r[j], j, 64);
      ok = ok && d > 0.0;
      const double ljj = sqrt(d > 0.0 ? d : 1.0);
      if (i == j) r[j] = ljj;
      else if (i > j) r[j] /= ljj;
#pragma unroll
      for (int k = j + 1; k < NB; ++k) {
        const double lkj = __shfl(r[j], k, 64);
        if (k < nb && i >= k) r[k] -= r[j] * lkj;
      }
    }
  }
  if (i < nb) {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (k <= i) {
        H[(int64_t)(kb + i) * n + kb + k] = r[k];
        Ld[i][k] = r[k];
      }
  }
  return ok;
}

// Panel below the diagonal block: L21 = A21 L11^-T, one row per thread.
__device__ __noinline__ void panel_solve(double* H, int n, int kb, int nb, const double (*Ld)[NB + 1]) {
  const int t = threadIdx.x, T = blockDim.x;
    const int m0 = kb + nb;
    for (int i = m0 + t; i < n; i += T) {
      double* row = H + (int64_t)i * n + kb;
      double x[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nb) {
          double v = row[j];
#pragma unroll
          for (int k = 0; k < NB; ++k)
            if (k < j) v -= x[k] * Ld[j][k];
          x[j] = v / Ld[j][j];
        } else {
          x[j] = 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (j < nb) row[j] = x[j];
    }
}

// Trailing update of the lower triangle: A22 -= L21 L21^T in 4x4 register
// tiles.  The panel L21 is read from LDS (P, row stride NB) when it fits, else
// from global memory.
constexpr int kPanelRows = 896;  // LDS panel capacity: 896 x 16 doubles = 112 KB
__device__ __noinline__ void trailing_update(double* H, int n, int kb, int nb, const double* P) {
  const int t = threadIdx.x, T = blockDim.x;
  const int m0 = kb + nb;
  const int m = n - m0;
  const bool lds = m <= kPanelRows;
  const int tiles = (m + 3) / 4;
  const int n_tiles = tiles * (tiles + 1) / 2;
  for (int tt = t; tt < n_tiles; tt += T) {
    // tile (ti, tk) with ti >= tk, enumerated row by row of the tile triangle
    int ti = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= tt) ++ti;
    while (ti * (ti + 1) / 2 > tt) --ti;
    const int tk = tt - ti * (ti + 1) / 2;
    const int i0 = 4 * ti, k0 = 4 * tk;  // panel-relative rows
    double acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
    for (int j0 = 0; j0 < nb; j0 += 4) {
      double li[4][4], lk[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool okj = j0 + j < nb;
          const int ri = i0 + p, rk = k0 + p;
          li[p][j] = (okj && ri < m) ? (lds ? P[ri * NB + j0 + j] : H[(int64_t)(m0 + ri) * n + kb + j0 + j]) : 0.0;
          lk[p][j] = (okj && rk < m) ? (lds ? P[rk * NB + j0 + j] : H[(int64_t)(m0 + rk) * n + kb + j0 + j]) : 0.0;
        }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[p][q] = fma(li[p][j], lk[q][j], acc[p][q]);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = m0 + i0 + p, k = m0 + k0 + q;
        if (i < n && k <= i) H[(int64_t)i * n + k] -= acc[p][q];
      }
  }
}

// Damped Cholesky solve of one problem's system and its pose update.  Every
// return is block-uniform.
__device__ __noinline__ void solve_one(const ProbSys& S, const SolveArgs& a, double* Ld, double* P, double* sh,
                                       int* fail_flag, int32_t* status) {
  const int n = S.n;
  const int t = threadIdx.x, T = blockDim.x;
  double* H = a.H + S.h_off;
  double* y = a.delta + S.v_off;
  const double* b = a.b + S.v_off;
  double tr = 0.0;
  for (int i = t; i < n; i += T) tr += H[(int64_t)i * n + i];
  tr = block_sum(tr, sh);
  if (!(tr > 0.0)) return;  // no pair touches a free frame: nothing moves
  const double mu = S.damping_rel * tr / n;
  for (int i = t; i < n; i += T) {
    H[(int64_t)i * n + i] += mu;
    y[i] = -b[i];
  }
  if (t == 0) *fail_flag = 0;
  __syncthreads();

  // ---- blocked Cholesky, lower triangle in place
  for (int kb = 0; kb < n; kb += NB) {
    const int nb = min(NB, n - kb);
    if (t < 64) {
      const bool ok = factor_diag(H, n, kb, nb, reinterpret_cast<double(*)[NB + 1]>(Ld));
      if (t == 0 && !ok) *fail_flag = 1;
    }
    __syncthreads();
    if (*fail_flag) break;
    panel_solve(H, n, kb, nb, reinterpret_cast<double(*)[NB + 1]>(Ld));
    __syncthreads();
    if (n - (kb + nb) <= kPanelRows) {  // stage the panel in LDS for the trailing update
      for (int idx = threadIdx.x; idx < (n - kb - nb) * NB; idx += blockDim.x) {
        const int r = idx / NB, j = idx % NB;
        P[idx] = j < nb ? H[(int64_t)(kb + nb + r) * n + kb + j] : 0.0;
      }
      __syncthreads();
    }
    trailing_update(H, n, kb, nb, P);
    __syncthreads();
  }
  if (*fail_flag) {
    if (t == 0) *status = -4;
    return;
  }

  // ---- L y' = -b: diagonal blocks in wave 0, off-diagonal updates by all threads
  for (int kb = 0; kb < n; kb += NB) {
    const int nb = min(NB, n - kb);
    if (t < 64) {
      double v = t < nb ? y[kb + t] : 0.0;
      for (int j = 0; j < nb; ++j) {
        const double yj = __shfl(v, j, 64) / H[(int64_t)(kb + j) * n + kb + j];
        if (t == j) v = yj;
        else if (t > j && t < nb) v -= H[(int64_t)(kb + t) * n + kb + j] * yj;
      }
      if (t < nb) y[kb + t] = v;
    }
    __syncthreads();
    for (int i = kb + nb + t; i < n; i += T) {
      double v = y[i];
      for (int j = 0; j < nb; ++j) v -= H[(int64_t)i * n + kb + j] * y[kb + j];
      y[i] = v;
    }
    __syncthreads();
  }
  // ---- L^T delta = y'
  for (int kb = ((n - 1) / NB) * NB; kb >= 0; kb -= NB) {
    const int nb = min(NB, n - kb);
    if (t < 64) {
      double v = t < nb ? y[kb + t] : 0.0;
      for (int j = nb - 1; j >= 0; --j) {
        const double xj = __shfl(v, j, 64) / H[(int64_t)(kb + j) * n + kb + j];
        if (t == j) v = xj;
        else if (t < j) v -= H[(int64_t)(kb + j) * n + kb + t] * xj;
      }
      if (t < nb) y[kb + t] = v;
    }
    __syncthreads();
    for (int i = t; i < kb; i += T) {
      double v = y[i];
      for (int j = 0; j < nb; ++j) v -= H[(int64_t)(kb + j) * n + i] * y[kb + j];
      y[i] = v;
    }
    __syncthreads();
  }
  for (int k = t; k < n / 6; k += T)
    right_update(a.poses + 12 * (S.slot0 + frame_of_reduced(k, S.fixed)), y + 6 * k);
}

// One workgroup per problem.  A problem whose iteration count has reached
// n_iter (its last evaluation gave the final loss) is left unchanged.
__global__ __launch_bounds__(kSolveThreads) void k_solve_update(SolveArgs a) {
  __shared__ double Ld[NB * (NB + 1)];
  __shared__ double P[kPanelRows * NB];
  __shared__ double sh[kSolveThreads / 64];
  __shared__ int fail;
  const ProbSys S = a.sys[blockIdx.x];
  int32_t* st = a.state + S.state_off;
  const int iter = st[0];
  const bool run = iter < S.n_iter && st[1] == 0 && S.n > 0;
  __syncthreads();
  if (run) solve_one(S, a, Ld, P, sh, &fail, st + 1);
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
