// Normal-equation assembly, FP64 Cholesky solve and SE(3) pose update of one
// Gauss-Newton / IRLS step (Sec. V-A): with the weights frozen, the step
// solves (H_red + mu I) delta = -b_red over every frame except the fixed one
// and moves T_m <- T_m exp(delta_m^) (right perturbation, eps = [rho; phi]).
// Single-workgroup kernels: the system is 6(K-1) <= a few hundred unknowns.
#include "rkhsba_device.h"

namespace rkhsba {
namespace {

constexpr int kSolveThreads = 256;

__device__ inline int sym_index(int r, int c) {
  if (r > c) { const int t = r; r = c; c = t; }
  return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

__device__ inline int reduced(int frame, int fixed) {
  if (fixed < 0) return frame;
  return frame == fixed ? -1 : (frame < fixed ? frame : frame - 1);
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

// Scatters the per-edge blocks into the dense system (rows/columns of the
// fixed frame dropped when fixed >= 0).  Edges are added one after another,
// so the sums are deterministic.  Also records F (times sigma^2) and the pair
// count of this evaluation.
__global__ __launch_bounds__(kSolveThreads) void k_assemble(SolveArgs a) {
  const int Kr = a.fixed >= 0 ? a.K - 1 : a.K;
  const int n = 6 * Kr;
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) a.H[i] = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a.b[i] = 0.0;
  __syncthreads();
  const int t = threadIdx.x;
  for (int e = 0; e < a.E; ++e) {
    const double* v = a.edge_out + (int64_t)e * kEdgeVals;
    const int rm = reduced(a.edges[e].m, a.fixed), rn = reduced(a.edges[e].n, a.fixed);
    if (t < 36) {
      const int r = t / 6, c = t % 6;
      const double mm = v[13 + sym_index(r, c)], nn = v[34 + sym_index(r, c)], mn = v[55 + 6 * r + c];
      if (rm >= 0) a.H[(int64_t)(6 * rm + r) * n + 6 * rm + c] += mm;
      if (rn >= 0) a.H[(int64_t)(6 * rn + r) * n + 6 * rn + c] += nn;
      if (rm >= 0 && rn >= 0) {
        a.H[(int64_t)(6 * rm + r) * n + 6 * rn + c] += mn;
        a.H[(int64_t)(6 * rn + c) * n + 6 * rm + r] += mn;
      }
    } else if (t < 42) {
      if (rm >= 0) a.b[6 * rm + t - 36] += v[1 + t - 36];
    } else if (t < 48) {
      if (rn >= 0) a.b[6 * rn + t - 42] += v[7 + t - 42];
    }
    __syncthreads();
  }
  if (t == 0) {
    double F = 0.0, np = 0.0;
    for (int e = 0; e < a.E; ++e) {
      F += a.edge_out[(int64_t)e * kEdgeVals];
      np += a.edge_out[(int64_t)e * kEdgeVals + 91];
    }
    if (a.loss_hist) a.loss_hist[a.iter] = a.sigma2 * F;
    if (a.pairs_hist) a.pairs_hist[a.iter] = np;
  }
}

// Loss-only evaluation: F and the pair count from the per-edge sums.
__global__ void k_loss_only(SolveArgs a) {
  if (threadIdx.x != 0) return;
  double F = 0.0, np = 0.0;
  for (int e = 0; e < a.E; ++e) {
    F += a.edge_out[(int64_t)e * kEdgeVals];
    np += a.edge_out[(int64_t)e * kEdgeVals + 91];
  }
  if (a.loss_hist) a.loss_hist[a.iter] = a.sigma2 * F;
  if (a.pairs_hist) a.pairs_hist[a.iter] = np;
}

// T <- T exp(xi^): closed-form SE(3) exponential (Rodrigues for the rotation,
// V = I + B K + C K^2 for the translation), series for small angles.
__device__ void right_update(double* T, const double* xi) {
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

// Damped Cholesky solve of the reduced system and pose update.  A failed
// factorisation sets *status = -4 and leaves the poses untouched; once set,
// later steps do nothing.
__global__ __launch_bounds__(kSolveThreads) void k_solve_update(SolveArgs a) {
  __shared__ double sh[kSolveThreads / 64];
  __shared__ int fail;
  if (*a.status != 0) return;
  const int n = 6 * (a.K - 1);
  const int t = threadIdx.x, T = blockDim.x;
  double* H = a.H;
  double* y = a.delta;
  double tr = 0.0;
  for (int i = t; i < n; i += T) tr += H[(int64_t)i * n + i];
  tr = block_sum(tr, sh);
  if (!(tr > 0.0)) return;  // no pair touches a free frame: nothing moves
  const double mu = a.damping_rel * tr / n;
  for (int i = t; i < n; i += T) {
    H[(int64_t)i * n + i] += mu;
    y[i] = -a.b[i];
  }
  if (t == 0) fail = 0;
  __syncthreads();
  // right-looking Cholesky, lower triangle in place
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      const double d = H[(int64_t)j * n + j];
      if (d > 0.0) H[(int64_t)j * n + j] = sqrt(d);
      else fail = 1;
    }
    __syncthreads();
    if (fail) break;
    const double ljj = H[(int64_t)j * n + j];
    for (int i = j + 1 + t; i < n; i += T) H[(int64_t)i * n + j] /= ljj;
    __syncthreads();
    const int m = n - j - 1;
    for (int idx = t; idx < m * m; idx += T) {
      const int i = j + 1 + idx / m, k = j + 1 + idx % m;
      if (k <= i) H[(int64_t)i * n + k] -= H[(int64_t)i * n + j] * H[(int64_t)k * n + j];
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) *a.status = -4;
    return;
  }
  // L y' = -b  (column-oriented forward substitution)
  for (int j = 0; j < n; ++j) {
    if (t == 0) y[j] /= H[(int64_t)j * n + j];
    __syncthreads();
    const double yj = y[j];
    for (int i = j + 1 + t; i < n; i += T) y[i] -= H[(int64_t)i * n + j] * yj;
    __syncthreads();
  }
  // L^T delta = y'
  for (int j = n - 1; j >= 0; --j) {
    if (t == 0) y[j] /= H[(int64_t)j * n + j];
    __syncthreads();
    const double xj = y[j];
    for (int i = t; i < j; i += T) y[i] -= H[(int64_t)j * n + i] * xj;
    __syncthreads();
  }
  for (int k = t; k < a.K - 1; k += T) {
    const int f = k < a.fixed ? k : k + 1;
    right_update(a.poses + 12 * f, y + 6 * k);
  }
}

}  // namespace

hipError_t launch_assemble(const SolveArgs& a, hipStream_t st) {
  k_assemble<<<1, kSolveThreads, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_solve_update(const SolveArgs& a, hipStream_t st) {
  k_solve_update<<<1, kSolveThreads, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_loss_only(const SolveArgs& a, hipStream_t st) {
  k_loss_only<<<1, 64, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rkhsba
