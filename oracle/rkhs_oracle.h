/*
 * FP64 CPU oracle for the RKHS-BA hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It is a plain, slow, brute-force restatement of the
 * paper's definitions and shares no code with the GPU library.
 *
 * Paper: "RKHS-BA: A Robust Correspondence-Free Multi-View Bundle Adjustment
 * Framework for Semantic Point Clouds" (arXiv 2403.01254).
 *
 * Conventions
 *   pose      12 doubles, [R row-major 3x3 | t], maps frame-local -> world
 *   edge      (m, n) int32: one factor F^{mn} of Eq. (eq:inner_product_all)
 *   tangent   eps = [rho; phi], right perturbation T exp(eps^) (Sec. V-A)
 *   b         6K vector  sum w J^T u          (grad F = -(sigma^2/ell^2) b)
 *   H         6K x 6K    sum w J^T J          (Gauss-Newton matrix of the
 *                                              IRLS cost, Eq. (eq:irls_final))
 */
#ifndef RKHS_ORACLE_H
#define RKHS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_FEAT_CLASS = 0, ORACLE_FEAT_DENSE = 1 };
enum { ORACLE_MEMBER_FP64 = 0, ORACLE_MEMBER_FP32_RULE = 1 };
/* Neighbour search: every point pair (the definition), or the targets of the
 * 27 world-coordinate cells around each source point (same pairs, sums in
 * another order; see rkhs_oracle.c). */
enum { ORACLE_SEARCH_BRUTE = 0, ORACLE_SEARCH_CELLS = 1 };

typedef struct {
  int K;                       /* frames */
  const int64_t* n_points;     /* K */
  const float* const* xyz;     /* K pointers to N_m*3 floats (frame-local) */
  int feat_kind;               /* ORACLE_FEAT_* */
  int D;                       /* dense feature dimension (ignored for class ids) */
  const void* const* feats;    /* K pointers: uint16 ids or N_m*D floats */
  double ell;                  /* lengthscale */
  double cutoff_factor;        /* truncation radius r_c = cutoff_factor * ell */
  double sigma;                /* kernel amplitude */
  int clamp_negative_c;        /* use max(c, 0) */
  int top_k;                   /* > 0: each source point keeps its top_k largest-weight pairs */
  int search;                  /* ORACLE_SEARCH_* */
} oracle_problem;

/* Loss F, b and H at `poses` (K*12), over every point pair of every edge
 * (or, with the cell search, over each source point's 27 nearby cells).  membership: ORACLE_MEMBER_FP64 keeps pairs with r^2 <= r_c^2
 * in FP64 (the definition); ORACLE_MEMBER_FP32_RULE keeps the pairs of the
 * documented FP32 membership rule.  b, H, F_edge, n_pairs may be NULL.
 * Returns 0, -1 on invalid arguments, or -2 when a world coordinate is too
 * far out for the cell list's keys (cell search only). */
int oracle_normal_eqs(const oracle_problem* P, const double* poses, int E, const int32_t* edges,
                      int membership, double* F, double* b, double* H, double* F_edge, int64_t* n_pairs);

/* Per-edge F and W = sum over the kept pairs of w |u|^2 (u the world residual,
 * w = c exp(-|u|^2 / 2 ell^2), no sigma^2).  Edges may be self-pairs (m == n).
 * F_edge, W_edge: E doubles (nullable).  Returns 0, -1, or -2 (as oracle_normal_eqs). */
int oracle_edge_sums(const oracle_problem* P, const double* poses, int E, const int32_t* edges, int membership,
                     double* F_edge, double* W_edge);

/* n_iter Gauss-Newton / IRLS steps in place on poses (frame `fixed_frame`
 * untouched).  loss_per_iter (n_iter+1, nullable) receives F at the poses
 * entering each step and after the last one; pose_trace ((n_iter+1)*K*12,
 * nullable) the poses at the same points.  Returns 0, -1 invalid,
 * -2 (as oracle_normal_eqs), -4 Cholesky failure. */
int oracle_gn(const oracle_problem* P, double* poses, int E, const int32_t* edges, int n_iter,
              int fixed_frame, double damping_rel, int membership, double* loss_per_iter, double* pose_trace);

/* Point pairs (i, j) (original indices, i in frame m, j in frame n) kept by
 * the FP32 membership rule, in (i, j) order.  With class ids only pairs of
 * equal labels are listed; with top_k > 0 only each source point's top_k
 * pairs (c > 0, ranked by weight).  Writes at most cap pairs, returns the total
 * count (or -1).  The list does not depend on the search mode. */
int64_t oracle_pairs(const oracle_problem* P, const double* poses, int m, int n, int64_t cap, int32_t* pairs);

/* Voxel structure of one frame: cell coordinates k = floor(x * inv_cell)
 * (FP64), grid origin = min k - margin, dims = max k - min k + 1 + 2 margin,
 * linear key ((kz-oz)*NY + (ky-oy))*NX + (kx-ox), points stably sorted by
 * key.  With class ids (labels != NULL) the frame is label-stacked: the z
 * index becomes label*NZ + (kz-oz), one layer of NZ cells per class id.
 * Outputs perm (sorted position -> original index), sorted keys, and
 * origin[3], dims[3] (the geometric grid).  Returns 0 or -1 (keys would not
 * fit 32 bits). */
int oracle_voxels(const float* xyz, const uint16_t* labels, int64_t N, double inv_cell, int margin,
                  int32_t* perm, uint32_t* keys, int32_t* origin, int32_t* dims);

/* SE(3) exponential of xi = [rho; phi] (closed form); T: 12 doubles. */
void oracle_se3_exp(const double* xi, double* T);

/* Solve A x = b for symmetric positive definite A (n x n row-major) by
 * Cholesky.  Returns 0, or -4 when a pivot is not positive. */
int oracle_cholesky_solve(int n, const double* A, const double* b, double* x);

#ifdef __cplusplus
}
#endif
#endif
