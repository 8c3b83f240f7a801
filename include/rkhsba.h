/*
 * rkhsba -- MI355X (gfx950) library for the data-parallel hot path of RKHS-BA
 * (arXiv 2403.01254): the correspondence-free multi-frame RKHS objective, its
 * Gauss-Newton / IRLS normal equations and the pose update.
 *
 * Objective (Sec. III-B, Eq. (eq:inner_product_actual_ba)):
 *     F(T) = sum_{(m,n) in C} sum_{i,j} sigma^2 exp(-|T_m x_i - T_n z_j|^2 / (2 ell^2)) c_ij
 * with c_ij = <l(x_i), l(z_j)> the inner product of the points' pose-invariant
 * features (Sec. III-A, Eq. (eq:double_sum)), summed over the point pairs
 * inside the truncation radius r_c = cutoff_factor * ell (the double sum is
 * sparse, Sec. III-B).  The solver of Sec. V-A freezes the weights
 * w_ij = c_ij exp(-|u|^2 / (2 ell^2)) (Eq. (eq:irls_weight)), u = T_m x_i - T_n z_j,
 * and takes Gauss-Newton steps on the weighted least squares of
 * Eq. (eq:irls_final) with right perturbations T exp(eps^), eps = [rho; phi],
 * holding one frame fixed and recomputing the weights after every step.
 *
 * Conventions shared by every call
 *   - All pointers are HOST pointers unless an argument says otherwise.  The
 *     caller owns every buffer it passes; the library copies what it keeps.
 *   - pose: 12 doubles [R (3x3 row-major) | t], mapping frame-local -> world.
 *     poses: K*12 doubles, frame-major.
 *   - edges: E*2 int32 (m, n), 0-based, m != n; each listed entry is one factor
 *     F^{mn} (a duplicated entry counts twice).
 *   - b: 6K doubles, b = sum w J^T u (so grad_eps F = -(sigma^2/ell^2) b).
 *     H: (6K)^2 doubles row-major, H = sum w J^T J, J = du/d eps (Gauss-Newton
 *     matrix with the weights frozen).  Frame-major, [rho(3); phi(3)] per frame.
 *   - Every call returns an rkhsba_status; rkhsba_last_error() describes the
 *     last failure on that context.  Calls on one context must not overlap.
 *     Contexts on one device may be used from different threads, with one
 *     limit: a call that has to grow one of its context's device pools (a
 *     build, or the first solve of a larger problem) waits for the whole
 *     device, which the HIP runtime refuses while another thread's call is
 *     capturing its HIP graph (use_graphs); that call then fails with
 *     RKHSBA_EDEVICE.  Serialize such calls across threads (the request
 *     server does so for its two lanes).
 *   - Membership in the truncation radius is decided by the FP32 rule below,
 *     so the pair set is exactly reproducible on a CPU.
 *   - Values: the pair terms are FP32, from d = q32 - z of the rule.  F is
 *     their sum.  b and H take q in FP64 and move each source point's sums to
 *     d = q - z to first order in q - q32 (q32 is off by up to half an FP32
 *     ulp of |q|, which matters for points far from their frame's origin).
 *     Sums past the per-point stage run in FP64 (or Kahan FP32, option).
 *
 * FP32 membership rule (pair (i in frame m, j in frame n)):
 *   R_nm[a][b] = fma(Rn[2][a], Rm[2][b], fma(Rn[1][a], Rm[1][b], Rn[0][a]*Rm[0][b]))
 *   dt = t_m - t_n;  t_nm[a] = fma(Rn[2][a], dt[2], fma(Rn[1][a], dt[1], Rn[0][a]*dt[0]))
 *   q[a] = fma(R_nm[a][2], x[2], fma(R_nm[a][1], x[1], fma(R_nm[a][0], x[0], t_nm[a])))
 *   (all FP64, fma correctly rounded); q32 = float(q) (round to nearest even);
 *   in float: d = q32 - z; s2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx));
 *   inside iff s2 <= float(r_c * r_c), r_c = cutoff_factor * ell in FP64.
 *   With class-id features a pair also needs equal labels (c_ij = 0 otherwise).
 *
 * Voxel structure: each frame is hashed once, in its own local coordinates,
 * into cubic cells of edge r_c / cell_subdiv: k = floor(x * inv_cell) in FP64
 * with inv_cell = 1 / ((cutoff_factor * ell) / cell_subdiv), origin = min k,
 * dims = max k - min k + 1, key = ((kz-oz)*NY + (ky-oy))*NX + (kx-ox); points
 * are stably sorted by key (ties keep input order).
 */
#ifndef RKHSBA_H
#define RKHSBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkhsba_ctx rkhsba_ctx;

typedef enum {
  RKHSBA_OK = 0,
  RKHSBA_EINVAL = -1,   /* invalid argument (sizes, indices, NaN/Inf, ell <= 0, ...) */
  RKHSBA_ENOMEM = -2,   /* device allocation failed or a grid does not fit its limits */
  RKHSBA_EDEVICE = -3,  /* HIP runtime error */
  RKHSBA_ENOTPD = -4,   /* Cholesky pivot <= 0 in a Gauss-Newton step */
  RKHSBA_ESTATE = -5,   /* call out of order (e.g. no frames built yet), or a request cancelled */
  RKHSBA_EBUSY = -6     /* a served request has not finished within the wait's timeout */
} rkhsba_status;

typedef enum {
  RKHSBA_FEAT_CLASS_ID = 0,    /* one-hot labels passed as uint16 class ids (N_m values) */
  RKHSBA_FEAT_DENSE_F32 = 1,   /* dense float32 rows (N_m * D values), D <= 64 */
  RKHSBA_FEAT_DENSE_BF16 = 2,  /* float32 rows as DENSE_F32, stored rounded to bfloat16 (nearest even); inner
                                  products on the matrix cores with FP32 accumulation */
  RKHSBA_FEAT_DENSE_FP8 = 3    /* as DENSE_BF16 with OCP fp8 e4m3 storage (nearest even, saturating at 448) */
} rkhsba_feat_kind;

typedef struct {
  double ell;            /* lengthscale of Eq. (eq:kernel), > 0 */
  double cutoff_factor;  /* truncation radius r_c = cutoff_factor * ell (default 3) */
  double sigma;          /* kernel amplitude of Eq. (eq:kernel) (default 1) */
  double damping_rel;    /* GN damping mu = damping_rel * trace(H_red) / dim(H_red) (default 1e-10) */
  int fixed_frame;       /* gauge: this frame is not moved (default 0, Sec. V-A) */
  int clamp_negative_c;  /* use max(c_ij, 0) for dense features (default 1) */
  int device;            /* HIP device ordinal (default 0) */
  int cell_subdiv;       /* voxel cells per truncation radius, 1..8; 0 = chosen at each build from the
                            points per occupied r_c-cube (the table rkhsba_autotune fills, else a default
                            rule) (default 0) */
  int pass_points;       /* source points per candidate sweep: 16, 32 or 64 (8 with class ids) share one
                            walk over the cells around their box; 1 = every point walks its own cells
                            (sparse frames); 0 = chosen with cell_subdiv (default 0) */
  int moment_path;       /* 16-point sweep, Gauss-Newton moments accumulated on 0 = library choice,
                            1 = vector ALU, 2 = matrix cores (default 0) */
  int use_graphs;        /* 1 = capture one Gauss-Newton iteration in a HIP graph and replay it (default 1;
                            stage timing, when enabled, runs the launches one by one instead) */
  int hessian_fp32;      /* 1 = per-edge sums of the normal-equation terms in FP32 with Kahan compensation,
                            0 = FP64 (default) */
  int top_k;             /* 0 = every pair inside r_c (default); 1..8 = per source point and edge only the
                            top_k pairs with the largest kernel values c exp(-r^2/2 ell^2) (Sec. VI-G: eight
                            such neighbours sufficed on LiDAR), ranked in FP64 with ties broken by the
                            smaller FP32 squared distance, then the smaller original index; class ids or
                            float32 features; the per-point walks (pass_points 1) run the selection.
                            rkhsba_export_pairs lists the selected pairs. */
  void* stream;          /* hipStream_t to run on; NULL = a stream owned by the context */
} rkhsba_options;

/* Fills *opt with the defaults listed above (ell = 0.1). */
void rkhsba_default_options(rkhsba_options* opt);

/* Creates a context on opt->device.  *out is set to NULL on failure. */
int rkhsba_create(rkhsba_ctx** out, const rkhsba_options* opt);

/* Releases every device buffer of the context.  NULL is allowed. */
void rkhsba_destroy(rkhsba_ctx* ctx);

/* Text of the last failure on ctx ("" if none).  Valid until the next call on ctx. */
const char* rkhsba_last_error(const rkhsba_ctx* ctx);

/* Stages K frames (Sec. III, problem setup: point sets X_m with pose-invariant
 * features l(x), Eq. (eq:pc_function)) and builds each frame's voxel structure
 * in local coordinates.
 *   n_points: K counts (each >= 1).
 *   xyz:      K pointers to N_m*3 float32 (x,y,z rows), frame-local coordinates.
 *   feats:    K pointers: uint16 class ids (kind CLASS_ID) or N_m*D float32 rows.
 *   is_device: 0 = xyz/feats are host pointers, 1 = device pointers on ctx's
 *             device (read once on the context's stream).
 * Replaces any frames built before.  Poses are not needed here. */
int rkhsba_build_neighbors(rkhsba_ctx* ctx, int K, const int64_t* n_points, const float* const* xyz,
                           int feat_kind, int D, const void* const* feats, int is_device);

/* F at `poses` (Eq. (eq:inner_product_actual_ba), truncated), total and per
 * edge (loss_per_edge: E doubles, nullable), and the number of in-radius pairs
 * with c_ij != 0 (n_pairs, nullable). */
int rkhsba_eval_loss(rkhsba_ctx* ctx, const double* poses, int E, const int32_t* edges,
                     double* loss_total, double* loss_per_edge, int64_t* n_pairs);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): rkhsba_eval_loss on the frames built before, with the same
 * arguments, outputs and results (the same kernels; loss_per_edge, loss_total and n_pairs equal
 * rkhsba_eval_loss's), but with no device allocation and no free: the edge layout and the evaluation's
 * scratch (binning keys and values, their sort buffers, per-point sums, per-edge sums) live in a static
 * device array of 64 MiB that each GPU the library runs on holds until the process ends.  That bounds
 * one call to about 2 million (edge, source point) entries (each edge contributes its source frame's
 * point count); a call that needs more returns RKHSBA_ENOMEM with a message and changes nothing.  Host
 * bookkeeping only (no device memory) is allocated.  Every call on a GPU, from any context, shares that
 * GPU's array and overwrites what the last call left there: calls that overlap on one GPU (from two
 * threads, or on two streams whose work is in flight at once) race and must not be made. */
int rkhsba_eval_loss_noalloc(rkhsba_ctx* ctx, const double* poses, int E, const int32_t* edges,
                             double* loss_total, double* loss_per_edge, int64_t* n_pairs);

/* H (6K x 6K, full, no frame removed), b (6K) and F at `poses` (Sec. V-A,
 * normal equations of Eq. (eq:irls_final) with the weights of
 * Eq. (eq:irls_weight) frozen).  H, b, loss_total, n_pairs are nullable. */
int rkhsba_accumulate_normal_eqs(rkhsba_ctx* ctx, const double* poses, int E, const int32_t* edges,
                                 double* H, double* b, double* loss_total, int64_t* n_pairs);

/* n_iter Gauss-Newton / IRLS steps in place on poses_inout (Sec. V-A): each
 * step recomputes the weights at the current poses, solves
 * (H_red + mu I) delta = -b_red over every frame except fixed_frame (FP64
 * Cholesky on the GPU) and applies T_m <- T_m exp(delta_m^).
 * loss_per_iter (n_iter+1, nullable): F at the poses entering each step and
 * after the last; pairs_per_iter (n_iter+1, nullable): in-radius pair counts.
 * Returns RKHSBA_ENOTPD if a Cholesky pivot is not positive (poses then hold
 * the last successful step). */
int rkhsba_gn_step(rkhsba_ctx* ctx, double* poses_inout, int E, const int32_t* edges, int n_iter,
                   double* loss_per_iter, int64_t* pairs_per_iter);

/* Autotuner for the launch configuration.  Builds the frames (arguments as
 * rkhsba_build_neighbors) with every cell size in {1,2,3,4,6,8} cells per r_c
 * and every sweep size in {1,16,32,64} source points (and 8 with class ids), times `trials` normal-
 * equation evaluations of each at `poses` / `edges` (HIP events on the
 * context's stream, after one warm-up), and leaves the context built with the
 * fastest pair; outputs (nullable): that pair and its time per evaluation in
 * ms.  The choice is also recorded, for this feature layout and the frames'
 * points per occupied r_c-cube, in a process-wide table that builds with
 * cell_subdiv = 0 / pass_points = 0 consult.  Results (pair sets, F, b, H) do not depend on the
 * configuration beyond FP32 summation order. */
int rkhsba_autotune(rkhsba_ctx* ctx, int K, const int64_t* n_points, const float* const* xyz, int feat_kind, int D,
                    const void* const* feats, int is_device, const double* poses, int E, const int32_t* edges,
                    int trials, int* best_cell_subdiv, int* best_pass_points, double* best_ms);

/* The configuration of the resident frames: cells per r_c, sweep size, and
 * points per occupied r_c-cube (0 if that was not measured).  Nullable outputs. */
int rkhsba_get_config(rkhsba_ctx* ctx, int* cell_subdiv, int* pass_points, double* occupancy);

/* Lengthscale outer loop (Sec. V-C).  The RKHS distance of the graph is
 * d_H = sum over edges of <f_m,f_m> + <f_n,f_n> - 2 <f_m,f_n> (Eq. (eq:dist_rkhs),
 * truncated inner products of Eq. (eq:double_sum)); its derivative in ell is
 * sigma^2 / ell^3 times sum(W_mm + W_nn - 2 W_mn), W = sum over pairs of w r^2
 * (the truncation radius moving with ell is not differentiated).
 * rkhsba_ell_gradient returns both at `poses` and the context's lengthscale. */
int rkhsba_ell_gradient(rkhsba_ctx* ctx, const double* poses, int E, const int32_t* edges, double* d,
                        double* dd_dell);

typedef struct {
  double ell_init;     /* starting lengthscale (large: wide basin, Sec. VII) */
  double ell_min;      /* lengthscale range */
  double ell_max;
  double step;         /* fixed fractional change per outer iteration (0 < step < 1) */
  double elasticity;   /* ell shrinks when -ell (d d_H / d ell) / d_H >= elasticity, grows otherwise */
  double tol;          /* an inner loop raising F by at most tol |F| counts as converged */
  int inner_iter;      /* Gauss-Newton steps per lengthscale */
  int max_outer;       /* bound on outer iterations */
} rkhsba_ell_schedule;

/* Defaults for a base lengthscale ell: ell_init 4 ell, range [ell, 8 ell], step 0.1, elasticity 1,
 * tol 1e-6, 5 inner steps, at most 30 outer iterations. */
void rkhsba_default_ell_schedule(rkhsba_ell_schedule* s, double ell);

/* Inner-outer loop: at the current ell, inner_iter Gauss-Newton steps (as rkhsba_gn_step); then
 * d_H and its derivative at the new poses decide the fixed-percentage update of ell (elasticity
 * rule above), clamped to the range.  Stops when the clamped update leaves ell unchanged and the
 * inner loop no longer increased F (tol), or after max_outer.  The cell grid of the build is kept
 * (any lengthscale is correct on it).  poses_inout is updated; n_outer (nullable) receives the
 * outer iterations run; trace (nullable, 5 * max_outer doubles) one row per outer iteration:
 * ell, F entering and leaving its inner loop, d_H and d d_H / d ell after it.  The context's own
 * lengthscale is unchanged afterwards. */
int rkhsba_gn_lengthscale(rkhsba_ctx* ctx, double* poses_inout, int E, const int32_t* edges,
                          const rkhsba_ell_schedule* schedule, int* n_outer, double* trace);

/* Frame-to-frame tracking (Sec. III-A: the two-frame registration that
 * initialises the graph, solved by gradient ascent on the inner product of
 * Eq. (eq:double_sum)).  Frame m stays fixed; frame n moves by right
 * perturbations along grad F = -(sigma^2/ell^2) b_n (normalised) with a step
 * length s: a step is accepted when F increases (then s grows by 1.5),
 * otherwise s halves and the step is retried; the run ends after max_iter
 * accepted steps or when s drops below step_min.  step0: the first step
 * length (e.g. ell).  poses_inout: K*12, frame n's pose is updated.
 * iters (nullable): accepted steps; loss (nullable): the final F of the edge. */
int rkhsba_track(rkhsba_ctx* ctx, double* poses_inout, int m, int n, int max_iter, double step0, double step_min,
                 int* iters, double* loss);

/* Cosine alignment of frames m and n at `poses`: <f_m, f_n> / sqrt(<f_m,f_m> <f_n,f_n>)
 * (Sec. IV-A and the keyframe rule of Sec. VI-C: a new frame becomes a keyframe when
 * its alignment with the latest keyframe falls below a threshold). */
int rkhsba_cosine(rkhsba_ctx* ctx, const double* poses, int m, int n, double* cos_out);

/* The 60 rotations of the icosahedral group (Sec. IV-A: the identity, 15
 * half-turns about edge axes, 20 third-turns about face axes, 24 fifth-turns
 * about vertex axes), 9 doubles each (row-major), in the library's order. */
void rkhsba_icosahedral_rotations(double* out);

/* Global rotation initialisation of frame n against frame m (Sec. IV-A):
 * F of the edge (m, n) is evaluated with frame n's pose replaced by
 * T_n G_k, G_k(x) = R_k (x - c) + c (c = centroid of frame n's points in its
 * local coordinates), for every candidate rotation R_k -- all candidates in
 * one batched evaluation.  The norms of the two point-cloud functions do not
 * depend on the poses, so the largest F is the largest cosine alignment.
 *   rotations: n_rot row-major 3x3 (1 <= n_rot <= 4096), or NULL with n_rot 0
 *              or 60 for the icosahedral group (rkhsba_icosahedral_rotations).
 *   scores:    n_rot doubles (nullable); best: index of the largest score (the
 *              first one on ties; nullable); best_pose: 12 doubles (nullable).
 * poses: K*12 as elsewhere; only frame m's and frame n's are used. */
int rkhsba_rotation_search(rkhsba_ctx* ctx, const double* poses, int m, int n, int n_rot, const double* rotations,
                           double* scores, int* best, double* best_pose);

/* Debug/parity: the in-radius pairs of edge (m, n) at `poses` under the FP32
 * membership rule (and equal labels for class ids), as (i, j) original point
 * indices sorted by (i, j).  Writes min(total, cap) pairs to pairs (cap*2
 * int32) and the total count to *n_out. */
int rkhsba_export_pairs(rkhsba_ctx* ctx, const double* poses, int m, int n, int64_t cap, int32_t* pairs,
                        int64_t* n_out);

/* Debug/parity: how many pairs of edge (m, n) at `poses` each source point has
 * inside the truncation radius with c_ij != 0 (Eq. (eq:double_sum) truncated as
 * in Sec. III-B), as counted by the same candidate sweep (launch shape, cell
 * size, pass table) that sums them in rkhsba_accumulate_normal_eqs: the sweep
 * runs once with each source point's own count written out.  counts: N_m
 * int64, indexed by the original point index of frame m (host buffer). */
int rkhsba_export_source_counts(rkhsba_ctx* ctx, const double* poses, int m, int n, int64_t* counts);

/* Debug/parity: the voxel structure of one frame.  perm (N_m int32): sorted
 * position -> original index; keys (N_m uint32): sorted cell keys; origin[3],
 * dims[3]: the frame's cell grid (cells of edge r_c / cell_subdiv, keys
 * ((kz * NY) + ky) * NX + kx relative to the origin).  label_layers: 0, or for
 * class ids in a label-stacked frame the number of class-id layers (largest id
 * + 1); the key's z index is then id * NZ + kz, so that the points of one id
 * are contiguous.  Class ids are stacked when every frame's keys fit 32 bits
 * and the cell-row tables stay within 16 rows per point (+ 2^20).  Any pointer
 * may be NULL. */
int rkhsba_export_voxels(rkhsba_ctx* ctx, int frame, int32_t* perm, uint32_t* keys, int32_t* origin,
                         int32_t* dims, int32_t* label_layers);

/* Stage timing for measurement.  When enabled, the context brackets each
 * stage's launches with HIP events on its own stream and, at the end of every
 * call, adds the elapsed GPU time per stage.  Stages: */
enum {
  RKHSBA_PROF_BUILD = 0,       /* voxel build of rkhsba_build_neighbors */
  RKHSBA_PROF_BIN = 1,         /* relative transforms + source binning sort, per evaluation */
  RKHSBA_PROF_PAIRS = 2,       /* candidate sweep accumulating moments (Gauss-Newton evaluations) */
  RKHSBA_PROF_PAIRS_LOSS = 3,  /* candidate sweep, loss-only evaluations */
  RKHSBA_PROF_FINALIZE = 4,    /* per-point finalisation + per-edge reduction */
  RKHSBA_PROF_SOLVE = 5,       /* assembly + Cholesky + pose update */
  RKHSBA_PROF_STAGES = 6
};
int rkhsba_profile_enable(rkhsba_ctx* ctx, int on);
/* total_ms / launches (nullable) accumulated for `stage` since the last reset. */
int rkhsba_profile_read(rkhsba_ctx* ctx, int stage, double* total_ms, int64_t* launches, int reset);

/* ------------------------------------------------------------------------
 * Request loop (continuous batching of whole solves).
 *
 * A server runs one or two lanes, each a worker thread with its own engine
 * and device stream.  Each request is one multi-frame problem (its own
 * frames, edge list, ell, n_iter and initial poses) solved exactly as
 * rkhsba_gn_step solves it; with two lanes, large requests (by their
 * (edge, source point) entries) go to the second lane, so that small ones do
 * not wait for their iterations, and the lanes' batch iterations take turns
 * on the device in proportion to lane0_weight.  In a lane, requests wait in FIFO order and
 * are admitted while fewer than max_active are active in the lane and the sum
 * of the estimated device footprints of all admitted requests stays within
 * hbm_budget_bytes (one request is always admitted when its lane is idle).  Admission builds the
 * request's voxel structures into memory that stays resident until it
 * finishes; every batch iteration then advances every active request by one
 * Gauss-Newton step in shared launches (one edge table over all requests, one
 * Cholesky workgroup per request).  A request joins at the batch iteration
 * after its admission and leaves after its final loss evaluation, so the
 * requests in flight overlap on the device.  A request's result does not
 * depend on the other requests in flight beyond FP32 summation order in its
 * last loss value (the final evaluation may run with or without the
 * Gauss-Newton moments).
 */
typedef struct rkhsba_server rkhsba_server;

typedef struct {
  int device;
  int feat_kind;            /* feature kind of every request */
  int D;                    /* dense feature dimension of every request */
  int max_active;           /* requests iterating together (default 64) */
  int64_t hbm_budget_bytes; /* admission limit on the estimated footprints (0: 80% of free memory) */
  int pass_points;          /* sweep pass size for every request (0: chosen per request, default) */
  int use_graphs;           /* replay a batch iteration from a HIP graph while the active set is unchanged */
  int hessian_fp32;         /* as rkhsba_options.hessian_fp32 */
  void* stream;             /* hipStream_t of lane 0; NULL = a stream owned by the server (lane 1 always runs
                               on a stream of its own) */
  int lanes;                /* 1 or 2 concurrent batches, each with its own engine and stream (default 1) */
  int64_t lane_split_entries; /* with 2 lanes: requests with more (edge, source point) entries (sum over the edges
                               of the source frame's points) go to lane 1 (default 2,000,000) */
  int64_t lane_work_entries;  /* a lane admits the request at the head of its queue only while the entries of its
                               active requests plus the request's stay within this (0: no limit, the default; a
                               request is always admitted into an idle lane).  It bounds the work of one batch
                               iteration, which every active request of the lane waits for. */
  int lane1_max_active;     /* with 2 lanes: requests active together in lane 1 (default 1: a large request fills
                               the device alone and large requests run one after another, in the order lane1_order
                               sets, beside lane 0's batch of small ones; 0: as max_active) */
  double lane_split_work;   /* with 2 lanes: a request admitted to lane 0 whose entries times the points per
                               occupied r_c-cube that its build measured (an estimate of the candidate pairs of one
                               iteration) exceed this moves to lane 1, in arrival order (default 5e8; 0: off) */
  double lane0_weight;      /* with 2 lanes: the two lanes' batch iterations take turns on the device; while both
                               have active requests, lane 0 launches its next iteration only when its measured
                               device time divided by this weight is not ahead of lane 1's time, which caps its
                               share at w / (1 + w) (default 0.25; must be > 0) */
  int lane1_order;          /* with 2 lanes and lane1_max_active 1: 1 (default) builds up to four of lane 1's
                               waiting requests ahead while it runs one, and starts the built request whose
                               estimated service time (its entries x the points per occupied r_c-cube its build
                               measured x its evaluations, at the rate of lane 1's completed requests) less the time
                               it has waited since submission is smallest; 0 starts them in arrival order.  Results
                               do not depend on the order. */
} rkhsba_server_options;

typedef struct {
  int K;                       /* frames */
  const int64_t* n_points;     /* K counts */
  const float* const* xyz;     /* K pointers to N_m*3 float32 (frame-local) */
  const void* const* feats;    /* K pointers (class ids or N_m*D float32) */
  int is_device;               /* xyz/feats are device pointers on the server's device */
  int feat_kind, D;            /* must equal the server's */
  const double* poses;         /* K*12 initial poses (copied at submit) */
  int E;
  const int32_t* edges;        /* E*2 (copied at submit) */
  double ell, cutoff_factor, sigma, damping_rel;
  int fixed_frame;
  int clamp_negative_c;
  int cell_subdiv;             /* 1..8, or 0 = chosen from the frames' occupancy */
  int n_iter;                  /* Gauss-Newton steps */
} rkhsba_request;

typedef struct {
  int64_t submitted, completed, failed, queued;
  int64_t batch_iterations;    /* shared launches of Gauss-Newton iterations */
  int64_t max_active;          /* most requests seen in one batch iteration */
  int64_t peak_device_bytes;   /* largest engine footprint observed */
  int64_t pair_evals;          /* in-radius pairs summed over every evaluation of completed requests */
} rkhsba_server_stats;

void rkhsba_server_default_options(rkhsba_server_options* opt);
int rkhsba_server_create(rkhsba_server** out, const rkhsba_server_options* opt);
/* Stops the worker after its current batch iteration; requests still queued
 * or active finish with RKHSBA_ESTATE.  NULL is allowed. */
void rkhsba_server_destroy(rkhsba_server* srv);
/* Queues a request and returns at once with its ticket.  xyz and feats are
 * read when the request is admitted: the caller keeps them valid until
 * rkhsba_server_wait has returned for the ticket. */
int rkhsba_server_submit(rkhsba_server* srv, const rkhsba_request* req, int64_t* ticket);
/* Waits up to timeout_s seconds (< 0: no limit) for the ticket; returns the
 * request's status (RKHSBA_EBUSY on timeout, the ticket stays valid).  On
 * RKHSBA_OK / RKHSBA_ENOTPD the outputs (nullable) receive the final poses
 * (K*12), loss and pair count per evaluation (n_iter+1 each, as
 * rkhsba_gn_step), the time from submission to completion and the time spent
 * queued before admission (seconds). */
int rkhsba_server_wait(rkhsba_server* srv, int64_t ticket, double timeout_s, double* poses_out,
                       double* loss_per_iter, int64_t* pairs_per_iter, double* latency_s, double* queue_s);
int rkhsba_server_stats_get(rkhsba_server* srv, rkhsba_server_stats* out);
/* Text of the failure of the last request waited for. */
const char* rkhsba_server_last_error(const rkhsba_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RKHSBA_H */
