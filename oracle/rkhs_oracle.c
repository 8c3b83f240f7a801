/*
 * FP64 CPU oracle for the RKHS-BA hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow restatement of the paper's definitions, written to be checked
 * by eye against the paper: brute force over every point pair, or (search
 * mode) a world-coordinate cell list that visits a superset of the pairs
 * inside the truncation radius.  Only tests/, the smoke check and the
 * benchmark's CPU-baseline leg use it; it shares no code with the GPU library.
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math).
 *
 * Paper: arXiv 2403.01254, Sec. III (representation and objective) and
 * Sec. V-A (IRLS solver).
 */
#include "rkhs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ small linear algebra */

static void pose_split(const double* T, double R[3][3], double t[3]) {
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) R[a][b] = T[3 * a + b];
    t[a] = T[9 + a];
  }
}

static void apply(const double R[3][3], const double t[3], const double x[3], double y[3]) {
  for (int a = 0; a < 3; ++a) y[a] = R[a][0] * x[0] + R[a][1] * x[1] + R[a][2] * x[2] + t[a];
}

/* [v]_x, the matrix with [v]_x y = v x y. */
static void skew(const double v[3], double S[3][3]) {
  S[0][0] = 0.0;   S[0][1] = -v[2]; S[0][2] = v[1];
  S[1][0] = v[2];  S[1][1] = 0.0;   S[1][2] = -v[0];
  S[2][0] = -v[1]; S[2][1] = v[0];  S[2][2] = 0.0;
}

static void mat3_mul(const double A[3][3], const double B[3][3], double C[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[a][b] = A[a][0] * B[0][b] + A[a][1] * B[1][b] + A[a][2] * B[2][b];
}

/* Jacobian of u = T_m x - T_n z w.r.t. the right perturbation T exp(eps^),
 * eps = [rho; phi] (Sec. V-A):  d(R (x + phi x x + rho) + t)/d eps = R [I | -[x]_x].
 * sign = +1 for the frame carrying x (u = +T x ...), -1 for the frame carrying z. */
static void jacobian(const double R[3][3], const double x[3], double sign, double J[3][6]) {
  double S[3][3], RS[3][3];
  skew(x, S);
  mat3_mul(R, S, RS);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      J[a][b] = sign * R[a][b];
      J[a][3 + b] = -sign * RS[a][b];
    }
}

/* ------------------------------------------------------------------ FP32 membership rule */

/* The documented FP32 rule deciding whether a pair lies inside the truncation
 * radius.  Relative transform T_nm = T_n^-1 T_m in FP64 with this exact
 * operation order (fma = fused multiply-add, correctly rounded):
 *   R_nm[a][b] = fma(Rn[2][a], Rm[2][b], fma(Rn[1][a], Rm[1][b], Rn[0][a]*Rm[0][b]))
 *   dt = t_m - t_n
 *   t_nm[a]    = fma(Rn[2][a], dt[2], fma(Rn[1][a], dt[1], Rn[0][a]*dt[0]))
 *   q[a]       = fma(R_nm[a][2], x[2], fma(R_nm[a][1], x[1], fma(R_nm[a][0], x[0], t_nm[a])))
 *   q32 = round-to-nearest float(q)
 * then in float: d = q32 - z; s2 = fmaf(dz,dz, fmaf(dy,dy, dx*dx)); in iff
 * s2 <= float(r_c * r_c). */
static void rule_relative(const double* Tm, const double* Tn, double Rnm[3][3], double tnm[3]) {
  double Rm[3][3], tm[3], Rn[3][3], tn[3], dt[3];
  pose_split(Tm, Rm, tm);
  pose_split(Tn, Rn, tn);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      Rnm[a][b] = fma(Rn[2][a], Rm[2][b], fma(Rn[1][a], Rm[1][b], Rn[0][a] * Rm[0][b]));
  for (int k = 0; k < 3; ++k) dt[k] = tm[k] - tn[k];
  for (int a = 0; a < 3; ++a) tnm[a] = fma(Rn[2][a], dt[2], fma(Rn[1][a], dt[1], Rn[0][a] * dt[0]));
}

static void rule_q32(const double Rnm[3][3], const double tnm[3], const float* x, float q32[3]) {
  for (int a = 0; a < 3; ++a) {
    double q = fma(Rnm[a][2], (double)x[2], fma(Rnm[a][1], (double)x[1], fma(Rnm[a][0], (double)x[0], tnm[a])));
    q32[a] = (float)q;
  }
}

static int rule_inside(const float q32[3], const float* z, float rc2_32) {
  float dx = q32[0] - z[0], dy = q32[1] - z[1], dz = q32[2] - z[2];
  float s2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  return s2 <= rc2_32;
}

/* ------------------------------------------------------------------ label inner product */

/* c_ij = <l(x_i), l(z_j)> (Sec. III-A, Eq. (eq:double_sum)).  Class ids are
 * one-hot vectors, whose inner product is 1 for equal labels and 0 otherwise. */
static double label_product(const oracle_problem* P, int m, int64_t i, int n, int64_t j) {
  if (P->feat_kind == ORACLE_FEAT_CLASS) {
    const uint16_t* lm = (const uint16_t*)P->feats[m];
    const uint16_t* ln = (const uint16_t*)P->feats[n];
    return lm[i] == ln[j] ? 1.0 : 0.0;
  }
  const float* fm = (const float*)P->feats[m] + i * P->D;
  const float* fn = (const float*)P->feats[n] + j * P->D;
  double c = 0.0;
  for (int k = 0; k < P->D; ++k) c += (double)fm[k] * (double)fn[k];
  if (P->clamp_negative_c && c < 0.0) c = 0.0;
  return c;
}

/* ------------------------------------------------------------------ cell-list neighbour search */

/* The truncation radius makes the double sum of Eq. (eq:double_sum) sparse
 * (Sec. III-B): a pair farther apart than r_c adds nothing.  With search =
 * ORACLE_SEARCH_CELLS an edge's target points are hashed, in WORLD
 * coordinates at the current poses, into cubic cells of edge h slightly above
 * r_c, and each source point visits only the targets of the 27 cells around
 * its own.  Every pair the membership test can accept is among them, so the
 * sums are those of the brute-force search up to the order of summation
 * (cells in a fixed order, targets by ascending index within a cell).
 *
 * h = r_c (1 + 2^-10) + 2^-20 (M + r_c), M the largest absolute local
 * coordinate of the target frame: the FP32 rule's rounding of q and of the
 * squared distance moves a pair's decision by at most ~2^-22 r_c + 2^-23 (M + r_c),
 * and the FP64 world coordinates by far less, so an accepted pair is always
 * less than h apart in every axis and its cells differ by at most one. */
#define CELL_BITS 21
#define CELL_HALF (1LL << (CELL_BITS - 1))

typedef struct {
  double inv_h;
  int64_t n_runs;
  int64_t* order;  /* target indices sorted by (cell key, index) */
  int64_t* start;  /* n_runs + 1: first position of each cell's run in order */
  uint64_t* key;   /* cell key of each run */
  int64_t* slot;   /* open addressing table: run index, or -1 */
  uint64_t mask;
} cell_list;

typedef struct {
  uint64_t key;
  int64_t j;
} keyed_index;

static int cmp_keyed_index(const void* pa, const void* pb) {
  const keyed_index* a = (const keyed_index*)pa;
  const keyed_index* b = (const keyed_index*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return a->j < b->j ? -1 : (a->j > b->j ? 1 : 0);
}

/* 1 and the packed key of cell (cx, cy, cz) if every coordinate fits CELL_BITS bits, else 0. */
static int cell_key(int64_t cx, int64_t cy, int64_t cz, uint64_t* key) {
  if (cx < -CELL_HALF || cx >= CELL_HALF || cy < -CELL_HALF || cy >= CELL_HALF || cz < -CELL_HALF ||
      cz >= CELL_HALF)
    return 0;
  *key = ((uint64_t)(cx + CELL_HALF) << (2 * CELL_BITS)) | ((uint64_t)(cy + CELL_HALF) << CELL_BITS) |
         (uint64_t)(cz + CELL_HALF);
  return 1;
}

static uint64_t mix64(uint64_t x) { /* splitmix64 finaliser */
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ULL;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

static void cell_of_point(const cell_list* cl, const double w[3], int64_t c[3]) {
  for (int a = 0; a < 3; ++a) c[a] = (int64_t)floor(w[a] * cl->inv_h);
}

/* Cell list of the world points Wz (N rows of 3); h from r_c and the target's local coordinates Z.
 * Returns 0, or -1 when a cell coordinate does not fit the key. */
static int cell_list_build(cell_list* cl, const double* Wz, const float* Z, int64_t N, double rc) {
  double M = 0.0;
  for (int64_t i = 0; i < 3 * N; ++i) M = fmax(M, fabs((double)Z[i]));
  const double h = rc * (1.0 + ldexp(1.0, -10)) + ldexp(M + rc, -20);
  cl->inv_h = 1.0 / h;
  keyed_index* ki = (keyed_index*)malloc(sizeof(keyed_index) * (size_t)(N > 0 ? N : 1));
  for (int64_t j = 0; j < N; ++j) {
    int64_t c[3];
    cell_of_point(cl, Wz + 3 * j, c);
    if (!cell_key(c[0], c[1], c[2], &ki[j].key)) {
      free(ki);
      return -1;
    }
    ki[j].j = j;
  }
  qsort(ki, (size_t)N, sizeof(keyed_index), cmp_keyed_index);
  cl->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
  cl->start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  cl->key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N > 0 ? N : 1));
  int64_t runs = 0;
  for (int64_t p = 0; p < N; ++p) {
    cl->order[p] = ki[p].j;
    if (p == 0 || ki[p].key != ki[p - 1].key) {
      cl->start[runs] = p;
      cl->key[runs] = ki[p].key;
      ++runs;
    }
  }
  cl->start[runs] = N;
  cl->n_runs = runs;
  uint64_t size = 16;
  while (size < 2 * (uint64_t)runs) size <<= 1;
  cl->mask = size - 1;
  cl->slot = (int64_t*)malloc(sizeof(int64_t) * size);
  for (uint64_t s = 0; s < size; ++s) cl->slot[s] = -1;
  for (int64_t r = 0; r < runs; ++r) {
    uint64_t s = mix64(cl->key[r]) & cl->mask;
    while (cl->slot[s] >= 0) s = (s + 1) & cl->mask;
    cl->slot[s] = r;
  }
  free(ki);
  return 0;
}

static void cell_list_free(cell_list* cl) {
  free(cl->order);
  free(cl->start);
  free(cl->key);
  free(cl->slot);
}

/* Targets in the 27 cells around world point w, appended to out (capacity N); returns their count. */
static int64_t cell_list_gather(const cell_list* cl, const double w[3], int64_t* out) {
  int64_t c[3], n = 0;
  cell_of_point(cl, w, c);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        uint64_t key;
        if (!cell_key(c[0] + dx, c[1] + dy, c[2] + dz, &key)) continue;
        uint64_t s = mix64(key) & cl->mask;
        for (; cl->slot[s] >= 0; s = (s + 1) & cl->mask) {
          const int64_t r = cl->slot[s];
          if (cl->key[r] != key) continue;
          for (int64_t p = cl->start[r]; p < cl->start[r + 1]; ++p) out[n++] = cl->order[p];
          break;
        }
      }
  return n;
}

/* ------------------------------------------------------------------ loss, gradient, GN matrix */

typedef struct {
  double F, bm[6], bn[6], Hmm[36], Hnn[36], Hmn[36];
  double W;  /* sum of w |u|^2: the ell-derivative of the factor is sigma^2 W / ell^3 */
  int64_t pairs;
} edge_acc;

static int check_problem(const oracle_problem* P) {
  if (!P || P->K < 1 || !P->n_points || !P->xyz || !P->feats) return -1;
  if (!(P->ell > 0.0) || !(P->cutoff_factor > 0.0)) return -1;
  if (P->feat_kind != ORACLE_FEAT_CLASS && (P->feat_kind != ORACLE_FEAT_DENSE || P->D < 1)) return -1;
  if (P->search != ORACLE_SEARCH_BRUTE && P->search != ORACLE_SEARCH_CELLS) return -1;
  return 0;
}

static int check_edges(const oracle_problem* P, int E, const int32_t* edges) {
  if (E < 0 || (E > 0 && !edges)) return -1;
  for (int e = 0; e < E; ++e) {
    int m = edges[2 * e], n = edges[2 * e + 1];
    if (m < 0 || n < 0 || m >= P->K || n >= P->K || m == n) return -1;
  }
  return 0;
}

#define ORACLE_CHUNK 256

/* One kept pair (i, j) of an edge: w = c exp(-r^2 / 2 ell^2) and the terms
 * it adds to F, W, b and H (see edge_terms). */
static void add_pair(edge_acc* a, double s2sig, double inv_2l2, const double Jm[3][6], const double Rn[3][3],
                     const float* zj, const double u[3], double r2, double c) {
  double w = c * exp(-r2 * inv_2l2);
  a->F += s2sig * w;
  a->W += w * r2;
  a->pairs += 1;
  double z[3] = {zj[0], zj[1], zj[2]};
  double Jn[3][6];
  jacobian(Rn, z, -1.0, Jn);
  for (int r = 0; r < 6; ++r) {
    double gm = 0.0, gn = 0.0;
    for (int k = 0; k < 3; ++k) {
      gm += Jm[k][r] * u[k];
      gn += Jn[k][r] * u[k];
    }
    a->bm[r] += w * gm;
    a->bn[r] += w * gn;
    for (int s = 0; s < 6; ++s) {
      double mm = 0.0, nn = 0.0, mn = 0.0;
      for (int k = 0; k < 3; ++k) {
        mm += Jm[k][r] * Jm[k][s];
        nn += Jn[k][r] * Jn[k][s];
        mn += Jm[k][r] * Jn[k][s];
      }
      a->Hmm[6 * r + s] += w * mm;
      a->Hnn[6 * r + s] += w * nn;
      a->Hmn[6 * r + s] += w * mn;
    }
  }
}

/* ------------------------------------------------------------------ top-k truncation */

/* Per-point truncation of the Time-Analysis paragraph of Sec. VI: each source
 * point keeps only the top_k pairs with the largest kernel values.  The
 * ranking value is the pair's weight c exp(-r^2 / 2 ell^2); only pairs inside
 * the truncation radius with c > 0 are candidates.  Which pairs are kept is
 * an integer decision, so with the FP32 membership rule it is taken on the
 * rule's quantities: c rounded to float (class ids: 1; dense features: a
 * float fused multiply-add chain in element order, clamped at 0 when
 * negative c are clamped), s2 the rule's float squared distance, value
 * (double)c * exp(-(double)s2 / 2 ell^2).  With FP64 membership the value
 * uses the FP64 c and r^2.  Equal values: smaller squared distance first,
 * then the smaller target index j. */
typedef struct {
  double key, s2;
  int64_t j;
} candidate;

static int candidate_order(const void* pa, const void* pb) {
  const candidate* a = (const candidate*)pa;
  const candidate* b = (const candidate*)pb;
  if (a->key != b->key) return a->key > b->key ? -1 : 1;
  if (a->s2 != b->s2) return a->s2 < b->s2 ? -1 : 1;
  return a->j < b->j ? -1 : (a->j > b->j ? 1 : 0);
}

static float label_product_f32(const oracle_problem* P, int m, int64_t i, int n, int64_t j) {
  if (P->feat_kind == ORACLE_FEAT_CLASS) {
    const uint16_t* lm = (const uint16_t*)P->feats[m];
    const uint16_t* ln = (const uint16_t*)P->feats[n];
    return lm[i] == ln[j] ? 1.0f : 0.0f;
  }
  const float* fm = (const float*)P->feats[m] + i * P->D;
  const float* fn = (const float*)P->feats[n] + j * P->D;
  float c = 0.0f;
  for (int k = 0; k < P->D; ++k) c = fmaf(fm[k], fn[k], c);
  if (P->clamp_negative_c) c = fmaxf(c, 0.0f);
  return c;
}

/* Ranking candidate of pair (i, j); returns 0 when the pair is no candidate. */
static int make_candidate(const oracle_problem* P, int m, int64_t i, int n, int64_t j, int membership,
                          const float q32[3], double r2, double inv_2l2, candidate* out) {
  if (membership == ORACLE_MEMBER_FP32_RULE) {
    const float* z = P->xyz[n] + 3 * j;
    float dx = q32[0] - z[0], dy = q32[1] - z[1], dz = q32[2] - z[2];
    float s2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float c = label_product_f32(P, m, i, n, j);
    if (!(c > 0.0f)) return 0;
    out->key = (double)c * exp(-(double)s2 * inv_2l2);
    out->s2 = (double)s2;
  } else {
    double c = label_product(P, m, i, n, j);
    if (!(c > 0.0)) return 0;
    out->key = c * exp(-r2 * inv_2l2);
    out->s2 = r2;
  }
  out->j = j;
  return 1;
}

/* One edge (m, n): the factor F^{mn} = sum_ij h(T_m x_i, T_n z_j) c_ij of
 * Eq. (eq:inner_product_actual_ba) over the pairs inside the truncation
 * radius (the sparsity remark of Sec. III-B), with
 *   h = sigma^2 exp(-|u|^2 / (2 ell^2))          Eq. (eq:kernel)
 *   w = c_ij exp(-|u|^2 / (2 ell^2))             Eq. (eq:irls_weight)
 *   u = T_m x_i - T_n z_j                        residual d(.,.) of Sec. V-A
 * and the IRLS normal-equation terms of Eq. (eq:irls_final) with the weights
 * frozen: b += w J^T u, H += w J^T J, J = du/d[eps_m, eps_n].  With top_k > 0
 * only each source point's top_k pairs (see make_candidate) are summed. */
static int edge_terms(const oracle_problem* P, const double* poses, int m, int n, int membership,
                      edge_acc* out) {
  const int64_t Nm = P->n_points[m], Nn = P->n_points[n];
  const float* X = P->xyz[m];
  const float* Z = P->xyz[n];
  double Rm[3][3], tm[3], Rn[3][3], tn[3];
  pose_split(poses + 12 * m, Rm, tm);
  pose_split(poses + 12 * n, Rn, tn);
  const double rc = P->cutoff_factor * P->ell;
  const double rc2 = rc * rc;
  const float rc2_32 = (float)rc2;
  const double inv_2l2 = 1.0 / (2.0 * P->ell * P->ell);
  const double s2sig = P->sigma * P->sigma;
  const int top_k = P->top_k;
  double Rnm[3][3], tnm[3];
  rule_relative(poses + 12 * m, poses + 12 * n, Rnm, tnm);

  /* world coordinates of the target points, computed once per edge */
  double* Wz = (double*)malloc(sizeof(double) * 3 * (size_t)(Nn > 0 ? Nn : 1));
  for (int64_t j = 0; j < Nn; ++j) {
    double z[3] = {Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]};
    apply(Rn, tn, z, Wz + 3 * j);
  }
  const int cells = P->search == ORACLE_SEARCH_CELLS;
  cell_list cl;
  if (cells && cell_list_build(&cl, Wz, Z, Nn, rc)) {
    free(Wz);
    return -1;
  }
  const int64_t n_chunks = (Nm + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
  edge_acc* acc = (edge_acc*)calloc((size_t)(n_chunks > 0 ? n_chunks : 1), sizeof(edge_acc));

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ch = 0; ch < n_chunks; ++ch) {
    edge_acc a;
    memset(&a, 0, sizeof(a));
    candidate* cand = top_k > 0 ? (candidate*)malloc(sizeof(candidate) * (size_t)(Nn > 0 ? Nn : 1)) : NULL;
    int64_t* near = cells ? (int64_t*)malloc(sizeof(int64_t) * (size_t)(Nn > 0 ? Nn : 1)) : NULL;
    const int64_t i1 = (ch + 1) * ORACLE_CHUNK < Nm ? (ch + 1) * ORACLE_CHUNK : Nm;
    for (int64_t i = ch * ORACLE_CHUNK; i < i1; ++i) {
      double x[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
      double p[3];
      apply(Rm, tm, x, p);
      float q32[3];
      rule_q32(Rnm, tnm, X + 3 * i, q32);
      double Jm[3][6];
      jacobian(Rm, x, +1.0, Jm);
      int64_t nc = 0;
      /* brute force: every target point; cell list: the targets of the 27 cells around p */
      const int64_t n_near = cells ? cell_list_gather(&cl, p, near) : Nn;
      for (int64_t t = 0; t < n_near; ++t) {
        const int64_t j = cells ? near[t] : t;
        const double* q = Wz + 3 * j;
        double u[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
        double r2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        int inside = membership == ORACLE_MEMBER_FP32_RULE ? rule_inside(q32, Z + 3 * j, rc2_32) : (r2 <= rc2);
        if (!inside) continue;
        if (top_k > 0) {
          nc += make_candidate(P, m, i, n, j, membership, q32, r2, inv_2l2, cand + nc);
          continue;
        }
        double c = label_product(P, m, i, n, j);
        if (c == 0.0) continue;
        add_pair(&a, s2sig, inv_2l2, Jm, Rn, Z + 3 * j, u, r2, c);
      }
      if (top_k > 0) {
        qsort(cand, (size_t)nc, sizeof(candidate), candidate_order);
        for (int64_t t = 0; t < nc && t < top_k; ++t) {
          const int64_t j = cand[t].j;
          const double* q = Wz + 3 * j;
          double u[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
          double r2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
          add_pair(&a, s2sig, inv_2l2, Jm, Rn, Z + 3 * j, u, r2, label_product(P, m, i, n, j));
        }
      }
    }
    free(cand);
    free(near);
    acc[ch] = a;
  }
  if (cells) cell_list_free(&cl);
  /* chunks summed in a fixed order: the result does not depend on the thread count */
  memset(out, 0, sizeof(*out));
  for (int64_t ch = 0; ch < n_chunks; ++ch) {
    out->F += acc[ch].F;
    out->W += acc[ch].W;
    out->pairs += acc[ch].pairs;
    for (int r = 0; r < 6; ++r) {
      out->bm[r] += acc[ch].bm[r];
      out->bn[r] += acc[ch].bn[r];
    }
    for (int r = 0; r < 36; ++r) {
      out->Hmm[r] += acc[ch].Hmm[r];
      out->Hnn[r] += acc[ch].Hnn[r];
      out->Hmn[r] += acc[ch].Hmn[r];
    }
  }
  free(acc);
  free(Wz);
  return 0;
}

/* Per-edge F and W = sum w |u|^2 (no sigma^2).  An edge may pair a frame with
 * itself: that is the self inner product <f_X, f_X> of the RKHS distance,
 * Eq. (eq:dist_rkhs), whose pair (i, i) has u = 0. */
int oracle_edge_sums(const oracle_problem* P, const double* poses, int E, const int32_t* edges, int membership,
                     double* F_edge, double* W_edge) {
  if (check_problem(P) || !poses || E < 0 || (E > 0 && !edges)) return -1;
  for (int e = 0; e < E; ++e) {
    const int m = edges[2 * e], n = edges[2 * e + 1];
    if (m < 0 || n < 0 || m >= P->K || n >= P->K) return -1;
    edge_acc a;
    if (edge_terms(P, poses, m, n, membership, &a)) return -2;
    if (F_edge) F_edge[e] = a.F;
    if (W_edge) W_edge[e] = a.W;
  }
  return 0;
}

int oracle_normal_eqs(const oracle_problem* P, const double* poses, int E, const int32_t* edges,
                      int membership, double* F, double* b, double* H, double* F_edge, int64_t* n_pairs) {
  if (check_problem(P) || !poses || check_edges(P, E, edges)) return -1;
  const int K = P->K, n6 = 6 * K;
  double Ftot = 0.0;
  int64_t ptot = 0;
  if (b) memset(b, 0, sizeof(double) * n6);
  if (H) memset(H, 0, sizeof(double) * (size_t)n6 * n6);
  for (int e = 0; e < E; ++e) {
    const int m = edges[2 * e], n = edges[2 * e + 1];
    edge_acc a;
    if (edge_terms(P, poses, m, n, membership, &a)) return -2;
    Ftot += a.F;
    ptot += a.pairs;
    if (F_edge) F_edge[e] = a.F;
    if (b)
      for (int r = 0; r < 6; ++r) {
        b[6 * m + r] += a.bm[r];
        b[6 * n + r] += a.bn[r];
      }
    if (H)
      for (int r = 0; r < 6; ++r)
        for (int s = 0; s < 6; ++s) {
          H[(size_t)(6 * m + r) * n6 + 6 * m + s] += a.Hmm[6 * r + s];
          H[(size_t)(6 * n + r) * n6 + 6 * n + s] += a.Hnn[6 * r + s];
          H[(size_t)(6 * m + r) * n6 + 6 * n + s] += a.Hmn[6 * r + s];
          H[(size_t)(6 * n + s) * n6 + 6 * m + r] += a.Hmn[6 * r + s];
        }
  }
  if (F) *F = Ftot;
  if (n_pairs) *n_pairs = ptot;
  return 0;
}

/* ------------------------------------------------------------------ SE(3) exponential, Cholesky */

void oracle_se3_exp(const double* xi, double* T) {
  const double* rho = xi;
  const double* phi = xi + 3;
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) { /* Taylor series of sin(t)/t, (1-cos t)/t^2, (t-sin t)/t^3 */
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  double S[3][3], S2[3][3];
  skew(phi, S);
  mat3_mul(S, S, S2);
  double V[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double I = a == b ? 1.0 : 0.0;
      T[3 * a + b] = I + A * S[a][b] + B * S2[a][b];
      V[a][b] = I + B * S[a][b] + C * S2[a][b];
    }
  for (int a = 0; a < 3; ++a) T[9 + a] = V[a][0] * rho[0] + V[a][1] * rho[1] + V[a][2] * rho[2];
}

int oracle_cholesky_solve(int n, const double* A, const double* b, double* x) {
  if (n < 0) return -1;
  double* L = (double*)calloc((size_t)(n > 0 ? n : 1) * (n > 0 ? n : 1), sizeof(double));
  double* y = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  int status = 0;
  for (int j = 0; j < n && !status; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0)) {
      status = -4;
      break;
    }
    const double ljj = sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = s / ljj;
    }
  }
  if (!status) {
    for (int i = 0; i < n; ++i) { /* L y = b */
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
      y[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) { /* L^T x = y */
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
      x[i] = s / L[(size_t)i * n + i];
    }
  }
  free(L);
  free(y);
  return status;
}

/* ------------------------------------------------------------------ Gauss-Newton / IRLS */

/* Sec. V-A: with the weights w frozen, Eq. (eq:irls_gradient) is the
 * stationarity condition of the weighted least squares Eq. (eq:irls_final);
 * one Gauss-Newton step solves (H + mu I) delta = -b over every frame but the
 * fixed one and moves T_m <- T_m exp(delta_m^).  The weights are recomputed
 * from the new poses before the next step. */
int oracle_gn(const oracle_problem* P, double* poses, int E, const int32_t* edges, int n_iter,
              int fixed_frame, double damping_rel, int membership, double* loss_per_iter, double* pose_trace) {
  if (check_problem(P) || !poses || check_edges(P, E, edges) || n_iter < 0) return -1;
  if (fixed_frame < 0 || fixed_frame >= P->K || damping_rel < 0.0) return -1;
  const int K = P->K, n6 = 6 * K, nr = 6 * (K - 1);
  double* b = (double*)malloc(sizeof(double) * n6);
  double* H = (double*)malloc(sizeof(double) * (size_t)n6 * n6);
  double* Hr = (double*)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1) * (nr > 0 ? nr : 1));
  double* br = (double*)malloc(sizeof(double) * (nr > 0 ? nr : 1));
  double* dr = (double*)malloc(sizeof(double) * (nr > 0 ? nr : 1));
  int* frame_of = (int*)malloc(sizeof(int) * (K > 1 ? K - 1 : 1));
  for (int m = 0, k = 0; m < K; ++m)
    if (m != fixed_frame) frame_of[k++] = m;
  int status = 0;
  for (int it = 0; it <= n_iter; ++it) {
    double F;
    status = oracle_normal_eqs(P, poses, E, edges, membership, &F, b, H, NULL, NULL);
    if (status) break;
    if (loss_per_iter) loss_per_iter[it] = F;
    if (pose_trace) memcpy(pose_trace + (size_t)it * 12 * K, poses, sizeof(double) * 12 * K);
    if (it == n_iter || nr == 0) continue;
    double tr = 0.0;
    for (int r = 0; r < nr; ++r) {
      const int gr = 6 * frame_of[r / 6] + r % 6;
      br[r] = -b[gr];
      for (int s = 0; s < nr; ++s) Hr[(size_t)r * nr + s] = H[(size_t)gr * n6 + 6 * frame_of[s / 6] + s % 6];
      tr += Hr[(size_t)r * nr + r];
    }
    if (tr == 0.0) continue; /* no pair at all: nothing moves */
    const double mu = damping_rel * tr / nr;
    for (int r = 0; r < nr; ++r) Hr[(size_t)r * nr + r] += mu;
    status = oracle_cholesky_solve(nr, Hr, br, dr);
    if (status) break;
    for (int k = 0; k < K - 1; ++k) {
      double* T = poses + 12 * frame_of[k];
      double Ex[12], R[3][3], t[3], Re[3][3], te[3], Rn[3][3];
      oracle_se3_exp(dr + 6 * k, Ex);
      pose_split(T, R, t);
      pose_split(Ex, Re, te);
      mat3_mul(R, Re, Rn);
      double tn[3];
      apply(R, t, te, tn);
      for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) T[3 * a + c] = Rn[a][c];
        T[9 + a] = tn[a];
      }
    }
  }
  free(b); free(H); free(Hr); free(br); free(dr); free(frame_of);
  return status;
}

/* ------------------------------------------------------------------ neighbour list */

static int cmp_i64(const void* pa, const void* pb) {
  const int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
  return a < b ? -1 : (a > b ? 1 : 0);
}

int64_t oracle_pairs(const oracle_problem* P, const double* poses, int m, int n, int64_t cap, int32_t* pairs) {
  if (check_problem(P) || !poses || m < 0 || n < 0 || m >= P->K || n >= P->K || m == n || cap < 0) return -1;
  const int64_t Nm = P->n_points[m], Nn = P->n_points[n];
  const float* X = P->xyz[m];
  const float* Z = P->xyz[n];
  const double rc = P->cutoff_factor * P->ell;
  const float rc2_32 = (float)(rc * rc);
  const double inv_2l2 = 1.0 / (2.0 * P->ell * P->ell);
  double Rnm[3][3], tnm[3];
  rule_relative(poses + 12 * m, poses + 12 * n, Rnm, tnm);
  /* cell search: the targets' world coordinates at the given poses */
  const int cells = P->search == ORACLE_SEARCH_CELLS;
  double Rm[3][3], tm[3], Rn[3][3], tn[3];
  pose_split(poses + 12 * m, Rm, tm);
  pose_split(poses + 12 * n, Rn, tn);
  cell_list cl;
  if (cells) {
    double* Wz = (double*)malloc(sizeof(double) * 3 * (size_t)(Nn > 0 ? Nn : 1));
    for (int64_t j = 0; j < Nn; ++j) {
      double z[3] = {Z[3 * j], Z[3 * j + 1], Z[3 * j + 2]};
      apply(Rn, tn, z, Wz + 3 * j);
    }
    const int bad = cell_list_build(&cl, Wz, Z, Nn, rc);
    free(Wz);
    if (bad) return -1;
  }
  int64_t* cnt = (int64_t*)calloc((size_t)(Nm + 1), sizeof(int64_t));
  const uint16_t* lm = (const uint16_t*)P->feats[m];
  const uint16_t* ln = (const uint16_t*)P->feats[n];
  const int classes = P->feat_kind == ORACLE_FEAT_CLASS;
  for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel
    {
      int64_t* near = (int64_t*)malloc(sizeof(int64_t) * (size_t)(Nn > 0 ? Nn : 1));
      candidate* cand = P->top_k > 0 ? (candidate*)malloc(sizeof(candidate) * (size_t)(Nn > 0 ? Nn : 1)) : NULL;
#pragma omp for schedule(dynamic, 64)
      for (int64_t i = 0; i < Nm; ++i) {
        float q32[3];
        rule_q32(Rnm, tnm, X + 3 * i, q32);
        /* candidate targets: all of them, or those of the 27 cells around the source's world point */
        int64_t n_near = Nn;
        if (cells) {
          double x[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]}, p[3];
          apply(Rm, tm, x, p);
          n_near = cell_list_gather(&cl, p, near);
        }
        int64_t c = 0, o = pass ? cnt[i] : 0;
        if (P->top_k > 0) { /* the top_k candidates of make_candidate, listed by j */
          for (int64_t t = 0; t < n_near; ++t) {
            const int64_t j = cells ? near[t] : t;
            if (rule_inside(q32, Z + 3 * j, rc2_32))
              c += make_candidate(P, m, i, n, j, ORACLE_MEMBER_FP32_RULE, q32, 0.0, inv_2l2, cand + c);
          }
          qsort(cand, (size_t)c, sizeof(candidate), candidate_order);
          if (c > P->top_k) c = P->top_k;
          for (int64_t t = 0; t < c; ++t) near[t] = cand[t].j;
        } else {
          for (int64_t t = 0; t < n_near; ++t) {
            const int64_t j = cells ? near[t] : t;
            if (!rule_inside(q32, Z + 3 * j, rc2_32)) continue;
            if (classes && lm[i] != ln[j]) continue;
            near[c++] = j; /* c <= t: overwrites only entries already read */
          }
        }
        qsort(near, (size_t)c, sizeof(int64_t), cmp_i64);
        for (int64_t t = 0; pass && t < c; ++t)
          if (o + t < cap) {
            pairs[2 * (o + t)] = (int32_t)i;
            pairs[2 * (o + t) + 1] = (int32_t)near[t];
          }
        if (!pass) cnt[i] = c;
      }
      free(cand);
      free(near);
    }
    if (!pass) { /* exclusive prefix sum: output offset of each source point */
      int64_t s = 0;
      for (int64_t i = 0; i < Nm; ++i) {
        int64_t c = cnt[i];
        cnt[i] = s;
        s += c;
      }
      cnt[Nm] = s;
    }
  }
  if (cells) cell_list_free(&cl);
  const int64_t total = cnt[Nm];
  free(cnt);
  return total;
}

/* ------------------------------------------------------------------ voxel structure */

typedef struct {
  uint32_t key;
  int32_t idx;
} key_idx;

static int cmp_key_idx(const void* a, const void* b) {
  const key_idx* x = (const key_idx*)a;
  const key_idx* y = (const key_idx*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

int oracle_voxels(const float* xyz, const uint16_t* labels, int64_t N, double inv_cell, int margin,
                  int32_t* perm, uint32_t* keys, int32_t* origin, int32_t* dims) {
  if (N < 1 || N > 0x7fffffff || !(inv_cell > 0.0) || margin < 0) return -1;
  int64_t lo[3], hi[3];
  int64_t* k = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)N);
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) {
      k[3 * i + a] = (int64_t)floor((double)xyz[3 * i + a] * inv_cell);
      if (i == 0 || k[3 * i + a] < lo[a]) lo[a] = k[3 * i + a];
      if (i == 0 || k[3 * i + a] > hi[a]) hi[a] = k[3 * i + a];
    }
  int64_t d[3], total = 1;
  for (int a = 0; a < 3; ++a) {
    d[a] = hi[a] - lo[a] + 1 + 2 * (int64_t)margin;
    total *= d[a];
    origin[a] = (int32_t)(lo[a] - margin);
    dims[a] = (int32_t)d[a];
  }
  int64_t layers = 1;
  if (labels)
    for (int64_t i = 0; i < N; ++i)
      if ((int64_t)labels[i] + 1 > layers) layers = (int64_t)labels[i] + 1;
  if (total * layers >= 0xffffffffLL) {
    free(k);
    return -1;
  }
  key_idx* ki = (key_idx*)malloc(sizeof(key_idx) * (size_t)N);
  for (int64_t i = 0; i < N; ++i) {
    int64_t kx = k[3 * i] - origin[0], ky = k[3 * i + 1] - origin[1], kz = k[3 * i + 2] - origin[2];
    if (labels) kz += (int64_t)labels[i] * d[2];
    ki[i].key = (uint32_t)((kz * d[1] + ky) * d[0] + kx);
    ki[i].idx = (int32_t)i;
  }
  qsort(ki, (size_t)N, sizeof(key_idx), cmp_key_idx);
  for (int64_t p = 0; p < N; ++p) {
    perm[p] = ki[p].idx;
    keys[p] = ki[p].key;
  }
  free(ki);
  free(k);
  return 0;
}
