// Internal declarations shared by the rkhsba HIP translation units.
// Device data layout (all frames concatenated, HBM-resident between calls):
//   pts   float4[N_total]  frame-local xyz of each frame's points in cell-key order;
//                          .w holds the class id bits (class features) or 0
//   feat  float[N_total*Dp] dense feature rows in the same order (zero padded to Dp)
//   perm  int32[N_total]   sorted position -> original index within the frame
//   keys  uint32[N_total]  sorted cell keys, ((kz' * NY) + ky) * NX + kx with kz' = kz, or for class ids in a
//                          label-stacked frame kz' = label * NZ + kz (each class id has a layer of NZ cells)
//   rows  int4[sum NY*NZ*L] per (ky,kz') row of cells: (x_lo, x_hi, xtab offset, 0); L label layers (1 unstacked)
//   xtab  uint32[...]      per row, for x in [x_lo, x_hi+1]: first point of cell x
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace rkhsba {

// Binning keys: a 30-bit Morton code of the source point's target-frame cell (clamped to the grid and its
// margin), with this bit set when the point lies outside both (it has no pair).  The sort orders the code
// bits only, so a point keeps its place when a later evaluation with the same binning flips the bit.
constexpr uint32_t kInvalidBit = 0x80000000u;
constexpr int kMaxDense = 64;

enum Mode { MODE_LOSS = 0, MODE_NORMAL = 1 };
// Feature paths (values equal the public feature kinds): class ids, dense
// FP32 rows, dense rows stored in bfloat16 or fp8 e4m3 (inner products on the
// matrix cores with FP32 accumulation).
enum FeatPath { FEAT_CLASS = 0, FEAT_DENSE = 1, FEAT_BF16 = 2, FEAT_FP8 = 3 };
__host__ __device__ constexpr bool feat_low_precision(int f) { return f == FEAT_BF16 || f == FEAT_FP8; }
__host__ __device__ constexpr int feat_elem_bytes(int f) { return f == FEAT_DENSE ? 4 : f == FEAT_BF16 ? 2 : 1; }

// Per-frame grid description (device and host copies).
struct FrameInfo {
  int64_t pt_off;    // first point of the frame in pts/feat/perm/keys
  int32_t n;         // points
  int32_t org[3];    // cell coordinates of the grid origin
  int32_t dim[3];    // cells per axis
  int32_t mort_shift;  // source-binning Morton code: (k + reach) >> mort_shift
  int64_t row_off;   // first row descriptor of the frame
  int64_t xt_off;    // first xtab entry of the frame
  int32_t n_lab;     // label layers of a label-stacked frame (class id + 1 of its largest id), 0: not stacked
  int32_t key_sub;   // source-binning key resolution: 2^key_sub sub-cells per cell and axis
};

// First row descriptor (relative to row_off) of the layer of class id lbl: 0 in a frame that is not
// label-stacked, -1 where the frame has no layer for that id (no point of the frame carries it).
__host__ __device__ inline int64_t label_rows(const FrameInfo& T, uint32_t lbl) {
  if (T.n_lab <= 0) return 0;
  if (lbl >= (uint32_t)T.n_lab) return -1;
  return (int64_t)lbl * T.dim[1] * T.dim[2];
}

// Static per-edge layout of one edge list (host-computed once per list).
struct EdgeInfo {
  int32_t m, n;      // source frame, target frame
  int64_t ent_off;   // first binning entry (one per source point)
  int32_t n_src;     // source points (= frame m's count)
  int32_t pass_size; // source points per sweep pass of the edge (its problem's choice)
  int32_t n_pass;
  int32_t fin_off;   // first finalize block of the edge
  int32_t n_fin;
  int32_t fin_pt;    // entries per finalize thread (a block covers kFinThreads * fin_pt entries)
  int32_t prob;      // problem of the edge within the evaluated set (constants, system)
  int32_t pass0;     // first pass of the edge in the set's pass table
  int32_t seg0;      // first binning segment of the edge (one per class id of a label-stacked source frame,
  int32_t n_seg;     // else one): passes never straddle a segment
};

// One sweep pass: up to pass-size consecutive binning entries of one segment of an edge.
struct PassInfo {
  int64_t entry0;    // first binning entry
  int64_t src_off;   // pool offset of the source frame's points
  int32_t e;         // edge (set-wide)
  int32_t count;     // entries in the pass
  int32_t tgt;       // target frame slot
  int32_t prob;      // problem (constants)
};

// Relative transform of an edge, T_nm = T_n^-1 T_m (FP64), written on device.
struct EdgeXf {
  double R[9];
  double t[3];
};

// Kernel constants derived from the options (host-computed in FP64).
struct KConst {
  double inv_cell;   // 1 / cell edge
  double cell;       // cell edge = r_c / cell_subdiv
  double reach;      // r_c * (1 + 2^-12): covers every pair the FP32 rule accepts
  double reach2;
  float rc2;         // float(r_c * r_c), the FP32 membership threshold
  float alpha;       // log2(e) / (2 ell^2), so that exp(-r^2/2l^2) = exp2(-alpha r^2)
  int reach_cells;   // cell_subdiv + 1
  int clamp;         // clamp negative c to 0 (only set when some feature value is negative)
  int Dp;            // padded dense feature width (0 for class ids)
  int topk;          // > 0: only the topk pairs with the largest kernel values per source point (per edge)
  double inv2l2;     // 1 / (2 ell^2), for the FP64 ranking key of the topk selection
  int c_positive;    // FP32 dense features, none negative, and one dimension >= 1e-18 in every row: every
                     // inner product is > 0 (its term in that dimension is >= 1e-36, above FLT_MIN)
  float spread_limit;  // class-id sweeps: passes whose box is wider than this walk per source point
};
constexpr int kMaxTopK = 8;

// Segmented LSD radix sort: tiles never straddle a segment.
struct SortTile {
  int64_t start;     // first element
  int32_t count;     // elements (<= kSortTile)
  int32_t seg;       // segment id
  int32_t edge;      // edge of the binning entries (edge sorts), or the frame (point sorts)
  int32_t pad_;
};
struct SortSeg {
  int64_t start;
  int64_t count;
  int32_t tile0;     // first tile
  int32_t n_tiles;
};
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the first HIP error.  All run on `st`.

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                             uint32_t* hist, const SortTile* d_tiles, int n_tiles, const SortSeg* d_segs,
                             int n_segs, int bits, hipStream_t st, bool* result_in_tmp);

hipError_t launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint64_t* d_total,
                                 hipStream_t st);
constexpr int kScanTileElems = 2048;

// Padded feature row length: 8, 16, 24, 32 or 64 (FP32), 32 or 64 (bfloat16, fp8: whole 32-wide MFMA slices).
int dense_pad(int D, int feat_path);

// d_label_max (class ids, else null): per frame, the largest class id (max-combined; the caller sets -1).
hipError_t launch_cell_coords(const float* const* d_xyz_ptrs, const int64_t* d_in_off, int K, int64_t n_total,
                              double inv_cell, const void* const* d_class_ptrs, int32_t* d_cell, int32_t* d_minmax,
                              int32_t* d_label_max, hipStream_t st);
// Cell keys; frames with n_lab > 0 take the class ids (d_class_ptrs) into kz'.
hipError_t launch_cell_keys(const int32_t* d_cell, const int64_t* d_in_off, const FrameInfo* d_frames, int K,
                            int64_t n_total, const void* const* d_class_ptrs, uint32_t* d_keys, uint32_t* d_vals,
                            hipStream_t st);
// For every label-stacked frame f (frame-local key order) and class id l in [0, n_lab]: the first point
// of layer l (l = n_lab: the frame's count), at d_out[d_lab_off[f] + l].
hipError_t launch_label_starts(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_lab_off, int K,
                               int32_t* d_out, hipStream_t st);
hipError_t launch_gather(const float* const* d_xyz_ptrs, const void* const* d_feat_ptrs, int feat_kind, int D, int Dp,
                         const FrameInfo* d_frames, const int64_t* d_in_off, int K, int64_t n_total,
                         const uint32_t* d_sorted_vals, float4* d_pts, void* d_feat, int32_t* d_perm,
                         int32_t* d_neg_flag, hipStream_t st);
// Per feature dimension d < Dp (<= 64), the smallest stored FP32 value over n rows, as its bit pattern (values
// >= 0; negative values count as 0), min-combined into d_min[d], which the caller sets to +inf first.
hipError_t launch_feature_min(const float* d_feat, int64_t n, int Dp, uint32_t* d_min, hipStream_t st);
hipError_t launch_rows(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_in_off, int K,
                       int64_t n_total, int4* d_rows, int64_t n_rows, uint32_t* d_sizes, uint32_t* d_scan_tmp,
                       uint64_t* d_total, hipStream_t st);
hipError_t launch_xtab(const uint32_t* d_keys, const FrameInfo* d_frames, const int64_t* d_in_off, int K,
                       int64_t n_total, const int4* d_rows, uint32_t* d_xtab, uint32_t* d_n_cells, hipStream_t st);

// Mean of n points' xyz in FP64 (one workgroup, fixed summation order) -> out[3].
hipError_t launch_frame_centroid(const float4* d_pts, int n, double* d_out, hipStream_t st);

// The pass table of a set from its edge table: passes pass0 .. pass0 + n_pass - 1
// of each edge cover each of its segments in runs of pass_size (64 for per-point walks).
hipError_t launch_fill_passes(const EdgeInfo* d_edges, int E, const FrameInfo* d_frames, const SortSeg* d_segs,
                              PassInfo* d_passes, hipStream_t st);
hipError_t launch_edge_setup(const double* d_poses, const EdgeInfo* d_edges, int E, EdgeXf* d_xf, hipStream_t st);
// Binning keys and source indices of every entry, one block per sort tile of an edge.  rebin_sorted: the
// entries hold the sorted source indices of an earlier binning (d_vals, read only); only the keys, and with
// them the invalid bits, are recomputed at the current transforms.
hipError_t launch_bin(const float4* d_pts, const FrameInfo* d_frames, const EdgeInfo* d_edges,
                      const SortTile* d_tiles, int n_tiles, const EdgeXf* d_xf, const KConst* d_kcs, uint32_t* d_keys,
                      uint32_t* d_vals, bool rebin_sorted, hipStream_t st);

struct PairArgs {
  const float4* pts;
  const void* feat;       // feature rows (element type by feature path), Dp elements per point
  const int4* rows;
  const uint32_t* xtab;
  const FrameInfo* frames;
  const EdgeInfo* edges;
  const EdgeXf* xf;
  const uint32_t* keys;   // sorted binning keys
  const uint32_t* vals;   // sorted binning values (source point, frame-local sorted index)
  float* mom;             // moments, component-major: mom[c * n_entries + entry]
  uint32_t* cnt;          // in-radius pair count per entry
  const KConst* kcs;      // per problem of the set, indexed by EdgeInfo::prob
  const int32_t* perm;    // sorted position -> original index (ties of the topk selection)
  const PassInfo* passes; // per sweep pass
  int64_t n_entries;
  int32_t E;
  int32_t pass0;          // first pass of this launch in the pass table
  int32_t n_pass;         // passes of this launch
  KConst kc;              // set-wide: Dp and clamp (clamping is exact for non-negative features)
  int32_t stacked;        // every frame of the set is label-stacked (class ids): a candidate of the pass's
                          // layer always carries the pass's class id, and the sweeps skip that test
};
// Passes of pass_points sources: 1 = each lane walks its own point's cells,
// 8 (class ids) and 16 (launch_sweep), 32, 64 = shared walk over the pass's box.
hipError_t launch_pairs(const PairArgs& a, int mode, int feat_path, int pass_points, bool topk, hipStream_t st);

// Tiled sweep for passes of 16 sources, or 8 with class ids.  source_counts (Gauss-Newton moments on the
// VALU only): each entry of a.cnt receives its own source point's pair count instead of the pass total on
// the pass's first entry (the per-edge sums are the same).
hipError_t launch_sweep(const PairArgs& a, int mode, int feat_path, int pass_points, bool matrix_moments,
                        bool source_counts, hipStream_t st);

struct FinArgs {
  const float4* pts;
  const EdgeInfo* edges;
  const EdgeXf* xf;
  const FrameInfo* frames;
  const uint32_t* keys;
  const uint32_t* vals;
  const float* mom;
  const uint32_t* cnt;
  const KConst* kcs;      // per problem of the set, indexed by EdgeInfo::prob
  double* partial;        // [n_fin_total][kFinStats]
  int64_t n_entries;
  int32_t E;
  int32_t n_fin_total;
};
constexpr int kEdgeVals = 93;  // F, b_m(6), b_n(6), H_mm(21), H_nn(21), H_mn(36), pair count, sum w r^2
constexpr int kFinThreads = 256;
constexpr int kFinStats = 40;  // per-edge sums the normal-equation blocks are expanded from, sum w r^2, F, pair count
// fp32_sums: per-point terms and their sums in FP32 with Kahan compensation,
// else FP64.  Pair counts are summed in FP64.
hipError_t launch_finalize(const FinArgs& a, const int32_t* d_fin_off, int mode, bool fp32_sums, hipStream_t st);
hipError_t launch_edge_reduce(const double* d_partial, const EdgeInfo* d_edges, const EdgeXf* d_xf, int E, int mode,
                              bool fp32_sums, double* d_edge_out, hipStream_t st);

// One problem's Gauss-Newton system within an evaluated set.
struct ProbSys {
  int32_t K;          // frames
  int32_t fixed;      // frame removed from the system (-1: none)
  int32_t n;          // system size: 6K, or 6(K-1) with a fixed frame
  int32_t e0, E;      // edges of the problem in the set's edge table
  int32_t blk0;       // first entry of the problem's K*K+1 block-contributor starts
  int32_t vec0;       // first entry of the problem's K+1 vector-contributor starts
  int32_t n_iter;     // Gauss-Newton iterations; solves stop once iter reaches it
  int64_t slot0;      // first frame slot (frame table, poses)
  int64_t h_off;      // offset of the problem's n x n matrix in the set's H buffer
  int64_t v_off;      // offset of its n-vectors in b and delta
  int64_t hist_off;   // offset of its loss and pair-count histories (n_iter + 1 each)
  int64_t state_off;  // offset of its (iter, status) pair
  double sigma2;
  double damping_rel;
};

struct SolveArgs {
  const double* edge_out;  // [E][kEdgeVals]
  const ProbSys* sys;      // [n_prob]
  int32_t n_prob;
  int32_t n_max;           // largest system size of the set
  double* H;
  double* b;
  double* delta;
  double* poses;           // [slot][12], updated in place by the solve
  double* loss_hist;       // F per evaluation, at hist_off + iter
  double* pairs_hist;      // in-radius pair count per evaluation
  int32_t* state;          // per problem: iter (evaluations whose solve ran), status (0 ok, -4 not PD; sticky)
  // contributors of each 6x6 block (frame a, frame c) of a problem's H, CSR over blk0 + a*K + c:
  // entries e*4 + role (set-wide edge index), role 0 H_mm, 1 H_nn, 2 H_mn, 3 H_mn^T
  const int32_t* blk_start;
  const int32_t* blk_list;
  // contributors of each frame's 6-vector of b, CSR over vec0 + a: entries e*2 + role, role 0 b_m, 1 b_n
  const int32_t* vec_start;
  const int32_t* vec_list;
};
// Writes H, b of every problem (and the loss / pair-count history entry of the
// current iteration).
hipError_t launch_assemble(const SolveArgs& a, hipStream_t st);
// Loss / pair-count history entry only (loss evaluations).
hipError_t launch_loss_only(const SolveArgs& a, hipStream_t st);
// Damped Cholesky solve and pose update of every problem whose iteration count
// is below its n_iter; advances the iteration count of every problem.
hipError_t launch_solve_update(const SolveArgs& a, hipStream_t st);

// out[0] = sum of F, out[1] = sum of pair counts over the E per-edge rows of edge_out (edge order).
hipError_t launch_edge_totals(const double* d_edge_out, int E, double* d_out, hipStream_t st);

hipError_t launch_export_pairs(const float4* d_pts, const int4* d_rows, const uint32_t* d_xtab,
                               const FrameInfo* d_frames, int n_src, const int32_t* d_perm, const void* d_feat,
                               const EdgeXf* d_xf, int m, int n, int feat_path, KConst kc, int64_t cap, int32_t* d_out,
                               unsigned long long* d_count, hipStream_t st);

}  // namespace rkhsba
