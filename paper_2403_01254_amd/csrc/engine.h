// Host-side engine of the rkhsba library: resident frame storage for any
// number of problems (sets of frames with their own length scale, grids and
// poses), the per-set work layout, and the launch sequence of one
// evaluation / Gauss-Newton iteration over every problem of a set.
//
// Storage.  Every problem's points, features, cell tables and poses live in
// device pools shared by all resident problems.  A pool is a growable device
// array whose sub-ranges are handed out first-fit; growing it copies the
// contents, so element offsets stay valid and the kernels address every
// problem through the same base pointers (FrameInfo holds pool offsets).
//
// Sets.  An evaluation runs over a set of (problem, edge list) items: one
// edge table over all items (each edge knows its problem), one launch per
// stage for the whole set, and one Gauss-Newton system per problem, solved by
// one workgroup each.  A set's launch sequence can be captured once in a HIP
// graph and replayed for every iteration while the set is unchanged.
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "rkhsba_internal.h"

namespace rkhsba {

// Error raised by engine code; the C ABI turns it into a status code.
struct Fail {
  int code;
  std::string msg;
};

[[noreturn]] void throw_hip(hipError_t e, const char* what);

#define RK_HIP(expr)                                           \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) ::rkhsba::throw_hip(e_, #expr);      \
  } while (0)

#define RK_REQUIRE(cond, code, msg)                            \
  do {                                                         \
    if (!(cond)) throw ::rkhsba::Fail{(code), (msg)};          \
  } while (0)

// Device buffer that grows on demand; contents are not preserved.  A buffer
// can instead view caller-provided device memory (attach): it is then never
// freed or grown.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  bool owned = true;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    n = 0;
    owned = true;
  }
  void attach(T* ptr, size_t count) {
    release();
    p = ptr;
    n = count;
    owned = false;
  }
  hipError_t reserve(size_t count) {
    if (count == 0) count = 1;
    if (count <= n) return hipSuccess;
    if (!owned) return hipErrorOutOfMemory;  // a view does not grow
    release();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = count;
    return hipSuccess;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Consecutive 256-byte aligned pieces of one caller-provided device region.
struct Arena {
  uint8_t* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  int mom_components = 10;  // moments per entry the evaluations need (1 for loss-only evaluations)
  template <typename T>
  T* take(size_t count) {
    if (count == 0) count = 1;
    const size_t off = (used + 255) & ~(size_t)255;
    if (off + count * sizeof(T) > cap) return nullptr;
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base + off);
  }
};

// Per-evaluation device scratch of an engine: relative transforms, binning
// keys and values (and their sort buffers), moments, pair counts, partial and
// per-edge sums, and the assembled systems.
struct EvalScratch {
  DBuf<EdgeXf> xf;
  DBuf<uint32_t> bk, bv, bk2, bv2, bhist;
  DBuf<float> mom;
  DBuf<uint32_t> cnt;
  DBuf<double> partial, edge_out;
  DBuf<double> H, b, delta;
};

// First-fit allocator of element ranges [0, capacity).
class RangeAlloc {
 public:
  int64_t alloc(int64_t n);  // -1 when no free range is large enough
  void free(int64_t off, int64_t n);
  void grow(int64_t new_cap);
  int64_t capacity() const { return cap_; }
  int64_t used() const { return used_; }
  int64_t largest_free() const;

 private:
  std::map<int64_t, int64_t> free_;  // offset -> length, disjoint, coalesced
  int64_t cap_ = 0;
  int64_t used_ = 0;
};

// A set of device arrays sharing one range allocator (element i of every
// array belongs to the same owner).  Growth preserves contents and offsets.
class Pool {
 public:
  explicit Pool(std::vector<size_t> elem_bytes) : eb_(std::move(elem_bytes)), ptr_(eb_.size(), nullptr) {}
  Pool(const Pool&) = delete;
  Pool& operator=(const Pool&) = delete;
  ~Pool();
  // Offset of n fresh elements; grows (copying on `st`, then synchronising it) when needed.
  int64_t alloc(int64_t n, hipStream_t st);
  void free(int64_t off, int64_t n) { ra_.free(off, n); }
  void* ptr(int i) const { return ptr_[i]; }
  int64_t capacity() const { return ra_.capacity(); }
  int64_t used() const { return ra_.used(); }
  size_t bytes() const;
  // Changes the element size of array i; only while the pool is empty.
  void set_elem_bytes(int i, size_t b);
  uint64_t generation() const { return gen_; }  // bumped whenever a base pointer changes

 private:
  std::vector<size_t> eb_;
  std::vector<void*> ptr_;
  RangeAlloc ra_;
  uint64_t gen_ = 0;
};

struct ProbParams {
  double ell = 0.1;
  double cutoff_factor = 3.0;
  double sigma = 1.0;
  double damping_rel = 1e-10;
  int fixed_frame = 0;
  int clamp_negative_c = 1;
  int cell_subdiv = 8;   // cells per r_c, 1..8 (0: chosen at the build)
  int pass_points = 16;  // sweep pass size: 1 (per-point walks), 16, 32, 64 (0: chosen at the build)
  int top_k = 0;         // > 0: keep the top_k largest-kernel pairs per source point (per-point walks)
};

// One resident problem: its frames, their voxel structures and poses.
struct Problem {
  int id = -1;
  ProbParams par;
  KConst kc{};
  bool negative_features = false;
  bool c_positive = false;  // every inner product of the features is > 0 (KConst::c_positive)
  int K = 0;
  int64_t N = 0;
  int64_t slot0 = -1;   // frame slots (frame table and poses)
  int64_t pbase = -1;   // point pool range [pbase, pbase + N)
  int64_t rbase = -1, n_rows = 0;
  int64_t xbase = -1, n_xt = 0;
  int64_t hbase = -1, n_hist = 0;   // history pool range (loss, pair count per evaluation)
  int64_t sbase = -1;               // state pool entry (iter, status)
  int bin_bits = 3;
  bool stacked = false;             // class ids stacked into label layers in every frame (FrameInfo::n_lab)
  std::vector<int64_t> lab_off;     // per frame: first entry of its layer starts in lab_start
  std::vector<int32_t> lab_start;   // per stacked frame, n_lab + 1 entries: first point of each layer
  std::vector<FrameInfo> frames;    // pool offsets
  std::vector<int64_t> n_points;
  int64_t resident_bytes = 0;       // pool bytes held by the problem
  // aliases: extra frame slots sharing one frame's resident points, each with its own pose
  // (local frame indices K .. K + n_alias - 1); used to evaluate a batch of candidate poses
  int kc_version = 0;               // bumped when the constants change (lengthscale updates)
  int alias_of = -1, n_alias = 0;
  int64_t alias_slot0 = -1;
  double occupancy = 0.0;           // points per occupied cell of the problem's grid
  double occupancy_r = 0.0;         // points per occupied cell of edge r_c (0: not measured)
};

// One item of an evaluated set.
struct SetItem {
  Problem* p;
  const int32_t* edges;  // E pairs of problem-local frame indices
  int E;
  int fixed;             // frame removed from the system (-1: none)
  int n_iter;            // Gauss-Newton iterations (history length n_iter + 1)
  bool allow_self = false;  // evaluation-only sets may pair a frame with itself (m == n)
};

// Work layout of a set (rebuilt when the set changes).
struct SetLayout {
  std::vector<int> ids;             // problem ids, in item order
  std::vector<int32_t> edge_key;    // pass size, problem ids, edge lists, fixed, n_iter (change detection)
  uint64_t gen = 0;                 // pool generation the tables were built for
  int n_prob = 0, n_max = 0, E = 0;
  int64_t n_entries = 0;
  int n_pass_total = 0, n_fin_total = 0, n_edge_tiles = 0, n_edge_segs = 0, bin_bits = 3;
  bool stacked = false;             // every problem of the set is label-stacked
  struct Group {
    int pass_points, pass0, n_pass;
    bool topk;
  };
  std::vector<Group> groups;        // contiguous runs of the pass table, one sweep launch each
  bool clamp = false;
  bool c_positive = false;          // every problem's inner products are > 0 (pair counts need no c != 0 test)
  DBuf<EdgeInfo> d_edges;
  DBuf<int64_t> d_ent_off;
  DBuf<int32_t> d_fin_off;
  DBuf<SortTile> d_etiles;
  DBuf<SortSeg> d_esegs;
  DBuf<KConst> d_kcs;
  DBuf<PassInfo> d_passes;
  DBuf<ProbSys> d_sys;
  DBuf<int32_t> d_blk_start, d_blk_list, d_vec_start, d_vec_list;
  std::vector<ProbSys> sys;         // host copy
  int64_t h_total = 0, v_total = 0;
  // graph of one Gauss-Newton iteration over the set
  hipGraphExec_t graph = nullptr;
  uint64_t graph_gen = 0;
  int graph_mode = -1;
  int uses = 0;                     // iterate() calls since the layout was built
  // the binning (sorted entries) of the layout's last full binning, while the scratch still holds it
  bool binned = false;
  uint64_t bin_gen = 0;             // scratch generation it was written under
  const void* bin_sc = nullptr;     // scratch set it lives in
  const uint32_t* bin_k = nullptr;
  const uint32_t* bin_v = nullptr;
  hipGraphExec_t graph_rest = nullptr;  // iterations after the first of an iterate() call (binning reused)
  uint64_t graph_rest_gen = 0;
  // pinned staging of the host tables' uploads, free again once stage_ev has completed
  uint8_t* stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
  ~SetLayout();
  void drop_graph();
  // The staging buffer, at least `bytes` large, once its previous uploads are done (nullptr when no_alloc
  // and it is too small).
  uint8_t* stage_for(size_t bytes, bool no_alloc);
};

class Engine {
 public:
  Engine(int device, hipStream_t stream, int moment_path);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  int device;
  hipStream_t st;
  hipStream_t build_st = nullptr;  // stream of add_problem's work (nullptr: st); st waits for a build's end
  int moment_path;
  bool use_graphs = true;
  int graph_min_uses = 1;  // iterate(lay, 1) captures a graph once the layout has been used this often
  bool fp32_sums = false;  // per-edge normal-equation sums in FP32 with Kahan compensation (else FP64)
  bool source_counts = false;  // sweeps write every source point's own pair count (parity checks)

  // feature layout shared by all resident problems
  int feat_kind = -1, D = 0, Dp = 0;

  // Builds the voxel structures of a new problem from K clouds (host or
  // device pointers) and keeps it resident.  Returns its id.
  int add_problem(const ProbParams& par, int K, const int64_t* n_points, const float* const* xyz, int kind, int D,
                  const void* const* feats, bool is_device);
  // As add_problem; cell_subdiv == 0 picks the cell size from the occupancy
  // of a first build with cells of edge r_c (tuned table, else a default rule).
  int add_problem_auto(const ProbParams& par, int K, const int64_t* n_points, const float* const* xyz, int kind,
                       int D, const void* const* feats, bool is_device);
  // (cell_subdiv, pass_points) for frames with this many points per occupied r_c-cube
  std::pair<int, int> choose_config(double occupancy_r) const;
  void tune_record(double occupancy_r, int subdiv, int pass_points);  // process-wide tuned table
  void remove_problem(int id);
  Problem* problem(int id);
  int n_problems() const { return (int)probs_.size(); }
  // Bytes the engine holds in HBM (pools, set buffers, build scratch).
  int64_t device_bytes() const;
  // Resident pool bytes a problem of this shape is expected to hold (admission estimate).
  int64_t estimate_problem_bytes(int K, const int64_t* n_points, int E) const {
    return estimate_bytes(K, n_points, E, feat_row_bytes());
  }
  // The same estimate for a given feature row size (bytes per point), without engine state.
  static int64_t estimate_bytes(int K, const int64_t* n_points, int E, int64_t row_bytes);
  // The resident (pool) part of estimate_bytes; a built problem's resident_bytes replaces it.
  static int64_t estimate_resident_bytes(int K, const int64_t* n_points, int64_t row_bytes);

  void upload_poses(Problem* p, const double* poses);   // host K*12
  // count alias slots of `frame` with the given host poses (count*12); replaces earlier aliases
  void set_aliases(Problem* p, int frame, int count, const double* poses);
  void clear_aliases(Problem* p);
  // New lengthscale on the existing grid: r_c, the reach (and the reach in cells) and the kernel
  // scale follow ell; the cells keep their size (correct for any ell, fastest near the build's).
  void set_ell(Problem* p, double ell);
  // FP64 centroid of a frame's local coordinates (fixed summation order)
  void frame_centroid(Problem* p, int frame, double c[3]);
  void download_poses(Problem* p, double* poses);       // host K*12 (synchronises the stream)
  void ensure_history(Problem* p, int n_iter);
  void reset_state(Problem* p);                          // iter = 0, status = 0 (stream-ordered copy)

  // Set layout for the items (cached in `lay`; rebuilt when the items change).
  void prepare(SetLayout& lay, const std::vector<SetItem>& items);
  // Allocation-free evaluations: while an arena is set, prepare() places the layout's tables and the
  // per-evaluation scratch in it (no device allocation; a layout too large for it fails with
  // RKHSBA_ENOMEM), skips the loss histories, and graphs and stage timing are off.  The layout must
  // be one used only under this arena; it is rebuilt on every prepare().
  void set_arena(Arena* a);
  // One evaluation of every item of the set at the device poses: per-edge sums in edge_out.
  // reuse_binning: keep the order of the layout's last binning (its passes stay spatially compact while
  // the poses move a little) and only recompute which sources fall outside their target grids; done in
  // full when the scratch no longer holds that binning.
  void evaluate(SetLayout& lay, int mode, bool reuse_binning = false);
  // Assembly (+ history entry) of every problem.
  void assemble(SetLayout& lay);
  // Damped solve + pose update of every problem still iterating.
  void solve(SetLayout& lay);
  // History entry only (after a loss evaluation).
  void loss_only(SetLayout& lay);
  // n Gauss-Newton iterations (evaluate, assemble, solve) over the set; graph-replayed when enabled.
  void iterate(SetLayout& lay, int n, bool continue_binning = false);
  SolveArgs solve_args(SetLayout& lay);

  // results
  void read_history(Problem* p, int count, double* loss, double* pairs);  // synchronises
  // Queues copies of the poses (K*12), `count` history entries and the (iter, status) pair to host
  // memory (pinned, for the copies to be asynchronous) on the engine's stream; does not wait.
  void copy_results_async(Problem* p, int count, double* poses, double* loss, double* pairs, int32_t* state);
  // After an evaluation with source_counts on, of a set whose first edge has source frame m of p:
  // every source point's pair count, by its original index (frame m's point count; synchronises).
  void read_source_counts(Problem* p, int m, int64_t* counts);
  int32_t read_status(Problem* p);                                         // synchronises
  const double* edge_out() const { return sc_->edge_out.p; }

  // device views
  const float4* pts() const { return static_cast<const float4*>(points_.ptr(0)); }
  const void* feat() const { return points_.ptr(3); }
  int64_t feat_row_bytes() const { return feat_kind <= 0 ? 4 : (int64_t)feat_elem_bytes(feat_kind) * Dp; }
  const int32_t* perm() const { return static_cast<const int32_t*>(points_.ptr(1)); }
  const uint32_t* keys() const { return static_cast<const uint32_t*>(points_.ptr(2)); }
  const int4* rows() const { return static_cast<const int4*>(rows_.ptr(0)); }
  const uint32_t* xtab() const { return static_cast<const uint32_t*>(xtab_.ptr(0)); }
  const FrameInfo* frames() const { return static_cast<const FrameInfo*>(slots_.ptr(0)); }
  double* poses() const { return static_cast<double*>(slots_.ptr(1)); }
  double* poses_ptr(const Problem* p) const { return poses() + 12 * p->slot0; }
  uint64_t generation() const;

  // stage timing with HIP events on the engine's stream (graphs are not used while on)
  bool prof = false;
  struct Stage {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0.0;
    int64_t launches = 0;
  };
  Stage stages[8];
  hipEvent_t prof_begin();
  void prof_end(int stage, hipEvent_t start);
  void prof_collect();

 private:
  void compute_constants(Problem* p);
  void record_iteration(SetLayout& lay, bool reuse_binning);
  const SetLayout* binned_lay_ = nullptr;  // layout whose binning the scratch holds

  std::map<int, std::unique_ptr<Problem>> probs_;
  int next_id_ = 0;

  Pool points_{{sizeof(float4), sizeof(int32_t), sizeof(uint32_t), sizeof(float)}};  // pts, perm, keys, feat (x Dp)
  Pool rows_{{sizeof(int4)}};
  Pool xtab_{{sizeof(uint32_t)}};
  Pool slots_{{sizeof(FrameInfo), 12 * sizeof(double)}};
  Pool hist_{{sizeof(double), sizeof(double)}};  // loss, pair count
  Pool state_{{2 * sizeof(int32_t)}};

  // build scratch
  DBuf<float> raw_xyz_;
  DBuf<uint8_t> raw_feat_;
  DBuf<const float*> d_xyz_ptrs_;
  DBuf<const void*> d_feat_ptrs_;
  DBuf<int64_t> d_in_off_;
  DBuf<FrameInfo> d_bframes_;
  DBuf<int32_t> cell_, minmax_;
  DBuf<uint32_t> k1_, v1_, k2_, v2_, hist_scratch_;
  DBuf<SortTile> d_tiles_;
  DBuf<SortSeg> d_segs_;
  DBuf<uint32_t> row_sizes_, scan_tmp_;
  DBuf<uint64_t> d_total_;
  DBuf<int64_t> d_lab_off_;
  DBuf<int32_t> d_lab_start_;

  template <typename T>
  void need(DBuf<T>& b, size_t count, const char* what);

  // per-evaluation scratch (sized for the largest set so far), or views of the arena
  EvalScratch own_sc_, arena_sc_;
  EvalScratch* sc_ = &own_sc_;
  Arena* arena_ = nullptr;
  const uint32_t* sorted_k_ = nullptr;
  const uint32_t* sorted_v_ = nullptr;
  uint64_t scratch_gen_ = 0;  // bumped when a scratch buffer moves

  std::vector<hipEvent_t> event_pool_;
};

}  // namespace rkhsba
