// Engine: resident problem storage, set layouts and the launch sequences of
// the voxel build, the evaluation and the Gauss-Newton iteration.
#include "engine.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/rkhsba.h"

namespace rkhsba {

void throw_hip(hipError_t e, const char* what) {
  throw Fail{e == hipErrorOutOfMemory ? RKHSBA_ENOMEM : RKHSBA_EDEVICE,
             std::string(what) + ": " + hipGetErrorString(e)};
}

// ---------------------------------------------------------------- RangeAlloc

int64_t RangeAlloc::alloc(int64_t n) {
  if (n <= 0) n = 1;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < n) continue;
    const int64_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > n) free_[off + n] = len - n;
    used_ += n;
    return off;
  }
  return -1;
}

void RangeAlloc::free(int64_t off, int64_t n) {
  if (n <= 0) n = 1;
  used_ -= n;
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + n == next->first) {
    n += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += n;
      return;
    }
  }
  free_[off] = n;
}

void RangeAlloc::grow(int64_t new_cap) {
  if (new_cap <= cap_) return;
  const int64_t add = new_cap - cap_;
  if (!free_.empty()) {
    auto last = std::prev(free_.end());
    if (last->first + last->second == cap_) {
      last->second += add;
      cap_ = new_cap;
      return;
    }
  }
  free_[cap_] = add;
  cap_ = new_cap;
}

int64_t RangeAlloc::largest_free() const {
  int64_t m = 0;
  for (const auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

// ---------------------------------------------------------------- Pool

Pool::~Pool() {
  for (void* p : ptr_)
    if (p) (void)hipFree(p);
}

size_t Pool::bytes() const {
  size_t b = 0;
  for (size_t e : eb_) b += e * (size_t)ra_.capacity();
  return b;
}

void Pool::set_elem_bytes(int i, size_t b) {
  if (eb_[i] == b) return;
  if (ptr_[i]) (void)hipFree(ptr_[i]);
  ptr_[i] = nullptr;
  eb_[i] = b;
  if (ra_.capacity() > 0) RK_HIP(hipMalloc(&ptr_[i], b * (size_t)ra_.capacity()));
  ++gen_;
}

int64_t Pool::alloc(int64_t n, hipStream_t st) {
  if (n <= 0) n = 1;
  int64_t off = ra_.alloc(n);
  if (off >= 0) return off;
  const int64_t cap = ra_.capacity();
  const int64_t new_cap = std::max<int64_t>({cap + n, cap + cap / 2, 1024});
  // The contents move to new arrays: work queued on any stream of the engine (a lane's iterations while
  // a build on its own stream grows the pool) must have finished writing to the old ones first, and must
  // not read them after they are freed.
  RK_HIP(hipDeviceSynchronize());
  std::vector<void*> fresh(eb_.size(), nullptr);
  for (size_t i = 0; i < eb_.size(); ++i) {
    hipError_t e = hipMalloc(&fresh[i], eb_[i] * (size_t)new_cap);
    if (e != hipSuccess) {
      for (void* p : fresh)
        if (p) (void)hipFree(p);
      throw_hip(e, "pool growth");
    }
    if (ptr_[i] && cap > 0) RK_HIP(hipMemcpyAsync(fresh[i], ptr_[i], eb_[i] * (size_t)cap, hipMemcpyDeviceToDevice, st));
  }
  RK_HIP(hipStreamSynchronize(st));
  for (size_t i = 0; i < eb_.size(); ++i) {
    if (ptr_[i]) (void)hipFree(ptr_[i]);
    ptr_[i] = fresh[i];
  }
  ++gen_;
  ra_.grow(new_cap);
  off = ra_.alloc(n);
  RK_REQUIRE(off >= 0, RKHSBA_ENOMEM, "pool allocation failed after growth");
  return off;
}

// ---------------------------------------------------------------- SetLayout

void SetLayout::drop_graph() {
  if (graph) (void)hipGraphExecDestroy(graph);
  if (graph_rest) (void)hipGraphExecDestroy(graph_rest);
  graph = nullptr;
  graph_rest = nullptr;
  graph_mode = -1;
}

uint8_t* SetLayout::stage_for(size_t bytes, bool no_alloc) {
  if (no_alloc && stage_cap < bytes) return nullptr;  // allocation-free callers upload from their tables
  if (stage_ev) RK_HIP(hipEventSynchronize(stage_ev));  // the last uploads from the buffer are done
  if (stage_cap < bytes) {
    if (stage) (void)hipHostFree(stage);
    stage = nullptr;
    stage_cap = 0;
    const size_t cap = std::max<size_t>(bytes + bytes / 2, 1 << 16);
    RK_HIP(hipHostMalloc(reinterpret_cast<void**>(&stage), cap, hipHostMallocDefault));
    stage_cap = cap;
  }
  if (!stage_ev) RK_HIP(hipEventCreateWithFlags(&stage_ev, hipEventDisableTiming));
  return stage;
}

SetLayout::~SetLayout() {
  drop_graph();
  if (stage_ev) {
    (void)hipEventSynchronize(stage_ev);
    (void)hipEventDestroy(stage_ev);
  }
  if (stage) (void)hipHostFree(stage);
}

// ---------------------------------------------------------------- Engine

Engine::Engine(int dev, hipStream_t stream, int mp) : device(dev), st(stream), moment_path(mp) {}

Engine::~Engine() {
  for (auto& s : stages)
    for (auto& pr : s.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t ev : event_pool_) (void)hipEventDestroy(ev);
}

uint64_t Engine::generation() const {
  return points_.generation() + rows_.generation() + xtab_.generation() + slots_.generation() +
         hist_.generation() + state_.generation() + scratch_gen_;
}

hipEvent_t Engine::prof_begin() {
  if (!prof || arena_) return nullptr;
  hipEvent_t ev = nullptr;
  if (!event_pool_.empty()) {
    ev = event_pool_.back();
    event_pool_.pop_back();
  } else if (hipEventCreate(&ev) != hipSuccess) {
    return nullptr;
  }
  (void)hipEventRecord(ev, st);
  return ev;
}

void Engine::prof_end(int stage, hipEvent_t start) {
  if (!prof || !start) return;
  hipEvent_t ev = nullptr;
  if (!event_pool_.empty()) {
    ev = event_pool_.back();
    event_pool_.pop_back();
  } else if (hipEventCreate(&ev) != hipSuccess) {
    return;
  }
  (void)hipEventRecord(ev, st);
  stages[stage].pending.emplace_back(start, ev);
}

void Engine::prof_collect() {
  for (auto& s : stages) {
    for (auto& pr : s.pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        s.ms += ms;
        s.launches += 1;
      }
      event_pool_.push_back(pr.first);
      event_pool_.push_back(pr.second);
    }
    s.pending.clear();
  }
}

Problem* Engine::problem(int id) {
  auto it = probs_.find(id);
  return it == probs_.end() ? nullptr : it->second.get();
}

int64_t Engine::device_bytes() const {
  int64_t b = (int64_t)(points_.bytes() + rows_.bytes() + xtab_.bytes() + slots_.bytes() + hist_.bytes() +
                        state_.bytes());
  b += (int64_t)(raw_xyz_.bytes() + raw_feat_.bytes() + cell_.bytes() + k1_.bytes() + v1_.bytes() + k2_.bytes() +
                 v2_.bytes() + hist_scratch_.bytes() + row_sizes_.bytes() + scan_tmp_.bytes());
  const EvalScratch& o = own_sc_;
  b += (int64_t)(o.xf.bytes() + o.bk.bytes() + o.bv.bytes() + o.bk2.bytes() + o.bv2.bytes() + o.bhist.bytes() +
                 o.mom.bytes() + o.cnt.bytes() + o.partial.bytes() + o.edge_out.bytes() + o.H.bytes() + o.b.bytes() +
                 o.delta.bytes());
  return b;
}

int64_t Engine::estimate_resident_bytes(int K, const int64_t* n_points, int64_t row_bytes) {
  int64_t N = 0;
  for (int f = 0; f < K; ++f) N += n_points[f];
  return N * (28 + row_bytes + 12);  // pools + cell tables (typical occupancy)
}

int64_t Engine::estimate_bytes(int K, const int64_t* n_points, int E, int64_t row_bytes) {
  int64_t nmax = 0;
  for (int f = 0; f < K; ++f) nmax = std::max(nmax, n_points[f]);
  const int64_t per_entry = 16 + 40 + 4 + 3;                // binning keys/values (x2), moments, count, partials
  const int64_t n = 6 * (int64_t)K;
  return estimate_resident_bytes(K, n_points, row_bytes) + (int64_t)E * nmax * per_entry + 2 * n * n * 8 +
         (int64_t)E * 2 * kEdgeVals * 8;
}

// Class-id sweep passes whose box is wider than this many truncation radii walk per source point.  On the
// LiDAR map (64 x 100,000 points, 20% outliers) a fifth of the 8-point passes span more than 4 r_c and hold
// under 1% of the pairs.  With the box filter, label layers and sub-cell keys of the shared walk, 16-point
// passes measured per launch against 3 r_c: 2.25 r_c +1%, 4.5 r_c -0.7%, 6 r_c -1.4%, 9 r_c -1%, 12 r_c
// -1.9%, 16 r_c +2.5%, 24 r_c +2.6%, no per-source walks +40%.
constexpr double kSpreadFactor = 6.0;

void Engine::compute_constants(Problem* p) {
  const ProbParams& o = p->par;
  const double rc = o.cutoff_factor * o.ell;
  const double cell = rc / o.cell_subdiv;
  KConst k{};
  k.inv_cell = 1.0 / cell;
  k.cell = cell;
  k.reach = rc * (1.0 + std::ldexp(1.0, -12));
  k.reach2 = k.reach * k.reach;
  k.rc2 = (float)(rc * rc);
  k.alpha = (float)(1.4426950408889634 / (2.0 * o.ell * o.ell));
  k.reach_cells = o.cell_subdiv + 1;
  k.clamp = (o.clamp_negative_c && p->negative_features) ? 1 : 0;
  k.c_positive = p->c_positive ? 1 : 0;
  k.Dp = Dp;
  k.topk = o.top_k;
  k.inv2l2 = 1.0 / (2.0 * o.ell * o.ell);
  k.spread_limit = (float)(kSpreadFactor * rc);
  p->kc = k;
}

int Engine::add_problem(const ProbParams& par, int K, const int64_t* n_points, const float* const* xyz, int kind,
                        int Din, const void* const* feats, bool is_device) {
  RK_REQUIRE(K >= 1 && n_points && xyz && feats, RKHSBA_EINVAL, "K >= 1 and non-NULL n_points/xyz/feats required");
  RK_REQUIRE(kind == RKHSBA_FEAT_CLASS_ID || kind == RKHSBA_FEAT_DENSE_F32 || kind == RKHSBA_FEAT_DENSE_BF16 ||
                 kind == RKHSBA_FEAT_DENSE_FP8,
             RKHSBA_EINVAL, "unknown feature kind");
  if (kind != RKHSBA_FEAT_CLASS_ID)
    RK_REQUIRE(Din >= 1 && Din <= kMaxDense, RKHSBA_EINVAL, "dense feature dimension must be in [1, 64]");
  RK_REQUIRE(par.ell > 0.0 && std::isfinite(par.ell) && par.cutoff_factor > 0.0 && std::isfinite(par.cutoff_factor) &&
                 par.cell_subdiv >= 1 && par.cell_subdiv <= 8 && std::isfinite(par.sigma) && par.damping_rel >= 0.0 &&
                 (par.pass_points == 1 || par.pass_points == 8 || par.pass_points == 16 || par.pass_points == 32 ||
                  par.pass_points == 64) &&
                 par.top_k >= 0 && par.top_k <= kMaxTopK,
             RKHSBA_EINVAL, "invalid problem parameters");
  RK_REQUIRE(par.top_k == 0 || kind == RKHSBA_FEAT_CLASS_ID || kind == RKHSBA_FEAT_DENSE_F32, RKHSBA_EINVAL,
             "top-k pair selection needs class ids or float32 dense features");
  RK_REQUIRE(par.top_k == 0 || par.pass_points == 1, RKHSBA_EINVAL, "top-k pair selection needs per-point walks");
  RK_REQUIRE(par.pass_points != 8 || kind == RKHSBA_FEAT_CLASS_ID, RKHSBA_EINVAL, "8-point passes need class ids");
  const int Dk = kind == RKHSBA_FEAT_CLASS_ID ? 0 : Din;
  // builds run on their own stream when the engine has one (the server's lanes: a build then does not wait
  // for the lane's queued iterations); the engine's stream is ordered after the build at the end
  hipStream_t bst = build_st ? build_st : st;
  if (probs_.empty()) {
    feat_kind = kind;
    D = Dk;
    Dp = kind == RKHSBA_FEAT_CLASS_ID ? 0 : dense_pad(Din, kind);
    points_.set_elem_bytes(3, kind == RKHSBA_FEAT_CLASS_ID ? 4 : (size_t)feat_elem_bytes(kind) * Dp);
  } else {
    RK_REQUIRE(kind == feat_kind && Dk == D, RKHSBA_EINVAL,
               "all resident problems share one feature kind and dimension");
  }
  std::vector<int64_t> off(K + 1, 0);
  for (int f = 0; f < K; ++f) {
    RK_REQUIRE(n_points[f] >= 1 && n_points[f] < (1LL << 31), RKHSBA_EINVAL, "each frame needs 1..2^31-1 points");
    RK_REQUIRE(xyz[f] && feats[f], RKHSBA_EINVAL, "NULL frame pointer");
    off[f + 1] = off[f] + n_points[f];
  }
  const int64_t N = off[K];
  RK_REQUIRE(N < (1LL << 32), RKHSBA_EINVAL, "too many points in one problem");

  auto P = std::make_unique<Problem>();
  Problem* p = P.get();
  p->par = par;
  p->K = K;
  p->N = N;
  p->n_points.assign(n_points, n_points + K);
  compute_constants(p);
  const KConst kc0 = p->kc;
  const size_t fbytes = kind == RKHSBA_FEAT_CLASS_ID ? sizeof(uint16_t) : sizeof(float) * (size_t)Din;

  auto release = [&]() {
    if (p->pbase >= 0) points_.free(p->pbase, N);
    if (p->rbase >= 0) rows_.free(p->rbase, p->n_rows);
    if (p->xbase >= 0) xtab_.free(p->xbase, p->n_xt);
    if (p->slot0 >= 0) slots_.free(p->slot0, K);
    if (p->sbase >= 0) state_.free(p->sbase, 1);
  };
  try {
    // stage inputs and per-frame pointers
    std::vector<const float*> xp(K);
    std::vector<const void*> fp(K);
    if (is_device) {
      for (int f = 0; f < K; ++f) {
        xp[f] = xyz[f];
        fp[f] = feats[f];
      }
    } else {
      for (int f = 0; f < K; ++f)
        for (int64_t i = 0; i < 3 * n_points[f]; ++i)
          RK_REQUIRE(std::isfinite(xyz[f][i]), RKHSBA_EINVAL, "non-finite point coordinate");
      if (kind != RKHSBA_FEAT_CLASS_ID)
        for (int f = 0; f < K; ++f) {
          const float* v = static_cast<const float*>(feats[f]);
          for (int64_t i = 0; i < (int64_t)Din * n_points[f]; ++i)
            RK_REQUIRE(std::isfinite(v[i]), RKHSBA_EINVAL, "non-finite feature value");
        }
      RK_HIP(raw_xyz_.reserve((size_t)N * 3));
      RK_HIP(raw_feat_.reserve((size_t)N * fbytes));
      for (int f = 0; f < K; ++f) {
        RK_HIP(hipMemcpyAsync(raw_xyz_.p + 3 * off[f], xyz[f], sizeof(float) * 3 * n_points[f],
                              hipMemcpyHostToDevice, bst));
        RK_HIP(hipMemcpyAsync(raw_feat_.p + fbytes * off[f], feats[f], fbytes * n_points[f], hipMemcpyHostToDevice,
                              bst));
        xp[f] = raw_xyz_.p + 3 * off[f];
        fp[f] = raw_feat_.p + fbytes * off[f];
      }
    }
    hipEvent_t tb = bst == st ? prof_begin() : nullptr;
    RK_HIP(d_xyz_ptrs_.reserve(K));
    RK_HIP(d_feat_ptrs_.reserve(K));
    RK_HIP(d_in_off_.reserve(K + 1));
    RK_HIP(hipMemcpyAsync(d_xyz_ptrs_.p, xp.data(), sizeof(void*) * K, hipMemcpyHostToDevice, bst));
    RK_HIP(hipMemcpyAsync(d_feat_ptrs_.p, fp.data(), sizeof(void*) * K, hipMemcpyHostToDevice, bst));
    RK_HIP(hipMemcpyAsync(d_in_off_.p, off.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, bst));

    // cell coordinates and per-frame bounds (and largest class ids)
    const int n_dmin = kind == RKHSBA_FEAT_DENSE_F32 ? Dp : 0;  // per-dimension minima of FP32 features
    const bool class_ids = kind == RKHSBA_FEAT_CLASS_ID;
    const int lab0 = 6 * K + 3 + n_dmin;                          // per-frame largest class id
    std::vector<int32_t> mm(lab0 + (class_ids ? K : 0), -1);
    for (int f = 0; f < K; ++f)
      for (int a = 0; a < 3; ++a) {
        mm[6 * f + a] = INT_MAX;
        mm[6 * f + 3 + a] = INT_MIN;
      }
    mm[6 * K] = 0;      // bad coordinate flag
    mm[6 * K + 1] = 0;  // negative feature flag
    mm[6 * K + 2] = 0;  // occupied cells
    for (int d = 0; d < n_dmin; ++d) mm[6 * K + 3 + d] = 0x7f800000;  // feature minima (+inf until the build)
    RK_HIP(cell_.reserve((size_t)N * 3));
    RK_HIP(minmax_.reserve(mm.size()));
    RK_HIP(hipMemcpyAsync(minmax_.p, mm.data(), sizeof(int32_t) * mm.size(), hipMemcpyHostToDevice, bst));
    RK_HIP(launch_cell_coords(d_xyz_ptrs_.p, d_in_off_.p, K, N, kc0.inv_cell, d_feat_ptrs_.p, cell_.p, minmax_.p,
                              class_ids ? minmax_.p + lab0 : nullptr, bst));
    RK_HIP(hipMemcpyAsync(mm.data(), minmax_.p, sizeof(int32_t) * mm.size(), hipMemcpyDeviceToHost, bst));
    RK_HIP(hipStreamSynchronize(bst));
    RK_REQUIRE(mm[6 * K] == 0, RKHSBA_EINVAL, "non-finite or out-of-range point coordinate");

    // grids (frame-local offsets for the build)
    std::vector<FrameInfo> fr(K);
    int64_t rows_total = 0;
    uint64_t max_cells = 1;
    int bin_axis_bits = 1;
    std::vector<int> frame_bits(K);  // per-axis bits of a frame's cell coordinates (negative: coarsened)
    for (int f = 0; f < K; ++f) {
      FrameInfo& F = fr[f];
      F.pt_off = off[f];
      F.n = (int32_t)n_points[f];
      uint64_t cells = 1;
      for (int a = 0; a < 3; ++a) {
        F.org[a] = mm[6 * f + a];
        const int64_t d = (int64_t)mm[6 * f + 3 + a] - mm[6 * f + a] + 1;
        RK_REQUIRE(d >= 1 && d < (1 << 24), RKHSBA_ENOMEM, "frame extent too large for its cell grid");
        F.dim[a] = (int32_t)d;
        cells *= (uint64_t)d;
      }
      RK_REQUIRE(cells < 0xffffffffull, RKHSBA_ENOMEM,
                 "frame spans more than 2^32 cells; raise ell or lower cell_subdiv");
      max_cells = std::max(max_cells, cells);
      F.xt_off = 0;
      F.n_lab = 0;
      F.key_sub = 0;
      int ext_max = 0;
      for (int a = 0; a < 3; ++a) ext_max = std::max(ext_max, F.dim[a] + 2 * kc0.reach_cells);
      int shift = 0;
      while (((ext_max - 1) >> shift) >= 1023) ++shift;
      F.mort_shift = shift;
      const int maxc = (ext_max - 1) >> shift;
      int bits = 1;
      while ((1 << bits) < maxc + 2) ++bits;
      frame_bits[f] = shift == 0 ? bits : -bits;
      bin_axis_bits = std::max(bin_axis_bits, bits);
    }
    // The binning keys order the source points of a cell by sub-cell (Morton order at a finer grid), as
    // far as that fits the radix passes the cells already take: the passes' groups of consecutive points
    // then span smaller boxes, whose walks hold fewer candidates that pair with none of the group.
    {
      const int axis_room = (8 * ((3 * bin_axis_bits + 7) / 8)) / 3;  // axis bits the same digit passes sort
      for (int f = 0; f < K; ++f) {
        if (frame_bits[f] < 0) continue;  // coarsened grid (mort_shift > 0)
        fr[f].key_sub = std::max(0, std::min({3, axis_room - frame_bits[f], 10 - frame_bits[f]}));
        bin_axis_bits = std::max(bin_axis_bits, frame_bits[f] + fr[f].key_sub);
      }
    }
    // Class ids: every frame stacks one layer of its z extent per class id (0 .. its largest id) along z,
    // so that points of one id are contiguous and the sweeps walk only the candidates that can pair.  Kept
    // only while the keys fit 32 bits and the row table stays within 16 rows per point (+ 2^20).
    bool stacked = class_ids;
    {
      int64_t rows_stacked = 0;
      for (int f = 0; f < K && stacked; ++f) {
        const int64_t n_lab = (int64_t)mm[lab0 + f] + 1;
        const uint64_t cells = (uint64_t)fr[f].dim[0] * fr[f].dim[1] * fr[f].dim[2];
        stacked = n_lab >= 1 && cells * (uint64_t)n_lab < 0xffffffffull;
        rows_stacked += (int64_t)fr[f].dim[1] * fr[f].dim[2] * n_lab;
      }
      stacked = stacked && rows_stacked < (1LL << 31) && rows_stacked <= 16 * N + (1LL << 20);
    }
    for (int f = 0; f < K; ++f) {
      FrameInfo& F = fr[f];
      F.n_lab = stacked ? mm[lab0 + f] + 1 : 0;
      F.row_off = rows_total;
      rows_total += (int64_t)F.dim[1] * F.dim[2] * std::max(F.n_lab, 1);
      max_cells = std::max(max_cells, (uint64_t)F.dim[0] * F.dim[1] * F.dim[2] * std::max(F.n_lab, 1));
    }
    p->stacked = stacked;
    RK_REQUIRE(rows_total < (1LL << 31), RKHSBA_ENOMEM, "cell-row table too large");
    p->bin_bits = 3 * bin_axis_bits;
    RK_HIP(d_bframes_.reserve(K));
    RK_HIP(hipMemcpyAsync(d_bframes_.p, fr.data(), sizeof(FrameInfo) * K, hipMemcpyHostToDevice, bst));

    // resident ranges
    p->pbase = points_.alloc(N, bst);
    p->n_rows = std::max<int64_t>(rows_total, 1);
    p->rbase = rows_.alloc(p->n_rows, bst);
    float4* d_pts = static_cast<float4*>(points_.ptr(0)) + p->pbase;
    int32_t* d_perm = static_cast<int32_t*>(points_.ptr(1)) + p->pbase;
    uint32_t* d_keys = static_cast<uint32_t*>(points_.ptr(2)) + p->pbase;
    void* d_feat = static_cast<uint8_t*>(points_.ptr(3)) + p->pbase * feat_row_bytes();
    int4* d_rows = static_cast<int4*>(rows_.ptr(0)) + p->rbase;

    // keys, segmented sort by frame, gather
    RK_HIP(k1_.reserve(N));
    RK_HIP(v1_.reserve(N));
    RK_HIP(k2_.reserve(N));
    RK_HIP(v2_.reserve(N));
    RK_HIP(launch_cell_keys(cell_.p, d_in_off_.p, d_bframes_.p, K, N, d_feat_ptrs_.p, k1_.p, v1_.p, bst));
    std::vector<SortTile> tiles;
    std::vector<SortSeg> segs(K);
    for (int f = 0; f < K; ++f) {
      segs[f].start = off[f];
      segs[f].count = n_points[f];
      segs[f].tile0 = (int32_t)tiles.size();
      for (int64_t s = 0; s < n_points[f]; s += kSortTile)
        tiles.push_back(SortTile{off[f] + s, (int32_t)std::min<int64_t>(kSortTile, n_points[f] - s), f, f, 0});
      segs[f].n_tiles = (int32_t)tiles.size() - segs[f].tile0;
    }
    RK_HIP(d_tiles_.reserve(tiles.size()));
    RK_HIP(d_segs_.reserve(K));
    RK_HIP(hist_scratch_.reserve(tiles.size() * 256));
    RK_HIP(hipMemcpyAsync(d_tiles_.p, tiles.data(), sizeof(SortTile) * tiles.size(), hipMemcpyHostToDevice, bst));
    RK_HIP(hipMemcpyAsync(d_segs_.p, segs.data(), sizeof(SortSeg) * K, hipMemcpyHostToDevice, bst));
    int key_bits = 1;
    while (key_bits < 32 && (1ull << key_bits) < max_cells) ++key_bits;
    bool in_tmp = false;
    RK_HIP(launch_radix_sort(k1_.p, v1_.p, k2_.p, v2_.p, hist_scratch_.p, d_tiles_.p, (int)tiles.size(), d_segs_.p, K,
                             key_bits, bst, &in_tmp));
    uint32_t* sk = in_tmp ? k2_.p : k1_.p;
    uint32_t* sv = in_tmp ? v2_.p : v1_.p;
    RK_HIP(launch_gather(d_xyz_ptrs_.p, d_feat_ptrs_.p, kind, D, std::max(Dp, 1),
                         d_bframes_.p, d_in_off_.p, K, N, sv, d_pts, d_feat, d_perm, minmax_.p + 6 * K + 1, bst));
    RK_HIP(hipMemcpyAsync(d_keys, sk, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, bst));
    RK_HIP(launch_feature_min(static_cast<const float*>(d_feat), N, n_dmin,
                              reinterpret_cast<uint32_t*>(minmax_.p + 6 * K + 3), bst));

    // cell-row tables
    RK_HIP(row_sizes_.reserve(rows_total));
    RK_HIP(scan_tmp_.reserve(rows_total / kScanTileElems + 2));
    RK_HIP(d_total_.reserve(1));
    RK_HIP(launch_rows(d_keys, d_bframes_.p, d_in_off_.p, K, N, d_rows, rows_total, row_sizes_.p, scan_tmp_.p,
                       d_total_.p, bst));
    // first point of every label layer (pass segments of the edges that start in the frame)
    p->lab_off.assign(K, -1);
    p->lab_start.clear();
    if (stacked) {
      int64_t n_ls = 0;
      for (int f = 0; f < K; ++f) {
        p->lab_off[f] = n_ls;
        n_ls += fr[f].n_lab + 1;
      }
      p->lab_start.resize(n_ls);
      RK_HIP(d_lab_off_.reserve(K));
      RK_HIP(d_lab_start_.reserve(n_ls));
      RK_HIP(hipMemcpyAsync(d_lab_off_.p, p->lab_off.data(), sizeof(int64_t) * K, hipMemcpyHostToDevice, bst));
      RK_HIP(launch_label_starts(d_keys, d_bframes_.p, d_lab_off_.p, K, d_lab_start_.p, bst));
      RK_HIP(hipMemcpyAsync(p->lab_start.data(), d_lab_start_.p, sizeof(int32_t) * n_ls, hipMemcpyDeviceToHost, bst));
    }
    uint64_t xt_total = 0;
    int32_t neg = 0;
    RK_HIP(hipMemcpyAsync(&xt_total, d_total_.p, sizeof(uint64_t), hipMemcpyDeviceToHost, bst));
    RK_HIP(hipMemcpyAsync(&neg, minmax_.p + 6 * K + 1, sizeof(int32_t), hipMemcpyDeviceToHost, bst));
    std::vector<uint32_t> dmin(std::max(n_dmin, 1));
    if (n_dmin > 0)
      RK_HIP(hipMemcpyAsync(dmin.data(), minmax_.p + 6 * K + 3, sizeof(uint32_t) * n_dmin, hipMemcpyDeviceToHost, bst));
    RK_HIP(hipStreamSynchronize(bst));
    p->negative_features = neg != 0;
    p->c_positive = false;
    if (!p->negative_features)
      for (int d = 0; d < n_dmin; ++d) {
        float v;
        std::memcpy(&v, &dmin[d], sizeof(v));
        p->c_positive = p->c_positive || v >= 1e-18f;
      }
    compute_constants(p);
    RK_REQUIRE(xt_total < (1ull << 31), RKHSBA_ENOMEM, "cell table too large");
    p->n_xt = std::max<int64_t>((int64_t)xt_total, 1);
    p->xbase = xtab_.alloc(p->n_xt, bst);
    RK_HIP(launch_xtab(d_keys, d_bframes_.p, d_in_off_.p, K, N, d_rows,
                       static_cast<uint32_t*>(xtab_.ptr(0)) + p->xbase,
                       reinterpret_cast<uint32_t*>(minmax_.p + 6 * K + 2), bst));
    uint32_t n_cells = 0;
    RK_HIP(hipMemcpyAsync(&n_cells, minmax_.p + 6 * K + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, bst));

    // frame table entries with pool offsets
    p->slot0 = slots_.alloc(K, bst);
    p->sbase = state_.alloc(1, bst);
    for (int f = 0; f < K; ++f) {
      fr[f].pt_off += p->pbase;
      fr[f].row_off += p->rbase;
      fr[f].xt_off = p->xbase;
    }
    RK_HIP(hipMemcpyAsync(static_cast<FrameInfo*>(slots_.ptr(0)) + p->slot0, fr.data(), sizeof(FrameInfo) * K,
                          hipMemcpyHostToDevice, bst));
    prof_end(RKHSBA_PROF_BUILD, tb);
    RK_HIP(hipStreamSynchronize(bst));
    prof_collect();
    p->frames = std::move(fr);
    p->occupancy = (double)N / std::max<uint32_t>(n_cells, 1u);
    p->resident_bytes = N * (int64_t)(28 + feat_row_bytes()) + p->n_rows * 16 + p->n_xt * 4 +
                        (int64_t)K * (int64_t)(sizeof(FrameInfo) + 96) + 8;
  } catch (...) {
    release();
    throw;
  }
  if (par.cell_subdiv == 1) p->occupancy_r = p->occupancy;
  p->id = next_id_++;
  probs_[p->id] = std::move(P);
  return p->id;
}

// ---------------------------------------------------------------- cell-size choice

namespace {
std::mutex g_tune_mu;
// (feature kind, Dp, occupancy bucket) -> (cell_subdiv, pass_points)
std::map<std::vector<int>, std::pair<int, int>> g_tune;
}  // namespace

int occupancy_bucket(double occ) {
  const double b = std::floor(2.0 * std::log2(std::max(occ, 1.0)));
  return (int)std::min(40.0, std::max(0.0, b));
}

void Engine::tune_record(double occ_r, int subdiv, int pp) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{feat_kind, Dp, occupancy_bucket(occ_r)}] = {subdiv, pp};
}

std::pair<int, int> Engine::choose_config(double occ_r) const {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find({feat_kind, Dp, occupancy_bucket(occ_r)});
    if (it != g_tune.end()) return it->second;
  }
  // Untuned default: finer cells and shared 16-point walks as the points per
  // truncation-radius cube grow; per-point walks for sparse frames.
  if (occ_r < 3.0) return {1, 1};
  if (occ_r < 12.0) return {2, 16};
  if (occ_r < 48.0) return {4, 16};
  return {8, 16};
}

int Engine::add_problem_auto(const ProbParams& par_in, int K, const int64_t* n_points, const float* const* xyz,
                             int kind, int Din, const void* const* feats, bool is_device) {
  ProbParams par = par_in;
  if (par.top_k > 0) par.pass_points = 1;  // the top-k selection runs in the per-point walks
  if (par.cell_subdiv != 0 && par.pass_points != 0)
    return add_problem(par, K, n_points, xyz, kind, Din, feats, is_device);
  ProbParams probe = par;
  probe.cell_subdiv = 1;  // cells of one truncation radius: occupancy probe
  if (probe.pass_points == 0) probe.pass_points = 16;
  const int id = add_problem(probe, K, n_points, xyz, kind, Din, feats, is_device);
  const double occ = problem(id)->occupancy;
  const std::pair<int, int> cfg = choose_config(occ);
  ProbParams fine = par;
  if (fine.cell_subdiv == 0) fine.cell_subdiv = cfg.first;
  if (fine.pass_points == 0) fine.pass_points = cfg.second;
  if (fine.cell_subdiv == 1) {
    Problem* p = problem(id);
    p->par.pass_points = fine.pass_points;  // same grid; only the sweep choice changes
    return id;
  }
  remove_problem(id);
  const int id2 = add_problem(fine, K, n_points, xyz, kind, Din, feats, is_device);
  problem(id2)->occupancy_r = occ;
  return id2;
}

void Engine::remove_problem(int id) {
  auto it = probs_.find(id);
  if (it == probs_.end()) return;
  Problem* p = it->second.get();
  points_.free(p->pbase, p->N);
  rows_.free(p->rbase, p->n_rows);
  xtab_.free(p->xbase, p->n_xt);
  slots_.free(p->slot0, p->K);
  state_.free(p->sbase, 1);
  if (p->hbase >= 0) hist_.free(p->hbase, p->n_hist);
  clear_aliases(p);
  probs_.erase(it);
}

void Engine::upload_poses(Problem* p, const double* poses) {
  RK_REQUIRE(poses != nullptr, RKHSBA_EINVAL, "poses is NULL");
  for (int i = 0; i < 12 * p->K; ++i) RK_REQUIRE(std::isfinite(poses[i]), RKHSBA_EINVAL, "non-finite pose entry");
  RK_HIP(hipMemcpyAsync(poses_ptr(p), poses, sizeof(double) * 12 * p->K, hipMemcpyHostToDevice, st));
}

void Engine::set_aliases(Problem* p, int frame, int count, const double* alias_poses) {
  RK_REQUIRE(frame >= 0 && frame < p->K && count >= 1 && alias_poses, RKHSBA_EINVAL, "bad alias request");
  for (int i = 0; i < 12 * count; ++i) RK_REQUIRE(std::isfinite(alias_poses[i]), RKHSBA_EINVAL, "non-finite pose entry");
  if (p->n_alias != count) {
    clear_aliases(p);
    p->alias_slot0 = slots_.alloc(count, st);
    p->n_alias = count;
  }
  p->alias_of = frame;
  std::vector<FrameInfo> fr(count, p->frames[frame]);
  RK_HIP(hipMemcpyAsync(static_cast<FrameInfo*>(slots_.ptr(0)) + p->alias_slot0, fr.data(), sizeof(FrameInfo) * count,
                        hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(poses() + 12 * p->alias_slot0, alias_poses, sizeof(double) * 12 * count, hipMemcpyHostToDevice,
                        st));
  RK_HIP(hipStreamSynchronize(st));  // the host FrameInfo copies go out of scope
}

void Engine::set_ell(Problem* p, double ell) {
  RK_REQUIRE(ell > 0.0 && std::isfinite(ell), RKHSBA_EINVAL, "lengthscale must be positive");
  p->par.ell = ell;
  KConst k = p->kc;
  const double rc = p->par.cutoff_factor * ell;
  k.reach = rc * (1.0 + std::ldexp(1.0, -12));
  k.reach2 = k.reach * k.reach;
  k.rc2 = (float)(rc * rc);
  k.alpha = (float)(1.4426950408889634 / (2.0 * ell * ell));
  k.reach_cells = (int)std::ceil(k.reach * k.inv_cell) + 1;
  k.inv2l2 = 1.0 / (2.0 * ell * ell);
  k.spread_limit = (float)(kSpreadFactor * rc);
  p->kc = k;
  ++p->kc_version;
}

void Engine::clear_aliases(Problem* p) {
  if (p->n_alias > 0) slots_.free(p->alias_slot0, p->n_alias);
  p->alias_slot0 = -1;
  p->n_alias = 0;
  p->alias_of = -1;
}

void Engine::frame_centroid(Problem* p, int frame, double c[3]) {
  RK_REQUIRE(frame >= 0 && frame < p->K, RKHSBA_EINVAL, "frame out of range");
  DBuf<double> d;
  RK_HIP(d.reserve(3));
  const FrameInfo& F = p->frames[frame];
  RK_HIP(launch_frame_centroid(pts() + F.pt_off, F.n, d.p, st));
  RK_HIP(hipMemcpyAsync(c, d.p, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
  RK_HIP(hipStreamSynchronize(st));
}

void Engine::download_poses(Problem* p, double* poses) {
  RK_HIP(hipMemcpyAsync(poses, poses_ptr(p), sizeof(double) * 12 * p->K, hipMemcpyDeviceToHost, st));
  RK_HIP(hipStreamSynchronize(st));
}

void Engine::ensure_history(Problem* p, int n_iter) {
  const int64_t need = (int64_t)n_iter + 1;
  if (p->hbase >= 0 && p->n_hist >= need) return;
  if (p->hbase >= 0) hist_.free(p->hbase, p->n_hist);
  p->hbase = -1;
  p->hbase = hist_.alloc(need, st);
  p->n_hist = need;
}

void Engine::reset_state(Problem* p) {
  static const int32_t zero[2] = {0, 0};
  RK_HIP(hipMemcpyAsync(static_cast<int32_t*>(state_.ptr(0)) + 2 * p->sbase, zero, sizeof(zero),
                        hipMemcpyHostToDevice, st));
}

void Engine::read_history(Problem* p, int count, double* loss, double* pairs) {
  RK_REQUIRE(p->hbase >= 0 && count <= p->n_hist, RKHSBA_ESTATE, "no history of that length");
  if (loss)
    RK_HIP(hipMemcpyAsync(loss, static_cast<double*>(hist_.ptr(0)) + p->hbase, sizeof(double) * count,
                          hipMemcpyDeviceToHost, st));
  if (pairs)
    RK_HIP(hipMemcpyAsync(pairs, static_cast<double*>(hist_.ptr(1)) + p->hbase, sizeof(double) * count,
                          hipMemcpyDeviceToHost, st));
  RK_HIP(hipStreamSynchronize(st));
}

void Engine::read_source_counts(Problem* p, int m, int64_t* counts) {
  RK_REQUIRE(m >= 0 && m < p->K && sorted_k_ && sorted_v_, RKHSBA_ESTATE, "no evaluation to read");
  const FrameInfo& F = p->frames[m];
  std::vector<uint32_t> c(F.n), v(F.n);
  std::vector<int32_t> perm(F.n);
  RK_HIP(hipMemcpyAsync(c.data(), sc_->cnt.p, sizeof(uint32_t) * F.n, hipMemcpyDeviceToHost, st));
  RK_HIP(hipMemcpyAsync(v.data(), sorted_v_, sizeof(uint32_t) * F.n, hipMemcpyDeviceToHost, st));
  RK_HIP(hipMemcpyAsync(perm.data(), this->perm() + F.pt_off, sizeof(int32_t) * F.n, hipMemcpyDeviceToHost, st));
  RK_HIP(hipStreamSynchronize(st));
  for (int32_t i = 0; i < F.n; ++i) counts[i] = 0;
  for (int32_t e = 0; e < F.n; ++e) {
    RK_REQUIRE(v[e] < (uint32_t)F.n, RKHSBA_EDEVICE, "binning value out of range");
    counts[perm[v[e]]] = (int64_t)c[e];  // (the sweeps count zero for a source outside the target grid)
  }
}

void Engine::copy_results_async(Problem* p, int count, double* poses, double* loss, double* pairs, int32_t* state) {
  RK_REQUIRE(p->hbase >= 0 && count <= p->n_hist, RKHSBA_ESTATE, "no history of that length");
  RK_HIP(hipMemcpyAsync(poses, poses_ptr(p), sizeof(double) * 12 * p->K, hipMemcpyDeviceToHost, st));
  RK_HIP(hipMemcpyAsync(loss, static_cast<double*>(hist_.ptr(0)) + p->hbase, sizeof(double) * count,
                        hipMemcpyDeviceToHost, st));
  RK_HIP(hipMemcpyAsync(pairs, static_cast<double*>(hist_.ptr(1)) + p->hbase, sizeof(double) * count,
                        hipMemcpyDeviceToHost, st));
  RK_HIP(hipMemcpyAsync(state, static_cast<int32_t*>(state_.ptr(0)) + 2 * p->sbase, 2 * sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
}

int32_t Engine::read_status(Problem* p) {
  int32_t s[2] = {0, 0};
  RK_HIP(hipMemcpyAsync(s, static_cast<int32_t*>(state_.ptr(0)) + 2 * p->sbase, sizeof(s), hipMemcpyDeviceToHost,
                        st));
  RK_HIP(hipStreamSynchronize(st));
  return s[1];
}

// ---------------------------------------------------------------- set layout

template <typename T>
void Engine::need(DBuf<T>& b, size_t count, const char* what) {
  if (!arena_) {
    // growing frees the old buffer, which work still queued on the stream may use
    if (std::max<size_t>(count, 1) > b.n && b.p) RK_HIP(hipStreamSynchronize(st));
    RK_HIP(b.reserve(count));
    return;
  }
  T* p = arena_->take<T>(count);
  RK_REQUIRE(p != nullptr, RKHSBA_ENOMEM,
             std::string("allocation-free evaluation: the static scratch (") + std::to_string(arena_->cap) +
                 " bytes) cannot hold the layout (exhausted at '" + what + "'); use fewer edges or points");
  b.attach(p, count);
}

void Engine::set_arena(Arena* a) {
  arena_ = a;
  sc_ = a ? &arena_sc_ : &own_sc_;
  if (a) a->used = 0;
}

void Engine::prepare(SetLayout& lay, const std::vector<SetItem>& items) {
  RK_REQUIRE(!items.empty(), RKHSBA_EINVAL, "empty set");
  for (const SetItem& it : items) {
    RK_REQUIRE(it.p != nullptr, RKHSBA_ESTATE, "no frames: call rkhsba_build_neighbors first");
    RK_REQUIRE(it.E >= 1, RKHSBA_EINVAL, "need at least one edge");
    RK_REQUIRE(it.edges != nullptr, RKHSBA_EINVAL, "edges is NULL");
    RK_REQUIRE(it.fixed >= -1 && it.fixed < it.p->K, RKHSBA_EINVAL, "fixed_frame out of range");
    RK_REQUIRE(it.n_iter >= 0, RKHSBA_EINVAL, "n_iter must be >= 0");
    for (int e = 0; e < it.E; ++e) {
      const int m = it.edges[2 * e], n = it.edges[2 * e + 1];
      const int Kx = it.p->K + it.p->n_alias;
      RK_REQUIRE(m >= 0 && n >= 0 && m < Kx && n < Kx, RKHSBA_EINVAL, "edge frame index out of range");
      RK_REQUIRE(m != n || it.allow_self, RKHSBA_EINVAL, "self-edge (m == n)");
    }
    if (!arena_) ensure_history(it.p, it.n_iter);
  }
  std::vector<int32_t> key;  // (pass sizes and finalisation splits follow from the problems)
  std::vector<int> ids;
  for (const SetItem& it : items) {
    ids.push_back(it.p->id);
    key.push_back(it.p->id);
    key.push_back(it.E);
    key.push_back(it.fixed);
    key.push_back(it.n_iter);
    key.push_back((int32_t)it.p->hbase);
    key.push_back((int32_t)it.p->alias_slot0);
    key.push_back(it.allow_self ? 1 : 0);
    key.push_back(it.p->kc_version);
    key.insert(key.end(), it.edges, it.edges + 2 * it.E);
  }
  if (key == lay.edge_key && !lay.sys.empty() && !arena_) return;
  lay.drop_graph();

  int E_total = 0;
  for (const SetItem& it : items) E_total += it.E;
  std::vector<EdgeInfo> info(E_total);
  std::vector<int64_t> ent(E_total);
  std::vector<int32_t> foff(E_total);
  std::vector<SortTile> tiles;
  std::vector<SortSeg> segs;
  segs.reserve(E_total);
  std::vector<KConst> kcs(items.size());
  bool all_stacked = !items.empty();
  // one launch per group of equal pass size; group 4: per-point walks with top-k selection
  const int group_order[6] = {16, 1, 32, 64, 1, 8};
  int64_t gcount[6] = {0, 0, 0, 0, 0, 0};  // passes per group
  std::vector<int8_t> egroup(E_total);
  std::vector<ProbSys> sys(items.size());
  std::vector<int32_t> bstart_all, blist, vstart_all, vlist;
  int64_t entries = 0, passes = 0, fins = 0, h_total = 0, v_total = 0;
  int bin_bits = 3, n_max = 0;
  bool clamp = false, positive = true;
  int e_glob = 0;
  for (size_t pi = 0; pi < items.size(); ++pi) {
    const SetItem& it = items[pi];
    Problem* p = it.p;
    kcs[pi] = p->kc;
    kcs[pi].Dp = Dp;
    clamp = clamp || p->kc.clamp;
    positive = positive && p->kc.c_positive;
    bin_bits = std::max(bin_bits, p->bin_bits);
    all_stacked = all_stacked && p->stacked;
    ProbSys& S = sys[pi];
    S.K = p->K;
    S.fixed = it.fixed;
    S.n = 6 * (it.fixed >= 0 ? p->K - 1 : p->K);
    S.e0 = e_glob;
    S.E = it.E;
    S.n_iter = it.n_iter;
    S.slot0 = p->slot0;
    S.h_off = h_total;
    S.v_off = v_total;
    S.hist_off = p->hbase;
    S.state_off = 2 * p->sbase;
    S.sigma2 = p->par.sigma * p->par.sigma;
    S.damping_rel = p->par.damping_rel;
    h_total += (int64_t)S.n * S.n;
    v_total += S.n;
    n_max = std::max(n_max, S.n);
    const int K = p->K;
    std::vector<std::vector<int32_t>> blk((size_t)K * K), vec(K);
    for (int e = 0; e < it.E; ++e, ++e_glob) {
      const int m = it.edges[2 * e], n = it.edges[2 * e + 1];
      EdgeInfo& I = info[e_glob];
      auto slot_of = [&](int f) { return f < p->K ? p->slot0 + f : p->alias_slot0 + (f - p->K); };
      auto frame_of = [&](int f) -> const FrameInfo& { return p->frames[f < p->K ? f : p->alias_of]; };
      I.m = (int32_t)slot_of(m);
      I.n = (int32_t)slot_of(n);
      I.ent_off = entries;
      I.n_src = frame_of(m).n;
      const int pp = p->par.pass_points;
      const int P = pp == 1 ? 64 : pp;  // per-point walks: 64 sources (one per lane) per pass
      const int gi = p->par.top_k > 0 ? 4 : pp == 16 ? 0 : pp == 1 ? 1 : pp == 32 ? 2 : pp == 64 ? 3 : 5;
      I.pass_size = pp;
      // binning segments: the source frame's label layers (a pass's sources then share one class id), or
      // the whole frame
      I.seg0 = (int32_t)segs.size();
      I.n_pass = 0;
      {
        const int mf = m < K ? m : p->alias_of;
        std::vector<std::pair<int64_t, int64_t>> parts;  // (first source point, count)
        if (p->stacked) {
          const int32_t* ls = p->lab_start.data() + p->lab_off[mf];
          for (int L = 0; L < p->frames[mf].n_lab; ++L)
            if (ls[L + 1] > ls[L]) parts.emplace_back(ls[L], ls[L + 1] - ls[L]);
        } else if (I.n_src > 0) {
          parts.emplace_back(0, I.n_src);
        }
        for (const auto& pr : parts) {
          SortSeg S0;
          S0.start = entries + pr.first;
          S0.count = pr.second;
          S0.tile0 = (int32_t)tiles.size();
          for (int64_t s = 0; s < pr.second; s += kSortTile)
            tiles.push_back(SortTile{S0.start + s, (int32_t)std::min<int64_t>(kSortTile, pr.second - s),
                                     (int32_t)segs.size(), e_glob, 0});
          S0.n_tiles = (int32_t)tiles.size() - S0.tile0;
          segs.push_back(S0);
          I.n_pass += (int32_t)((pr.second + P - 1) / P);
        }
      }
      I.n_seg = (int32_t)segs.size() - I.seg0;
      I.fin_off = (int32_t)fins;
      // finalisation split from the edge's own size: 1..16 entries per thread
      I.fin_pt = std::min(16, std::max(1, I.n_src / 4096));
      I.n_fin = (I.n_src + kFinThreads * I.fin_pt - 1) / (kFinThreads * I.fin_pt);
      I.prob = (int32_t)pi;
      gcount[gi] += I.n_pass;  // pass0 is assigned below, once every edge's target is known
      egroup[e_glob] = (int8_t)gi;
      ent[e_glob] = entries;
      foff[e_glob] = I.fin_off;
      entries += I.n_src;
      passes += I.n_pass;
      fins += I.n_fin;
      if (m != n && m < K && n < K) {  // self and alias edges are evaluated but never assembled
        blk[(size_t)m * K + m].push_back(e_glob * 4 + 0);
        blk[(size_t)n * K + n].push_back(e_glob * 4 + 1);
        blk[(size_t)m * K + n].push_back(e_glob * 4 + 2);
        blk[(size_t)n * K + m].push_back(e_glob * 4 + 3);
        vec[m].push_back(e_glob * 2 + 0);
        vec[n].push_back(e_glob * 2 + 1);
      }
    }
    S.blk0 = (int32_t)bstart_all.size();
    for (size_t k = 0; k < blk.size(); ++k) {
      bstart_all.push_back((int32_t)blist.size());
      blist.insert(blist.end(), blk[k].begin(), blk[k].end());
    }
    bstart_all.push_back((int32_t)blist.size());
    S.vec0 = (int32_t)vstart_all.size();
    for (int k = 0; k < K; ++k) {
      vstart_all.push_back((int32_t)vlist.size());
      vlist.insert(vlist.end(), vec[k].begin(), vec[k].end());
    }
    vstart_all.push_back((int32_t)vlist.size());
  }
  RK_REQUIRE(passes < INT_MAX && fins < INT_MAX && entries < (int64_t)INT_MAX * 4 && blist.size() < INT_MAX,
             RKHSBA_EINVAL, "edge list too large");
  if (blist.empty()) blist.push_back(0);
  if (vlist.empty()) vlist.push_back(0);
  need(lay.d_edges, E_total, "edges");
  need(lay.d_ent_off, E_total, "ent_off");
  need(lay.d_fin_off, E_total, "fin_off");
  need(lay.d_etiles, tiles.size(), "etiles");
  need(lay.d_esegs, std::max<size_t>(segs.size(), 1), "esegs");
  // the pass table: the groups one after another, each edge's passes contiguous (filled on the device)
  std::vector<SetLayout::Group> groups;
  int64_t gbase[6], n_pass_table = 0;
  for (int gi = 0; gi < 6; ++gi) {
    gbase[gi] = n_pass_table;
    if (gcount[gi] == 0) continue;
    groups.push_back(SetLayout::Group{group_order[gi], (int)n_pass_table, (int)gcount[gi], gi == 4});
    n_pass_table += gcount[gi];
  }
  // Inside a group, the passes of edges that share a target frame are placed next to each other: the
  // passes in flight at one time then read candidates from the same frame, which stays in the L2.  The
  // results do not depend on this order (every pass writes its own entries).
  {
    std::vector<int> order(E_total);
    for (int e = 0; e < E_total; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return egroup[x] != egroup[y] ? egroup[x] < egroup[y] : info[x].n < info[y].n;
    });
    int64_t run[6] = {0, 0, 0, 0, 0, 0};
    for (int e : order) {
      const int gi = egroup[e];
      info[e].pass0 = (int32_t)(gbase[gi] + run[gi]);
      run[gi] += info[e].n_pass;
    }
  }
  need(lay.d_kcs, items.size(), "kcs");
  need(lay.d_passes, (size_t)n_pass_table, "passes");
  need(lay.d_sys, items.size(), "sys");
  need(lay.d_blk_start, bstart_all.size(), "blk_start");
  need(lay.d_blk_list, blist.size(), "blk_list");
  need(lay.d_vec_start, vstart_all.size(), "vec_start");
  need(lay.d_vec_list, vlist.size(), "vec_list");
  // The host tables go to the device through the layout's pinned staging buffer, whose previous uploads
  // must have completed before it is rewritten (the host then need not wait for the stream here).
  size_t stage_bytes = 0;
  auto stage_size = [&](size_t bytes) { stage_bytes += (bytes + 255) & ~(size_t)255; };
  stage_size(sizeof(EdgeInfo) * E_total);
  stage_size(sizeof(int64_t) * E_total);
  stage_size(sizeof(int32_t) * E_total);
  stage_size(sizeof(SortTile) * tiles.size());
  stage_size(sizeof(SortSeg) * segs.size());
  stage_size(sizeof(KConst) * kcs.size());
  stage_size(sizeof(ProbSys) * sys.size());
  stage_size(sizeof(int32_t) * bstart_all.size());
  stage_size(sizeof(int32_t) * blist.size());
  stage_size(sizeof(int32_t) * vstart_all.size());
  stage_size(sizeof(int32_t) * vlist.size());
  uint8_t* stage = lay.stage_for(stage_bytes, arena_ != nullptr);
  size_t stage_off = 0;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (!stage) {
      RK_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
      return;
    }
    std::memcpy(stage + stage_off, src, bytes);
    RK_HIP(hipMemcpyAsync(dst, stage + stage_off, bytes, hipMemcpyHostToDevice, st));
    stage_off += (bytes + 255) & ~(size_t)255;
  };
  up(lay.d_edges.p, info.data(), sizeof(EdgeInfo) * E_total);
  up(lay.d_ent_off.p, ent.data(), sizeof(int64_t) * E_total);
  up(lay.d_fin_off.p, foff.data(), sizeof(int32_t) * E_total);
  up(lay.d_etiles.p, tiles.data(), sizeof(SortTile) * tiles.size());
  up(lay.d_esegs.p, segs.data(), sizeof(SortSeg) * segs.size());
  up(lay.d_kcs.p, kcs.data(), sizeof(KConst) * kcs.size());
  RK_HIP(launch_fill_passes(lay.d_edges.p, E_total, frames(), lay.d_esegs.p, lay.d_passes.p, st));
  up(lay.d_sys.p, sys.data(), sizeof(ProbSys) * sys.size());
  up(lay.d_blk_start.p, bstart_all.data(), sizeof(int32_t) * bstart_all.size());
  up(lay.d_blk_list.p, blist.data(), sizeof(int32_t) * blist.size());
  up(lay.d_vec_start.p, vstart_all.data(), sizeof(int32_t) * vstart_all.size());
  up(lay.d_vec_list.p, vlist.data(), sizeof(int32_t) * vlist.size());

  // per-evaluation scratch
  const void* before[] = {sc_->xf.p, sc_->bk.p, sc_->bv.p, sc_->bk2.p, sc_->bv2.p, sc_->bhist.p, sc_->mom.p, sc_->cnt.p, sc_->partial.p, sc_->edge_out.p,
                          sc_->H.p, sc_->b.p, sc_->delta.p};
  need(sc_->xf, E_total, "xf");
  need(sc_->bk, entries, "bk");
  need(sc_->bv, entries, "bv");
  need(sc_->bk2, entries, "bk2");
  need(sc_->bv2, entries, "bv2");
  need(sc_->bhist, tiles.size() * 256, "bhist");
  need(sc_->mom, (size_t)entries * (arena_ ? arena_->mom_components : 10), "mom");
  need(sc_->cnt, entries, "cnt");
  need(sc_->partial, (size_t)fins * kFinStats, "partial");
  need(sc_->edge_out, (size_t)E_total * kEdgeVals, "edge_out");
  need(sc_->H, h_total, "H");
  need(sc_->b, v_total, "b");
  need(sc_->delta, v_total, "delta");
  const void* after[] = {sc_->xf.p, sc_->bk.p, sc_->bv.p, sc_->bk2.p, sc_->bv2.p, sc_->bhist.p, sc_->mom.p, sc_->cnt.p, sc_->partial.p, sc_->edge_out.p,
                         sc_->H.p, sc_->b.p, sc_->delta.p};
  if (!arena_)
    for (size_t i = 0; i < sizeof(before) / sizeof(before[0]); ++i)
      if (before[i] != after[i]) ++scratch_gen_;
  if (stage) {
    RK_HIP(hipEventRecord(lay.stage_ev, st));  // the staging buffer is free again once this completes
  } else {
    RK_HIP(hipStreamSynchronize(st));  // host tables above go out of scope
  }

  lay.uses = 0;
  lay.binned = false;
  lay.ids = std::move(ids);
  lay.edge_key = std::move(key);
  lay.sys = std::move(sys);
  lay.n_prob = (int)items.size();
  lay.n_max = n_max;
  lay.E = E_total;
  lay.n_entries = entries;
  lay.n_pass_total = (int)passes;
  lay.groups = std::move(groups);
  lay.n_fin_total = (int)fins;
  lay.n_edge_tiles = (int)tiles.size();
  lay.n_edge_segs = (int)segs.size();
  lay.stacked = all_stacked;
  lay.bin_bits = bin_bits;
  lay.clamp = clamp;
  lay.c_positive = positive && !items.empty();
  lay.h_total = h_total;
  lay.v_total = v_total;
}

// ---------------------------------------------------------------- launches

// Pass sizes that the tiled sweep takes (16 points; 8 or 32 with class ids); the others (per-point walks, 32 or
// 64 points with dense features) run in the untiled pass kernel.
static bool tiled_sweep(int pass_points, int feat_kind) {
  return pass_points == 16 || ((pass_points == 8 || pass_points == 32) && feat_kind == RKHSBA_FEAT_CLASS_ID);
}

void Engine::evaluate(SetLayout& lay, int mode, bool reuse_binning) {
  RK_REQUIRE(!arena_ || mode == MODE_LOSS || arena_->mom_components == 10, RKHSBA_ESTATE,
             "the arena holds loss-evaluation moments only");
  hipEvent_t t0 = prof_begin();
  RK_HIP(launch_edge_setup(poses(), lay.d_edges.p, lay.E, sc_->xf.p, st));
  const bool reuse = reuse_binning && lay.binned && binned_lay_ == &lay && lay.bin_sc == sc_ &&
                     lay.bin_gen == scratch_gen_;
  if (reuse) {
    sorted_k_ = lay.bin_k;
    sorted_v_ = lay.bin_v;
    // The keys are read only for their out-of-grid bit, and only by the per-point walks and the larger passes:
    // the tiled sweeps test the grid from the transformed point themselves.
    bool keys_read = false;
    for (const SetLayout::Group& gr : lay.groups) keys_read = keys_read || !tiled_sweep(gr.pass_points, feat_kind);
    if (keys_read)
      RK_HIP(launch_bin(pts(), frames(), lay.d_edges.p, lay.d_etiles.p, lay.n_edge_tiles, sc_->xf.p, lay.d_kcs.p,
                        const_cast<uint32_t*>(sorted_k_), const_cast<uint32_t*>(sorted_v_), true, st));
  } else {
    RK_HIP(launch_bin(pts(), frames(), lay.d_edges.p, lay.d_etiles.p, lay.n_edge_tiles, sc_->xf.p, lay.d_kcs.p,
                      sc_->bk.p, sc_->bv.p, false, st));
    bool in_tmp = false;
    RK_HIP(launch_radix_sort(sc_->bk.p, sc_->bv.p, sc_->bk2.p, sc_->bv2.p, sc_->bhist.p, lay.d_etiles.p,
                             lay.n_edge_tiles, lay.d_esegs.p, lay.n_edge_segs, lay.bin_bits, st, &in_tmp));
    sorted_k_ = in_tmp ? sc_->bk2.p : sc_->bk.p;
    sorted_v_ = in_tmp ? sc_->bv2.p : sc_->bv.p;
    lay.binned = true;
    lay.bin_gen = scratch_gen_;
    lay.bin_sc = sc_;
    lay.bin_k = sorted_k_;
    lay.bin_v = sorted_v_;
    binned_lay_ = &lay;
  }
  prof_end(RKHSBA_PROF_BIN, t0);
  PairArgs pa{};
  pa.pts = pts();
  pa.feat = feat();
  pa.rows = rows();
  pa.xtab = xtab();
  pa.frames = frames();
  pa.edges = lay.d_edges.p;
  pa.xf = sc_->xf.p;
  pa.keys = sorted_k_;
  pa.vals = sorted_v_;
  pa.mom = sc_->mom.p;
  pa.cnt = sc_->cnt.p;
  pa.kcs = lay.d_kcs.p;
  pa.passes = lay.d_passes.p;
  pa.perm = perm();
  pa.n_entries = lay.n_entries;
  pa.E = lay.E;

  pa.kc.Dp = Dp;
  pa.kc.clamp = lay.clamp ? 1 : 0;
  pa.kc.c_positive = lay.c_positive ? 1 : 0;
  pa.stacked = lay.stacked && feat_kind == RKHSBA_FEAT_CLASS_ID ? 1 : 0;
  const int feat_path = feat_kind;
  hipEvent_t t1 = prof_begin();
  for (const SetLayout::Group& gr : lay.groups) {
    pa.pass0 = gr.pass0;
    pa.n_pass = gr.n_pass;
    if (tiled_sweep(gr.pass_points, feat_kind))
      RK_HIP(launch_sweep(pa, mode, feat_path, gr.pass_points, moment_path == 2 && !source_counts,
                          source_counts && mode == MODE_NORMAL, st));
    else
      RK_HIP(launch_pairs(pa, mode, feat_path, gr.pass_points, gr.topk, st));
  }
  prof_end(mode == MODE_NORMAL ? RKHSBA_PROF_PAIRS : RKHSBA_PROF_PAIRS_LOSS, t1);
  FinArgs fa{};
  fa.pts = pts();
  fa.edges = lay.d_edges.p;
  fa.xf = sc_->xf.p;
  fa.frames = frames();
  fa.keys = sorted_k_;
  fa.vals = sorted_v_;
  fa.mom = sc_->mom.p;
  fa.cnt = sc_->cnt.p;
  fa.kcs = lay.d_kcs.p;
  fa.partial = sc_->partial.p;
  fa.n_entries = lay.n_entries;
  fa.E = lay.E;
  fa.n_fin_total = lay.n_fin_total;
  hipEvent_t t2 = prof_begin();
  RK_HIP(launch_finalize(fa, lay.d_fin_off.p, mode, fp32_sums, st));
  RK_HIP(launch_edge_reduce(sc_->partial.p, lay.d_edges.p, sc_->xf.p, lay.E, mode, fp32_sums, sc_->edge_out.p, st));
  prof_end(RKHSBA_PROF_FINALIZE, t2);
}

SolveArgs Engine::solve_args(SetLayout& lay) {
  SolveArgs s{};
  s.edge_out = sc_->edge_out.p;
  s.sys = lay.d_sys.p;
  s.n_prob = lay.n_prob;
  s.n_max = lay.n_max;
  s.H = sc_->H.p;
  s.b = sc_->b.p;
  s.delta = sc_->delta.p;
  s.poses = poses();
  s.loss_hist = static_cast<double*>(hist_.ptr(0));
  s.pairs_hist = static_cast<double*>(hist_.ptr(1));
  s.state = static_cast<int32_t*>(state_.ptr(0));
  s.blk_start = lay.d_blk_start.p;
  s.blk_list = lay.d_blk_list.p;
  s.vec_start = lay.d_vec_start.p;
  s.vec_list = lay.d_vec_list.p;
  return s;
}

void Engine::assemble(SetLayout& lay) { RK_HIP(launch_assemble(solve_args(lay), st)); }

void Engine::loss_only(SetLayout& lay) { RK_HIP(launch_loss_only(solve_args(lay), st)); }

void Engine::solve(SetLayout& lay) {
  hipEvent_t t = prof_begin();
  RK_HIP(launch_solve_update(solve_args(lay), st));
  prof_end(RKHSBA_PROF_SOLVE, t);
}

void Engine::record_iteration(SetLayout& lay, bool reuse_binning) {
  evaluate(lay, MODE_NORMAL, reuse_binning);
  hipEvent_t t = prof_begin();
  RK_HIP(launch_assemble(solve_args(lay), st));
  RK_HIP(launch_solve_update(solve_args(lay), st));
  prof_end(RKHSBA_PROF_SOLVE, t);
}

void Engine::iterate(SetLayout& lay, int n, bool continue_binning) {
  if (n <= 0) return;
  // A graph pays for its capture only when it is replayed: capture on a
  // layout's second use, or when this call runs several iterations.
  const bool graph = use_graphs && !prof && (n > 1 || lay.uses >= graph_min_uses);
  ++lay.uses;
  // The first iteration bins the sources afresh; the later ones keep its order (see evaluate).  With
  // continue_binning, an iteration right after one of the same layout keeps that order too.
  const bool warm = continue_binning && lay.binned && binned_lay_ == &lay && lay.bin_sc == sc_ &&
                    lay.bin_gen == scratch_gen_;
  if (!graph) {
    for (int i = 0; i < n; ++i) record_iteration(lay, i > 0 || warm);
    return;
  }
  const uint64_t g = generation();
  auto capture = [&](bool reuse) -> hipGraphExec_t {
    RK_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipGraph_t graph = nullptr;
    try {
      record_iteration(lay, reuse);
    } catch (...) {
      (void)hipStreamEndCapture(st, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    RK_HIP(hipStreamEndCapture(st, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    RK_HIP(e);
    return exec;
  };
  if (!warm && (!lay.graph || lay.graph_gen != g)) {
    if (lay.graph) (void)hipGraphExecDestroy(lay.graph);
    lay.graph = nullptr;
    lay.graph = capture(false);
    lay.graph_gen = g;
    lay.graph_mode = MODE_NORMAL;
  }
  // the replay bins into the scratch as the capture did: the host-side record of the binning follows it
  binned_lay_ = &lay;
  lay.binned = true;
  if ((warm || n > 1) && (!lay.graph_rest || lay.graph_rest_gen != g)) {
    if (lay.graph_rest) (void)hipGraphExecDestroy(lay.graph_rest);
    lay.graph_rest = nullptr;
    lay.graph_rest = capture(true);
    lay.graph_rest_gen = g;
  }
  if (!warm) RK_HIP(hipGraphLaunch(lay.graph, st));
  for (int i = warm ? 0 : 1; i < n; ++i) RK_HIP(hipGraphLaunch(lay.graph_rest, st));
}

}  // namespace rkhsba
