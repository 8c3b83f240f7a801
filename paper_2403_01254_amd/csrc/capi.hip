// Host side of the rkhsba C ABI: context, HBM buffers, argument validation and
// the launch sequences of build_neighbors / eval_loss /
// accumulate_normal_eqs / gn_step.  No exception crosses the ABI.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rkhsba.h"
#include "rkhsba_internal.h"


using namespace rkhsba;

namespace {

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  // Ensures room for `count` elements; contents are not preserved.
  hipError_t reserve(size_t count) {
    if (count == 0) count = 1;
    if (count <= n) return hipSuccess;
    release();
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = count;
    return hipSuccess;
  }
};

struct Fail {
  int code;
};

}  // namespace

struct rkhsba_ctx {
  rkhsba_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  KConst kc{};

  // frames (resident between calls)
  int K = 0;
  int feat_kind = 0, D = 0, Dp = 0;
  int64_t n_total = 0;
  std::vector<FrameInfo> frames;
  std::vector<int64_t> in_off;  // K+1
  int bin_bits = 0;
  bool negative_features = false;  // some dense feature value < 0: inner products may be negative
  DBuf<float4> pts;
  DBuf<float> feat;
  DBuf<int32_t> perm;
  DBuf<uint32_t> keys;
  DBuf<int4> rows;
  DBuf<uint32_t> xtab;
  DBuf<FrameInfo> d_frames;
  DBuf<int64_t> d_in_off;

  // build scratch
  DBuf<float> raw_xyz;
  DBuf<uint8_t> raw_feat;
  DBuf<const float*> d_xyz_ptrs;
  DBuf<const void*> d_feat_ptrs;
  DBuf<int32_t> cell;
  DBuf<int32_t> minmax;
  DBuf<uint32_t> k1, v1, k2, v2;
  DBuf<uint32_t> hist;
  DBuf<SortTile> d_tiles;
  DBuf<SortSeg> d_segs;
  DBuf<uint32_t> row_sizes, scan_tmp;
  DBuf<uint64_t> d_total;

  // edge list layout (cached for the last edge list)
  std::vector<int32_t> edge_list;
  int E = 0;
  int64_t n_entries = 0;
  int n_pass_total = 0, n_fin_total = 0, n_edge_tiles = 0;
  std::vector<EdgeInfo> edges;
  DBuf<EdgeInfo> d_edges;
  DBuf<int64_t> d_ent_off;
  DBuf<int32_t> d_pass_off, d_fin_off;
  DBuf<SortTile> d_etiles;
  DBuf<SortSeg> d_esegs;
  DBuf<int32_t> d_blk_start, d_blk_list, d_vec_start, d_vec_list;  // system assembly lists

  // per-evaluation buffers
  DBuf<double> d_poses;
  DBuf<EdgeXf> d_xf;
  DBuf<uint32_t> bk, bv, bk2, bv2, bhist;
  DBuf<float> mom;
  DBuf<uint32_t> cnt;
  DBuf<double> partial, edge_out;
  DBuf<double> H, b, delta, loss_hist, pairs_hist;
  DBuf<int32_t> status;
  const uint32_t* sorted_k = nullptr;
  const uint32_t* sorted_v = nullptr;

  // stage timing (HIP events on the context's stream), off unless enabled
  bool prof = false;
  struct Stage {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0.0;
    int64_t launches = 0;
  } stages[RKHSBA_PROF_STAGES];
  std::vector<hipEvent_t> event_pool;
  ~rkhsba_ctx() {
    for (auto& st : stages)
      for (auto& pr : st.pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
    for (hipEvent_t ev : event_pool) (void)hipEventDestroy(ev);
  }
};

namespace {

int fail(rkhsba_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define RK_HIP(expr)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) {                                                                        \
      throw Fail{fail(c, e_ == hipErrorOutOfMemory ? RKHSBA_ENOMEM : RKHSBA_EDEVICE,              \
                      std::string(#expr) + ": " + hipGetErrorString(e_))};                         \
    }                                                                                              \
  } while (0)

#define RK_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw Fail{fail(c, (code), (msg))}; \
  } while (0)

template <typename F>
int guarded(rkhsba_ctx* c, F&& body) {
  if (!c) return RKHSBA_EINVAL;
  c->err.clear();
  try {
    if (hipSetDevice(c->opt.device) != hipSuccess) return fail(c, RKHSBA_EDEVICE, "hipSetDevice failed");
    return body();
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::bad_alloc&) {
    return fail(c, RKHSBA_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(c, RKHSBA_EDEVICE, "unexpected exception");
  }
}

hipEvent_t prof_event(rkhsba_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t ev = c->event_pool.back();
    c->event_pool.pop_back();
    return ev;
  }
  hipEvent_t ev = nullptr;
  if (hipEventCreate(&ev) != hipSuccess) return nullptr;
  return ev;
}

// Brackets the launches of one stage with events when profiling is on.
hipEvent_t prof_begin(rkhsba_ctx* c) {
  if (!c->prof) return nullptr;
  hipEvent_t ev = prof_event(c);
  if (ev) (void)hipEventRecord(ev, c->stream);
  return ev;
}

void prof_end(rkhsba_ctx* c, int stage, hipEvent_t start) {
  if (!c->prof || !start) return;
  hipEvent_t ev = prof_event(c);
  if (!ev) return;
  (void)hipEventRecord(ev, c->stream);
  c->stages[stage].pending.emplace_back(start, ev);
}

// After the stream has been synchronised: accumulate the recorded intervals.
void prof_collect(rkhsba_ctx* c) {
  for (auto& st : c->stages) {
    for (auto& pr : st.pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        st.ms += ms;
        st.launches += 1;
      }
      c->event_pool.push_back(pr.first);
      c->event_pool.push_back(pr.second);
    }
    st.pending.clear();
  }
}

void compute_constants(rkhsba_ctx* c) {
  const rkhsba_options& o = c->opt;
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
  k.clamp = (o.clamp_negative_c && c->negative_features) ? 1 : 0;
  k.Dp = c->Dp;
  c->kc = k;
}

void check_poses(rkhsba_ctx* c, const double* poses) {
  RK_REQUIRE(poses != nullptr, RKHSBA_EINVAL, "poses is NULL");
  for (int i = 0; i < 12 * c->K; ++i) RK_REQUIRE(std::isfinite(poses[i]), RKHSBA_EINVAL, "non-finite pose entry");
}

// Host-side layout of an edge list: binning entries (one per source point),
// sweep passes of pass_points entries, finalisation blocks and sort tiles.
void prepare_edges(rkhsba_ctx* c, int E, const int32_t* edges) {
  RK_REQUIRE(c->K > 0, RKHSBA_ESTATE, "no frames: call rkhsba_build_neighbors first");
  RK_REQUIRE(E >= 1, RKHSBA_EINVAL, "need at least one edge");
  RK_REQUIRE(edges != nullptr, RKHSBA_EINVAL, "edges is NULL");
  for (int e = 0; e < E; ++e) {
    const int m = edges[2 * e], n = edges[2 * e + 1];
    RK_REQUIRE(m >= 0 && n >= 0 && m < c->K && n < c->K, RKHSBA_EINVAL, "edge frame index out of range");
    RK_REQUIRE(m != n, RKHSBA_EINVAL, "self-edge (m == n)");
  }
  std::vector<int32_t> list(edges, edges + 2 * E);
  if (list == c->edge_list) return;
  const int P = c->opt.pass_points;
  std::vector<EdgeInfo> info(E);
  std::vector<int64_t> ent(E);
  std::vector<int32_t> poff(E), foff(E);
  std::vector<SortTile> tiles;
  std::vector<SortSeg> segs(E);
  int64_t entries = 0;
  int64_t passes = 0, fins = 0;
  for (int e = 0; e < E; ++e) {
    EdgeInfo& I = info[e];
    I.m = edges[2 * e];
    I.n = edges[2 * e + 1];
    I.ent_off = entries;
    I.n_src = c->frames[I.m].n;
    I.pass_off = (int32_t)passes;
    I.n_pass = (I.n_src + P - 1) / P;
    I.fin_off = (int32_t)fins;
    I.n_fin = (I.n_src + kFinThreads - 1) / kFinThreads;
    I.pad = 0;
    ent[e] = entries;
    poff[e] = I.pass_off;
    foff[e] = I.fin_off;
    segs[e].start = entries;
    segs[e].count = I.n_src;
    segs[e].tile0 = (int32_t)tiles.size();
    for (int64_t s = 0; s < I.n_src; s += kSortTile)
      tiles.push_back(SortTile{entries + s, (int32_t)std::min<int64_t>(kSortTile, I.n_src - s), e});
    segs[e].n_tiles = (int32_t)tiles.size() - segs[e].tile0;
    entries += I.n_src;
    passes += I.n_pass;
    fins += I.n_fin;
  }
  RK_REQUIRE(passes < INT_MAX && fins < INT_MAX && entries < (int64_t)INT_MAX * 4, RKHSBA_EINVAL,
             "edge list too large");
  hipStream_t st = c->stream;
  RK_HIP(c->d_edges.reserve(E));
  RK_HIP(c->d_ent_off.reserve(E));
  RK_HIP(c->d_pass_off.reserve(E));
  RK_HIP(c->d_fin_off.reserve(E));
  RK_HIP(c->d_etiles.reserve(tiles.size()));
  RK_HIP(c->d_esegs.reserve(E));
  RK_HIP(hipMemcpyAsync(c->d_edges.p, info.data(), sizeof(EdgeInfo) * E, hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_ent_off.p, ent.data(), sizeof(int64_t) * E, hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_pass_off.p, poff.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_fin_off.p, foff.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice, st));
  if (!tiles.empty())
    RK_HIP(hipMemcpyAsync(c->d_etiles.p, tiles.data(), sizeof(SortTile) * tiles.size(), hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_esegs.p, segs.data(), sizeof(SortSeg) * E, hipMemcpyHostToDevice, st));
  // contributors of every 6x6 block of H and every 6-vector of b, in edge order
  const int K = c->K;
  std::vector<std::vector<int32_t>> blk((size_t)K * K), vec(K);
  for (int e = 0; e < E; ++e) {
    const int m = info[e].m, n = info[e].n;
    blk[(size_t)m * K + m].push_back(e * 4 + 0);
    blk[(size_t)n * K + n].push_back(e * 4 + 1);
    blk[(size_t)m * K + n].push_back(e * 4 + 2);
    blk[(size_t)n * K + m].push_back(e * 4 + 3);
    vec[m].push_back(e * 2 + 0);
    vec[n].push_back(e * 2 + 1);
  }
  std::vector<int32_t> bstart((size_t)K * K + 1, 0), blist, vstart(K + 1, 0), vlist;
  for (size_t k = 0; k < blk.size(); ++k) {
    bstart[k] = (int32_t)blist.size();
    blist.insert(blist.end(), blk[k].begin(), blk[k].end());
  }
  bstart[blk.size()] = (int32_t)blist.size();
  for (int k = 0; k < K; ++k) {
    vstart[k] = (int32_t)vlist.size();
    vlist.insert(vlist.end(), vec[k].begin(), vec[k].end());
  }
  vstart[K] = (int32_t)vlist.size();
  RK_HIP(c->d_blk_start.reserve(bstart.size()));
  RK_HIP(c->d_blk_list.reserve(blist.size()));
  RK_HIP(c->d_vec_start.reserve(vstart.size()));
  RK_HIP(c->d_vec_list.reserve(vlist.size()));
  RK_HIP(hipMemcpyAsync(c->d_blk_start.p, bstart.data(), sizeof(int32_t) * bstart.size(), hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_blk_list.p, blist.data(), sizeof(int32_t) * blist.size(), hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_vec_start.p, vstart.data(), sizeof(int32_t) * vstart.size(), hipMemcpyHostToDevice, st));
  RK_HIP(hipMemcpyAsync(c->d_vec_list.p, vlist.data(), sizeof(int32_t) * vlist.size(), hipMemcpyHostToDevice, st));
  // per-evaluation buffers sized for this list
  RK_HIP(c->d_xf.reserve(E));
  RK_HIP(c->bk.reserve(entries));
  RK_HIP(c->bv.reserve(entries));
  RK_HIP(c->bk2.reserve(entries));
  RK_HIP(c->bv2.reserve(entries));
  RK_HIP(c->bhist.reserve(tiles.size() * 256));
  RK_HIP(c->mom.reserve((size_t)entries * 10));
  RK_HIP(c->cnt.reserve(entries));
  RK_HIP(c->partial.reserve((size_t)fins * kEdgeVals));
  RK_HIP(c->edge_out.reserve((size_t)E * kEdgeVals));
  RK_HIP(hipStreamSynchronize(st));  // host vectors above go out of scope
  c->edges = std::move(info);
  c->E = E;
  c->n_entries = entries;
  c->n_pass_total = (int)passes;
  c->n_fin_total = (int)fins;
  c->n_edge_tiles = (int)tiles.size();
  c->edge_list = std::move(list);
}

void upload_poses(rkhsba_ctx* c, const double* poses) {
  check_poses(c, poses);
  RK_HIP(c->d_poses.reserve((size_t)12 * c->K));
  RK_HIP(hipMemcpyAsync(c->d_poses.p, poses, sizeof(double) * 12 * c->K, hipMemcpyHostToDevice, c->stream));
}

// Transforms, binning, sweep, finalisation and per-edge reduction at the
// device poses; leaves per-edge sums in c->edge_out.
void evaluate(rkhsba_ctx* c, int mode) {
  hipStream_t st = c->stream;
  hipEvent_t t0 = prof_begin(c);
  RK_HIP(launch_edge_setup(c->d_poses.p, c->d_edges.p, c->E, c->d_xf.p, st));
  RK_HIP(launch_bin(c->pts.p, c->d_frames.p, c->d_edges.p, c->d_ent_off.p, c->d_xf.p, c->E, c->n_entries, c->kc,
                    c->bk.p, c->bv.p, st));
  bool in_tmp = false;
  RK_HIP(launch_radix_sort(c->bk.p, c->bv.p, c->bk2.p, c->bv2.p, c->bhist.p, c->d_etiles.p, c->n_edge_tiles,
                           c->d_esegs.p, c->E, c->bin_bits, st, &in_tmp));
  c->sorted_k = in_tmp ? c->bk2.p : c->bk.p;
  c->sorted_v = in_tmp ? c->bv2.p : c->bv.p;
  prof_end(c, RKHSBA_PROF_BIN, t0);
  PairArgs pa{};
  pa.pts = c->pts.p;
  pa.feat = c->feat.p;
  pa.rows = c->rows.p;
  pa.xtab = c->xtab.p;
  pa.frames = c->d_frames.p;
  pa.edges = c->d_edges.p;
  pa.xf = c->d_xf.p;
  pa.keys = c->sorted_k;
  pa.vals = c->sorted_v;
  pa.mom = c->mom.p;
  pa.cnt = c->cnt.p;
  pa.n_entries = c->n_entries;
  pa.E = c->E;
  pa.n_pass_total = c->n_pass_total;
  pa.kc = c->kc;
  const int feat_path = c->feat_kind == RKHSBA_FEAT_CLASS_ID ? FEAT_CLASS : FEAT_DENSE;
  hipEvent_t t1 = prof_begin(c);
  if (c->opt.pass_points == 16) {
    // vector-ALU moments measured faster on both feature kinds; the matrix-core variant stays selectable
    const bool mm = c->opt.moment_path == 2;
    RK_HIP(launch_sweep16(pa, c->d_pass_off.p, mode, feat_path, mm, st));
  }
  else
    RK_HIP(launch_pairs(pa, c->d_pass_off.p, mode, feat_path, c->opt.pass_points, st));
  prof_end(c, mode == MODE_NORMAL ? RKHSBA_PROF_PAIRS : RKHSBA_PROF_PAIRS_LOSS, t1);
  FinArgs fa{};
  fa.pts = c->pts.p;
  fa.edges = c->d_edges.p;
  fa.xf = c->d_xf.p;
  fa.frames = c->d_frames.p;
  fa.keys = c->sorted_k;
  fa.vals = c->sorted_v;
  fa.mom = c->mom.p;
  fa.cnt = c->cnt.p;
  fa.partial = c->partial.p;
  fa.n_entries = c->n_entries;
  fa.E = c->E;
  fa.n_fin_total = c->n_fin_total;
  hipEvent_t t2 = prof_begin(c);
  RK_HIP(launch_finalize(fa, c->d_fin_off.p, mode, st));
  RK_HIP(launch_edge_reduce(c->partial.p, c->d_edges.p, c->E, kEdgeVals, c->edge_out.p, st));
  prof_end(c, RKHSBA_PROF_FINALIZE, t2);
}

SolveArgs solve_args(rkhsba_ctx* c, int fixed, int iter) {
  SolveArgs s{};
  s.edge_out = c->edge_out.p;
  s.edges = c->d_edges.p;
  s.E = c->E;
  s.K = c->K;
  s.fixed = fixed;
  s.sigma2 = c->opt.sigma * c->opt.sigma;
  s.damping_rel = c->opt.damping_rel;
  s.H = c->H.p;
  s.b = c->b.p;
  s.delta = c->delta.p;
  s.poses = c->d_poses.p;
  s.loss_hist = c->loss_hist.p;
  s.pairs_hist = c->pairs_hist.p;
  s.status = c->status.p;
  s.iter = iter;
  s.blk_start = c->d_blk_start.p;
  s.blk_list = c->d_blk_list.p;
  s.vec_start = c->d_vec_start.p;
  s.vec_list = c->d_vec_list.p;
  return s;
}

void ensure_system(rkhsba_ctx* c, int n, int hist) {
  RK_HIP(c->H.reserve((size_t)n * n));
  RK_HIP(c->b.reserve(n));
  RK_HIP(c->delta.reserve(n));
  RK_HIP(c->loss_hist.reserve(hist));
  RK_HIP(c->pairs_hist.reserve(hist));
  RK_HIP(c->status.reserve(1));
}

}  // namespace

extern "C" {

void rkhsba_default_options(rkhsba_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->ell = 0.1;
  o->cutoff_factor = 3.0;
  o->sigma = 1.0;
  o->damping_rel = 1e-10;
  o->fixed_frame = 0;
  o->clamp_negative_c = 1;
  o->device = 0;
  o->cell_subdiv = 8;
  o->pass_points = 16;
  o->stream = nullptr;
}

int rkhsba_create(rkhsba_ctx** out, const rkhsba_options* opt) {
  if (!out) return RKHSBA_EINVAL;
  *out = nullptr;
  if (!opt) return RKHSBA_EINVAL;
  if (!(opt->ell > 0.0) || !std::isfinite(opt->ell) || !(opt->cutoff_factor > 0.0) ||
      !std::isfinite(opt->cutoff_factor) || !std::isfinite(opt->sigma) || !(opt->damping_rel >= 0.0) ||
      opt->cell_subdiv < 1 || opt->cell_subdiv > 8 ||
      (opt->pass_points != 16 && opt->pass_points != 32 && opt->pass_points != 64) || opt->fixed_frame < 0 ||
      opt->moment_path < 0 || opt->moment_path > 2)
    return RKHSBA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device < 0 || opt->device >= ndev) return RKHSBA_EDEVICE;
  rkhsba_ctx* c = new (std::nothrow) rkhsba_ctx();
  if (!c) return RKHSBA_ENOMEM;
  c->opt = *opt;
  if (hipSetDevice(opt->device) != hipSuccess) {
    delete c;
    return RKHSBA_EDEVICE;
  }
  if (opt->stream) {
    c->stream = static_cast<hipStream_t>(opt->stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return RKHSBA_EDEVICE;
    }
    c->own_stream = true;
  }
  compute_constants(c);
  *out = c;
  return RKHSBA_OK;
}

void rkhsba_destroy(rkhsba_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->opt.device);
  (void)hipStreamSynchronize(c->stream);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* rkhsba_last_error(const rkhsba_ctx* c) { return c ? c->err.c_str() : "null context"; }

int rkhsba_build_neighbors(rkhsba_ctx* c, int K, const int64_t* n_points, const float* const* xyz, int feat_kind,
                           int D, const void* const* feats, int is_device) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(K >= 1 && n_points && xyz && feats, RKHSBA_EINVAL, "K >= 1 and non-NULL n_points/xyz/feats required");
    RK_REQUIRE(feat_kind == RKHSBA_FEAT_CLASS_ID || feat_kind == RKHSBA_FEAT_DENSE_F32, RKHSBA_EINVAL,
               "feature kind not supported by this build (class ids or dense float32)");
    if (feat_kind != RKHSBA_FEAT_CLASS_ID)
      RK_REQUIRE(D >= 1 && D <= kMaxDense, RKHSBA_EINVAL, "dense feature dimension must be in [1, 64]");
    std::vector<int64_t> off(K + 1, 0);
    for (int f = 0; f < K; ++f) {
      RK_REQUIRE(n_points[f] >= 1 && n_points[f] < (1LL << 31), RKHSBA_EINVAL, "each frame needs 1..2^31-1 points");
      RK_REQUIRE(xyz[f] && feats[f], RKHSBA_EINVAL, "NULL frame pointer");
      off[f + 1] = off[f] + n_points[f];
    }
    const int64_t N = off[K];
    RK_REQUIRE(N < (1LL << 32), RKHSBA_EINVAL, "too many points in total");
    hipStream_t st = c->stream;
    c->K = 0;  // invalid until the build completes
    c->edge_list.clear();
    c->feat_kind = feat_kind;
    c->D = feat_kind == RKHSBA_FEAT_CLASS_ID ? 0 : D;
    c->Dp = feat_kind == RKHSBA_FEAT_CLASS_ID ? 0 : dense_pad(D);
    compute_constants(c);
    const size_t fbytes = feat_kind == RKHSBA_FEAT_CLASS_ID ? sizeof(uint16_t) : sizeof(float) * (size_t)D;

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
      if (feat_kind != RKHSBA_FEAT_CLASS_ID)
        for (int f = 0; f < K; ++f) {
          const float* v = static_cast<const float*>(feats[f]);
          for (int64_t i = 0; i < (int64_t)D * n_points[f]; ++i)
            RK_REQUIRE(std::isfinite(v[i]), RKHSBA_EINVAL, "non-finite feature value");
        }
      RK_HIP(c->raw_xyz.reserve((size_t)N * 3));
      RK_HIP(c->raw_feat.reserve((size_t)N * fbytes));
      for (int f = 0; f < K; ++f) {
        RK_HIP(hipMemcpyAsync(c->raw_xyz.p + 3 * off[f], xyz[f], sizeof(float) * 3 * n_points[f],
                              hipMemcpyHostToDevice, st));
        RK_HIP(hipMemcpyAsync(c->raw_feat.p + fbytes * off[f], feats[f], fbytes * n_points[f], hipMemcpyHostToDevice,
                              st));
        xp[f] = c->raw_xyz.p + 3 * off[f];
        fp[f] = c->raw_feat.p + fbytes * off[f];
      }
    }
    hipEvent_t tb = prof_begin(c);
    RK_HIP(c->d_xyz_ptrs.reserve(K));
    RK_HIP(c->d_feat_ptrs.reserve(K));
    RK_HIP(c->d_in_off.reserve(K + 1));
    RK_HIP(hipMemcpyAsync(c->d_xyz_ptrs.p, xp.data(), sizeof(void*) * K, hipMemcpyHostToDevice, st));
    RK_HIP(hipMemcpyAsync(c->d_feat_ptrs.p, fp.data(), sizeof(void*) * K, hipMemcpyHostToDevice, st));
    RK_HIP(hipMemcpyAsync(c->d_in_off.p, off.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, st));

    // cell coordinates and per-frame bounds
    std::vector<int32_t> mm(6 * K + 2);
    for (int f = 0; f < K; ++f)
      for (int a = 0; a < 3; ++a) {
        mm[6 * f + a] = INT_MAX;
        mm[6 * f + 3 + a] = INT_MIN;
      }
    mm[6 * K] = 0;
    mm[6 * K + 1] = 0;
    RK_HIP(c->cell.reserve((size_t)N * 3));
    RK_HIP(c->minmax.reserve(mm.size()));
    RK_HIP(hipMemcpyAsync(c->minmax.p, mm.data(), sizeof(int32_t) * mm.size(), hipMemcpyHostToDevice, st));
    RK_HIP(launch_cell_coords(c->d_xyz_ptrs.p, c->d_in_off.p, K, N, c->kc.inv_cell, c->cell.p, c->minmax.p, st));
    RK_HIP(hipMemcpyAsync(mm.data(), c->minmax.p, sizeof(int32_t) * mm.size(), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    RK_REQUIRE(mm[6 * K] == 0, RKHSBA_EINVAL, "non-finite or out-of-range point coordinate");

    // grids
    std::vector<FrameInfo> fr(K);
    int64_t rows_total = 0;
    uint64_t max_cells = 1;
    int bin_axis_bits = 1;
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
      F.row_off = rows_total;
      rows_total += (int64_t)F.dim[1] * F.dim[2];
      F.xt_off = 0;
      int ext_max = 0;
      for (int a = 0; a < 3; ++a) ext_max = std::max(ext_max, F.dim[a] + 2 * c->kc.reach_cells);
      int shift = 0;
      while (((ext_max - 1) >> shift) >= 1023) ++shift;
      F.mort_shift = shift;
      const int maxc = (ext_max - 1) >> shift;
      int bits = 1;
      while ((1 << bits) < maxc + 2) ++bits;
      bin_axis_bits = std::max(bin_axis_bits, bits);
    }
    RK_REQUIRE(rows_total < (1LL << 31), RKHSBA_ENOMEM, "cell-row table too large");
    c->bin_bits = 3 * bin_axis_bits;
    RK_HIP(c->d_frames.reserve(K));
    RK_HIP(hipMemcpyAsync(c->d_frames.p, fr.data(), sizeof(FrameInfo) * K, hipMemcpyHostToDevice, st));

    // keys, segmented sort by frame, gather
    RK_HIP(c->k1.reserve(N));
    RK_HIP(c->v1.reserve(N));
    RK_HIP(c->k2.reserve(N));
    RK_HIP(c->v2.reserve(N));
    RK_HIP(launch_cell_keys(c->cell.p, c->d_in_off.p, c->d_frames.p, K, N, c->k1.p, c->v1.p, st));
    std::vector<SortTile> tiles;
    std::vector<SortSeg> segs(K);
    for (int f = 0; f < K; ++f) {
      segs[f].start = off[f];
      segs[f].count = n_points[f];
      segs[f].tile0 = (int32_t)tiles.size();
      for (int64_t s = 0; s < n_points[f]; s += kSortTile)
        tiles.push_back(SortTile{off[f] + s, (int32_t)std::min<int64_t>(kSortTile, n_points[f] - s), f});
      segs[f].n_tiles = (int32_t)tiles.size() - segs[f].tile0;
    }
    RK_HIP(c->d_tiles.reserve(tiles.size()));
    RK_HIP(c->d_segs.reserve(K));
    RK_HIP(c->hist.reserve(tiles.size() * 256));
    RK_HIP(hipMemcpyAsync(c->d_tiles.p, tiles.data(), sizeof(SortTile) * tiles.size(), hipMemcpyHostToDevice, st));
    RK_HIP(hipMemcpyAsync(c->d_segs.p, segs.data(), sizeof(SortSeg) * K, hipMemcpyHostToDevice, st));
    int key_bits = 1;
    while (key_bits < 32 && (1ull << key_bits) < max_cells) ++key_bits;
    bool in_tmp = false;
    RK_HIP(launch_radix_sort(c->k1.p, c->v1.p, c->k2.p, c->v2.p, c->hist.p, c->d_tiles.p, (int)tiles.size(),
                             c->d_segs.p, K, key_bits, st, &in_tmp));
    uint32_t* sk = in_tmp ? c->k2.p : c->k1.p;
    uint32_t* sv = in_tmp ? c->v2.p : c->v1.p;
    RK_HIP(c->pts.reserve(N));
    RK_HIP(c->perm.reserve(N));
    RK_HIP(c->keys.reserve(N));
    RK_HIP(c->feat.reserve(c->Dp > 0 ? (size_t)N * c->Dp : 1));
    RK_HIP(launch_gather(c->d_xyz_ptrs.p, c->d_feat_ptrs.p, feat_kind == RKHSBA_FEAT_CLASS_ID ? 0 : 1, c->D, c->Dp,
                         c->d_frames.p, c->d_in_off.p, K, N, sv, c->pts.p, c->feat.p, c->perm.p, c->minmax.p + 6 * K + 1,
                         st));
    RK_HIP(hipMemcpyAsync(c->keys.p, sk, sizeof(uint32_t) * N, hipMemcpyDeviceToDevice, st));

    // cell-row tables
    RK_HIP(c->rows.reserve(rows_total));
    RK_HIP(c->row_sizes.reserve(rows_total));
    RK_HIP(c->scan_tmp.reserve(rows_total / kScanTileElems + 2));
    RK_HIP(c->d_total.reserve(1));
    RK_HIP(launch_rows(c->keys.p, c->d_frames.p, c->d_in_off.p, K, N, c->rows.p, rows_total, c->row_sizes.p,
                       c->scan_tmp.p, c->d_total.p, st));
    uint64_t xt_total = 0;
    int32_t neg = 0;
    RK_HIP(hipMemcpyAsync(&xt_total, c->d_total.p, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    RK_HIP(hipMemcpyAsync(&neg, c->minmax.p + 6 * K + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    c->negative_features = neg != 0;
    compute_constants(c);
    RK_REQUIRE(xt_total < (1ull << 31), RKHSBA_ENOMEM, "cell table too large");
    RK_HIP(c->xtab.reserve(xt_total));
    RK_HIP(launch_xtab(c->keys.p, c->d_frames.p, c->d_in_off.p, K, N, c->rows.p, c->xtab.p, st));
    prof_end(c, RKHSBA_PROF_BUILD, tb);
    RK_HIP(hipStreamSynchronize(st));
    prof_collect(c);
    c->frames = std::move(fr);
    c->in_off = std::move(off);
    c->n_total = N;
    c->K = K;
    return RKHSBA_OK;
  });
}

int rkhsba_eval_loss(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* loss_total,
                     double* loss_per_edge, int64_t* n_pairs) {
  return guarded(c, [&]() -> int {
    prepare_edges(c, E, edges);
    upload_poses(c, poses);
    ensure_system(c, 6, 1);
    evaluate(c, MODE_LOSS);
    std::vector<double> eo((size_t)E * kEdgeVals);
    RK_HIP(hipMemcpyAsync(eo.data(), c->edge_out.p, sizeof(double) * eo.size(), hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    prof_collect(c);
    const double s2 = c->opt.sigma * c->opt.sigma;
    double F = 0.0, np = 0.0;
    for (int e = 0; e < E; ++e) {
      const double fe = s2 * eo[(size_t)e * kEdgeVals];
      if (loss_per_edge) loss_per_edge[e] = fe;
      F += eo[(size_t)e * kEdgeVals];
      np += eo[(size_t)e * kEdgeVals + 91];
    }
    if (loss_total) *loss_total = s2 * F;
    if (n_pairs) *n_pairs = (int64_t)np;
    return RKHSBA_OK;
  });
}

int rkhsba_accumulate_normal_eqs(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* H, double* b,
                                 double* loss_total, int64_t* n_pairs) {
  return guarded(c, [&]() -> int {
    prepare_edges(c, E, edges);
    upload_poses(c, poses);
    const int n = 6 * c->K;
    ensure_system(c, n, 1);
    evaluate(c, MODE_NORMAL);
    RK_HIP(launch_assemble(solve_args(c, -1, 0), c->stream));
    if (H) RK_HIP(hipMemcpyAsync(H, c->H.p, sizeof(double) * n * n, hipMemcpyDeviceToHost, c->stream));
    if (b) RK_HIP(hipMemcpyAsync(b, c->b.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    double F = 0.0, np = 0.0;
    RK_HIP(hipMemcpyAsync(&F, c->loss_hist.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipMemcpyAsync(&np, c->pairs_hist.p, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    prof_collect(c);
    if (loss_total) *loss_total = F;
    if (n_pairs) *n_pairs = (int64_t)np;
    return RKHSBA_OK;
  });
}

int rkhsba_gn_step(rkhsba_ctx* c, double* poses, int E, const int32_t* edges, int n_iter, double* loss_per_iter,
                   int64_t* pairs_per_iter) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(n_iter >= 0, RKHSBA_EINVAL, "n_iter must be >= 0");
    prepare_edges(c, E, edges);
    RK_REQUIRE(c->opt.fixed_frame < c->K, RKHSBA_EINVAL, "fixed_frame out of range");
    upload_poses(c, poses);
    const int n = 6 * (c->K - 1);
    ensure_system(c, std::max(n, 6), n_iter + 1);
    hipStream_t st = c->stream;
    RK_HIP(hipMemsetAsync(c->status.p, 0, sizeof(int32_t), st));
    for (int it = 0; it < n_iter; ++it) {
      evaluate(c, MODE_NORMAL);
      const SolveArgs sa = solve_args(c, c->opt.fixed_frame, it);
      hipEvent_t t3 = prof_begin(c);
      RK_HIP(launch_assemble(sa, st));
      RK_HIP(launch_solve_update(sa, st));
      prof_end(c, RKHSBA_PROF_SOLVE, t3);
    }
    evaluate(c, MODE_LOSS);
    RK_HIP(launch_loss_only(solve_args(c, c->opt.fixed_frame, n_iter), st));
    std::vector<double> lh(n_iter + 1), ph(n_iter + 1);
    int32_t status = 0;
    RK_HIP(hipMemcpyAsync(poses, c->d_poses.p, sizeof(double) * 12 * c->K, hipMemcpyDeviceToHost, st));
    RK_HIP(hipMemcpyAsync(lh.data(), c->loss_hist.p, sizeof(double) * (n_iter + 1), hipMemcpyDeviceToHost, st));
    RK_HIP(hipMemcpyAsync(ph.data(), c->pairs_hist.p, sizeof(double) * (n_iter + 1), hipMemcpyDeviceToHost, st));
    RK_HIP(hipMemcpyAsync(&status, c->status.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    prof_collect(c);
    for (int i = 0; i <= n_iter; ++i) {
      if (loss_per_iter) loss_per_iter[i] = lh[i];
      if (pairs_per_iter) pairs_per_iter[i] = (int64_t)ph[i];
    }
    if (status != 0) return fail(c, RKHSBA_ENOTPD, "Cholesky pivot not positive in a Gauss-Newton step");
    return RKHSBA_OK;
  });
}

int rkhsba_export_pairs(rkhsba_ctx* c, const double* poses, int m, int n, int64_t cap, int32_t* pairs,
                        int64_t* n_out) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(c->K > 0, RKHSBA_ESTATE, "no frames: call rkhsba_build_neighbors first");
    RK_REQUIRE(m >= 0 && n >= 0 && m < c->K && n < c->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    RK_REQUIRE(cap >= 0 && (cap == 0 || pairs), RKHSBA_EINVAL, "bad output buffer");
    upload_poses(c, poses);
    hipStream_t st = c->stream;
    EdgeInfo one{};
    one.m = m;
    one.n = n;
    DBuf<EdgeInfo> d_one;
    DBuf<EdgeXf> d_xf;
    DBuf<unsigned long long> d_cnt;
    RK_HIP(d_one.reserve(1));
    RK_HIP(d_xf.reserve(1));
    RK_HIP(d_cnt.reserve(1));
    RK_HIP(hipMemcpyAsync(d_one.p, &one, sizeof(one), hipMemcpyHostToDevice, st));
    RK_HIP(launch_edge_setup(c->d_poses.p, d_one.p, 1, d_xf.p, st));
    const int fp = c->feat_kind == RKHSBA_FEAT_CLASS_ID ? FEAT_CLASS : FEAT_DENSE;
    RK_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(unsigned long long), st));
    RK_HIP(launch_export_pairs(c->pts.p, c->rows.p, c->xtab.p, c->d_frames.p, c->frames[m].n, c->perm.p, d_xf.p, m, n,
                               fp, c->kc, 0, nullptr, d_cnt.p, st));
    unsigned long long total = 0;
    RK_HIP(hipMemcpyAsync(&total, d_cnt.p, sizeof(total), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    if (n_out) *n_out = (int64_t)total;
    if (cap == 0 || total == 0) return RKHSBA_OK;
    DBuf<int32_t> d_out;
    RK_HIP(d_out.reserve((size_t)total * 2));
    RK_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(unsigned long long), st));
    RK_HIP(launch_export_pairs(c->pts.p, c->rows.p, c->xtab.p, c->d_frames.p, c->frames[m].n, c->perm.p, d_xf.p, m, n,
                               fp, c->kc, (int64_t)total, d_out.p, d_cnt.p, st));
    std::vector<int32_t> h((size_t)total * 2);
    RK_HIP(hipMemcpyAsync(h.data(), d_out.p, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    std::vector<uint64_t> packed(total);
    for (size_t k = 0; k < total; ++k)
      packed[k] = ((uint64_t)(uint32_t)h[2 * k] << 32) | (uint32_t)h[2 * k + 1];
    std::sort(packed.begin(), packed.end());
    const int64_t w = std::min<int64_t>(cap, (int64_t)total);
    for (int64_t k = 0; k < w; ++k) {
      pairs[2 * k] = (int32_t)(packed[k] >> 32);
      pairs[2 * k + 1] = (int32_t)(packed[k] & 0xffffffffu);
    }
    return RKHSBA_OK;
  });
}

int rkhsba_export_voxels(rkhsba_ctx* c, int frame, int32_t* perm, uint32_t* keys, int32_t* origin, int32_t* dims) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(c->K > 0, RKHSBA_ESTATE, "no frames: call rkhsba_build_neighbors first");
    RK_REQUIRE(frame >= 0 && frame < c->K, RKHSBA_EINVAL, "frame out of range");
    const FrameInfo& F = c->frames[frame];
    if (perm)
      RK_HIP(hipMemcpyAsync(perm, c->perm.p + F.pt_off, sizeof(int32_t) * F.n, hipMemcpyDeviceToHost, c->stream));
    if (keys)
      RK_HIP(hipMemcpyAsync(keys, c->keys.p + F.pt_off, sizeof(uint32_t) * F.n, hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    for (int a = 0; a < 3; ++a) {
      if (origin) origin[a] = F.org[a];
      if (dims) dims[a] = F.dim[a];
    }
    return RKHSBA_OK;
  });
}

int rkhsba_profile_enable(rkhsba_ctx* c, int on) {
  if (!c) return RKHSBA_EINVAL;
  c->prof = on != 0;
  return RKHSBA_OK;
}

int rkhsba_profile_read(rkhsba_ctx* c, int stage, double* total_ms, int64_t* launches, int reset) {
  if (!c || stage < 0 || stage >= RKHSBA_PROF_STAGES) return RKHSBA_EINVAL;
  if (total_ms) *total_ms = c->stages[stage].ms;
  if (launches) *launches = c->stages[stage].launches;
  if (reset) {
    c->stages[stage].ms = 0.0;
    c->stages[stage].launches = 0;
  }
  return RKHSBA_OK;
}

}  // extern "C"
