// C ABI of the single-problem context: one resident problem in an engine,
// argument validation, and the call sequences of build_neighbors /
// eval_loss / accumulate_normal_eqs / gn_step.  No exception crosses the ABI.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rkhsba.h"
#include "engine.h"

using namespace rkhsba;

// Device scratch of rkhsba_eval_loss_noalloc: one static array per device the library runs on, held
// until the process ends.  Its device address comes from hipGetSymbolAddress (per device, at context
// creation); host code uses that address, never the array's name.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch_ptr;  // device ordinal -> address of that device's `scratch`

// The device address of `scratch` on the current device `dev` (looked up once per device).
hipError_t scratch_address(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = static_cast<uint8_t*>(ptr);
  *out = static_cast<uint8_t*>(ptr);
  return hipSuccess;
}
}  // namespace

struct rkhsba_ctx {
  rkhsba_options opt{};
  uint8_t* scratch_dev = nullptr;  // this device's static scratch (rkhsba_eval_loss_noalloc)
  SetLayout lay_noalloc;           // layout tables of rkhsba_eval_loss_noalloc, in that scratch
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::unique_ptr<Engine> eng;
  int prob = -1;         // the resident problem
  SetLayout lay_eval;    // evaluations without a fixed frame (loss, normal equations)
  SetLayout lay_gn;      // Gauss-Newton runs
  SetLayout lay_rot;     // candidate-pose batches
  SetLayout lay_ell;     // RKHS distance terms (graph edges and self inner products)
  double occ_r = 0.0;    // points per occupied r_c-cube of the frames last measured
};

namespace {

template <typename F>
int guarded(rkhsba_ctx* c, F&& body) {
  if (!c) return RKHSBA_EINVAL;
  c->err.clear();
  try {
    if (hipSetDevice(c->opt.device) != hipSuccess) {
      c->err = "hipSetDevice failed";
      return RKHSBA_EDEVICE;
    }
    return body();
  } catch (const Fail& f) {
    c->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return RKHSBA_ENOMEM;
  } catch (...) {
    c->err = "unexpected exception";
    return RKHSBA_EDEVICE;
  }
}

Problem* resident(rkhsba_ctx* c) {
  Problem* p = c->prob >= 0 ? c->eng->problem(c->prob) : nullptr;
  RK_REQUIRE(p != nullptr, RKHSBA_ESTATE, "no frames: call rkhsba_build_neighbors first");
  return p;
}

// The rotation group of the icosahedron (Sec. IV-A): closure of the 3-fold
// rotation about (1,1,1) (cyclic permutation of the axes) and the 5-fold
// rotation about the vertex direction (0, 1, golden ratio), in breadth-first
// order from the identity.
std::vector<std::array<double, 9>> icosahedral_group() {
  typedef std::array<double, 9> M;
  auto mul = [](const M& A, const M& B) {
    M C{};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
    return C;
  };
  const M P = {0, 0, 1, 1, 0, 0, 0, 1, 0};
  const double phi = 0.5 * (1.0 + std::sqrt(5.0));
  double ax[3] = {0.0, 1.0, phi};
  const double nrm = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
  for (double& v : ax) v /= nrm;
  const double th = 2.0 * M_PI / 5.0, cs = std::cos(th), sn = std::sin(th);
  M Q{};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const double K[3][3] = {{0, -ax[2], ax[1]}, {ax[2], 0, -ax[0]}, {-ax[1], ax[0], 0}};
      Q[3 * r + c] = (r == c ? cs : 0.0) + sn * K[r][c] + (1.0 - cs) * ax[r] * ax[c];
    }
  std::vector<M> G = {M{1, 0, 0, 0, 1, 0, 0, 0, 1}};
  for (size_t i = 0; i < G.size() && G.size() < 64; ++i)
    for (const M& g : {P, Q}) {
      const M x = mul(G[i], g);
      bool seen = false;
      for (const M& y : G) {
        double d = 0.0;
        for (int k = 0; k < 9; ++k) d = std::max(d, std::fabs(x[k] - y[k]));
        if (d < 1e-9) {
          seen = true;
          break;
        }
      }
      if (!seen) G.push_back(x);
    }
  return G;
}

ProbParams params_of(const rkhsba_options& o) {
  ProbParams p;
  p.ell = o.ell;
  p.cutoff_factor = o.cutoff_factor;
  p.sigma = o.sigma;
  p.damping_rel = o.damping_rel;
  p.fixed_frame = o.fixed_frame;
  p.clamp_negative_c = o.clamp_negative_c;
  p.cell_subdiv = o.cell_subdiv;
  p.pass_points = o.pass_points;
  p.top_k = o.top_k;
  return p;
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
  o->cell_subdiv = 0;
  o->pass_points = 0;
  o->moment_path = 0;
  o->use_graphs = 1;
  o->hessian_fp32 = 0;
  o->top_k = 0;
  o->stream = nullptr;
}

int rkhsba_create(rkhsba_ctx** out, const rkhsba_options* opt) {
  if (!out) return RKHSBA_EINVAL;
  *out = nullptr;
  if (!opt) return RKHSBA_EINVAL;
  if (!(opt->ell > 0.0) || !std::isfinite(opt->ell) || !(opt->cutoff_factor > 0.0) ||
      !std::isfinite(opt->cutoff_factor) || !std::isfinite(opt->sigma) || !(opt->damping_rel >= 0.0) ||
      opt->cell_subdiv < 0 || opt->cell_subdiv > 8 ||
      (opt->pass_points != 0 && opt->pass_points != 1 && opt->pass_points != 8 && opt->pass_points != 16 &&
       opt->pass_points != 32 && opt->pass_points != 64) ||
      opt->fixed_frame < 0 ||
      opt->moment_path < 0 || opt->moment_path > 2 || opt->use_graphs < 0 || opt->use_graphs > 1 ||
      opt->hessian_fp32 < 0 || opt->hessian_fp32 > 1 || opt->top_k < 0 || opt->top_k > kMaxTopK)
    return RKHSBA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device < 0 || opt->device >= ndev) return RKHSBA_EDEVICE;
  rkhsba_ctx* c = new (std::nothrow) rkhsba_ctx();
  if (!c) return RKHSBA_ENOMEM;
  c->opt = *opt;
  if (hipSetDevice(opt->device) != hipSuccess || scratch_address(opt->device, &c->scratch_dev) != hipSuccess) {
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
  c->eng.reset(new (std::nothrow) Engine(opt->device, c->stream, opt->moment_path));
  if (!c->eng) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return RKHSBA_ENOMEM;
  }
  c->eng->use_graphs = opt->use_graphs != 0;
  c->eng->fp32_sums = opt->hessian_fp32 != 0;
  *out = c;
  return RKHSBA_OK;
}

void rkhsba_destroy(rkhsba_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->opt.device);
  (void)hipStreamSynchronize(c->stream);
  c->lay_eval.drop_graph();
  c->lay_gn.drop_graph();
  c->lay_rot.drop_graph();
  c->lay_ell.drop_graph();
  c->lay_noalloc.drop_graph();
  c->eng.reset();
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* rkhsba_last_error(const rkhsba_ctx* c) { return c ? c->err.c_str() : "null context"; }

int rkhsba_build_neighbors(rkhsba_ctx* c, int K, const int64_t* n_points, const float* const* xyz, int feat_kind,
                           int D, const void* const* feats, int is_device) {
  return guarded(c, [&]() -> int {
    if (c->prob >= 0) {
      c->eng->remove_problem(c->prob);
      c->prob = -1;
    }
    c->prob = c->eng->add_problem_auto(params_of(c->opt), K, n_points, xyz, feat_kind, D, feats, is_device != 0);
    const double occ = c->eng->problem(c->prob)->occupancy_r;
    if (occ > 0.0) c->occ_r = occ;
    return RKHSBA_OK;
  });
}

int rkhsba_autotune(rkhsba_ctx* c, int K, const int64_t* n_points, const float* const* xyz, int feat_kind, int D,
                    const void* const* feats, int is_device, const double* poses, int E, const int32_t* edges,
                    int trials, int* best_cell_subdiv, int* best_pass_points, double* best_ms) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(trials >= 1 && trials <= 100, RKHSBA_EINVAL, "trials must be in [1, 100]");
    Engine& g = *c->eng;
    const bool prof = g.prof;
    g.prof = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    RK_HIP(hipEventCreate(&ev[0]));
    RK_HIP(hipEventCreate(&ev[1]));
    struct Cleanup {
      hipEvent_t* ev;
      Engine& g;
      bool prof;
      ~Cleanup() {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        g.prof = prof;
      }
    } cleanup{ev, g, prof};
    const int subdivs[] = {1, 2, 3, 4, 6, 8};
    const int passes[] = {1, 8, 16, 32, 64};
    double best = 1e300, occ_r = 0.0;
    int bestS = 0, bestP = 0;
    for (int P : passes) {
      if (P == 8 && feat_kind != RKHSBA_FEAT_CLASS_ID) continue;  // 8-point passes: class ids only
      for (int S : subdivs) {
        if (c->prob >= 0) g.remove_problem(c->prob);
        c->prob = -1;
        ProbParams par = params_of(c->opt);
        par.cell_subdiv = S;
        par.pass_points = P;
        c->prob = g.add_problem(par, K, n_points, xyz, feat_kind, D, feats, is_device != 0);
        Problem* p = g.problem(c->prob);
        if (S == 1) occ_r = p->occupancy;
        g.prepare(c->lay_eval, {SetItem{p, edges, E, -1, 0}});
        g.upload_poses(p, poses);
        g.evaluate(c->lay_eval, MODE_NORMAL);  // warm-up
        RK_HIP(hipEventRecord(ev[0], c->stream));
        for (int t = 0; t < trials; ++t) g.evaluate(c->lay_eval, MODE_NORMAL);
        RK_HIP(hipEventRecord(ev[1], c->stream));
        RK_HIP(hipEventSynchronize(ev[1]));
        float ms = 0.f;
        RK_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        const double per = ms / trials;
        if (per < best) {
          best = per;
          bestS = S;
          bestP = P;
        }
      }
    }
    // leave the context on the best configuration
    c->opt.pass_points = bestP;
    c->opt.cell_subdiv = bestS;
    g.tune_record(occ_r, bestS, bestP);
    c->occ_r = occ_r;
    g.remove_problem(c->prob);
    c->prob = -1;
    c->prob = g.add_problem(params_of(c->opt), K, n_points, xyz, feat_kind, D, feats, is_device != 0);
    if (best_cell_subdiv) *best_cell_subdiv = bestS;
    if (best_pass_points) *best_pass_points = bestP;
    if (best_ms) *best_ms = best;
    return RKHSBA_OK;
  });
}

int rkhsba_get_config(rkhsba_ctx* c, int* cell_subdiv, int* pass_points, double* occupancy) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    if (cell_subdiv) *cell_subdiv = p->par.cell_subdiv;
    if (pass_points) *pass_points = p->par.pass_points;
    if (occupancy) *occupancy = p->occupancy_r > 0.0 ? p->occupancy_r : c->occ_r;
    return RKHSBA_OK;
  });
}

int rkhsba_eval_loss(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* loss_total,
                     double* loss_per_edge, int64_t* n_pairs) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    g.prepare(c->lay_eval, {SetItem{p, edges, E, -1, 0}});
    g.upload_poses(p, poses);
    g.reset_state(p);
    g.evaluate(c->lay_eval, MODE_LOSS);
    std::vector<double> eo((size_t)E * kEdgeVals);
    RK_HIP(hipMemcpyAsync(eo.data(), g.edge_out(), sizeof(double) * eo.size(), hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    g.prof_collect();
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

int rkhsba_eval_loss_noalloc(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* loss_total,
                             double* loss_per_edge, int64_t* n_pairs) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(c->scratch_dev != nullptr, RKHSBA_ESTATE, "no static scratch on this device");
    // the layout tables and the loss evaluation's scratch in this device's static array; the last 256
    // bytes hold the two totals
    Arena arena;
    arena.base = c->scratch_dev;
    arena.cap = kNoallocScratchBytes - 256;
    arena.mom_components = 1;
    double* d_totals = reinterpret_cast<double*>(c->scratch_dev + kNoallocScratchBytes - 256);
    g.set_arena(&arena);
    struct Restore {
      Engine& g;
      ~Restore() { g.set_arena(nullptr); }
    } restore{g};
    g.prepare(c->lay_noalloc, {SetItem{p, edges, E, -1, 0}});
    g.upload_poses(p, poses);
    g.evaluate(c->lay_noalloc, MODE_LOSS);
    RK_HIP(launch_edge_totals(g.edge_out(), E, d_totals, c->stream));
    double tot[2] = {0.0, 0.0};
    RK_HIP(hipMemcpyAsync(tot, d_totals, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    if (loss_per_edge)
      RK_HIP(hipMemcpy2DAsync(loss_per_edge, sizeof(double), g.edge_out(), sizeof(double) * kEdgeVals,
                              sizeof(double), (size_t)E, hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    const double s2 = c->opt.sigma * c->opt.sigma;
    if (loss_per_edge)
      for (int e = 0; e < E; ++e) loss_per_edge[e] *= s2;
    if (loss_total) *loss_total = s2 * tot[0];
    if (n_pairs) *n_pairs = (int64_t)tot[1];
    return RKHSBA_OK;
  });
}

int rkhsba_accumulate_normal_eqs(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* H, double* b,
                                 double* loss_total, int64_t* n_pairs) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    g.prepare(c->lay_eval, {SetItem{p, edges, E, -1, 0}});
    g.upload_poses(p, poses);
    g.reset_state(p);
    const int n = 6 * p->K;
    g.evaluate(c->lay_eval, MODE_NORMAL);
    g.assemble(c->lay_eval);
    const SolveArgs sa = g.solve_args(c->lay_eval);
    if (H) RK_HIP(hipMemcpyAsync(H, sa.H, sizeof(double) * n * n, hipMemcpyDeviceToHost, c->stream));
    if (b) RK_HIP(hipMemcpyAsync(b, sa.b, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    double F = 0.0, np = 0.0;
    g.read_history(p, 1, &F, &np);
    g.prof_collect();
    if (loss_total) *loss_total = F;
    if (n_pairs) *n_pairs = (int64_t)np;
    return RKHSBA_OK;
  });
}

int rkhsba_gn_step(rkhsba_ctx* c, double* poses, int E, const int32_t* edges, int n_iter, double* loss_per_iter,
                   int64_t* pairs_per_iter) {
  return guarded(c, [&]() -> int {
    RK_REQUIRE(n_iter >= 0, RKHSBA_EINVAL, "n_iter must be >= 0");
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(c->opt.fixed_frame < p->K, RKHSBA_EINVAL, "fixed_frame out of range");
    g.prepare(c->lay_gn, {SetItem{p, edges, E, c->opt.fixed_frame, n_iter}});
    g.upload_poses(p, poses);
    g.reset_state(p);
    g.iterate(c->lay_gn, n_iter);
    g.evaluate(c->lay_gn, MODE_LOSS, n_iter > 0);  // the binning of this call's first iteration
    g.loss_only(c->lay_gn);
    std::vector<double> lh(n_iter + 1), ph(n_iter + 1);
    g.download_poses(p, poses);
    g.read_history(p, n_iter + 1, lh.data(), ph.data());
    const int32_t status = g.read_status(p);
    g.prof_collect();
    for (int i = 0; i <= n_iter; ++i) {
      if (loss_per_iter) loss_per_iter[i] = lh[i];
      if (pairs_per_iter) pairs_per_iter[i] = (int64_t)ph[i];
    }
    if (status != 0) {
      c->err = "Cholesky pivot not positive in a Gauss-Newton step";
      return RKHSBA_ENOTPD;
    }
    return RKHSBA_OK;
  });
}

// d_H = sum over edges of <f_m,f_m> + <f_n,f_n> - 2 <f_m,f_n> and its ell-derivative
// sigma^2 / ell^3 * sum(W_mm + W_nn - 2 W_mn), at the device poses.
static void distance_terms(rkhsba_ctx* c, Problem* p, int E, const int32_t* edges, double* d, double* g) {
  Engine& eng = *c->eng;
  std::vector<int> frames;
  for (int e = 0; e < 2 * E; ++e) frames.push_back(edges[e]);
  std::sort(frames.begin(), frames.end());
  frames.erase(std::unique(frames.begin(), frames.end()), frames.end());
  std::vector<int32_t> all(edges, edges + 2 * E);
  for (int f : frames) {
    all.push_back(f);
    all.push_back(f);
  }
  const int Et = (int)all.size() / 2;
  SetItem it{p, all.data(), Et, -1, 0};
  it.allow_self = true;
  eng.prepare(c->lay_ell, {it});
  eng.evaluate(c->lay_ell, MODE_NORMAL);
  std::vector<double> eo((size_t)Et * kEdgeVals);
  RK_HIP(hipMemcpyAsync(eo.data(), eng.edge_out(), sizeof(double) * eo.size(), hipMemcpyDeviceToHost, c->stream));
  RK_HIP(hipStreamSynchronize(c->stream));
  eng.prof_collect();
  std::vector<double> S(p->K, 0.0), SW(p->K, 0.0);
  for (size_t k = 0; k < frames.size(); ++k) {
    S[frames[k]] = eo[(size_t)(E + k) * kEdgeVals];
    SW[frames[k]] = eo[(size_t)(E + k) * kEdgeVals + 92];
  }
  double dd = 0.0, gw = 0.0;
  for (int e = 0; e < E; ++e) {
    const int m = edges[2 * e], n = edges[2 * e + 1];
    dd += S[m] + S[n] - 2.0 * eo[(size_t)e * kEdgeVals];
    gw += SW[m] + SW[n] - 2.0 * eo[(size_t)e * kEdgeVals + 92];
  }
  const double s2 = p->par.sigma * p->par.sigma, ell = p->par.ell;
  *d = s2 * dd;
  *g = s2 * gw / (ell * ell * ell);
}

// F of one edge and the 6-vector b of frame n (Gauss-Newton sums, no frame removed) at host poses.
static double edge_value_and_b(rkhsba_ctx* c, Problem* p, const double* poses, int m, int n, double* bn) {
  Engine& eng = *c->eng;
  const int32_t edge[2] = {m, n};
  eng.prepare(c->lay_eval, {SetItem{p, edge, 1, -1, 0}});
  eng.upload_poses(p, poses);
  std::vector<double> eo(kEdgeVals);
  if (bn) {
    eng.evaluate(c->lay_eval, MODE_NORMAL);
  } else {
    eng.evaluate(c->lay_eval, MODE_LOSS);
  }
  RK_HIP(hipMemcpyAsync(eo.data(), eng.edge_out(), sizeof(double) * kEdgeVals, hipMemcpyDeviceToHost, c->stream));
  RK_HIP(hipStreamSynchronize(c->stream));
  eng.prof_collect();
  if (bn)
    for (int r = 0; r < 6; ++r) bn[r] = eo[7 + r];  // b_n of the edge: the 6-vector of its second frame
  return p->par.sigma * p->par.sigma * eo[0];
}

// T <- T exp(xi^), closed-form SE(3) exponential (host, FP64).
static void host_right_update(double* T, const double* xi) {
  const double* rho = xi;
  const double* phi = xi + 3;
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = std::sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    A = std::sin(th) / th;
    B = (1.0 - std::cos(th)) / th2;
    C = (th - std::sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0.0, -phi[2], phi[1]}, {phi[2], 0.0, -phi[0]}, {-phi[1], phi[0], 0.0}};
  double K2[3][3], Re[3][3], V[3][3], te[3], R[3][3], t[3];
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2) K2[r][c2] = K[r][0] * K[0][c2] + K[r][1] * K[1][c2] + K[r][2] * K[2][c2];
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2) {
      const double I = r == c2 ? 1.0 : 0.0;
      Re[r][c2] = I + A * K[r][c2] + B * K2[r][c2];
      V[r][c2] = I + B * K[r][c2] + C * K2[r][c2];
    }
  for (int r = 0; r < 3; ++r) te[r] = V[r][0] * rho[0] + V[r][1] * rho[1] + V[r][2] * rho[2];
  for (int r = 0; r < 3; ++r) {
    for (int c2 = 0; c2 < 3; ++c2) R[r][c2] = T[3 * r + c2];
    t[r] = T[9 + r];
  }
  for (int r = 0; r < 3; ++r) {
    for (int c2 = 0; c2 < 3; ++c2) T[3 * r + c2] = R[r][0] * Re[0][c2] + R[r][1] * Re[1][c2] + R[r][2] * Re[2][c2];
    T[9 + r] = R[r][0] * te[0] + R[r][1] * te[1] + R[r][2] * te[2] + t[r];
  }
}

int rkhsba_cosine(rkhsba_ctx* c, const double* poses, int m, int n, double* cos_out) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    RK_REQUIRE(m >= 0 && n >= 0 && m < p->K && n < p->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    c->eng->upload_poses(p, poses);
    const int32_t e[6] = {m, n, m, m, n, n};
    SetItem it{p, e, 3, -1, 0};
    it.allow_self = true;
    c->eng->prepare(c->lay_ell, {it});
    c->eng->evaluate(c->lay_ell, MODE_LOSS);
    std::vector<double> eo((size_t)3 * kEdgeVals);
    RK_HIP(hipMemcpyAsync(eo.data(), c->eng->edge_out(), sizeof(double) * eo.size(), hipMemcpyDeviceToHost,
                          c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    c->eng->prof_collect();
    const double Fmn = eo[0], Sm = eo[kEdgeVals], Sn = eo[2 * kEdgeVals];
    if (cos_out) *cos_out = (Sm > 0.0 && Sn > 0.0) ? Fmn / std::sqrt(Sm * Sn) : 0.0;
    return RKHSBA_OK;
  });
}

int rkhsba_track(rkhsba_ctx* c, double* poses, int m, int n, int max_iter, double step0, double step_min,
                 int* iters_out, double* loss_out) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    RK_REQUIRE(m >= 0 && n >= 0 && m < p->K && n < p->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    RK_REQUIRE(max_iter >= 0 && step0 > 0.0 && step_min > 0.0 && step_min <= step0, RKHSBA_EINVAL,
               "bad tracking parameters");
    for (int i = 0; i < 12 * p->K; ++i) RK_REQUIRE(std::isfinite(poses[i]), RKHSBA_EINVAL, "non-finite pose entry");
    const double s2 = p->par.sigma * p->par.sigma, l2 = p->par.ell * p->par.ell;
    std::vector<double> P(poses, poses + 12 * p->K), Pc;
    double bn[6];
    double F = edge_value_and_b(c, p, P.data(), m, n, bn);
    double s = step0;
    int it = 0;
    for (; it < max_iter && s >= step_min; ++it) {
      double g[6], gn = 0.0;
      for (int r = 0; r < 6; ++r) {
        g[r] = -(s2 / l2) * bn[r];  // grad of F w.r.t. the right perturbation of frame n
        gn += g[r] * g[r];
      }
      gn = std::sqrt(gn);
      if (!(gn > 0.0)) break;
      bool accepted = false;
      while (s >= step_min) {
        double xi[6];
        for (int r = 0; r < 6; ++r) xi[r] = s * g[r] / gn;
        Pc = P;
        host_right_update(&Pc[12 * n], xi);
        const double Fc = edge_value_and_b(c, p, Pc.data(), m, n, nullptr);
        if (Fc > F) {
          P.swap(Pc);
          s *= 1.5;
          accepted = true;
          break;
        }
        s *= 0.5;
      }
      if (!accepted) break;
      F = edge_value_and_b(c, p, P.data(), m, n, bn);
    }
    std::copy(P.begin(), P.end(), poses);
    if (iters_out) *iters_out = it;
    if (loss_out) *loss_out = F;
    return RKHSBA_OK;
  });
}

void rkhsba_default_ell_schedule(rkhsba_ell_schedule* s, double ell) {
  if (!s) return;
  s->ell_init = 4.0 * ell;
  s->ell_min = ell;
  s->ell_max = 8.0 * ell;
  s->step = 0.1;
  s->elasticity = 1.0;
  s->tol = 1e-6;
  s->inner_iter = 5;
  s->max_outer = 30;
}

int rkhsba_ell_gradient(rkhsba_ctx* c, const double* poses, int E, const int32_t* edges, double* d, double* dd_dell) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    RK_REQUIRE(E >= 1 && edges, RKHSBA_EINVAL, "need at least one edge");
    c->eng->upload_poses(p, poses);
    double dv = 0.0, gv = 0.0;
    distance_terms(c, p, E, edges, &dv, &gv);
    if (d) *d = dv;
    if (dd_dell) *dd_dell = gv;
    return RKHSBA_OK;
  });
}

int rkhsba_gn_lengthscale(rkhsba_ctx* c, double* poses, int E, const int32_t* edges, const rkhsba_ell_schedule* sc,
                          int* n_outer, double* trace) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(sc != nullptr, RKHSBA_EINVAL, "schedule is NULL");
    RK_REQUIRE(sc->ell_min > 0.0 && sc->ell_max >= sc->ell_min && std::isfinite(sc->ell_max) && sc->step > 0.0 &&
                   sc->step < 1.0 && sc->inner_iter >= 0 && sc->max_outer >= 1 && sc->tol >= 0.0,
               RKHSBA_EINVAL, "invalid lengthscale schedule");
    RK_REQUIRE(c->opt.fixed_frame < p->K, RKHSBA_EINVAL, "fixed_frame out of range");
    const double ell_build = p->par.ell;
    struct Restore {
      Engine& g;
      Problem* p;
      double ell;
      ~Restore() { g.set_ell(p, ell); }
    } restore{g, p, ell_build};
    double ell = std::min(std::max(sc->ell_init, sc->ell_min), sc->ell_max);
    const int ni = sc->inner_iter;
    std::vector<double> lh(ni + 1);
    int outer = 0;
    int status = 0;
    for (; outer < sc->max_outer; ++outer) {
      g.set_ell(p, ell);
      g.prepare(c->lay_gn, {SetItem{p, edges, E, c->opt.fixed_frame, ni}});
      g.upload_poses(p, poses);
      g.reset_state(p);
      g.iterate(c->lay_gn, ni);
      g.evaluate(c->lay_gn, MODE_LOSS);
      g.loss_only(c->lay_gn);
      g.download_poses(p, poses);
      g.read_history(p, ni + 1, lh.data(), nullptr);
      status = g.read_status(p);
      double d = 0.0, gr = 0.0;
      distance_terms(c, p, E, edges, &d, &gr);
      if (trace) {
        double* t = trace + 5 * outer;
        t[0] = ell;
        t[1] = lh[0];
        t[2] = lh[ni];
        t[3] = d;
        t[4] = gr;
      }
      if (status != 0) {
        ++outer;
        break;
      }
      const double eta = d > 0.0 ? -ell * gr / d : 0.0;
      double nxt = eta >= sc->elasticity ? ell * (1.0 - sc->step) : ell * (1.0 + sc->step);
      nxt = std::min(std::max(nxt, sc->ell_min), sc->ell_max);
      if (nxt == ell && lh[ni] - lh[0] <= sc->tol * std::fabs(lh[0])) {
        ++outer;
        break;
      }
      ell = nxt;
    }
    if (n_outer) *n_outer = outer;
    if (status != 0) {
      c->err = "Cholesky pivot not positive in a Gauss-Newton step";
      return RKHSBA_ENOTPD;
    }
    return RKHSBA_OK;
  });
}

void rkhsba_icosahedral_rotations(double* out) {
  if (!out) return;
  const auto G = icosahedral_group();
  for (size_t k = 0; k < G.size(); ++k)
    for (int i = 0; i < 9; ++i) out[9 * k + i] = G[k][i];
}

int rkhsba_rotation_search(rkhsba_ctx* c, const double* poses, int m, int n, int n_rot, const double* rotations,
                           double* scores, int* best, double* best_pose) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(m >= 0 && n >= 0 && m < p->K && n < p->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    std::vector<std::array<double, 9>> R;
    if (rotations) {
      RK_REQUIRE(n_rot >= 1 && n_rot <= 4096, RKHSBA_EINVAL, "n_rot must be in [1, 4096]");
      for (int k = 0; k < n_rot; ++k) {
        std::array<double, 9> r;
        for (int i = 0; i < 9; ++i) {
          r[i] = rotations[9 * k + i];
          RK_REQUIRE(std::isfinite(r[i]), RKHSBA_EINVAL, "non-finite rotation entry");
        }
        R.push_back(r);
      }
    } else {
      R = icosahedral_group();
      RK_REQUIRE(n_rot == 0 || n_rot == (int)R.size(), RKHSBA_EINVAL, "n_rot must be 0 or 60 without rotations");
    }
    const int nr = (int)R.size();
    g.upload_poses(p, poses);
    double ctr[3];
    g.frame_centroid(p, n, ctr);
    // candidate pose T_n G_k with G_k(x) = R_k (x - c) + c
    const double* Tn = poses + 12 * n;
    std::vector<double> cand((size_t)12 * nr);
    for (int k = 0; k < nr; ++k) {
      const auto& Rk = R[k];
      double* T = &cand[(size_t)12 * k];
      double gt[3];
      for (int a = 0; a < 3; ++a) gt[a] = ctr[a] - (Rk[3 * a] * ctr[0] + Rk[3 * a + 1] * ctr[1] + Rk[3 * a + 2] * ctr[2]);
      for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
          T[3 * a + b] = Tn[3 * a] * Rk[b] + Tn[3 * a + 1] * Rk[3 + b] + Tn[3 * a + 2] * Rk[6 + b];
        T[9 + a] = Tn[3 * a] * gt[0] + Tn[3 * a + 1] * gt[1] + Tn[3 * a + 2] * gt[2] + Tn[9 + a];
      }
    }
    g.set_aliases(p, n, nr, cand.data());
    std::vector<int32_t> edges((size_t)2 * nr);
    for (int k = 0; k < nr; ++k) {
      edges[2 * k] = m;
      edges[2 * k + 1] = p->K + k;
    }
    g.prepare(c->lay_rot, {SetItem{p, edges.data(), nr, -1, 0}});
    g.evaluate(c->lay_rot, MODE_LOSS);
    std::vector<double> eo((size_t)nr * kEdgeVals);
    RK_HIP(hipMemcpyAsync(eo.data(), g.edge_out(), sizeof(double) * eo.size(), hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    g.prof_collect();
    g.clear_aliases(p);
    const double s2 = c->opt.sigma * c->opt.sigma;
    int kb = 0;
    for (int k = 0; k < nr; ++k) {
      const double f = s2 * eo[(size_t)k * kEdgeVals];
      if (scores) scores[k] = f;
      if (f > s2 * eo[(size_t)kb * kEdgeVals]) kb = k;
    }
    if (best) *best = kb;
    if (best_pose) std::copy(&cand[(size_t)12 * kb], &cand[(size_t)12 * kb] + 12, best_pose);
    return RKHSBA_OK;
  });
}

int rkhsba_export_pairs(rkhsba_ctx* c, const double* poses, int m, int n, int64_t cap, int32_t* pairs,
                        int64_t* n_out) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(m >= 0 && n >= 0 && m < p->K && n < p->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    RK_REQUIRE(cap >= 0 && (cap == 0 || pairs), RKHSBA_EINVAL, "bad output buffer");
    g.upload_poses(p, poses);
    hipStream_t st = c->stream;
    const int mg = (int)(p->slot0 + m), ng = (int)(p->slot0 + n);
    EdgeInfo one{};
    one.m = mg;
    one.n = ng;
    DBuf<EdgeInfo> d_one;
    DBuf<EdgeXf> d_xf;
    DBuf<unsigned long long> d_cnt;
    RK_HIP(d_one.reserve(1));
    RK_HIP(d_xf.reserve(1));
    RK_HIP(d_cnt.reserve(1));
    RK_HIP(hipMemcpyAsync(d_one.p, &one, sizeof(one), hipMemcpyHostToDevice, st));
    RK_HIP(launch_edge_setup(g.poses(), d_one.p, 1, d_xf.p, st));
    const int fp = g.feat_kind == RKHSBA_FEAT_CLASS_ID ? FEAT_CLASS : FEAT_DENSE;
    RK_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(unsigned long long), st));
    RK_HIP(launch_export_pairs(g.pts(), g.rows(), g.xtab(), g.frames(), p->frames[m].n, g.perm(), g.feat(), d_xf.p, mg,
                               ng, fp,
                               p->kc, 0, nullptr, d_cnt.p, st));
    unsigned long long total = 0;
    RK_HIP(hipMemcpyAsync(&total, d_cnt.p, sizeof(total), hipMemcpyDeviceToHost, st));
    RK_HIP(hipStreamSynchronize(st));
    if (n_out) *n_out = (int64_t)total;
    if (cap == 0 || total == 0) return RKHSBA_OK;
    DBuf<int32_t> d_out;
    RK_HIP(d_out.reserve((size_t)total * 2));
    RK_HIP(hipMemsetAsync(d_cnt.p, 0, sizeof(unsigned long long), st));
    RK_HIP(launch_export_pairs(g.pts(), g.rows(), g.xtab(), g.frames(), p->frames[m].n, g.perm(), g.feat(), d_xf.p, mg,
                               ng, fp,
                               p->kc, (int64_t)total, d_out.p, d_cnt.p, st));
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

int rkhsba_export_source_counts(rkhsba_ctx* c, const double* poses, int m, int n, int64_t* counts) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(m >= 0 && n >= 0 && m < p->K && n < p->K && m != n, RKHSBA_EINVAL, "bad frame pair");
    RK_REQUIRE(counts != nullptr, RKHSBA_EINVAL, "counts is NULL");
    const int32_t edge[2] = {m, n};
    g.prepare(c->lay_eval, {SetItem{p, edge, 1, -1, 0}});
    g.upload_poses(p, poses);
    g.source_counts = true;
    struct Reset {
      Engine& g;
      ~Reset() { g.source_counts = false; }
    } reset{g};
    g.evaluate(c->lay_eval, MODE_NORMAL);
    g.read_source_counts(p, m, counts);
    g.prof_collect();
    return RKHSBA_OK;
  });
}

int rkhsba_export_voxels(rkhsba_ctx* c, int frame, int32_t* perm, uint32_t* keys, int32_t* origin, int32_t* dims,
                         int32_t* label_layers) {
  return guarded(c, [&]() -> int {
    Problem* p = resident(c);
    Engine& g = *c->eng;
    RK_REQUIRE(frame >= 0 && frame < p->K, RKHSBA_EINVAL, "frame out of range");
    const FrameInfo& F = p->frames[frame];
    if (perm)
      RK_HIP(hipMemcpyAsync(perm, g.perm() + F.pt_off, sizeof(int32_t) * F.n, hipMemcpyDeviceToHost, c->stream));
    if (keys)
      RK_HIP(hipMemcpyAsync(keys, g.keys() + F.pt_off, sizeof(uint32_t) * F.n, hipMemcpyDeviceToHost, c->stream));
    RK_HIP(hipStreamSynchronize(c->stream));
    for (int a = 0; a < 3; ++a) {
      if (origin) origin[a] = F.org[a];
      if (dims) dims[a] = F.dim[a];
    }
    if (label_layers) *label_layers = F.n_lab;
    return RKHSBA_OK;
  });
}

int rkhsba_profile_enable(rkhsba_ctx* c, int on) {
  if (!c) return RKHSBA_EINVAL;
  c->eng->prof = on != 0;
  return RKHSBA_OK;
}

int rkhsba_profile_read(rkhsba_ctx* c, int stage, double* total_ms, int64_t* launches, int reset) {
  if (!c || stage < 0 || stage >= RKHSBA_PROF_STAGES) return RKHSBA_EINVAL;
  Engine::Stage& s = c->eng->stages[stage];
  if (total_ms) *total_ms = s.ms;
  if (launches) *launches = s.launches;
  if (reset) {
    s.ms = 0.0;
    s.launches = 0;
  }
  return RKHSBA_OK;
}

}  // extern "C"
