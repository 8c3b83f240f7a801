// Request loop: continuous batching of whole solves (each request = the
// multi-frame Gauss-Newton problem of Sec. V-A on its own frames, graph and
// length scale).  The server runs one or two lanes; a lane is a worker thread
// with its own engine and stream.  With two lanes, requests with many
// (edge, source point) entries go to lane 1 and the others to lane 0, so small
// requests do not wait for the iterations of large ones, and the two lanes'
// launches overlap on the device.  In a lane, requests wait in a FIFO queue
// and are admitted while the number of active requests, the sum of their
// (edge, source point) entries (a bound on one batch iteration's work, and so
// on the time every active request waits per iteration) and the sum of the
// estimated device footprints of all admitted requests stay within the limits
// (a request is always admitted when its lane is idle).  Admission builds the
// request's voxel structures into the lane engine's resident pools; then every
// active request of the lane advances by one Gauss-Newton iteration per batch
// iteration, all of them in the same launches (one edge table, one system per
// request).  A request that has taken its n_iter steps gets its final loss
// evaluation in the next batch iteration and is retired: poses and histories
// are copied out, its pools are freed and its waiter is woken.  Requests that
// arrive meanwhile join at the next batch iteration.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rkhsba.h"
#include "engine.h"

using namespace rkhsba;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  int64_t ticket = 0;
  ProbParams par;
  int K = 0, E = 0, n_iter = 0, is_device = 0, feat_kind = 0, D = 0;
  std::vector<int64_t> n_points;
  std::vector<const float*> xyz;
  std::vector<const void*> feats;
  std::vector<double> poses;
  std::vector<int32_t> edges;
  int64_t est_bytes = 0;
  int64_t entries = 0;    // (edge, source point) entries: the request's share of every launch
  bool admitted = false;  // est_bytes counted in the server's committed total
  double work = 0.0;      // entries x measured points per occupied r_c-cube x evaluations (set at the build)
  bool timed = false;     // its service time feeds the estimate of lane 1's rate
  // progress (worker thread)
  int prob = -1;
  int evals = 0;
  // result (guarded by the server mutex once published)
  bool done = false;
  int status = RKHSBA_OK;
  std::string err;
  std::vector<double> loss, pairs;
  Clock::time_point t_submit, t_admit, t_done;
};

}  // namespace

namespace {

// A retiring request: its results on their way to a pinned host slot.
struct Retiring {
  std::shared_ptr<Req> q;
  hipEvent_t ev = nullptr;
  int slot = -1;
};

constexpr int kRetireSlots = 128;
constexpr size_t kRetireSlotBytes = 16384;  // poses, loss and pair-count histories, status

struct Lane {
  int id = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t build_stream = nullptr;        // admission builds (the lane's iterations keep running)
  std::unique_ptr<Engine> eng;
  SetLayout lay;
  std::thread worker;
  std::deque<std::shared_ptr<Req>> queue;    // guarded by the server mutex
  std::deque<std::shared_ptr<Req>> ready;    // built ahead, waiting to start (guarded by the server mutex)
  std::vector<std::shared_ptr<Req>> active;  // worker thread only
  int64_t dev_bytes = 0;                     // the engine's device memory, guarded by the server mutex
  hipEvent_t iter_ev[2] = {nullptr, nullptr};  // the last two batch iterations (bounds the host's lead)
  hipEvent_t iter_start[2] = {nullptr, nullptr};
  double iter_charge[2] = {0.0, 0.0};  // device ms charged to the lane when the iteration was launched
  int64_t iter_epoch[2] = {-1, -1};    // the sharing epoch of that charge (-1: none)
  int iter_next = 0;
  bool busy = false;  // has active requests (guarded by the server mutex)
  // Retirement: the worker queues the copy of a finished request's results to a pinned slot; the
  // completer thread waits for each copy in order, hands the results to the waiter, and returns the
  // request's problem to the worker, which frees its device memory (guarded by rmu).
  std::mutex rmu;
  std::condition_variable rcv;
  std::deque<Retiring> retiring;
  std::vector<int> done_probs;
  bool rstop = false;
  std::thread completer;
  uint8_t* pinned = nullptr;
  std::vector<int> free_slots;
  std::vector<hipEvent_t> free_events;
};

}  // namespace

struct rkhsba_server {
  rkhsba_server_options opt{};
  std::vector<std::unique_ptr<Lane>> lanes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<int64_t, std::shared_ptr<Req>> tickets;
  bool stop = false;
  int64_t next_ticket = 1;
  int64_t committed = 0;  // estimated bytes of admitted requests (all lanes)
  // lane 1's service rate: seconds from start to completion per unit of work, over its completed requests
  double l1_work = 0.0, l1_secs = 0.0;
  int64_t row_bytes = 4;  // stored feature bytes per point (admission estimates)
  rkhsba_server_stats stats{};
  std::string err;
  // Device time of the two lanes.  Their batch iterations run one after another on the device (each lane's
  // stream waits for the other lane's last launched iteration), and while both lanes have active requests a
  // lane launches its next iteration only when its device time so far, divided by its weight, is not ahead
  // of the other lane's: lane 0 (small requests) gets at most w / (1 + w) of the device, w = lane0_weight.
  // Run side by side instead, the small requests' short kernels waited behind the large requests' sweeps
  // for most of each iteration.  The times are measured with events over each iteration (charged with the
  // lane's running estimate at launch); a lane that becomes active while the other one is busy starts level
  // with it, and both restart from zero when the other one is idle.
  double used_ms[2] = {0.0, 0.0};
  double est_ms[2] = {0.0, 0.0};
  int64_t share_epoch = 0;
  hipEvent_t last_end[2] = {nullptr, nullptr};  // guarded by mu
  std::mutex launch_mu;                          // held by a lane while it launches an iteration (taken before mu)

  bool may_run(int id) const {
    const int o = 1 - id;
    if (!lanes[o]->busy) return true;
    const double w[2] = {opt.lane0_weight, 1.0};
    return used_ms[id] / w[id] <= used_ms[o] / w[o];
  }

  void set_busy(Lane& L, bool b) {
    std::lock_guard<std::mutex> lk(mu);
    if (b && !L.busy) {
      const int o = 1 - L.id;
      if (lanes[o]->busy) {
        // A lane that becomes active starts level with the other one (the same device time per weight), so
        // that neither lane's time before counts for or against it.
        const double w[2] = {opt.lane0_weight, 1.0};
        used_ms[L.id] = used_ms[o] / w[o] * w[L.id];
      } else {
        share_epoch += 1;
        used_ms[0] = used_ms[1] = 0.0;
      }
    }
    L.busy = b;
    cv_work.notify_all();
  }

  // The measured time of a completed iteration replaces its charge.
  void account(Lane& L, int slot) {
    if (L.iter_epoch[slot] < 0) return;
    float ms = 0.f;
    RK_HIP(hipEventElapsedTime(&ms, L.iter_start[slot], L.iter_ev[slot]));
    std::lock_guard<std::mutex> lk(mu);
    if (L.iter_epoch[slot] == share_epoch) used_ms[L.id] += (double)ms - L.iter_charge[slot];
    est_ms[L.id] = est_ms[L.id] > 0.0 ? 0.75 * est_ms[L.id] + 0.25 * (double)ms : (double)ms;
    L.iter_epoch[slot] = -1;
    cv_work.notify_all();
  }

  void finish(const std::shared_ptr<Req>& q, int status, const std::string& msg) {
    std::lock_guard<std::mutex> lk(mu);
    q->status = status;
    q->err = msg;
    q->done = true;
    q->t_done = Clock::now();
    if (status == RKHSBA_OK) stats.completed += 1;
    else stats.failed += 1;
    if (q->admitted) committed -= q->est_bytes;
    q->admitted = false;
    if (status == RKHSBA_OK && q->timed && q->work > 0.0) {
      l1_work += q->work;
      l1_secs += std::chrono::duration<double>(q->t_done - q->t_admit).count();
    }
    cv_done.notify_all();
    cv_work.notify_all();  // memory was released: other lanes may admit
  }

  void retire(Lane& L, const std::shared_ptr<Req>& q) {
    Problem* p = L.eng->problem(q->prob);
    int status = RKHSBA_OK;
    std::string msg;
    try {
      q->loss.assign(q->n_iter + 1, 0.0);
      q->pairs.assign(q->n_iter + 1, 0.0);
      L.eng->download_poses(p, q->poses.data());
      L.eng->read_history(p, q->n_iter + 1, q->loss.data(), q->pairs.data());
      if (L.eng->read_status(p) != 0) {
        status = RKHSBA_ENOTPD;
        msg = "Cholesky pivot not positive in a Gauss-Newton step";
      }
    } catch (const Fail& f) {
      status = f.code;
      msg = f.msg;
    }
    L.eng->remove_problem(q->prob);
    q->prob = -1;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (double v : q->pairs) stats.pair_evals += (int64_t)v;
    }
    finish(q, status, msg);
  }

  // Bytes of a request's results in a pinned slot: poses, loss and pair-count histories, (iter, status).
  static size_t result_bytes(const Req& q) { return sizeof(double) * (12 * (size_t)q.K + 2 * (size_t)(q.n_iter + 1)) + 8; }

  // Starts the copy of a finished request's results to a pinned slot and hands it to the lane's completer
  // thread; the request's device memory stays reserved until the copy has completed.  Falls back to the
  // synchronous retire() when no slot fits.
  void retire_async(Lane& L, const std::shared_ptr<Req>& q) {
    Retiring r;
    {
      std::lock_guard<std::mutex> lk(L.rmu);
      if (L.free_slots.empty() || result_bytes(*q) > kRetireSlotBytes) {
        r.slot = -1;
      } else {
        r.slot = L.free_slots.back();
        L.free_slots.pop_back();
        if (!L.free_events.empty()) {
          r.ev = L.free_events.back();
          L.free_events.pop_back();
        }
      }
    }
    if (r.slot < 0) {
      retire(L, q);
      return;
    }
    r.q = q;
    if (!r.ev) RK_HIP(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
    uint8_t* dst = L.pinned + (size_t)r.slot * kRetireSlotBytes;
    double* poses = reinterpret_cast<double*>(dst);
    double* loss = poses + 12 * q->K;
    double* pairs = loss + (q->n_iter + 1);
    L.eng->copy_results_async(L.eng->problem(q->prob), q->n_iter + 1, poses, loss, pairs,
                              reinterpret_cast<int32_t*>(pairs + q->n_iter + 1));
    RK_HIP(hipEventRecord(r.ev, L.stream));
    {
      std::lock_guard<std::mutex> lk(L.rmu);
      L.retiring.push_back(r);
    }
    L.rcv.notify_all();
  }

  // Completer thread of a lane: delivers results in the order their copies were queued.
  void complete(Lane& L) {
    (void)hipSetDevice(opt.device);
    for (;;) {
      Retiring r;
      {
        std::unique_lock<std::mutex> lk(L.rmu);
        L.rcv.wait(lk, [&] { return L.rstop || !L.retiring.empty(); });
        if (L.retiring.empty()) return;  // stopping and drained
        r = L.retiring.front();
      }
      const hipError_t e = hipEventSynchronize(r.ev);
      const std::shared_ptr<Req> q = r.q;
      int status = e == hipSuccess ? RKHSBA_OK : RKHSBA_EDEVICE;
      std::string msg = e == hipSuccess ? "" : std::string("result copy: ") + hipGetErrorString(e);
      if (e == hipSuccess) {
        const uint8_t* src = L.pinned + (size_t)r.slot * kRetireSlotBytes;
        const double* poses = reinterpret_cast<const double*>(src);
        const double* loss = poses + 12 * q->K;
        const double* pairs = loss + (q->n_iter + 1);
        const int32_t* state = reinterpret_cast<const int32_t*>(pairs + q->n_iter + 1);
        std::copy(poses, poses + 12 * q->K, q->poses.begin());
        q->loss.assign(loss, loss + q->n_iter + 1);
        q->pairs.assign(pairs, pairs + q->n_iter + 1);
        if (state[1] != 0) {
          status = RKHSBA_ENOTPD;
          msg = "Cholesky pivot not positive in a Gauss-Newton step";
        }
      }
      {
        std::lock_guard<std::mutex> lk(L.rmu);
        L.retiring.pop_front();
        L.free_slots.push_back(r.slot);
        L.free_events.push_back(r.ev);
        L.done_probs.push_back(q->prob);
      }
      L.rcv.notify_all();
      {
        std::lock_guard<std::mutex> lk(mu);
        for (double v : q->pairs) stats.pair_evals += (int64_t)v;
      }
      q->prob = -1;
      finish(q, status, msg);
    }
  }

  // Frees the device memory of the requests the completer has delivered (worker thread).
  void release_delivered(Lane& L) {
    std::vector<int> probs;
    {
      std::lock_guard<std::mutex> lk(L.rmu);
      probs.swap(L.done_probs);
    }
    for (int id : probs) L.eng->remove_problem(id);
  }

  void drop(Lane& L, const std::shared_ptr<Req>& q, int code, const std::string& msg) {
    if (q->prob >= 0) L.eng->remove_problem(q->prob);
    q->prob = -1;
    finish(q, code, msg);
  }

  // Builds a request's voxel structures in the lane's engine.  A build that grows a pool waits for the whole
  // device, which the runtime refuses while any stream is capturing a graph; with two lanes the build
  // therefore holds the launch lock, under which the other lane launches and captures its iterations.
  int build_problem(Lane& L, const Req& q) {
    std::unique_lock<std::mutex> dl(launch_mu, std::defer_lock);
    if (lanes.size() > 1) dl.lock();
    return L.eng->add_problem_auto(q.par, q.K, q.n_points.data(), q.xyz.data(), q.feat_kind, q.D, q.feats.data(),
                                   q.is_device != 0);
  }

  // Lane 1 with reordering: the built request to start next is the one whose estimated service time less
  // the time it has waited since submission is smallest (arrival order until a completed request has given
  // the lane a rate).  Waiting time enters one for one, so a long request is not passed over for ever.
  // Called with the server mutex held.
  std::shared_ptr<Req> pick_ready(Lane& L) {
    const double rate = l1_work > 0.0 ? l1_secs / l1_work : 0.0;
    const Clock::time_point now = Clock::now();
    size_t best = 0;
    double best_key = 0.0;
    for (size_t i = 0; i < L.ready.size(); ++i) {
      const double waited = std::chrono::duration<double>(now - L.ready[i]->t_submit).count();
      const double key = L.ready[i]->work * rate - waited;
      if (i == 0 || key < best_key) {
        best = i;
        best_key = key;
      }
    }
    std::shared_ptr<Req> q = L.ready[best];
    L.ready.erase(L.ready.begin() + (std::ptrdiff_t)best);
    return q;
  }

  // Estimated work of a built request: entries x the points per occupied r_c-cube its build measured (the
  // candidates of one iteration, up to a factor) x its evaluations.
  static double request_work(const Req& q, const Problem* p) {
    const double occ = p->occupancy_r > 0.0 ? p->occupancy_r : p->occupancy;
    return (double)q.entries * occ * (double)(q.n_iter + 1);
  }

  void run(Lane& L) {
    (void)hipSetDevice(opt.device);
    // lane 1 (large requests) runs at most lane1_max_active of them at once
    const int max_active = (L.id == 1 && opt.lane1_max_active > 0) ? std::min(opt.lane1_max_active, opt.max_active)
                                                                   : opt.max_active;
    // lane 1 running one request at a time may start its waiting requests out of arrival order: while it runs
    // one, it builds up to kReady of the next ahead (their builds measure the density that the service
    // estimate needs), and starts the built one that pick_ready chooses
    const bool reorder = L.id == 1 && max_active == 1 && opt.lane1_order == 1;
    constexpr size_t kReady = 4;
    for (;;) {
      std::vector<std::shared_ptr<Req>> admit;
      std::shared_ptr<Req> started, pre;
      release_delivered(L);
      {
        std::unique_lock<std::mutex> lk(mu);
        if (L.active.empty()) cv_work.wait(lk, [&] { return stop || !L.queue.empty() || !L.ready.empty(); });
        if (stop) break;
        const bool running = !L.active.empty();
        if (reorder && !running && !L.ready.empty()) started = pick_ready(L);
        int64_t work = 0;
        for (const auto& a : L.active) work += a->entries;
        while (!started && !L.queue.empty() && (int)(L.active.size() + admit.size()) < max_active) {
          const std::shared_ptr<Req>& q = L.queue.front();
          const bool idle = L.active.empty() && admit.empty();
          if (!idle && committed + q->est_bytes > opt.hbm_budget_bytes) break;
          if (!idle && opt.lane_work_entries > 0 && work + q->entries > opt.lane_work_entries) break;
          work += q->entries;
          committed += q->est_bytes;
          q->admitted = true;
          admit.push_back(q);
          L.queue.pop_front();
        }
        if (reorder && running && L.ready.size() < kReady && !L.queue.empty() &&
            committed + L.queue.front()->est_bytes <= opt.hbm_budget_bytes) {
          pre = L.queue.front();
          L.queue.pop_front();
          committed += pre->est_bytes;
          pre->admitted = true;
        }
      }
      if (started) {
        started->t_admit = Clock::now();
        started->timed = true;
        L.active.push_back(started);
      }
      for (auto& q : admit) {
        try {
          q->prob = build_problem(L, *q);
          Problem* p = L.eng->problem(q->prob);
          if (L.id == 0 && lanes.size() > 1 && opt.lane_split_work > 0.0) {
            // The build measured the points per occupied r_c-cube: entries x that occupancy estimates the
            // candidates a Gauss-Newton iteration tests.  A request above the split goes to lane 1 (it is
            // built there again), so that it does not slow the iterations of the small requests here.
            const double occ = p->occupancy_r > 0.0 ? p->occupancy_r : p->occupancy;
            if ((double)q->entries * occ > opt.lane_split_work) {
              L.eng->remove_problem(q->prob);
              q->prob = -1;
              {
                std::lock_guard<std::mutex> lk(mu);
                committed -= q->est_bytes;
                q->admitted = false;
                auto& Q = lanes[1]->queue;
                auto pos = std::find_if(Q.begin(), Q.end(), [&](const std::shared_ptr<Req>& o) {
                  return o->ticket > q->ticket;
                });
                Q.insert(pos, q);
              }
              cv_work.notify_all();
              continue;
            }
          }
          {
            // the admission estimate's resident part becomes the built problem's pools (label-stacked
            // class-id grids can hold several cell-row descriptors per point)
            const int64_t d = p->resident_bytes - Engine::estimate_resident_bytes(q->K, q->n_points.data(),
                                                                                  row_bytes);
            std::lock_guard<std::mutex> lk(mu);
            committed += d;
            q->est_bytes += d;
          }
          L.eng->upload_poses(p, q->poses.data());
          L.eng->reset_state(p);
          q->work = request_work(*q, p);
          q->timed = reorder;
          q->t_admit = Clock::now();
          L.active.push_back(q);
        } catch (const Fail& f) {
          drop(L, q, f.code, f.msg);
        } catch (...) {
          drop(L, q, RKHSBA_EDEVICE, "unexpected exception at admission");
        }
      }
      if (pre) {
        // built while the lane's iterations run (at most two are in flight); it starts later
        try {
          pre->prob = build_problem(L, *pre);
          Problem* p = L.eng->problem(pre->prob);
          L.eng->upload_poses(p, pre->poses.data());
          L.eng->reset_state(p);
          pre->work = request_work(*pre, p);
          const int64_t d = p->resident_bytes - Engine::estimate_resident_bytes(pre->K, pre->n_points.data(),
                                                                                row_bytes);
          std::lock_guard<std::mutex> lk(mu);
          committed += d;
          pre->est_bytes += d;
          L.ready.push_back(pre);
        } catch (const Fail& f) {
          drop(L, pre, f.code, f.msg);
        } catch (...) {
          drop(L, pre, RKHSBA_EDEVICE, "unexpected exception at admission");
        }
      }
      if (L.active.empty()) continue;
      try {
        std::vector<SetItem> items;
        bool all_final = true;
        for (auto& q : L.active) {
          items.push_back(SetItem{L.eng->problem(q->prob), q->edges.data(), q->E, q->par.fixed_frame, q->n_iter});
          all_final = all_final && q->evals == q->n_iter;
        }
        // at most two batch iterations in flight: the host prepares the next while the device runs one
        const int si = L.iter_next;
        hipEvent_t& slot = L.iter_ev[si];
        if (slot) {
          RK_HIP(hipEventSynchronize(slot));
          account(L, si);
        }
        const bool shared = lanes.size() > 1;
        if (shared) {
          set_busy(L, true);
          std::unique_lock<std::mutex> lk(mu);
          cv_work.wait(lk, [&] { return stop || may_run(L.id); });
        }
        L.eng->prepare(L.lay, items);
        if (!slot) RK_HIP(hipEventCreate(&slot));
        if (!L.iter_start[si]) RK_HIP(hipEventCreate(&L.iter_start[si]));
        {
          // The lanes launch one at a time, each iteration after the other lane's last one.  (The other
          // lane's event is then neither being recorded again nor on a stream in graph capture, which the
          // runtime would take as a dependency on captured work.)
          std::unique_lock<std::mutex> dl(launch_mu, std::defer_lock);
          hipEvent_t after = nullptr;
          if (shared) {
            dl.lock();
            std::lock_guard<std::mutex> lk(mu);
            after = last_end[1 - L.id];
          }
          if (after) RK_HIP(hipStreamWaitEvent(L.stream, after, 0));
          RK_HIP(hipEventRecord(L.iter_start[si], L.stream));
          // A lane that runs one request at a time keeps the binning order of the request's first
          // iteration, as rkhsba_gn_step does; a batch sorts afresh every iteration, so that a request's
          // result does not depend on when other requests join or leave.
          const bool solo = max_active == 1;
          if (all_final) {
            L.eng->evaluate(L.lay, MODE_LOSS, solo);
            L.eng->loss_only(L.lay);
          } else {
            L.eng->iterate(L.lay, 1, solo);
          }
          RK_HIP(hipEventRecord(slot, L.stream));
          if (shared) {
            std::lock_guard<std::mutex> lk(mu);
            last_end[L.id] = slot;
            L.iter_charge[si] = est_ms[L.id];
            L.iter_epoch[si] = share_epoch;
            used_ms[L.id] += est_ms[L.id];
            cv_work.notify_all();
          }
        }
        L.iter_next ^= 1;
        const int64_t mine = L.eng->device_bytes();
        {
          std::lock_guard<std::mutex> lk(mu);
          stats.batch_iterations += 1;
          stats.max_active = std::max<int64_t>(stats.max_active, (int64_t)L.active.size());
          L.dev_bytes = mine;
          int64_t dev = 0;
          for (const auto& l : lanes) dev += l->dev_bytes;
          stats.peak_device_bytes = std::max<int64_t>(stats.peak_device_bytes, dev);
        }
        std::vector<std::shared_ptr<Req>> still;
        for (auto& q : L.active) {
          q->evals += 1;
          if (q->evals > q->n_iter) retire_async(L, q);
          else still.push_back(q);
        }
        L.active.swap(still);
        if (L.active.empty() && lanes.size() > 1) set_busy(L, false);
      } catch (const Fail& f) {
        for (auto& q : L.active) drop(L, q, f.code, f.msg);
        L.active.clear();
        if (lanes.size() > 1) set_busy(L, false);
      }
    }
    // shutting down: results in flight are delivered; drop what is active or queued in this lane
    {
      std::unique_lock<std::mutex> lk(L.rmu);
      L.rcv.wait(lk, [&] { return L.retiring.empty(); });
      L.rstop = true;
    }
    L.rcv.notify_all();
    release_delivered(L);
    for (auto& q : L.active) drop(L, q, RKHSBA_ESTATE, "server shut down");
    L.active.clear();
    std::deque<std::shared_ptr<Req>> built;
    {
      std::lock_guard<std::mutex> lk(mu);
      built.swap(L.ready);
    }
    for (auto& q : built) drop(L, q, RKHSBA_ESTATE, "server shut down");
    std::deque<std::shared_ptr<Req>> rest;
    {
      std::lock_guard<std::mutex> lk(mu);
      rest.swap(L.queue);
    }
    for (auto& q : rest) finish(q, RKHSBA_ESTATE, "server shut down");
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_work.notify_all();
    for (auto& L : lanes)
      if (L->worker.joinable()) L->worker.join();
    for (auto& L : lanes) {
      {
        std::lock_guard<std::mutex> lk(L->rmu);
        L->rstop = true;
      }
      L->rcv.notify_all();
      if (L->completer.joinable()) L->completer.join();
    }
    (void)hipSetDevice(opt.device);
    for (auto& L : lanes) {
      if (L->stream) (void)hipStreamSynchronize(L->stream);
      if (L->build_stream) (void)hipStreamSynchronize(L->build_stream);
      L->lay.drop_graph();
      L->eng.reset();
      if (L->own_stream) (void)hipStreamDestroy(L->stream);
      if (L->build_stream) (void)hipStreamDestroy(L->build_stream);
      if (L->pinned) (void)hipHostFree(L->pinned);
      for (hipEvent_t ev : L->free_events) (void)hipEventDestroy(ev);
      for (hipEvent_t ev : L->iter_ev)
        if (ev) (void)hipEventDestroy(ev);
      for (hipEvent_t ev : L->iter_start)
        if (ev) (void)hipEventDestroy(ev);
    }
    lanes.clear();
  }
};

extern "C" {

void rkhsba_server_default_options(rkhsba_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->device = 0;
  o->feat_kind = RKHSBA_FEAT_CLASS_ID;
  o->D = 0;
  o->max_active = 64;
  o->hbm_budget_bytes = 0;
  o->pass_points = 0;
  o->use_graphs = 1;
  o->hessian_fp32 = 0;
  o->stream = nullptr;
  o->lanes = 1;
  o->lane_split_entries = 2000000;
  o->lane_work_entries = 0;
  o->lane1_max_active = 1;
  o->lane_split_work = 5e8;
  o->lane0_weight = 0.25;
  o->lane1_order = 1;
}

int rkhsba_server_create(rkhsba_server** out, const rkhsba_server_options* opt) {
  if (!out) return RKHSBA_EINVAL;
  *out = nullptr;
  if (!opt || opt->max_active < 1 || opt->hbm_budget_bytes < 0 ||
      (opt->pass_points != 0 && opt->pass_points != 1 && opt->pass_points != 8 && opt->pass_points != 16 &&
       opt->pass_points != 32 && opt->pass_points != 64) ||
      opt->feat_kind < RKHSBA_FEAT_CLASS_ID || opt->feat_kind > RKHSBA_FEAT_DENSE_FP8 ||
      (opt->feat_kind != RKHSBA_FEAT_CLASS_ID && (opt->D < 1 || opt->D > kMaxDense)) || opt->lanes < 1 ||
      opt->lanes > 2 || opt->lane_split_entries < 0 || opt->lane_work_entries < 0 || opt->lane1_max_active < 0 ||
      !(opt->lane_split_work >= 0.0) || !(opt->lane0_weight > 0.0 && opt->lane0_weight < 1e6) ||
      (opt->lane1_order != 0 && opt->lane1_order != 1))
    return RKHSBA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || opt->device < 0 || opt->device >= ndev) return RKHSBA_EDEVICE;
  if (hipSetDevice(opt->device) != hipSuccess) return RKHSBA_EDEVICE;
  rkhsba_server* s = new (std::nothrow) rkhsba_server();
  if (!s) return RKHSBA_ENOMEM;
  s->opt = *opt;
  if (s->opt.hbm_budget_bytes == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return RKHSBA_EDEVICE;
    }
    s->opt.hbm_budget_bytes = (int64_t)(0.8 * (double)free_b);
  }
  s->row_bytes = opt->feat_kind == RKHSBA_FEAT_CLASS_ID
                     ? 4
                     : (int64_t)feat_elem_bytes(opt->feat_kind) * dense_pad(opt->D, opt->feat_kind);
  int rc = RKHSBA_OK;
  try {
    for (int i = 0; i < opt->lanes && rc == RKHSBA_OK; ++i) {
      std::unique_ptr<Lane> L(new Lane());
      L->id = i;
      if (i == 0 && opt->stream) {
        L->stream = static_cast<hipStream_t>(opt->stream);
      } else if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) == hipSuccess) {
        L->own_stream = true;
      } else {
        rc = RKHSBA_EDEVICE;
        break;
      }
      L->eng.reset(new Engine(opt->device, L->stream, 0));
      L->eng->use_graphs = opt->use_graphs != 0;
      L->eng->fp32_sums = opt->hessian_fp32 != 0;
      // a batch iteration's graph pays for its capture only if the active set stays the same a while
      L->eng->graph_min_uses = 3;
      if (hipStreamCreateWithFlags(&L->build_stream, hipStreamNonBlocking) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void**>(&L->pinned), kRetireSlots * kRetireSlotBytes,
                        hipHostMallocDefault) != hipSuccess) {
        rc = RKHSBA_EDEVICE;
        s->lanes.push_back(std::move(L));
        break;
      }
      L->eng->build_st = L->build_stream;
      for (int k = kRetireSlots - 1; k >= 0; --k) L->free_slots.push_back(k);
      s->lanes.push_back(std::move(L));
    }
    if (rc == RKHSBA_OK)
      for (auto& L : s->lanes) {
        Lane* lp = L.get();
        L->worker = std::thread([s, lp] { s->run(*lp); });
        L->completer = std::thread([s, lp] { s->complete(*lp); });
      }
  } catch (...) {
    rc = RKHSBA_EDEVICE;
  }
  if (rc != RKHSBA_OK) {
    s->shutdown();
    delete s;
    return rc;
  }
  *out = s;
  return RKHSBA_OK;
}

void rkhsba_server_destroy(rkhsba_server* s) {
  if (!s) return;
  s->shutdown();
  delete s;
}

int rkhsba_server_submit(rkhsba_server* s, const rkhsba_request* r, int64_t* ticket) {
  if (!s || !r || !ticket) return RKHSBA_EINVAL;
  *ticket = 0;
  if (r->K < 1 || !r->n_points || !r->xyz || !r->feats || !r->poses || r->E < 1 || !r->edges || r->n_iter < 0 ||
      r->feat_kind != s->opt.feat_kind || (r->feat_kind != RKHSBA_FEAT_CLASS_ID && r->D != s->opt.D) ||
      !(r->ell > 0.0) || !(r->cutoff_factor > 0.0) || r->cell_subdiv < 0 || r->cell_subdiv > 8 ||
      r->fixed_frame < 0 || r->fixed_frame >= r->K)
    return RKHSBA_EINVAL;
  for (int e = 0; e < r->E; ++e) {
    const int m = r->edges[2 * e], n = r->edges[2 * e + 1];
    if (m < 0 || n < 0 || m >= r->K || n >= r->K || m == n) return RKHSBA_EINVAL;
  }
  for (int f = 0; f < r->K; ++f)
    if (r->n_points[f] < 1 || !r->xyz[f] || !r->feats[f]) return RKHSBA_EINVAL;
  try {
    auto q = std::make_shared<Req>();
    q->par.ell = r->ell;
    q->par.cutoff_factor = r->cutoff_factor;
    q->par.sigma = r->sigma;
    q->par.damping_rel = r->damping_rel;
    q->par.fixed_frame = r->fixed_frame;
    q->par.clamp_negative_c = r->clamp_negative_c;
    q->par.cell_subdiv = r->cell_subdiv;
    q->par.pass_points = s->opt.pass_points;
    q->K = r->K;
    q->E = r->E;
    q->n_iter = r->n_iter;
    q->is_device = r->is_device;
    q->feat_kind = r->feat_kind;
    q->D = r->feat_kind == RKHSBA_FEAT_CLASS_ID ? 0 : r->D;
    q->n_points.assign(r->n_points, r->n_points + r->K);
    q->xyz.assign(r->xyz, r->xyz + r->K);
    q->feats.assign(r->feats, r->feats + r->K);
    q->poses.assign(r->poses, r->poses + 12 * (size_t)r->K);
    q->edges.assign(r->edges, r->edges + 2 * (size_t)r->E);
    q->est_bytes = Engine::estimate_bytes(r->K, r->n_points, r->E, s->row_bytes);
    int64_t entries = 0;
    for (int e = 0; e < r->E; ++e) entries += r->n_points[r->edges[2 * e]];
    q->entries = entries;
    const size_t lane = (s->lanes.size() > 1 && entries > s->opt.lane_split_entries) ? 1 : 0;
    q->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) return RKHSBA_ESTATE;
      q->ticket = s->next_ticket++;
      s->tickets[q->ticket] = q;
      s->lanes[lane]->queue.push_back(q);
      s->stats.submitted += 1;
    }
    s->cv_work.notify_all();
    *ticket = q->ticket;
    return RKHSBA_OK;
  } catch (const std::bad_alloc&) {
    return RKHSBA_ENOMEM;
  }
}

int rkhsba_server_wait(rkhsba_server* s, int64_t ticket, double timeout_s, double* poses_out, double* loss_per_iter,
                       int64_t* pairs_per_iter, double* latency_s, double* queue_s) {
  if (!s) return RKHSBA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return RKHSBA_EINVAL;
  std::shared_ptr<Req> q = it->second;
  auto ready = [&] { return q->done; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return RKHSBA_EBUSY;
  }
  s->tickets.erase(it);
  if (q->status == RKHSBA_OK || q->status == RKHSBA_ENOTPD) {
    if (poses_out) std::copy(q->poses.begin(), q->poses.end(), poses_out);
    for (int i = 0; i <= q->n_iter && i < (int)q->loss.size(); ++i) {
      if (loss_per_iter) loss_per_iter[i] = q->loss[i];
      if (pairs_per_iter) pairs_per_iter[i] = (int64_t)q->pairs[i];
    }
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_submit).count();
  if (queue_s)
    *queue_s = q->t_admit.time_since_epoch().count() == 0
                   ? 0.0
                   : std::chrono::duration<double>(q->t_admit - q->t_submit).count();
  s->err = q->err;
  return q->status;
}

int rkhsba_server_stats_get(rkhsba_server* s, rkhsba_server_stats* out) {
  if (!s || !out) return RKHSBA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->queued = 0;
  for (const auto& L : s->lanes) out->queued += (int64_t)(L->queue.size() + L->ready.size());
  return RKHSBA_OK;
}

const char* rkhsba_server_last_error(const rkhsba_server* s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
