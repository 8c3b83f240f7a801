#!/usr/bin/env python3
"""Throughput of the RKHS-BA hot path on one MI355X.

One step = one whole solve of the LiDAR-mapping workload: the voxel build of
all frames from device-resident clouds (rkhsba_build_neighbors) followed by
the Gauss-Newton / IRLS iterations (rkhsba_gn_step: per iteration, transforms,
binning, candidate sweep, finalisation, assembly, Cholesky and pose update,
plus the final loss evaluation).  Workload: 64 spinning-LiDAR frames x
100,000 points over a 200 m street loop, 20% uniform outliers, 20-class
one-hot labels with 10% flipped, each frame paired with its 6 nearest poses
(384 directed pairs), ell = 0.3 m, cutoff 3 ell, 10 iterations (seeded
synthetic scene).  --workload selects the other configurations (odometry,
dense64, two_view) for kernel studies.

The printed JSON line reports pair evaluations per second (in-radius pairs
with c != 0, summed over every evaluation of the step), Gauss-Newton
iterations per second, the roofline position of the candidate-sweep kernel
measured with HIP events on the library's stream, the voxel build's
bandwidth, and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kernel pair-evals/s + GN iters/s at 1 GPU; p50/p99 solve latency at fixed QPS"
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak
# Algorithmic work per in-radius pair of the sweep (FMA = 2 flops, exp = 1):
# residual 3 + squared distance 5 + scale 1 + exp 1 + weight 1 + A 1 + w*d 3 + B 3 + C 12
FLOPS_PER_PAIR_GEOM = 30
# the sweep kernel and the engine that lays out its pass table (the pass order changes the kernel's traffic)
PAIR_KERNEL_SOURCES = [os.path.join(ROOT, "paper_2403_01254_amd", "csrc", f) for f in ("sweep.hip", "engine.hip")]
# calibrated HBM bytes per sweep launch from rocprofv3 counters, per workload (profiles/)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_{workload}_traffic.json")
WORKLOADS = {
    "odometry": "odometry: 8 depth-camera frames x 30,000 points, 23-dim soft-label+RGB features, all 28 frame "
                "pairs, ell=0.08 m, cutoff 3 ell, 15 Gauss-Newton iterations (one step = voxel build + 15 "
                "iterations + final loss)",
    "lidar": "lidar: 64 spinning-LiDAR frames x 100,000 points, 20% outliers, 20-class one-hot labels with 10% "
             "flipped, 384 directed 6-nearest-pose pairs, ell=0.3 m, cutoff 3 ell, 10 Gauss-Newton iterations",
    "two_view": "two_view: 2 frames x 5,000 points, 10-class one-hot labels, ell=0.1 m, cutoff 3 ell, "
                "10 Gauss-Newton iterations",
    "dense64": "dense64: as odometry with 64-dim unit-vector features (per-class mean + N(0, 0.1) jitter, "
               "renormalised; negative inner products clamped to 0)",
}


def kernel_source_hash():
    h = hashlib.sha256()
    for path in PAIR_KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload, config):
    """HBM bytes per launch of the sweep kernel from the committed rocprofv3
    counter summary of this workload, if it was taken on the current kernel
    source in the same launch configuration."""
    try:
        with open(TRAFFIC_FILE.format(workload=workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    for e in (t if isinstance(t, list) else [t]):  # one summary per profiled configuration
        if e.get("kernel_source_sha256_16") == kernel_source_hash() and e.get("config") == list(config):
            return e.get("bytes_per_launch")
    return None


def cpu_info():
    """Host description for the CPU baseline: CPUs this process may use and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), model


def build_bytes_per_point(p, cell_subdiv, kind, Dp):
    """Bytes the voxel build's kernels read and write per point, by design: cell coordinates (read xyz
    12, write 12), keys and values (read 12, write 8), each 8-bit digit pass of the radix sort (histogram
    read 4, scatter read 8 + write 8), the gather into key order (read value 4 + xyz 12 + feature, write
    point 16 + index 4 + stored feature), the key copy (8), and the row extents and cell tables (read
    keys 4 + 4).  Digit passes: ceil(key bits / 8) of the largest frame grid."""
    import math
    import numpy as np
    inv = 1.0 / ((p.cutoff_factor * p.ell) / cell_subdiv)
    cells = 1
    for x in p.points:
        k = np.floor(x.astype(np.float64) * inv)
        cells = max(cells, int(np.prod(k.max(0) - k.min(0) + 1)))
    key_bits = max(1, math.ceil(math.log2(cells)))
    passes = math.ceil(key_bits / 8)
    feat_in = 2 if kind == "class" else 4 * p.D
    feat_out = 0 if kind == "class" else {"dense": 4, "bf16": 2, "fp8": 1}[kind] * Dp
    return 24 + 20 + 20 * passes + (4 + 12 + feat_in + 16 + 4 + feat_out) + 8 + 8, passes


def _make_request(seed):
    import scenes
    return scenes.request(seed)


def start_request_generation(n, workers):
    """Generates the serving requests in worker processes (spawned, so the
    parent's GPU state is never inherited); returns the pending futures."""
    import concurrent.futures
    import multiprocessing
    if n <= 0:
        return None, []
    ex = concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
    return ex, [ex.submit(_make_request, 1000 + i) for i in range(n)]


def stop_request_generation(ex):
    """Joins the worker pool and the resource-tracker process that multiprocessing starts for its queues
    (it would otherwise outlive the pool until this process exits)."""
    ex.shutdown(wait=True)
    try:
        from multiprocessing import resource_tracker
        resource_tracker._resource_tracker._stop()
    except (ImportError, AttributeError, OSError):
        pass


def percentile_ms(lat, q):
    import numpy as np
    return float(np.percentile(np.asarray(lat) * 1e3, q)) if len(lat) else None


def serving_benchmark(reqs, rkhsba, torch, log, seed=0, lanes=2, work_entries=8_000_000):
    """Seeded Poisson stream of whole solves: capacity of the one-at-a-time
    FP32 form, then, at 0.5x and 0.9x of it, latency percentiles and
    throughput of the continuous-batching request loop and of the
    one-at-a-time form fed the same arrivals."""
    import threading
    import numpy as np
    dev = torch.device("cuda:0")
    staged = []
    for p in reqs:
        staged.append(([torch.from_numpy(x).to(dev) for x in p.points], [torch.from_numpy(f).to(dev) for f in p.feats]))
    torch.cuda.synchronize()
    D = reqs[0].D
    ctxs = {}

    def ctx_for(ell):
        if ell not in ctxs:
            ctxs[ell] = rkhsba.Context(ell=ell, cell_subdiv=0)
        return ctxs[ell]

    def solve_one(i):
        """One request on its own context; None if a Gauss-Newton step met a non-positive Cholesky pivot."""
        p = reqs[i]
        c = ctx_for(p.ell)
        c.build_neighbors(staged[i][0], staged[i][1], p.feat_kind)
        try:
            return c.gn_step(p.init_poses, p.edges, p.n_iter)
        except rkhsba.RkhsbaError as e:
            if e.code != rkhsba.ENOTPD:
                raise
            return None

    solve_one(0)  # warm-up (library load, first allocations)
    t0 = time.perf_counter()
    seq = [solve_one(i) for i in range(len(reqs))]
    cap_s = time.perf_counter() - t0
    capacity = len(reqs) / cap_s
    seq_pairs = sum(int(r[2].sum()) for r in seq if r is not None)
    not_pd = [i for i, r in enumerate(seq) if r is None]
    if not_pd:
        log(f"[serving] {len(not_pd)} request(s) met a non-positive Cholesky pivot: " +
            "; ".join(reqs[i].recipe for i in not_pd))
    log(f"[serving] one-at-a-time capacity {capacity:.2f} solves/s ({len(reqs)} requests in {cap_s:.2f} s)")
    rng = np.random.default_rng(seed)
    runs = []
    pose_diff = {}

    def run_batched(kind, arrivals):
        # two lanes: small requests batched in lane 0; requests whose measured work (entries x points per
        # occupied r_c-cube) is large run one at a time in lane 1; the lanes' iterations take turns on the device
        srv = rkhsba.Server(feat_kind=kind, D=D, max_active=64, lanes=lanes, lane_work_entries=work_entries)
        tickets = [None] * len(reqs)
        start = time.perf_counter() + 0.05

        def submitter():
            for i, p in enumerate(reqs):
                dt = start + arrivals[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(staged[i][0], staged[i][1], p.init_poses, p.edges, p.ell, p.n_iter)

        th = threading.Thread(target=submitter)
        th.start()
        lat, out = [], []
        for i in range(len(reqs)):
            while tickets[i] is None:
                time.sleep(1e-4)
            r = srv.wait(tickets[i], with_status=True)
            out.append(r)
            lat.append(r[3])
        th.join()
        end = time.perf_counter()
        st = srv.stats()
        srv.close()
        rot_d, tr_d = 0.0, 0.0
        for r, q in zip(out, seq):
            if q is None or r[5] != rkhsba.OK:
                continue
            for a, b in zip(r[0], q[0]):
                Ra, Rb = a[:9].reshape(3, 3), b[:9].reshape(3, 3)
                c = np.clip((np.trace(Ra.T @ Rb) - 1.0) / 2.0, -1.0, 1.0)
                rot_d = max(rot_d, float(np.arccos(c)))
                tr_d = max(tr_d, float(np.linalg.norm(a[9:] - b[9:])))
        not_pd_batched = sum(1 for r in out if r[5] != rkhsba.OK)
        prev = pose_diff.get(kind, (0.0, 0.0))
        pose_diff[kind] = (max(prev[0], rot_d), max(prev[1], tr_d))
        return {"p50_ms": percentile_ms(lat, 50), "p99_ms": percentile_ms(lat, 99),
                "solves_per_s": len(reqs) / (end - start), "pair_evals_per_s": st["pair_evals"] / (end - start),
                "max_active": st["max_active"], "batch_iterations": st["batch_iterations"],
                "mean_queue_ms": 1e3 * float(np.mean([r[4] for r in out])), "not_pd_requests": not_pd_batched,
                "max_pose_diff_vs_one_at_a_time_f32": {"rot_rad": rot_d, "trans_m": tr_d}}

    # capacity of the batched forms: every request submitted at once
    saturated = {}
    for k in ("dense", "bf16"):
        saturated[k] = run_batched(k, np.zeros(len(reqs)))
        log(f"[serving] all at once, batched {k}: {saturated[k]['solves_per_s']:.2f} solves/s "
            f"(up to {saturated[k]['max_active']} active, {saturated[k]['batch_iterations']} batch iterations)")
    for frac in (0.5, 0.9):
        qps = frac * capacity
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=len(reqs)))
        arrivals -= arrivals[0]
        batched = {}
        for k in ("dense", "bf16"):
            batched[k] = run_batched(k, arrivals)
            log(f"[serving] {qps:.2f} req/s: batched {k} done")
        # one at a time, FP32, same arrivals
        lat1 = []
        start1 = time.perf_counter()
        for i in range(len(reqs)):
            dt = start1 + arrivals[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            solve_one(i)
            lat1.append(time.perf_counter() - (start1 + arrivals[i]))
        end1 = time.perf_counter()
        single = {"p50_ms": percentile_ms(lat1, 50), "p99_ms": percentile_ms(lat1, 99),
                  "solves_per_s": len(reqs) / (end1 - start1), "pair_evals_per_s": seq_pairs / (end1 - start1)}
        for k, v in batched.items():
            log(f"[serving] {qps:.2f} req/s, batched {k}: p50 {v['p50_ms']:.1f} ms p99 {v['p99_ms']:.1f} ms "
                f"({v['solves_per_s']:.2f} solves/s, up to {v['max_active']} active)")
        log(f"[serving] {qps:.2f} req/s, one-at-a-time f32: p50 {single['p50_ms']:.1f} ms p99 {single['p99_ms']:.1f} ms")
        runs.append({"qps": qps, "load": frac, "batched_f32": batched["dense"], "batched_bf16": batched["bf16"],
                     "one_at_a_time_f32": single})
    for c in ctxs.values():
        c.close()
    return {"requests": len(reqs), "lanes": lanes, "lane_work_entries": work_entries,
            "lane1_order": "built ahead, shortest estimated service less waiting time first (library default)",
            "capacity_one_at_a_time_solves_per_s": capacity,
            "not_pd_requests_one_at_a_time": len(not_pd),
            "capacity_batched_f32_solves_per_s": saturated["dense"]["solves_per_s"],
            "capacity_batched_bf16_solves_per_s": saturated["bf16"]["solves_per_s"],
            "pair_evals_per_s_one_at_a_time": seq_pairs / cap_s, "runs": runs,
            "max_pose_diff_vs_one_at_a_time_f32": {k: {"rot_rad": v[0], "trans_m": v[1]} for k, v in pose_diff.items()},
            "pose_accuracy_vs_fp64_oracle": "tests/test_gpu_server.py::test_served_forms_against_oracle (FP32 forms "
                                            "within 1e-4 rad / 1e-4 m; the bf16 form within 1e-4 rad / 1e-4 m "
                                            "of the oracle on bf16-rounded features, its difference to the "
                                            "unrounded oracle printed)",
            "recipe": "requests: K ~ U{2..16} frames, N_m log-uniform in [5e3, 1.2e5], copies-of-a-scene or "
                      "depth-camera trajectory with a 0.3 m minimum range (p = 1/2), 20-class Dirichlet(0.3) soft "
                      "labels (D = 20), ell in {0.08, 0.3} m, all i<j pairs, 10 Gauss-Newton iterations, inputs "
                      "resident in HBM; Poisson arrivals at 0.5x and 0.9x of the measured one-at-a-time capacity"}


def cpu_baseline(p, workload, reps=5):
    """The oracle timed on the host cores: normal-equation evaluations (loss, b, H; FP64) of a fixed sample
    of the workload's frame pairs at the initial poses, one warm-up then `reps` timed runs; the value is
    the pairs of one evaluation over the median time.  Brute force over all point pairs (the definition)
    where that finishes in seconds, else the oracle's cell-list search (the same pairs and sums)."""
    import numpy as np
    import oracle
    stride, search = {"lidar": (48, "cells"), "dense64": (4, "cells"), "odometry": (4, "brute")}.get(
        workload, (1, "brute"))
    op = oracle.Problem.from_scene(p, search=search)
    edges = p.edges[::stride]
    times = []
    for r in range(reps + 1):
        t0 = time.perf_counter()
        _, _, _, _, npairs = oracle.normal_eqs(op, p.init_poses, edges)
        if r > 0:
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    nproc, model = cpu_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    mode = "brute force over all point pairs" if search == "brute" else "cell-list search (27 world cells per point)"
    return {"value": npairs / med, "unit": "pair-evals/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "cpu_model": model, "search": search,
            "sample": f"median of {reps} normal-equation evaluations (loss, b, H; FP64, {mode}) after one warm-up, "
                      f"of {len(edges)} of the {len(p.edges)} frame pairs (every {stride}th) at the initial poses: "
                      f"{npairs} in-radius pairs in {med:.3f} s (runs {min(times):.3f}-{max(times):.3f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--pass-points", type=int, default=0, help="0: chosen at the build (or by the autotuner)")
    ap.add_argument("--cell-subdiv", type=int, default=0, help="0: chosen at the build (or by the autotuner)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep --cell-subdiv/--pass-points instead of the autotuner's choice (made during warm-up)")
    ap.add_argument("--no-graphs", action="store_true", help="issue every launch eagerly (no HIP graph replay)")
    ap.add_argument("--moment-path", type=int, default=0, help="0 library choice, 1 vector ALU, 2 matrix cores")
    ap.add_argument("--features", default="f32", choices=["f32", "bf16", "fp8"],
                    help="storage / inner-product precision of dense features (bf16, fp8: matrix cores)")
    ap.add_argument("--workload", default="lidar", choices=["lidar", "odometry", "two_view", "dense64"],
                    help="lidar is the headline configuration; the others are for kernel studies")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=128,
                    help="requests in the serving measurement (0: skip); the serving workload's full stream is 512")
    ap.add_argument("--serving-lanes", type=int, default=2, choices=[1, 2],
                    help="concurrent batches of the request server (large requests in the second)")
    ap.add_argument("--serving-work-entries", type=int, default=8_000_000,
                    help="request server: most (edge, source point) entries active in one lane (0: no limit)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this size (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2403_01254_amd import rkhsba

    def log(msg):
        if not args.quiet:
            print(msg, file=sys.stderr, flush=True)

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = {"odometry": scenes.odometry, "lidar": scenes.lidar, "two_view": scenes.two_view,
         "dense64": scenes.dense64}[args.workload](0)
    kind = p.feat_kind
    if kind == "dense" and args.features != "f32":
        kind = args.features
    log(f"[bench] workload {p.recipe}: {len(p.edges)} edges, {p.n_iter} GN iterations")
    dev = torch.device("cuda:0")
    pts = [torch.from_numpy(x).to(dev) for x in p.points]
    # class ids travel as their 16-bit patterns
    feats = [torch.from_numpy(f.view(np.int16) if f.dtype == np.uint16 else f).to(dev) for f in p.feats]
    torch.cuda.synchronize()
    ctx = rkhsba.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, pass_points=args.pass_points,
                         cell_subdiv=args.cell_subdiv, moment_path=args.moment_path,
                         use_graphs=not args.no_graphs)
    if not args.no_autotune:
        S, P, ms = ctx.autotune(pts, feats, kind, p.init_poses, p.edges, trials=2)
        log(f"[bench] autotuner: cell_subdiv {S}, pass_points {P} ({ms:.3f} ms per normal-equation evaluation)")

    def step():
        ctx.build_neighbors(pts, feats, kind)
        return ctx.gn_step(p.init_poses, p.edges, p.n_iter)

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    for s in range(rkhsba.PROF_SOLVE + 1):
        ctx.profile_read(s, reset=True)
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs_total = 0
    for k in range(args.steps):
        poses, lpi, ppi = step()
        pairs_total += int(ppi.sum())
        log(f"[bench] step {k + 1}/{args.steps}: F {lpi[0]:.6g} -> {lpi[-1]:.6g}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.profile_enable(False)
    ms_per_step = 1e3 * elapsed / args.steps
    # the same steps without stage events: Gauss-Newton iterations replayed from a HIP graph
    graph_ms = None
    if not args.no_graphs:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            step()
        torch.cuda.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t1) / args.steps
        log(f"[bench] graph-replayed steps: {graph_ms:.3f} ms/step")
    prof = {rkhsba.PROF_NAMES[s]: ctx.profile_read(s) for s in range(rkhsba.PROF_SOLVE + 1)}
    cfg_subdiv, cfg_pass, cfg_occ = ctx.config()
    for name, (ms, n) in prof.items():
        log(f"[bench] stage {name:12s} {ms / args.steps:9.3f} ms/step over {n // max(args.steps, 1)} launches/step")

    # roofline of the sweep kernel (Gauss-Newton evaluations): algorithmic flops per launch / mean launch time
    pair_ms, pair_launches = prof["pairs"]
    gn_pairs_per_launch = float(np.mean(ppi[:-1])) if p.n_iter > 0 else 0.0
    # FP32 features: the inner products run on the FP32 matrix cores, whose published peak equals the
    # FP32 vector peak, and are counted in the same budget; bf16 / fp8 inner products run on the
    # low-precision matrix cores and are not counted against the FP32 peak.
    flops_per_pair = FLOPS_PER_PAIR_GEOM + (2 * p.D if kind == "dense" else 0)
    mean_launch_s = pair_ms / max(pair_launches, 1) / 1e3
    achieved = flops_per_pair * gn_pairs_per_launch / mean_launch_s / 1e12 if mean_launch_s > 0 else 0.0
    # committed counters hold for the workload, feature storage and launch configuration they were taken on
    traffic = load_traffic(args.workload, [kind, cfg_subdiv, cfg_pass]) if args.moment_path in (0, 1) else None
    # voxel build bandwidth: bytes its kernels move by design over the measured build time
    build_ms, build_n = prof["build"]
    Dp = 0 if kind == "class" else next(w for w in ((8, 16, 24, 32, 64) if kind == "dense" else (32, 64)) if w >= p.D)
    bpp, sort_passes = build_bytes_per_point(p, cfg_subdiv, kind, Dp)
    n_points = int(sum(len(x) for x in p.points))
    build_s = build_ms / max(build_n, 1) / 1e3

    result = {
        "metric": METRIC,
        "value": pairs_total / elapsed,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if kind in ("class", "dense") else f"f32+{kind}",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload],
            "frames": p.K, "points_per_frame": int(p.n_points[0]), "edges": int(len(p.edges)),
            "gn_iterations": p.n_iter, "feature_dim": p.D, "feature_storage": kind, "ell": p.ell,
            "pass_points": cfg_pass, "cell_subdiv": cfg_subdiv, "moment_path": args.moment_path,
            "autotuned": not args.no_autotune, "points_per_rc_cube": cfg_occ,
        },
        "gn_iters_per_s": p.n_iter * args.steps / elapsed,
        "graph_replay_ms_per_step": graph_ms,
        "pairs_per_step": pairs_total // args.steps,
        "stage_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "build": {"ms": build_s * 1e3, "points": n_points, "bytes_per_point": bpp, "sort_digit_passes": sort_passes,
                  "GB_per_s": bpp * n_points / build_s / 1e9 if build_s > 0 else None, "peak_GB_per_s": 8000.0},
        "roofline": {
            "bound": "alu",
            "kernel": "k_sweep (candidate sweep, Gauss-Newton moments)" if cfg_pass in (8, 16) else "k_pairs (candidate sweep, Gauss-Newton moments)",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "flops_per_pair": flops_per_pair,
            "pairs_per_launch": gn_pairs_per_launch,
            "mean_launch_ms": mean_launch_s * 1e3,
        },
    }
    rank = int(os.environ.get("RANK", "0"))
    if rank == 0 and not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(p, args.workload)
        log(f"[bench] CPU oracle: {result['cpu_baseline']['sample']}")
    # serving requests are generated only now, so that no worker process competes with the timed regions above
    gen_pool, gen_futures = start_request_generation(args.serving_requests, workers=8)
    if gen_futures:
        reqs = []
        for i, f in enumerate(gen_futures):
            reqs.append(f.result())
            if (i + 1) % 32 == 0 and i + 1 < len(gen_futures):
                log(f"[bench] serving: {i + 1} of {len(gen_futures)} requests generated")
        stop_request_generation(gen_pool)
        log(f"[bench] serving: {len(reqs)} requests generated")
        result["serving"] = serving_benchmark(reqs, rkhsba, torch, log, lanes=args.serving_lanes,
                                              work_entries=args.serving_work_entries)
    if rank == 0:
        print(json.dumps(result), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
