#!/usr/bin/env python3
"""Writes the oracle's Gauss-Newton trajectories of the full-size workloads.

    python tests/golden/make_trajectories.py [--conditioning] NAME [NAME ...]

For each workload the FP64 oracle (and nothing else) runs the workload's full
Gauss-Newton / IRLS iteration count (Sec. V-A) from its seeded initial poses,
with the FP32 membership rule, and the poses entering every step and after
the last, the loss per iteration and a digest of the inputs are written to
trajectory_NAME.json beside this script.  With --conditioning the oracle also
runs on the input with every point coordinate moved by one FP32 ulp in a
seeded random direction, and the largest per-frame rotation / translation
difference of the final poses is stored: pose parity at 1e-4 rad / 1e-4 m is
only meaningful where this spread stays well below it.

Workloads (seed 0, the benchmark sizes):
  two_view         2 x 5,000 points, class ids, 10 iterations, brute force
  odometry         8 x 30,000 points, 23-dim features, 28 pairs, 15 iterations, brute force
  lidar            64 x 100,000 points, class ids, 384 directed pairs, 10 iterations, cell-list search
  dense64          8 x 30,000 points, 64-dim unit vectors (FP32), 15 iterations, cell-list search
  dense64_bf16     the same features rounded to bfloat16 (nearest even), cell-list search
  dense64_fp8      the same features rounded to fp8 e4m3 (nearest even, saturating), cell-list search
The cell-list search gives the brute-force pairs and sums up to summation
order (tests/test_oracle_cells.py).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import scenes  # noqa: E402
from helpers import bf16_round, e4m3_round, pose_errors, scene_digest  # noqa: E402

WORKLOADS = {
    "two_view": (lambda: scenes.two_view(0), None, "brute"),
    "odometry": (lambda: scenes.odometry(0), None, "brute"),
    "lidar": (lambda: scenes.lidar(0), None, "cells"),
    "dense64": (lambda: scenes.dense64(0), None, "cells"),
    "dense64_bf16": (lambda: scenes.dense64(0), bf16_round, "cells"),
    "dense64_fp8": (lambda: scenes.dense64(0), e4m3_round, "cells"),
}


def ulp_perturbed(points, rng):
    out = []
    for x in points:
        toward = np.where(rng.random(x.shape) < 0.5, np.float32(np.inf), np.float32(-np.inf))
        out.append(np.nextafter(x, toward).astype(np.float32))
    return out


def path(name):
    return os.path.join(HERE, f"trajectory_{name}.json")


def run(name, conditioning):
    make, rounding, search = WORKLOADS[name]
    t0 = time.time()
    p = make()
    feats = [rounding(f) for f in p.feats] if rounding else p.feats
    prob = oracle.Problem(p.points, feats, p.feat_kind, p.ell, p.cutoff_factor, search=search)
    poses, lpi, trace = oracle.gn(prob, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE,
                                  trace=True)
    print(f"[{name}] {p.n_iter} iterations in {time.time() - t0:.0f} s, F {lpi[0]:.9g} -> {lpi[-1]:.9g}",
          flush=True)
    out = {
        "workload": name, "recipe": p.recipe, "search": search, "membership": "fp32_rule",
        "feature_rounding": None if rounding is None else rounding.__name__,
        "n_iter": int(p.n_iter), "fixed_frame": 0, "damping_rel": 1e-10,
        "input_sha256": scene_digest(p.points, p.feats, p.init_poses, p.edges),
        "loss": lpi.tolist(), "pose_trace": trace.tolist(),
    }
    if conditioning:
        rng = np.random.default_rng(123)
        moved = oracle.Problem(ulp_perturbed(p.points, rng), feats, p.feat_kind, p.ell, p.cutoff_factor,
                               search="cells")
        poses1, _ = oracle.gn(moved, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
        rot, tr = pose_errors(poses1, poses)
        out["conditioning"] = {"perturbation": "every point coordinate moved by one FP32 ulp (seeded direction)",
                               "rot_spread_rad": float(rot.max()), "trans_spread_m": float(tr.max())}
        print(f"[{name}] one-ulp spread: rotation {rot.max():.3g} rad, translation {tr.max():.3g} m", flush=True)
    with open(path(name), "w") as f:
        json.dump(out, f)
    print(f"[{name}] wrote {path(name)} ({time.time() - t0:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+", choices=list(WORKLOADS))
    ap.add_argument("--conditioning", action="store_true")
    a = ap.parse_args()
    for n in a.names:
        run(n, a.conditioning)


if __name__ == "__main__":
    main()
