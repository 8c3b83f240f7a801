"""Gauss-Newton poses at every workload's full size and full iteration count
against the oracle's trajectories (Sec. V-A: IRLS steps with the weights
recomputed after each step; pose tolerance 1e-4 rad / 1e-4 m per frame).

The oracle's trajectories are computed once on the CPU by
tests/golden/make_trajectories.py (FP64, FP32 membership rule; brute force,
or for the LiDAR map and the dense64 runs the cell-list search, which gives
the brute-force sums) and stored beside it with a digest of their inputs;
the GPU runs the same seeded workload in the benchmark's launch
configuration, from the same initial poses, for the same number of steps.
Each stored trajectory also records how far the oracle's own final poses
move when every input coordinate moves by one FP32 ulp: where that spread is
far below the tolerance, the comparison is meaningful (pinned by
conditioning).

Workloads: two_view 2 x 5,000 (10 steps); odometry 8 x 30,000 (15 steps);
LiDAR 64 x 100,000 with 384 directed pairs (10 steps); dense64 8 x 30,000
with 64-dim features in FP32, bfloat16 and fp8 (15 steps; the low-precision
runs against the oracle fed the rounded features).
"""
import json
import os
import sys

import numpy as np
import pytest

from helpers import REL_TOL, ROT_TOL, TRANS_TOL, pose_errors, scene_digest

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# (scene, feature storage, cell_subdiv, pass_points): the benchmark autotuner's choices
RUNS = {
    "two_view": ("two_view", "class", 1, 1),
    "odometry": ("odometry", "dense", 8, 16),
    "lidar": ("lidar", "class", 2, 8),
    "dense64": ("dense64", "dense", 6, 16),
    "dense64_bf16": ("dense64", "bf16", 6, 16),
    "dense64_fp8": ("dense64", "fp8", 4, 16),
}
# fp8 inner products on the matrix cores are not correctly rounded (see test_gpu_mixed): loss bar
LOSS_TOL = {"dense64_fp8": 2.5e-4}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


@pytest.mark.parametrize("name", list(RUNS))
def test_full_trajectory_matches_oracle(rk, full_scenes, name):
    path = os.path.join(GOLDEN, f"trajectory_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle trajectory for {name} (tests/golden/make_trajectories.py {name})")
    with open(path) as f:
        gold = json.load(f)
    scene, kind, S, P = RUNS[name]
    p = full_scenes.get(scene)
    assert scene_digest(p.points, p.feats, p.init_poses, p.edges) == gold["input_sha256"], \
        "the seeded workload differs from the one the stored trajectory was computed on"
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, cell_subdiv=S, pass_points=P)
    ctx.build_neighbors(p.points, p.feats, kind)
    poses, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, p.n_iter)
    ctx.close()
    trace = np.asarray(gold["pose_trace"])
    oloss = np.asarray(gold["loss"])
    rot, tr = pose_errors(poses, trace[-1])
    cond = gold.get("conditioning", {})
    lrel = np.abs(lpi - oloss) / np.abs(oloss)
    say(f"[trajectory] {name}: {p.n_iter} steps, rotation error {rot.max():.3g} rad, translation error "
        f"{tr.max():.3g} m (oracle one-ulp spread {cond.get('rot_spread_rad', float('nan')):.3g} rad, "
        f"{cond.get('trans_spread_m', float('nan')):.3g} m); loss rel error max {lrel.max():.3g}; "
        f"F {lpi[0]:.9g} -> {lpi[-1]:.9g}, {int(ppi.mean())} pairs per evaluation")
    assert len(lpi) == len(oloss) == p.n_iter + 1
    np.testing.assert_array_equal(poses[0], p.init_poses[0])  # the gauge frame
    assert lrel.max() <= LOSS_TOL.get(name, REL_TOL)
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
