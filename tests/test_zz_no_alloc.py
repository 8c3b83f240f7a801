"""The allocation-free loss evaluation (rkhsba_eval_loss_noalloc) against
rkhsba_eval_loss, through the C ABI: the same kernels on the same resident
frames, with the layout and scratch in the library's static device array
instead of allocated buffers.  Two calls in a row, the second with a smaller
input (fewer edges, then a smaller problem), so the second call runs on what
the first left in the array; results must match the allocating entry point's
(F, per-edge F and pair counts), and an input too large for the array is
rejected with RKHSBA_ENOMEM."""
import sys

import numpy as np
import pytest

import scenes
from helpers import REL_TOL

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


def compare(ctx, poses, edges, what):
    F0, Fe0, n0 = ctx.eval_loss(poses, edges)
    F1, Fe1, n1 = ctx.eval_loss_noalloc(poses, edges)
    say(f"[noalloc] {what}: F {F1:.12g} / {F0:.12g}, pairs {n1} / {n0}")
    assert n1 == n0 and n0 > 0
    assert abs(F1 - F0) <= REL_TOL * abs(F0)
    np.testing.assert_allclose(Fe1, Fe0, rtol=REL_TOL, atol=0)
    return F1, n1


def test_noalloc_loss_matches_eval_loss(rk):
    p = scenes.odometry(1, n_frames=6, n_points=8000, n_iter=2)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, sigma=1.3)
    ctx.build_neighbors(p.points, p.feats, p.feat_kind)
    compare(ctx, p.init_poses, p.edges, "odometry 6 x 8000, 15 edges")
    compare(ctx, p.gt_poses, p.edges[:4], "same frames, 4 edges (smaller second call)")
    ctx.close()
    q = scenes.lidar(2, n_frames=4, n_points=6000, n_neighbours=2, n_iter=3, spacing=3.125)
    ctx2 = rk.Context(ell=q.ell, cutoff_factor=q.cutoff_factor, cell_subdiv=2, pass_points=8)
    ctx2.build_neighbors(q.points, q.feats, q.feat_kind)
    compare(ctx2, q.init_poses, q.edges, "LiDAR 4 x 6000, class ids, 8-point passes")
    compare(ctx2, q.init_poses, q.edges[:1], "one edge")
    ctx2.close()


def test_noalloc_rejects_an_input_beyond_its_scratch(rk):
    rng = np.random.default_rng(5)
    pts = [rng.uniform(-5, 5, size=(600_000, 3)).astype(np.float32) for _ in range(2)]
    lab = [np.zeros(600_000, np.uint16)] * 2
    ctx = rk.Context(ell=0.05, cell_subdiv=1, pass_points=16)
    ctx.build_neighbors(pts, lab, "class")
    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    edges = [[0, 1], [1, 0]] * 3   # 3.6 million entries
    with pytest.raises(rk.RkhsbaError) as e:
        ctx.eval_loss_noalloc(np.stack([I, I]), edges)
    assert e.value.code == rk.ENOMEM and "static scratch" in str(e.value)
    # the array still serves a call that fits
    compare(ctx, np.stack([I, I]), [[0, 1]], "one 600k-point edge after the rejected call")
    ctx.close()
