"""GPU path of the per-point top-k truncation (the Time-Analysis paragraph of
Sec. VI) against the oracle: kept pair lists bit-exact, loss and normal
equations within the floating-point tolerance, Gauss-Newton poses."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from helpers import REL_TOL, ROT_TOL, TRANS_TOL, assert_blocks_close, normwise_rel, pose_errors

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


SCENES = {
    "odometry_small": lambda: scenes.odometry(1, n_frames=4, n_points=4000, n_iter=4),
    "two_view_ragged": lambda: scenes.two_view(3, n_points=1237),
    "dense64_small": lambda: scenes.dense64(5, n_frames=3, n_points=3000, n_iter=3),
    "lidar_small": lambda: scenes.lidar(2, n_frames=4, n_points=6000, n_neighbours=2, n_iter=3, spacing=3.125),
}


@pytest.fixture(scope="module", params=list(SCENES))
def scene(request):
    say(f"[scene] {request.param}")
    return request.param, SCENES[request.param]()


def contexts(rk, p, k):
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, top_k=k)
    ctx.build_neighbors(p.points, p.feats, p.feat_kind)
    return ctx, oracle.Problem.from_scene(p, top_k=k)


@pytest.mark.parametrize("k", [8, 1, 3])
def test_topk_pair_lists_bit_exact(rk, scene, k):
    name, p = scene
    ctx, op = contexts(rk, p, k)
    for poses in (p.init_poses, p.gt_poses):
        for (m, n) in p.edges[:2]:
            got = ctx.export_pairs(poses, m, n)
            ref = oracle.pairs(op, poses, m, n)
            say(f"[topk pairs] {name} k={k} edge ({m},{n}) gpu {len(got)} oracle {len(ref)}")
            assert len(ref) > 0
            assert np.bincount(ref[:, 0]).max() <= k
            np.testing.assert_array_equal(got, ref)
    ctx.close()


def test_topk_normal_equations_parity(rk, scene):
    name, p = scene
    ctx, op = contexts(rk, p, 8)
    H, b, F, npairs = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    oF, ob, oH, oFe, onp = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    say(f"[topk normal] {name} pairs {npairs} / {onp} F {F:.9g} / {oF:.9g} "
        f"b rel {normwise_rel(b, ob):.3g} H rel {normwise_rel(H, oH):.3g}")
    assert npairs == onp
    assert abs(F - oF) <= REL_TOL * abs(oF)
    assert_blocks_close(b, ob, 6, what=f"{name} b")
    assert_blocks_close(H, oH, 6, what=f"{name} H")
    F2, Fe, n2 = ctx.eval_loss(p.init_poses, p.edges)
    assert n2 == onp
    assert abs(F2 - oF) <= REL_TOL * abs(oF)
    assert normwise_rel(Fe, oFe) <= REL_TOL
    full = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor)
    full.build_neighbors(p.points, p.feats, p.feat_kind)
    Ff, _, nf = full.eval_loss(p.init_poses, p.edges)
    assert n2 <= nf and F2 <= Ff * (1 + REL_TOL)
    full.close()
    ctx.close()


def test_topk_gauss_newton_parity(rk, scene):
    name, p = scene
    ctx, op = contexts(rk, p, 8)
    n_iter = min(p.n_iter, 3)
    poses, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, n_iter)
    oposes, olpi = oracle.gn(op, p.init_poses, p.edges, n_iter, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(poses, oposes)
    say(f"[topk gn] {name} rot err {rot.max():.3g} trans err {tr.max():.3g} loss {lpi[-1]:.9g} / {olpi[-1]:.9g}")
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    ctx.close()


def test_topk_rejects_unsupported_settings(rk):
    p = scenes.dense64(5, n_frames=2, n_points=500, n_iter=1)
    with pytest.raises(rk.RkhsbaError):
        rk.Context(ell=p.ell, top_k=9)
    ctx = rk.Context(ell=p.ell, top_k=8)
    with pytest.raises(rk.RkhsbaError):
        ctx.build_neighbors(p.points, p.feats, "bf16")
    ctx.close()
