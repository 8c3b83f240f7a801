"""GPU path (through the C ABI) against the FP64 oracle.

Neighbour structures and pair lists must match bit for bit; F, b and H within
1e-5 normwise relative; poses after Gauss-Newton steps within 1e-4 rad and
1e-4 m.  Inputs are the seeded synthetic scenes at sizes the oracle finishes
in seconds (several sweep passes, finalisation blocks and sort tiles, with
ragged tails).
"""
import sys

import numpy as np
import pytest

import oracle
import scenes
from helpers import (REL_TOL, ROT_TOL, TRANS_TOL, assert_blocks_close, ident, inv_cell, label_stacked,
                     normwise_rel, pose_errors)

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


def make_ctx(rk, p, **kw):
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, **kw)
    ctx.build_neighbors(p.points, p.feats, p.feat_kind)
    return ctx


SCENES = {
    "two_view": lambda: scenes.two_view(0),
    "odometry_small": lambda: scenes.odometry(1, n_frames=4, n_points=4000, n_iter=4),
    "lidar_small": lambda: scenes.lidar(2, n_frames=4, n_points=6000, n_neighbours=2, n_iter=3, spacing=3.125),
    "two_view_ragged": lambda: scenes.two_view(3, n_points=1237),
    "dense64_small": lambda: scenes.dense64(5, n_frames=3, n_points=3000, n_iter=3),
    "lidar_k12": lambda: scenes.lidar(3, n_frames=12, n_points=3000, n_neighbours=4, n_iter=3, spacing=3.125),
}


@pytest.fixture(scope="module", params=list(SCENES))
def scene(request):
    say(f"[scene] {request.param}")
    return request.param, SCENES[request.param]()


def test_voxel_structure_bit_exact(rk, scene):
    name, p = scene
    for subdiv in (1, 3):
        ctx = make_ctx(rk, p, cell_subdiv=subdiv)
        inv = inv_cell(p.ell, p.cutoff_factor, subdiv)
        vox = [ctx.export_voxels(f, len(p.points[f])) for f in range(p.K)]
        stacked = p.feat_kind == "class" and label_stacked(p.feats, [v[3] for v in vox])
        say(f"[voxels] {name} subdiv {subdiv}: label-stacked {stacked}")
        for f in range(p.K):
            perm, keys, org, dims, layers = vox[f]
            assert layers == (int(p.feats[f].max()) + 1 if stacked else 0)
            operm, okeys, oorg, odims = oracle.voxels(p.points[f], inv, margin=0,
                                                      labels=p.feats[f] if stacked else None)
            np.testing.assert_array_equal(org, oorg)
            np.testing.assert_array_equal(dims, odims)
            np.testing.assert_array_equal(keys, okeys)
            np.testing.assert_array_equal(perm, operm)
        ctx.close()


def test_pair_lists_bit_exact(rk, scene):
    name, p = scene
    op = oracle.Problem.from_scene(p)
    ctx = make_ctx(rk, p)
    for poses in (p.init_poses, p.gt_poses):
        for (m, n) in p.edges[:3]:
            got = ctx.export_pairs(poses, m, n)
            ref = oracle.pairs(op, poses, m, n)
            say(f"[pairs] {name} edge ({m},{n}) gpu {len(got)} oracle {len(ref)}")
            assert len(ref) > 0
            np.testing.assert_array_equal(got, ref)


def test_loss_parity(rk, scene):
    name, p = scene
    op = oracle.Problem.from_scene(p)
    ctx = make_ctx(rk, p)
    F, Fe, npairs = ctx.eval_loss(p.init_poses, p.edges)
    oF, ob, oH, oFe, onp = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    say(f"[loss] {name} F gpu {F:.9g} oracle {oF:.9g} pairs {npairs} / {onp}")
    assert npairs == onp
    assert abs(F - oF) <= REL_TOL * abs(oF)
    assert normwise_rel(Fe, oFe) <= REL_TOL
    # the FP64 definition of membership differs only on the cutoff sphere
    dF = oracle.loss(op, p.init_poses, p.edges, oracle.MEMBER_FP64)
    assert abs(F - dF) <= REL_TOL * abs(dF)


def test_normal_equations_parity(rk, scene):
    name, p = scene
    op = oracle.Problem.from_scene(p)
    ctx = make_ctx(rk, p)
    H, b, F, npairs = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    oF, ob, oH, oFe, onp = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    say(f"[normal] {name} |b| {np.linalg.norm(ob):.4g} rel {normwise_rel(b, ob):.3g} "
        f"|H| {np.linalg.norm(oH):.4g} rel {normwise_rel(H, oH):.3g}")
    assert npairs == onp
    assert abs(F - oF) <= REL_TOL * abs(oF)
    assert_blocks_close(b, ob, 6, what=f"{name} b")
    assert_blocks_close(H, oH, 6, what=f"{name} H")
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())


@pytest.mark.parametrize("moment_path", [1, 2])
def test_normal_equations_parity_per_moment_path(rk, scene, moment_path):
    """The 16-point tiled sweep with its Gauss-Newton moments summed on the vector ALU (1) or on the matrix
    cores (2: moments about the pass's box centre, A, B, C recovered from them) against the oracle, at
    1-r_c and 1/2-r_c cells."""
    name, p = scene
    op = oracle.Problem.from_scene(p)
    oF, ob, oH, oFe, onp = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    for subdiv in (1, 2):
        ctx = make_ctx(rk, p, pass_points=16, cell_subdiv=subdiv, moment_path=moment_path)
        H, b, F, npairs = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
        say(f"[moments] {name} path {moment_path} subdiv {subdiv}: b rel {normwise_rel(b, ob):.3g} "
            f"H rel {normwise_rel(H, oH):.3g}")
        assert npairs == onp
        assert abs(F - oF) <= REL_TOL * abs(oF)
        assert_blocks_close(b, ob, 6, what=f"{name} b")
        assert_blocks_close(H, oH, 6, what=f"{name} H")
        ctx.close()


def test_gauss_newton_parity(rk, scene):
    name, p = scene
    op = oracle.Problem.from_scene(p)
    ctx = make_ctx(rk, p)
    n_iter = min(p.n_iter, 4)
    poses, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, n_iter)
    oposes, olpi = oracle.gn(op, p.init_poses, p.edges, n_iter, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(poses, oposes)
    say(f"[gn] {name} rot err {rot.max():.3g} trans err {tr.max():.3g} loss {lpi[-1]:.9g} / {olpi[-1]:.9g}")
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    np.testing.assert_array_equal(poses[0], p.init_poses[0])  # the fixed frame does not move


@pytest.mark.parametrize("pass_points,subdiv", [(1, 1), (32, 2), (64, 1), (8, 1)])
def test_gauss_newton_parity_kept_binning(rk, pass_points, subdiv):
    """Gauss-Newton steps that keep the first iteration's binning order with the untiled pass kernel (per-point
    walks, 32- and 64-point passes: the later iterations recompute the keys' out-of-grid bit) and with the
    tiled 8-point class-id sweep (which tests the grid itself), against the oracle's steps."""
    if pass_points == 8:
        p = scenes.lidar(2, n_frames=3, n_points=4000, n_neighbours=2, n_iter=3, spacing=3.125)
    else:
        p = scenes.odometry(4, n_frames=3, n_points=3000, n_iter=3)
    op = oracle.Problem.from_scene(p)
    ctx = make_ctx(rk, p, pass_points=pass_points, cell_subdiv=subdiv)
    poses, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, p.n_iter)
    oposes, olpi = oracle.gn(op, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(poses, oposes)
    say(f"[gn-kept] pass {pass_points} subdiv {subdiv}: rot err {rot.max():.3g} trans err {tr.max():.3g}")
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    ctx.close()


# scenes whose inner products are decided exactly on both sides (class ids, or features that are all
# positive): a pair's c != 0 test cannot differ between the GPU's FP32 sums and the oracle's FP64 ones
COUNT_SCENES = ["two_view_ragged", "odometry_small", "lidar_small", "lidar_k12"]
_scene_cache = {}


def scene_named(name):
    if name not in _scene_cache:
        _scene_cache[name] = SCENES[name]()
    return _scene_cache[name]


@pytest.mark.parametrize("pass_points,subdiv", [(16, 8), (16, 1), (8, 2), (8, 1), (32, 2), (64, 1), (1, 1), (1, 3)])
def test_sweep_source_counts_bit_exact(rk, pass_points, subdiv):
    """The pair set of the truncated double sum (Eq. (eq:double_sum), Sec. III-B) as the summing sweep
    itself enumerates it: every source point's count of in-radius pairs with c != 0, written by the same
    sweep launch (pass size, cell size, pass table) that accumulates the normal equations, equals the
    oracle's count from its brute-force FP32-rule pair list, point by point."""
    for name in COUNT_SCENES:
        p = scene_named(name)
        if pass_points == 8 and p.feat_kind != "class":
            continue  # 8-point passes take class ids only
        op = oracle.Problem.from_scene(p)
        ctx = make_ctx(rk, p, pass_points=pass_points, cell_subdiv=subdiv)
        assert ctx.config()[:2] == (subdiv, pass_points)
        for poses in (p.init_poses, p.gt_poses):
            for (m, n) in p.edges[:2]:
                got = ctx.export_source_counts(poses, m, n, len(p.points[m]))
                ref = np.bincount(oracle.pairs(op, poses, m, n)[:, 0], minlength=len(p.points[m]))
                assert ref.sum() > 0
                np.testing.assert_array_equal(got, ref)
                # the same sweep's per-edge total, as the normal equations report it
                _, _, _, npairs = ctx.accumulate_normal_eqs(poses, [[m, n]])
                assert npairs == ref.sum()
        say(f"[counts] {name} pass {pass_points} subdiv {subdiv}: per-source counts equal")
        ctx.close()


@pytest.mark.parametrize("pass_points", [8, 16])
def test_sparse_frames_walk_per_source(rk, pass_points):
    """Frames so sparse that every sweep pass spans many truncation radii (the case of isolated outliers):
    the class-id sweep then walks each source point's own cells.  Each point of frame 1 has a noisy copy in
    frame 2 and a few random neighbours; per-source pair counts, F, b, H and Gauss-Newton poses against the
    oracle."""
    rng = np.random.default_rng(41)
    n = 4000
    x = rng.uniform(-100.0, 100.0, size=(n, 3))
    near = x[rng.integers(0, n, size=n // 4)] + rng.normal(scale=0.1, size=(n // 4, 3))
    pts = [np.concatenate([x, near]).astype(np.float32),
           (np.concatenate([x, near]) + rng.normal(scale=0.05, size=(n + n // 4, 3))).astype(np.float32)]
    lab = [rng.integers(0, 3, size=n + n // 4).astype(np.uint16)] * 2
    ell = 0.1
    op = oracle.Problem(pts, lab, "class", ell)
    ctx = rk.Context(ell=ell, cell_subdiv=2, pass_points=pass_points)
    ctx.build_neighbors(pts, lab, "class")
    poses = np.stack([ident(), ident()])
    got = ctx.export_source_counts(poses, 0, 1, len(pts[0]))
    ref = np.bincount(oracle.pairs(op, poses, 0, 1)[:, 0], minlength=len(pts[0]))
    np.testing.assert_array_equal(got, ref)
    H, b, F, npairs = ctx.accumulate_normal_eqs(poses, [[0, 1], [1, 0]])
    oF, ob, oH, _, onp = oracle.normal_eqs(op, poses, [[0, 1], [1, 0]], oracle.MEMBER_FP32_RULE)
    say(f"[sparse] pass {pass_points}: {npairs} pairs / {onp}, F rel {abs(F - oF) / oF:.3g}")
    assert npairs == onp and abs(F - oF) <= REL_TOL * oF
    assert_blocks_close(b, ob, 6, what="sparse b")
    assert_blocks_close(H, oH, 6, what="sparse H")
    gposes, lpi, _ = ctx.gn_step(poses, [[0, 1]], 3)
    oposes, olpi = oracle.gn(op, poses, [[0, 1]], 3, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(gposes, oposes)
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    ctx.close()


@pytest.mark.parametrize("pass_points,subdiv", [(16, 1), (32, 2), (64, 3), (16, 4), (64, 1), (1, 1), (1, 3), (8, 1),
                                                (8, 3)])
def test_launch_shapes_agree(rk, pass_points, subdiv):
    """Every sweep shape and cell size gives the same pair count and, up to
    FP32 summation order, the same F, b and H (8-point passes: class ids)."""
    if pass_points == 8:
        p = scenes.lidar(2, n_frames=3, n_points=4000, n_neighbours=2, n_iter=1, spacing=3.125)
        with pytest.raises(rk.RkhsbaError):
            make_ctx(rk, scenes.odometry(4, n_frames=2, n_points=500), pass_points=8, cell_subdiv=subdiv)
    else:
        p = scenes.odometry(4, n_frames=3, n_points=3000)
    ref = make_ctx(rk, p, pass_points=16, cell_subdiv=8)
    H0, b0, F0, n0 = ref.accumulate_normal_eqs(p.init_poses, p.edges)
    ctx = make_ctx(rk, p, pass_points=pass_points, cell_subdiv=subdiv)
    H, b, F, n = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    assert n == n0
    assert abs(F - F0) <= REL_TOL * abs(F0)
    assert normwise_rel(b, b0) <= REL_TOL and normwise_rel(H, H0) <= REL_TOL


def test_degenerate_inputs(rk):
    """One-point frames, a frame with no pair in range, duplicated edges and
    zero pairs overall."""
    rng = np.random.default_rng(5)
    x = (rng.normal(size=(500, 3)) * 0.3).astype(np.float32)
    lone = np.array([[50.0, 50.0, 50.0]], np.float32)
    one = x[:1].copy()
    pts = [x, x + np.float32(0.01), lone, one]
    feats = [np.zeros(len(a), np.uint16) for a in pts]
    ctx = rk.Context(ell=0.1)
    ctx.build_neighbors(pts, feats, "class")
    poses = np.stack([ident()] * 4)
    op = oracle.Problem(pts, feats, "class", 0.1)
    edges = [[0, 1], [0, 2], [3, 0], [0, 1]]
    H, b, F, n = ctx.accumulate_normal_eqs(poses, edges)
    oF, ob, oH, _, on = oracle.normal_eqs(op, poses, edges, oracle.MEMBER_FP32_RULE)
    assert n == on and abs(F - oF) <= REL_TOL * oF
    assert normwise_rel(H, oH) <= REL_TOL and normwise_rel(b, ob) <= REL_TOL
    assert np.all(H[12:18] == 0) and np.all(b[12:18] == 0)   # the lone frame sees nothing
    F2, Fe2, n2 = ctx.eval_loss(poses, [[0, 2]])
    assert F2 == 0.0 and n2 == 0 and Fe2[0] == 0.0
    # a Gauss-Newton step leaves an isolated frame in place
    out, lpi, ppi = ctx.gn_step(poses, edges, 2)
    np.testing.assert_array_equal(out[2], poses[2])


def test_frame_of_coincident_points(rk):
    """A frame whose points all lie at one location (a depth camera placed on a
    surface returns such a view): a zero-extent voxel grid, passes of identical
    points, and exactly zero rotational terms in the oracle.  Pair counts are
    exact; F, b and H agree with the oracle within the tolerance."""
    rng = np.random.default_rng(11)
    x = (rng.normal(size=(400, 3)) * 0.1).astype(np.float32)
    spot = np.repeat(np.array([[0.02, -0.01, 0.03]], np.float32), 300, axis=0)
    pts = [x, spot]
    feats = [rng.dirichlet(np.full(6, 0.5), size=len(a)).astype(np.float32) for a in pts]
    poses = np.stack([ident(), ident()])
    poses[1, 9:] = [0.01, 0.0, -0.02]
    op = oracle.Problem(pts, feats, "dense", 0.08)
    for subdiv in (1, 8):
        ctx = rk.Context(ell=0.08, cell_subdiv=subdiv, pass_points=16)
        ctx.build_neighbors(pts, feats, "dense")
        for edges in ([[0, 1]], [[1, 0]], [[0, 1], [1, 0]]):
            H, b, F, n = ctx.accumulate_normal_eqs(poses, edges)
            oF, ob, oH, _, on = oracle.normal_eqs(op, poses, edges, oracle.MEMBER_FP32_RULE)
            say(f"[coincident] subdiv {subdiv} edges {edges}: pairs {n} / {on}, F {F:.9g} / {oF:.9g}")
            assert n == on > 0 and abs(F - oF) <= REL_TOL * oF
            assert_blocks_close(b, ob, 6, what="coincident b")
            assert_blocks_close(H, oH, 6, what="coincident H")
        ctx.close()


def test_zero_feature_rows_are_not_pairs(rk):
    """Pairs whose feature inner product is exactly 0 are not pairs (skipped by
    the oracle).  With strictly positive soft labels every product is > 0 and
    the sweep counts pairs from the membership mask alone; one all-zero row
    (or a zero in every row of each dimension) must switch that off: the counts
    stay equal to the oracle's."""
    rng = np.random.default_rng(12)
    x = (rng.normal(size=(600, 3)) * 0.1).astype(np.float32)
    y = (x[:500] + rng.normal(scale=0.01, size=(500, 3))).astype(np.float32)
    base = [rng.dirichlet(np.full(5, 0.5), size=len(a)).astype(np.float32) for a in (x, y)]
    poses = np.stack([ident(), ident()])
    zero_row = [f.copy() for f in base]
    zero_row[1][7] = 0.0
    staggered = [f.copy() for f in base]
    for d in range(5):
        staggered[0][d, d] = 0.0
    for name, feats in (("positive", base), ("zero row", zero_row), ("a zero per dimension", staggered)):
        op = oracle.Problem([x, y], feats, "dense", 0.08)
        ctx = rk.Context(ell=0.08, cell_subdiv=4, pass_points=16)
        ctx.build_neighbors([x, y], feats, "dense")
        H, b, F, n = ctx.accumulate_normal_eqs(poses, [[0, 1], [1, 0]])
        oF, ob, oH, _, on = oracle.normal_eqs(op, poses, [[0, 1], [1, 0]], oracle.MEMBER_FP32_RULE)
        say(f"[zero rows] {name}: pairs {n} / {on}")
        assert n == on and abs(F - oF) <= REL_TOL * oF
        assert_blocks_close(H, oH, 6, what=f"{name} H")
        ctx.close()


def test_frame_above_2_24_points(rk):
    """A frame of 2^24 + 250,000 points (more than FP32 counts exactly), against
    a small frame at a rotated pose: the pair lists of both directions must be
    bit-exact, with indices above 2^24 on the large side, and F, b and H within
    the usual tolerance.  The points near the small frame are the last ones of
    the large frame, so most pairs use its highest indices."""
    rng = np.random.default_rng(21)
    n_far, n_tail, n_small = 1 << 24, 250_000, 150
    big = np.empty((n_far + n_tail, 3), np.float32)
    big[:n_far, :2] = rng.uniform(-200.0, 200.0, size=(n_far, 2))
    big[n_far:, :2] = rng.uniform(-20.0, 20.0, size=(n_tail, 2)) + np.array([3.0, 150.0])
    big[:, 2] = rng.normal(scale=0.01, size=len(big))
    small = np.empty((n_small, 3), np.float32)
    small[:, 0] = rng.uniform(-2.0, 2.0, n_small)
    small[:, 1] = rng.uniform(-1.75, 1.75, n_small)
    small[:, 2] = rng.normal(scale=0.01, size=n_small)
    labels = [rng.integers(0, 3, len(a)).astype(np.uint16) for a in (big, small)]
    pose1 = ident()
    c, s = np.cos(0.2), np.sin(0.2)
    pose1[:9] = [c, -s, 0.0, s, c, 0.0, 0.0, 0.0, 1.0]
    pose1[9:] = [3.0, 150.0, 0.0]
    poses = np.stack([ident(), pose1])
    edges = [[0, 1], [1, 0]]
    say(f"[2^24] building {len(big)} + {n_small} points")
    ctx = rk.Context(ell=0.1, cell_subdiv=2, pass_points=16)
    ctx.build_neighbors([big, small], labels, "class")
    op = oracle.Problem([big, small], labels, "class", 0.1)
    for m, n in edges:
        got = ctx.export_pairs(poses, m, n)
        ref = oracle.pairs(op, poses, m, n)
        big_side = got[:, 0] if m == 0 else got[:, 1]
        say(f"[2^24] edge ({m},{n}) gpu {len(got)} oracle {len(ref)}, above 2^24: {(big_side >= n_far).sum()}")
        assert len(ref) > 1000 and (big_side >= n_far).sum() > len(ref) // 2
        np.testing.assert_array_equal(got, ref)
    H, b, F, npairs = ctx.accumulate_normal_eqs(poses, edges)
    oF, ob, oH, _, onp = oracle.normal_eqs(op, poses, edges, oracle.MEMBER_FP32_RULE)
    say(f"[2^24] F gpu {F:.9g} oracle {oF:.9g} pairs {npairs} / {onp}")
    assert npairs == onp and abs(F - oF) <= REL_TOL * oF
    assert_blocks_close(b, ob, 6, what="2^24 b")
    assert_blocks_close(H, oH, 6, what="2^24 H")
    # F is the plain sum of the pair terms in both evaluations (only b and H
    # take the correction for the rounding of q), so the two agree far below
    # the size of that correction here (2e-7 of F)
    F_loss, _, n_loss = ctx.eval_loss(poses, edges)
    say(f"[2^24] F loss-only {F_loss:.12g} normal equations {F:.12g}")
    assert n_loss == npairs and abs(F_loss - F) <= 1e-8 * F
    ctx.close()


def test_points_far_from_frame_origins(rk):
    """The same world geometry with every frame's points stored about 300 m
    from the frame's origin (poses compensate): the FP32 transformed points
    then carry rounding up to 2^-17 m, which the finalisation corrects to first
    order.  Pair counts are exact; F, b, H and Gauss-Newton poses agree with
    the oracle within the usual tolerances."""
    p = scenes.odometry(1, n_frames=4, n_points=4000, n_iter=3)
    shift = np.array([200.0, -150.0, 160.0])
    pts = [(a.astype(np.float64) + shift).astype(np.float32) for a in p.points]
    def moved(poses):
        out = np.array(poses, dtype=np.float64).copy()
        for q in out:
            q[9:] -= q[:9].reshape(3, 3) @ shift
        return out
    init = moved(p.init_poses)
    op = oracle.Problem(pts, p.feats, p.feat_kind, p.ell, p.cutoff_factor)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor)
    ctx.build_neighbors(pts, p.feats, p.feat_kind)
    H, b, F, n = ctx.accumulate_normal_eqs(init, p.edges)
    oF, ob, oH, _, on = oracle.normal_eqs(op, init, p.edges, oracle.MEMBER_FP32_RULE)
    say(f"[far] pairs {n} / {on}, F rel {abs(F - oF) / oF:.3g}, b rel {normwise_rel(b, ob):.3g}, "
        f"H rel {normwise_rel(H, oH):.3g}")
    assert n == on and abs(F - oF) <= REL_TOL * oF
    assert_blocks_close(b, ob, 6, what="far b")
    assert_blocks_close(H, oH, 6, what="far H")
    poses, lpi, _ = ctx.gn_step(init, p.edges, 3)
    oposes, olpi = oracle.gn(op, init, p.edges, 3, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(poses, oposes)
    say(f"[far] gn rot err {rot.max():.3g} trans err {tr.max():.3g}")
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    # the RKHS distance and its lengthscale derivative (Sec. V-C), whose W = sum w |d|^2 also takes the
    # first-order correction for the FP32 rounding of the transformed points
    from oracle import lengthscale as ls
    d, g = ctx.ell_gradient(init, p.edges)
    od, og = ls.distance_and_derivative(lambda ell: oracle.Problem(pts, p.feats, p.feat_kind, ell, p.cutoff_factor),
                                        p.ell, init, p.edges, oracle.MEMBER_FP32_RULE)
    say(f"[far] d_H {d:.9g} / {od:.9g}, derivative {g:.9g} / {og:.9g} (rel {abs(g - og) / abs(og):.3g})")
    assert abs(d - od) <= REL_TOL * abs(od) and abs(g - og) <= REL_TOL * abs(og)
    ctx.close()


@pytest.mark.parametrize("name,fixed,sigma,damping", [("odometry_small", 2, 1.7, 1e-3), ("two_view", 1, 0.6, 1e-10),
                                                      ("lidar_k12", 5, 2.5, 1e-6)])
def test_fixed_frame_sigma_and_damping_parity(rk, name, fixed, sigma, damping):
    """Options the default parity cases leave at their defaults: the gauge
    frame (Sec. V-A keeps the first frame fixed; any frame may be chosen), the
    kernel amplitude sigma of Eq. (eq:kernel) (it scales F, not b or H) and the
    relative damping of the step.  Loss, normal equations and Gauss-Newton
    poses against the oracle run with the same options."""
    p = SCENES[name]()
    op = oracle.Problem(p.points, p.feats, p.feat_kind, p.ell, p.cutoff_factor, sigma)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, sigma=sigma, fixed_frame=fixed, damping_rel=damping)
    ctx.build_neighbors(p.points, p.feats, p.feat_kind)
    F, Fe, npairs = ctx.eval_loss(p.init_poses, p.edges)
    oF, ob, oH, oFe, onp = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    assert npairs == onp and abs(F - oF) <= REL_TOL * abs(oF) and normwise_rel(Fe, oFe) <= REL_TOL
    H, b, F2, n2 = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    assert n2 == onp and abs(F2 - oF) <= REL_TOL * abs(oF)
    assert_blocks_close(b, ob, 6, what=f"{name} b (sigma {sigma})")
    assert_blocks_close(H, oH, 6, what=f"{name} H (sigma {sigma})")
    n_iter = 3
    poses, lpi, _ = ctx.gn_step(p.init_poses, p.edges, n_iter)
    oposes, olpi = oracle.gn(op, p.init_poses, p.edges, n_iter, fixed_frame=fixed, damping_rel=damping,
                             membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(poses, oposes)
    moved = max(np.abs(oposes[k] - p.init_poses[k]).max() for k in range(p.K) if k != fixed)
    say(f"[options] {name} fixed {fixed} sigma {sigma} damping {damping}: rot err {rot.max():.3g} "
        f"trans err {tr.max():.3g}, F {lpi[-1]:.9g} / {olpi[-1]:.9g}, largest move {moved:.3g}")
    np.testing.assert_array_equal(poses[fixed], p.init_poses[fixed])
    assert moved > 1e-4
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)
    ctx.close()


def test_common_rigid_motion_invariance_gpu(rk):
    p = scenes.odometry(6, n_frames=3, n_points=3000)
    ctx = make_ctx(rk, p)
    H0, b0, F0, n0 = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    from scipy.spatial.transform import Rotation
    G = np.eye(4)
    G[:3, :3] = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    G[:3, 3] = [1.5, -2.0, 0.7]
    moved = []
    for q in p.init_poses:
        T = np.eye(4)
        T[:3, :3] = q[:9].reshape(3, 3)
        T[:3, 3] = q[9:]
        T = G @ T
        moved.append(np.concatenate([T[:3, :3].reshape(9), T[:3, 3]]))
    H1, b1, F1, n1 = ctx.accumulate_normal_eqs(np.stack(moved), p.edges)
    assert abs(n1 - n0) <= max(2, 1e-5 * n0)   # membership is decided in FP32 after the motion
    assert abs(F1 - F0) <= 1e-5 * F0
    assert normwise_rel(b1, b0) <= 1e-4 and normwise_rel(H1, H0) <= 1e-5


def test_invalid_arguments(rk):
    p = scenes.two_view(7, n_points=300)
    ctx = make_ctx(rk, p)
    with pytest.raises(rk.RkhsbaError) as e:
        ctx.eval_loss(p.init_poses, [[0, 0]])
    assert e.value.code == rk.EINVAL
    with pytest.raises(rk.RkhsbaError) as e:
        ctx.eval_loss(p.init_poses, [[0, 5]])
    assert e.value.code == rk.EINVAL
    bad = p.init_poses.copy()
    bad[1, 9] = np.nan
    with pytest.raises(rk.RkhsbaError) as e:
        ctx.gn_step(bad, p.edges, 1)
    assert e.value.code == rk.EINVAL
    with pytest.raises(rk.RkhsbaError) as e:
        ctx.build_neighbors([np.full((3, 3), np.inf, np.float32)], [np.zeros(3, np.uint16)], "class")
    assert e.value.code == rk.EINVAL
    fresh = rk.Context(ell=0.1)
    fresh.K = 2  # the library itself holds no frames yet
    with pytest.raises(rk.RkhsbaError) as e:
        fresh.eval_loss(np.stack([ident(), ident()]), [[0, 1]])
    assert e.value.code == rk.ESTATE


def chain_of_copies(n_frames, n_points=400, seed=9):
    """n_frames noisy copies of one small cloud of class-labelled points, each frame paired with the next two:
    a quick way to a large reduced system."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    base = rng.uniform(-1.0, 1.0, size=(n_points, 3))
    labels = rng.integers(0, 4, size=n_points).astype(np.uint16)
    pts, poses = [], []
    for _ in range(n_frames):
        pts.append((base + rng.normal(scale=0.01, size=base.shape)).astype(np.float32))
        T = np.concatenate([Rotation.from_rotvec(rng.normal(scale=0.01, size=3)).as_matrix().reshape(9),
                            rng.normal(scale=0.02, size=3)])
        poses.append(T)
    edges = np.array([(k, k + d) for k in range(n_frames) for d in (1, 2) if k + d < n_frames], np.int32)
    return scenes.Problem(name=f"chain{n_frames}", points=pts, feat_kind="class", feats=[labels] * n_frames, D=4,
                          gt_poses=np.stack(poses), init_poses=np.stack(poses), edges=edges, ell=0.1)


@pytest.mark.parametrize("n_frames", [40, 90])
def test_gauss_newton_step_matches_host_solve_large_system(rk, n_frames):
    """One Gauss-Newton step on 40 frames (a 234-unknown system, several
    Cholesky panels with a ragged last one) or 90 frames (534 unknowns: the
    first panels too tall for the column-major panel in LDS) equals the step
    computed on the host from the library's own H and b (numpy solve, scipy
    SE(3) exp)."""
    import scipy.linalg
    if n_frames == 40:
        p = scenes.lidar(4, n_frames=40, n_points=2000, n_neighbours=4, spacing=3.125)
    else:
        p = chain_of_copies(n_frames)
    ctx = make_ctx(rk, p)
    H, b, F, n = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    Hr, br = H[6:, 6:], b[6:]
    nr = len(br)
    mu = 1e-10 * np.trace(Hr) / nr
    delta = np.linalg.solve(Hr + mu * np.eye(nr), -br)
    expect = p.init_poses.copy()
    for k in range(1, p.K):
        xi = delta[6 * (k - 1): 6 * k]
        W = np.zeros((4, 4))
        W[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
        W[:3, 3] = xi[:3]
        T = np.eye(4)
        T[:3, :3] = p.init_poses[k][:9].reshape(3, 3)
        T[:3, 3] = p.init_poses[k][9:]
        T = T @ scipy.linalg.expm(W)
        expect[k] = np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])
    got, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, 1)
    rot, tr = pose_errors(got, expect)
    say(f"[solve] n={nr} |delta| {np.linalg.norm(delta):.3g} rot {rot.max():.3g} trans {tr.max():.3g}")
    assert rot.max() <= 1e-9 and tr.max() <= 1e-9


def test_graph_replay_matches_eager(rk):
    """Gauss-Newton iterations replayed from a captured HIP graph give the
    same bits as the same launches issued one by one, on repeated calls and
    with other work on the stream between them."""
    p = scenes.odometry(8, n_frames=4, n_points=3000, n_iter=4)
    g = make_ctx(rk, p, use_graphs=True)
    e = make_ctx(rk, p, use_graphs=False)
    want = e.gn_step(p.init_poses, p.edges, 4)
    for rep in range(3):
        got = g.gn_step(p.init_poses, p.edges, 4)
        for x, y in zip(got, want):
            np.testing.assert_array_equal(x, y)
        g.eval_loss(p.init_poses, p.edges[:2])   # eager work between replays
        g.accumulate_normal_eqs(p.init_poses, p.edges)
    # a rebuild (new resident problem) invalidates the graph
    q = scenes.odometry(9, n_frames=3, n_points=2000, n_iter=2)
    g.build_neighbors(q.points, q.feats, q.feat_kind)
    e.build_neighbors(q.points, q.feats, q.feat_kind)
    for x, y in zip(g.gn_step(q.init_poses, q.edges, 2), e.gn_step(q.init_poses, q.edges, 2)):
        np.testing.assert_array_equal(x, y)


def test_autotune_and_auto_cell_size(rk):
    """The autotuner leaves the context on the configuration it reports, the
    results stay those of the default configuration, and a build with
    cell_subdiv = 0 on the same kind of frames picks the tuned cell size."""
    p = scenes.odometry(10, n_frames=3, n_points=3000, n_iter=2)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor)
    S, P, ms = ctx.autotune(p.points, p.feats, p.feat_kind, p.init_poses, p.edges, trials=1)
    say(f"[tune] best cell_subdiv {S} pass_points {P}: {ms:.3f} ms per evaluation")
    assert S in (1, 2, 3, 4, 6, 8) and P in (16, 32, 64) and ms > 0
    cS, cP, occ = ctx.config()
    assert (cS, cP) == (S, P) and occ > 0
    ref = make_ctx(rk, p)
    H0, b0, F0, n0 = ref.accumulate_normal_eqs(p.init_poses, p.edges)
    H, b, F, n = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    assert n == n0 and abs(F - F0) <= REL_TOL * abs(F0)
    assert normwise_rel(b, b0) <= REL_TOL and normwise_rel(H, H0) <= REL_TOL
    auto = make_ctx(rk, p, cell_subdiv=0, pass_points=0)
    aS, aP, aocc = auto.config()
    assert (aS, aP) == (S, P) and aocc == occ
    H2, b2, F2, n2 = auto.accumulate_normal_eqs(p.init_poses, p.edges)
    assert n2 == n0 and normwise_rel(H2, H0) <= REL_TOL
