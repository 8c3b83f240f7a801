"""Pins of the oracle's cell-list search against its brute-force search.

The cell-list mode (the targets of the 27 world-coordinate cells around each
source point) exists so that the oracle can evaluate the large LiDAR-scale
problems; it must visit every pair the brute-force search (every point pair,
the definition of the truncated double sum of Eq. (eq:double_sum), Sec. III-B)
accepts.  Both searches then sum the same terms in different orders: pair
counts and pair lists must agree exactly, F, b and H to 1e-12 relative.
Inputs include pairs lying exactly at the truncation radius and across cell
boundaries, points hundreds of metres from the origin, and top-k selection.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenes
from helpers import normwise_rel

pytestmark = pytest.mark.usefixtures("oracle_lib")

SCENES = {
    "two_view_ragged": lambda: scenes.two_view(3, n_points=1237),
    "odometry_small": lambda: scenes.odometry(1, n_frames=4, n_points=4000, n_iter=4),
    "lidar_small": lambda: scenes.lidar(2, n_frames=4, n_points=6000, n_neighbours=2, n_iter=3, spacing=3.125),
    "dense64_small": lambda: scenes.dense64(5, n_frames=3, n_points=3000, n_iter=3),
}
MEMBERSHIP = {"fp64": oracle.MEMBER_FP64, "fp32_rule": oracle.MEMBER_FP32_RULE}


def moved(poses, rng, rot=0.02, trans=0.05):
    out = poses.copy()
    for k in range(1, len(out)):
        R = out[k][:9].reshape(3, 3) @ Rotation.from_rotvec(rng.normal(size=3) * rot).as_matrix()
        out[k] = np.concatenate([R.reshape(9), out[k][9:] + rng.normal(size=3) * trans])
    return out


def assert_same_sums(pb, pc, poses, edges, membership, what):
    Fb, bb, Hb, Feb, nb = oracle.normal_eqs(pb, poses, edges, membership)
    Fc, bc, Hc, Fec, nc = oracle.normal_eqs(pc, poses, edges, membership)
    assert nb == nc and nb > 0, f"{what}: pair counts {nc} (cells) vs {nb} (brute force)"
    assert abs(Fc - Fb) <= 1e-12 * abs(Fb), what
    np.testing.assert_allclose(Fec, Feb, rtol=1e-12, atol=1e-300)
    assert normwise_rel(bc, bb) <= 1e-12, what
    assert normwise_rel(Hc, Hb) <= 1e-12, what
    return nb


@pytest.mark.parametrize("membership", list(MEMBERSHIP))
@pytest.mark.parametrize("name", list(SCENES))
def test_cell_search_equals_brute_force(name, membership):
    p = SCENES[name]()
    pb = oracle.Problem.from_scene(p)
    pc = pb.with_search("cells")
    rng = np.random.default_rng(17)
    for poses in (p.init_poses, moved(p.init_poses, rng)):
        n = assert_same_sums(pb, pc, poses, p.edges, MEMBERSHIP[membership], name)
    print(f"[cells] {name} ({membership}): {n} pairs, equal counts and sums")


@pytest.mark.parametrize("name", list(SCENES))
def test_cell_search_pair_lists_identical(name):
    p = SCENES[name]()
    pb = oracle.Problem.from_scene(p)
    pc = pb.with_search("cells")
    for m, n in p.edges[:3]:
        lb = oracle.pairs(pb, p.init_poses, m, n)
        lc = oracle.pairs(pc, p.init_poses, m, n)
        assert len(lb) > 0
        np.testing.assert_array_equal(lc, lb)


def lattice_problem(spacing, offset, n=7):
    """Two frames holding the same cubic lattice of spacing `spacing` (one the
    other's copy shifted by `offset`): many pairs lie exactly at the lattice
    spacing, across every cell boundary."""
    g = np.stack(np.meshgrid(*[np.arange(n)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
    x = (g * spacing + offset).astype(np.float32)
    z = (g * spacing).astype(np.float32)
    lab = [np.zeros(len(x), np.uint16)] * 2
    return [x, z], lab


@pytest.mark.parametrize("factor", [1.0, 1.0 - 1e-7, 1.0 + 1e-7])
def test_cell_search_at_the_truncation_radius(factor):
    """Lattice spacing equal to r_c (and one FP32 step either side): pairs at
    exactly the truncation radius, in neighbouring cells, must be found."""
    ell = 0.1
    rc = 3 * ell
    pts, lab = lattice_problem(rc * factor, np.array([0.0, 0.0, 0.0]))
    pb = oracle.Problem(pts, lab, "class", ell)
    pc = pb.with_search("cells")
    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    rng = np.random.default_rng(18)
    for poses in (np.stack([I, I]), moved(np.stack([I, I]), rng, 1e-3, 1e-3)):
        for mem in MEMBERSHIP.values():
            assert_same_sums(pb, pc, poses, [[0, 1], [1, 0]], mem, f"lattice x{factor}")
        np.testing.assert_array_equal(oracle.pairs(pc, poses, 0, 1), oracle.pairs(pb, poses, 0, 1))


def test_cell_search_far_from_the_origin():
    """Frames whose points lie about 300 m from their origins and from the
    world origin: the FP32 rule's rounding is largest there."""
    p = scenes.two_view(4, n_points=1500)
    shift = np.array([300.0, -250.0, 120.0])
    pts = [(x.astype(np.float64) + shift).astype(np.float32) for x in p.points]
    poses = p.init_poses.copy()
    for k in range(len(poses)):
        R = poses[k][:9].reshape(3, 3)
        poses[k][9:] = poses[k][9:] - R @ shift   # T (x + shift) = T x: the same world geometry
    pb = oracle.Problem(pts, p.feats, p.feat_kind, p.ell, p.cutoff_factor)
    pc = pb.with_search("cells")
    for mem in MEMBERSHIP.values():
        assert_same_sums(pb, pc, poses, p.edges, mem, "far from origin")
    np.testing.assert_array_equal(oracle.pairs(pc, poses, 0, 1), oracle.pairs(pb, poses, 0, 1))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_cell_search_top_k(k):
    p = scenes.odometry(1, n_frames=3, n_points=2500, n_iter=2)
    pb = oracle.Problem.from_scene(p, top_k=k)
    pc = pb.with_search("cells")
    assert_same_sums(pb, pc, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE, f"top-{k}")
    np.testing.assert_array_equal(oracle.pairs(pc, p.init_poses, 0, 2), oracle.pairs(pb, p.init_poses, 0, 2))


def test_cell_search_gauss_newton():
    p = scenes.odometry(1, n_frames=4, n_points=3000, n_iter=3)
    pb = oracle.Problem.from_scene(p)
    pc = pb.with_search("cells")
    P1, l1 = oracle.gn(pb, p.init_poses, p.edges, 3, membership=oracle.MEMBER_FP32_RULE)
    P2, l2 = oracle.gn(pc, p.init_poses, p.edges, 3, membership=oracle.MEMBER_FP32_RULE)
    np.testing.assert_allclose(l2, l1, rtol=1e-12)
    np.testing.assert_allclose(P2, P1, atol=1e-11)


def test_cell_search_pairs_just_inside_the_radius_anywhere():
    """20,000 sparse points, each with one partner just inside r_c along an
    axis or a diagonal: wherever a point falls in its cell, its partner must
    be found (a cell edge even slightly below r_c would lose the pairs whose
    source lies near the top of a cell)."""
    rng = np.random.default_rng(19)
    ell = 0.1
    rc = 3 * ell
    n = 20000
    x = rng.uniform(-30.0, 30.0, size=(n, 3))
    dirs = np.concatenate([np.eye(3), -np.eye(3), np.ones((1, 3)) / np.sqrt(3), -np.ones((1, 3)) / np.sqrt(3)])
    d = dirs[rng.integers(0, len(dirs), size=n)] * rc * (1 - 2 ** -16)
    pts = [x.astype(np.float32), (x + d).astype(np.float32)]
    lab = [np.zeros(n, np.uint16)] * 2
    pb = oracle.Problem(pts, lab, "class", ell)
    pc = pb.with_search("cells")
    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    poses = np.stack([I, I])
    for mem in MEMBERSHIP.values():
        assert assert_same_sums(pb, pc, poses, [[0, 1], [1, 0]], mem, "pairs at the radius") >= 2 * n
    np.testing.assert_array_equal(oracle.pairs(pc, poses, 0, 1), oracle.pairs(pb, poses, 0, 1))
