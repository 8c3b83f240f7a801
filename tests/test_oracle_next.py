"""Pins of the oracle's global rotation initialisation (Sec. IV-A)."""
import numpy as np
import pytest

import oracle
from oracle import global_init as gi

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_icosahedral_group_structure():
    R = gi.icosahedral_rotations()
    assert R.shape == (60, 3, 3)
    for r in R:
        np.testing.assert_allclose(r @ r.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(r) - 1.0) < 1e-12
    flat = R.reshape(60, 9)
    d = np.abs(flat[:, None, :] - flat[None, :, :]).max(axis=2)
    assert np.all(d[~np.eye(60, dtype=bool)] > 1e-6)            # 60 distinct elements
    for a in R[::7]:                                            # closed under composition
        for b in R[::5]:
            assert np.abs(flat - (a @ b).reshape(9)).max(axis=1).min() < 1e-9
    # rotation angles (in [0, pi]) against the element classes the paper lists (tests/golden)
    ang = np.arccos(np.clip((np.trace(R, axis1=1, axis2=2) - 1) / 2, -1, 1)) / np.pi
    want, total = golden_icosahedral_classes()
    assert total == 60 == sum(want.values())
    got = {a: int(np.sum(np.abs(ang - a) < 1e-9)) for a in want}
    assert got == want


def golden_icosahedral_classes():
    """{rotation angle / pi: number of group elements} and the stated total."""
    from fractions import Fraction
    import os
    want, total = {}, None
    path = os.path.join(os.path.dirname(__file__), "golden", "icosahedral_group.txt")
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "total":
            total = int(f[1])
        if f[0] != "class":
            continue
        axes = int(f[2].split("=")[1])
        for t in f[3].split("=")[1].split(","):
            a = Fraction(t)
            a = float(min(a, 2 - a))          # a turn by a pi is a rotation by min(a, 2 - a) pi
            want[a] = want.get(a, 0) + axes
    return want, total


def test_rotation_search_recovers_a_group_rotation():
    """Frame 1 is frame 0 turned about its centroid by a group element; at
    identity poses the search must pick the inverse turn, whose candidate
    coincides with frame 0 (the largest possible F, the identical-cloud value)."""
    rng = np.random.default_rng(3)
    x = (rng.normal(size=(300, 3)) * [1.0, 0.6, 0.3]).astype(np.float64)
    x[:, 0] += 0.4 * x[:, 1] ** 2                       # no symmetry of the cloud itself
    R = gi.icosahedral_rotations()
    k_true = 37
    c = x.mean(axis=0)
    z = ((x - c) @ R[k_true].T + c).astype(np.float32)
    pts = [x.astype(np.float32), z]
    feats = [np.zeros(len(x), np.uint16), np.zeros(len(x), np.uint16)]
    prob = oracle.Problem(pts, feats, "class", 0.15)
    ident = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    poses = np.stack([ident, ident])
    scores, best, Rc = gi.rotation_search(lambda P, e: oracle.normal_eqs(prob, P, e, oracle.MEMBER_FP32_RULE)[0],
                                          z, poses, 0, 1)
    np.testing.assert_allclose(Rc[best] @ R[k_true], np.eye(3), atol=1e-9)
    same = oracle.Problem([pts[0], pts[0]], feats, "class", 0.15)
    F_same = oracle.normal_eqs(same, poses, [[0, 1]], oracle.MEMBER_FP32_RULE)[0]
    assert abs(scores[best] - F_same) <= 1e-5 * F_same            # the candidate re-aligns the copy
    assert np.partition(scores, -2)[-2] < 0.9 * scores[best]       # and is clearly the largest


# ---------------------------------------------------------------- lengthscale (Sec. V-C)

from oracle import lengthscale as ls  # noqa: E402


def test_edge_sum_W_two_points():
    """W of one pair is w |u|^2 (closed form)."""
    x = np.array([[0.1, -0.2, 0.05]], np.float32)
    z = np.array([[0.15, -0.1, 0.0]], np.float32)
    feats = [np.array([[0.6, 0.8]], np.float32), np.array([[1.0, 0.5]], np.float32)]
    prob = oracle.Problem([x, z], feats, "dense", 0.1, 3.0, sigma=1.7)
    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    F, W = oracle.edge_sums(prob, np.stack([I, I]), [[0, 1]])
    r2 = float(np.sum((x.astype(np.float64) - z) ** 2))
    c = float(np.dot(feats[0][0].astype(np.float64), feats[1][0].astype(np.float64)))
    w = c * np.exp(-r2 / (2 * 0.1 ** 2))
    assert abs(W[0] - w * r2) <= 1e-14 * w * r2 and abs(F[0] - 1.7 ** 2 * w) <= 1e-14 * F[0]


def test_distance_derivative_matches_finite_differences():
    """d d_H / d ell = sigma^2 sum(W) / ell^3 against a central difference of
    d_H (truncation at 12 ell, where the moving boundary carries < e^-72)."""
    import scenes
    p = scenes.odometry(7, n_frames=3, n_points=700)

    def make(ell):
        return oracle.Problem(p.points, p.feats, p.feat_kind, ell, 12.0, sigma=1.3)

    for ell in (0.08, 0.2):
        d, g = ls.distance_and_derivative(make, ell, p.init_poses, p.edges, oracle.MEMBER_FP64)
        h = ell * 1e-4
        dp, _ = ls.distance_and_derivative(make, ell + h, p.init_poses, p.edges, oracle.MEMBER_FP64)
        dm, _ = ls.distance_and_derivative(make, ell - h, p.init_poses, p.edges, oracle.MEMBER_FP64)
        fd = (dp - dm) / (2 * h)
        assert abs(fd - g) <= 1e-6 * abs(g), (ell, fd, g)


def test_distance_vanishes_for_identical_frames():
    x = (np.random.default_rng(2).normal(size=(400, 3)) * 0.3).astype(np.float32)
    ids = np.random.default_rng(3).integers(0, 4, size=400).astype(np.uint16)

    def make(ell):
        return oracle.Problem([x, x], [ids, ids], "class", ell)

    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    d, g = ls.distance_and_derivative(make, 0.1, np.stack([I, I]), [[0, 1]], oracle.MEMBER_FP64)
    assert abs(d) <= 1e-9 * make(0.1).K * 400 and abs(g) <= 1e-6


def test_lengthscale_loop_refines_and_stops():
    """From a coarse start the loop ends at the finest allowed lengthscale with
    the objective no longer increasing, and the poses approach the ground truth."""
    import scenes
    p = scenes.two_view(1, n_points=800)

    def make(ell):
        return oracle.Problem(p.points, p.feats, p.feat_kind, ell, 3.0)

    poses, trace = ls.gn_lengthscale(make, p.init_poses, p.edges, ell_init=0.4, ell_min=0.1, ell_max=0.8,
                                     inner_iter=4, max_outer=25)
    assert trace[-1, 0] == 0.1 and trace[:, 0].max() <= 0.8
    assert trace[-1, 2] - trace[-1, 1] <= 1e-6 * abs(trace[-1, 1])
    R = poses[1][:9].reshape(3, 3) @ p.gt_poses[1][:9].reshape(3, 3).T
    assert np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))) < 0.5


# ---------------------------------------------------------------- tracking and keyframe alignment

from oracle import tracking as tk  # noqa: E402


def test_tracking_ascends_and_recovers_a_small_motion():
    import scenes
    p = scenes.two_view(2, n_points=600)
    prob = oracle.Problem.from_scene(p)
    F0 = oracle.normal_eqs(prob, p.init_poses, p.edges)[0]
    poses, it, F = tk.track(prob, p.init_poses, 0, 1, 60, p.ell, 1e-4 * p.ell)
    assert it > 0 and F > F0
    R = poses[1][:9].reshape(3, 3) @ p.gt_poses[1][:9].reshape(3, 3).T
    assert np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))) < 1.0
    assert np.linalg.norm(poses[1][9:] - p.gt_poses[1][9:]) < 0.03


def test_cosine_alignment():
    x = (np.random.default_rng(4).normal(size=(300, 3)) * 0.4).astype(np.float32)
    ids = np.random.default_rng(5).integers(0, 3, size=300).astype(np.uint16)
    prob = oracle.Problem([x, x], [ids, ids], "class", 0.1)
    I = np.concatenate([np.eye(3).reshape(9), np.zeros(3)])
    assert abs(tk.cosine(prob, np.stack([I, I]), 0, 1) - 1.0) < 1e-14
    far = I.copy()
    far[9] = 100.0
    assert tk.cosine(prob, np.stack([I, far]), 0, 1) == 0.0
    near = I.copy()
    near[9] = 0.05
    assert 0.0 < tk.cosine(prob, np.stack([I, near]), 0, 1) < 1.0
