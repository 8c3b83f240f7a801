"""Pins of the oracle's per-point top-k truncation (the Time-Analysis
paragraph of Sec. VI: each source point keeps only the pairs with the largest
kernel values).

The kept pairs are checked against routines that do not share the oracle's
ranking code: with class ids (every candidate has c = 1) the top-k pairs are
the k nearest same-label neighbours inside the truncation radius (scipy's
KD-tree); with coincident target points the ranking is by c alone (numpy
argsort of the feature dot products); with equal feature rows it is by
distance alone.  The pair count follows from the full pair list, a top_k
above every point's candidate count reproduces the untruncated sums, and the
truncated loss has the gradient -(sigma^2/ell^2) b by central differences
(the kept set is locally constant).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")


def ident():
    return np.concatenate([np.eye(3).reshape(9), np.zeros(3)])


def rand_pose(rng, ang=0.1, trans=0.1):
    R = Rotation.from_rotvec(rng.normal(size=3) * ang / np.sqrt(3)).as_matrix()
    return np.concatenate([R.reshape(9), rng.normal(size=3) * trans])


def right_perturb(p, xi):
    from scipy.linalg import expm
    W = np.zeros((4, 4))
    W[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
    W[:3, 3] = xi[:3]
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:]
    T = T @ expm(W)
    return np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])


def class_problem(seed, n=400, n_lab=3, ell=0.08, cutoff=3.0, top_k=0):
    rng = np.random.default_rng(seed)
    pts = [rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32) for _ in range(2)]
    labs = [rng.integers(0, n_lab, n).astype(np.uint16) for _ in range(2)]
    return pts, labs, oracle.Problem(pts, labs, "class", ell, cutoff, 1.0, top_k=top_k)


def as_set(pairs):
    return set(map(tuple, np.asarray(pairs).tolist()))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_class_topk_is_k_nearest_same_label_neighbours(k):
    pts, labs, P = class_problem(11, top_k=k)
    poses = np.stack([ident(), ident()])
    got = as_set(oracle.pairs(P, poses, 0, 1))
    rc = 3.0 * 0.08
    want = set()
    for lab in range(3):
        src = np.nonzero(labs[0] == lab)[0]
        tgt = np.nonzero(labs[1] == lab)[0]
        tree = cKDTree(pts[1][tgt].astype(np.float64))
        d, idx = tree.query(pts[0][src].astype(np.float64), k=k, distance_upper_bound=rc)
        d = d.reshape(len(src), k)
        idx = idx.reshape(len(src), k)
        for a, i in enumerate(src):
            for t in range(k):
                if np.isfinite(d[a, t]):
                    want.add((int(i), int(tgt[idx[a, t]])))
    assert len(want) > 0
    assert got == want


def test_topk_count_is_min_of_k_and_candidates():
    k = 4
    pts, labs, Pk = class_problem(12, top_k=k)
    _, _, P0 = class_problem(12)
    poses = np.stack([ident(), rand_pose(np.random.default_rng(5), 0.05, 0.02)])
    full = oracle.pairs(P0, poses, 0, 1)
    per_src = np.bincount(full[:, 0], minlength=len(pts[0]))
    expect = int(np.minimum(per_src, k).sum())
    assert len(oracle.pairs(Pk, poses, 0, 1)) == expect
    *_, n_pairs = oracle.normal_eqs(Pk, poses, [[0, 1]], oracle.MEMBER_FP32_RULE)
    assert n_pairs == expect
    assert as_set(oracle.pairs(Pk, poses, 0, 1)) <= as_set(full)


def test_topk_above_every_candidate_count_is_the_full_sum():
    pts, labs, P0 = class_problem(13, ell=0.04)
    poses = np.stack([ident(), rand_pose(np.random.default_rng(6), 0.05, 0.02)])
    full = oracle.pairs(P0, poses, 0, 1)
    kmax = int(np.bincount(full[:, 0]).max())
    assert kmax <= 8
    _, _, Pk = class_problem(13, ell=0.04, top_k=8)
    a = oracle.normal_eqs(P0, poses, [[0, 1]], oracle.MEMBER_FP32_RULE)
    b = oracle.normal_eqs(Pk, poses, [[0, 1]], oracle.MEMBER_FP32_RULE)
    assert a[4] == b[4]
    np.testing.assert_allclose(b[0], a[0], rtol=1e-13)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-12, atol=1e-12 * np.abs(a[1]).max())
    np.testing.assert_allclose(b[2], a[2], rtol=1e-12, atol=1e-12 * np.abs(a[2]).max())


def test_coincident_targets_rank_by_feature_product():
    """All target points at one position: every pair has the same distance,
    so the kept pairs are the k largest positive dot products."""
    rng = np.random.default_rng(14)
    D, n_src, n_tgt, k = 6, 20, 50, 5
    src = rng.uniform(-0.05, 0.05, (n_src, 3)).astype(np.float32)
    tgt = np.tile(np.float32([[0.01, -0.02, 0.015]]), (n_tgt, 1))
    fs = rng.normal(size=(n_src, D)).astype(np.float32)
    ft = rng.normal(size=(n_tgt, D)).astype(np.float32)
    P = oracle.Problem([src, tgt], [fs, ft], "dense", 0.1, 3.0, 1.0, top_k=k)
    got = as_set(oracle.pairs(P, np.stack([ident(), ident()]), 0, 1))
    c = fs.astype(np.float64) @ ft.astype(np.float64).T
    want = set()
    for i in range(n_src):
        order = np.argsort(-c[i], kind="stable")
        want |= {(i, int(j)) for j in order[:k] if c[i, j] > 0}
    assert got == want


def test_equal_features_rank_by_distance():
    """Equal positive feature rows: c is the same for every pair, so the kept
    pairs are the k nearest targets inside the radius."""
    rng = np.random.default_rng(15)
    n, k, ell = 300, 6, 0.1
    src = rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    tgt = rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    f = np.tile(np.float32([[0.5, 0.25, 0.125]]), (n, 1))
    P = oracle.Problem([src, tgt], [f, f], "dense", ell, 3.0, 1.0, top_k=k)
    got = as_set(oracle.pairs(P, np.stack([ident(), ident()]), 0, 1))
    d, idx = cKDTree(tgt.astype(np.float64)).query(src.astype(np.float64), k=k, distance_upper_bound=3.0 * ell)
    want = {(i, int(idx[i, t])) for i in range(n) for t in range(k) if np.isfinite(d[i, t])}
    assert got == want


def test_truncated_loss_gradient_matches_central_differences():
    """grad F = -(sigma^2/ell^2) b for the truncated objective, by central
    differences over every frame's tangent coordinates (FP64 membership; the
    step is small enough that no kept set changes)."""
    rng = np.random.default_rng(16)
    D, ell = 4, 0.3
    pts = [rng.uniform(0.0, 0.6, (n, 3)).astype(np.float32) for n in (40, 35, 30)]
    feats = [np.abs(rng.normal(size=(len(p), D))).astype(np.float32) for p in pts]
    P = oracle.Problem(pts, feats, "dense", ell, 20.0, 1.0, top_k=3)
    P_full = oracle.Problem(pts, feats, "dense", ell, 20.0, 1.0)
    poses = np.stack([rand_pose(rng) for _ in range(3)])
    edges = [[0, 1], [1, 2], [2, 0]]
    F, b, H, Fe, npairs = oracle.normal_eqs(P, poses, edges)
    assert npairs == 3 * (40 + 35 + 30)
    assert F < oracle.loss(P_full, poses, edges)
    h = 1e-6
    g = np.zeros(18)
    for m in range(3):
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = h
            pp, pm = poses.copy(), poses.copy()
            pp[m] = right_perturb(poses[m], xi)
            pm[m] = right_perturb(poses[m], -xi)
            g[6 * m + k] = (oracle.loss(P, pp, edges) - oracle.loss(P, pm, edges)) / (2 * h)
    expect = -(1.0 / ell ** 2) * b
    np.testing.assert_allclose(g, expect, rtol=2e-6, atol=2e-6 * np.abs(expect).max())
