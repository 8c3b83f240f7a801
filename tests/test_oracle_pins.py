"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
derived by hand for tiny inputs, finite differences, invariances of the
objective of Eq. (eq:inner_product_actual_ba), textbook routines (scipy expm,
numpy solve, weighted Kabsch) and brute force on tiny inputs.  A plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg
from scipy.spatial.transform import Rotation

import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")


def rand_pose(rng, ang=0.5, trans=1.0):
    R = Rotation.from_rotvec(rng.normal(size=3) * ang / np.sqrt(3)).as_matrix()
    return np.concatenate([R.reshape(9), rng.normal(size=3) * trans])


def ident():
    return np.concatenate([np.eye(3).reshape(9), np.zeros(3)])


def skew(v):
    return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])


def wedge(xi):
    W = np.zeros((4, 4))
    W[:3, :3] = skew(xi[3:])
    W[:3, 3] = xi[:3]
    return W


def to44(p):
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:]
    return T


def from44(T):
    return np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])


def right_perturb(p, xi):
    return from44(to44(p) @ scipy.linalg.expm(wedge(xi)))


def dense_problem(rng, sizes, D=5, ell=0.3, cutoff=20.0, spread=0.6):
    pts = [rng.normal(size=(n, 3)).astype(np.float32) * spread for n in sizes]
    feats = [rng.uniform(0.1, 1.0, size=(n, D)).astype(np.float32) for n in sizes]
    return oracle.Problem(pts, feats, "dense", ell, cutoff), pts, feats


# ----------------------------------------------------------------------------- closed forms

def test_two_points_identity_closed_form():
    """Two single points at identity poses: F = c exp(-r^2/2l^2) and the
    hand-derived blocks b_m = w[x-z; -x cross z], b_n = w[z-x; x cross z],
    H_mm = w[[I,-[x]],[[x],-[x]^2]], H_mn = -w[[I,-[z]],[[x],-[x][z]]]."""
    x = np.array([0.3, -0.2, 0.5], np.float32)
    z = np.array([0.35, -0.15, 0.47], np.float32)
    ell = 0.1
    P = oracle.Problem([x[None], z[None]], [np.array([3]), np.array([3])], "class", ell)
    poses = np.stack([ident(), ident()])
    F, b, H, Fe, n = oracle.normal_eqs(P, poses, [[0, 1]])
    xd, zd = x.astype(np.float64), z.astype(np.float64)
    r2 = np.sum((xd - zd) ** 2)
    w = np.exp(-r2 / (2 * ell * ell))
    assert n == 1
    assert F == pytest.approx(w, rel=1e-14)
    np.testing.assert_allclose(b[:6], w * np.r_[xd - zd, -np.cross(xd, zd)], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(b[6:], w * np.r_[zd - xd, np.cross(xd, zd)], rtol=1e-13, atol=1e-16)
    X, Zs = skew(xd), skew(zd)
    Hmm = w * np.block([[np.eye(3), -X], [X, -X @ X]])
    Hnn = w * np.block([[np.eye(3), -Zs], [Zs, -Zs @ Zs]])
    Hmn = -w * np.block([[np.eye(3), -Zs], [X, -X @ Zs]])
    np.testing.assert_allclose(H[:6, :6], Hmm, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(H[6:, 6:], Hnn, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(H[:6, 6:], Hmn, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(H[6:, :6], Hmn.T, rtol=1e-13, atol=1e-15)


def test_two_points_posed_closed_form():
    """Two single points at arbitrary poses: with v = R_m^T u and v' = R_n^T u,
    b_m = w[v; x cross v] and b_n = -w[v'; z cross v'] (right perturbation)."""
    rng = np.random.default_rng(1)
    x = np.array([0.2, 0.1, -0.3], np.float32)
    Tm, Tn = rand_pose(rng), ident()
    # place z so that T_n z is 4 cm away from T_m x
    pw = to44(Tm)[:3, :3] @ x + Tm[9:]
    z = (pw + np.array([0.02, -0.03, 0.02])).astype(np.float32)
    ell, sigma = 0.05, 1.7
    P = oracle.Problem([x[None], z[None]], [np.array([[0.5, 0.5]], np.float32), np.array([[0.75, 0.25]], np.float32)],
                       "dense", ell, 3.0, sigma)
    F, b, H, Fe, n = oracle.normal_eqs(P, np.stack([Tm, Tn]), [[0, 1]])
    Rm = Tm[:9].reshape(3, 3)
    u = Rm @ x + Tm[9:] - z.astype(np.float64)
    c = 0.5 * 0.75 + 0.5 * 0.25
    w = c * np.exp(-u @ u / (2 * ell ** 2))
    assert F == pytest.approx(sigma ** 2 * w, rel=1e-13)
    v = Rm.T @ u
    np.testing.assert_allclose(b[:6], w * np.r_[v, np.cross(x, v)], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(b[6:], -w * np.r_[u, np.cross(z, u)], rtol=1e-12, atol=1e-16)


def test_identical_clouds_identity_zero_gradient():
    """Identical clouds at identity poses: F >= sum_i c_ii (each point meets its
    own copy at r=0) and b = 0 by the antisymmetry of the pair terms."""
    rng = np.random.default_rng(2)
    x = (rng.normal(size=(300, 3)) * 0.3).astype(np.float32)
    lab = rng.integers(0, 4, size=300).astype(np.uint16)
    P = oracle.Problem([x, x.copy()], [lab, lab.copy()], "class", 0.1)
    F, b, H, Fe, n = oracle.normal_eqs(P, np.stack([ident(), ident()]), [[0, 1]])
    assert F >= 300 - 1e-9
    scale = np.abs(H).max()
    assert np.abs(b).max() <= 1e-13 * scale


# ----------------------------------------------------------------------------- derivatives

def test_gradient_matches_central_differences():
    """grad_eps F = -(sigma^2/l^2) b (Sec. V-A, Eq. (eq:inner_product_reformat)),
    checked by central finite differences of F over each frame's 6 tangent
    coordinates; the truncation radius is far (20 l) so F is smooth."""
    rng = np.random.default_rng(3)
    P, pts, feats = dense_problem(rng, [40, 35, 30], ell=0.4)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    edges = [[0, 1], [1, 2], [2, 0]]
    sigma = 1.0
    F, b, H, Fe, n = oracle.normal_eqs(P, poses, edges)
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
    expect = -(sigma ** 2 / P.c.ell ** 2) * b
    np.testing.assert_allclose(g, expect, rtol=2e-6, atol=2e-6 * np.abs(expect).max())


def test_gn_matrix_from_fd_jacobians():
    """H = sum w J^T J and b = sum w J^T u with J = du/d[eps_m, eps_n] rebuilt
    from finite differences of the residual u = T_m x - T_n z under right
    perturbations (textbook Gauss-Newton), on a brute-force pair list."""
    rng = np.random.default_rng(4)
    P, pts, feats = dense_problem(rng, [12, 10], D=3, ell=0.5)
    poses = np.stack([rand_pose(rng, 0.2, 0.2), rand_pose(rng, 0.2, 0.2)])
    F, b, H, Fe, n = oracle.normal_eqs(P, poses, [[0, 1]])
    ell = 0.5
    Hr = np.zeros((12, 12))
    br = np.zeros(12)
    h = 1e-6

    def resid(pm, pn, x, z):
        return to44(pm)[:3, :3] @ x + pm[9:] - (to44(pn)[:3, :3] @ z + pn[9:])

    for i in range(12):
        for j in range(10):
            x = pts[0][i].astype(np.float64)
            z = pts[1][j].astype(np.float64)
            u = resid(poses[0], poses[1], x, z)
            c = float(feats[0][i].astype(np.float64) @ feats[1][j].astype(np.float64))
            w = c * np.exp(-u @ u / (2 * ell ** 2))
            J = np.zeros((3, 12))
            for k in range(6):
                xi = np.zeros(6)
                xi[k] = h
                J[:, k] = (resid(right_perturb(poses[0], xi), poses[1], x, z)
                           - resid(right_perturb(poses[0], -xi), poses[1], x, z)) / (2 * h)
                J[:, 6 + k] = (resid(poses[0], right_perturb(poses[1], xi), x, z)
                               - resid(poses[0], right_perturb(poses[1], -xi), x, z)) / (2 * h)
            Hr += w * J.T @ J
            br += w * J.T @ u
    np.testing.assert_allclose(H, Hr, rtol=1e-7, atol=1e-7 * np.abs(Hr).max())
    np.testing.assert_allclose(b, br, rtol=1e-7, atol=1e-7 * np.abs(br).max())


# ----------------------------------------------------------------------------- invariances

def test_common_rigid_motion_invariance():
    """Moving every frame by the same rigid motion G leaves F, b and H (in the
    frames' right-perturbation coordinates) unchanged."""
    rng = np.random.default_rng(5)
    P, pts, feats = dense_problem(rng, [60, 50, 40], ell=0.3, cutoff=3.0)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    edges = [[0, 1], [0, 2], [1, 2]]
    G = to44(rand_pose(rng, 1.0, 3.0))
    moved = np.stack([from44(G @ to44(p)) for p in poses])
    F0, b0, H0, _, n0 = oracle.normal_eqs(P, poses, edges)
    F1, b1, H1, _, n1 = oracle.normal_eqs(P, moved, edges)
    assert n0 == n1
    assert F1 == pytest.approx(F0, rel=1e-12)
    np.testing.assert_allclose(b1, b0, atol=1e-11 * np.abs(b0).max())
    np.testing.assert_allclose(H1, H0, atol=1e-11 * np.abs(H0).max())


def test_edge_swap_symmetry():
    """The world residual is antisymmetric under swapping the frames of an
    edge, so (m, n) and (n, m) give the same F, b and H."""
    rng = np.random.default_rng(6)
    P, pts, feats = dense_problem(rng, [50, 45], ell=0.3, cutoff=3.0)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(2)])
    F0, b0, H0, _, _ = oracle.normal_eqs(P, poses, [[0, 1]])
    F1, b1, H1, _, _ = oracle.normal_eqs(P, poses, [[1, 0]])
    assert F1 == pytest.approx(F0, rel=1e-12)
    np.testing.assert_allclose(b1, b0, atol=1e-12 * np.abs(b0).max())
    np.testing.assert_allclose(H1, H0, atol=1e-12 * np.abs(H0).max())


def test_hessian_structure_and_gauge():
    """H is symmetric positive semidefinite for c >= 0; a common world
    translation (eps_m = [R_m^T tau; 0]) is in its null space; b is orthogonal
    to all six common-motion directions v_m = Ad(T_m^-1) eta."""
    rng = np.random.default_rng(7)
    P, pts, feats = dense_problem(rng, [60, 50, 40], ell=0.3, cutoff=3.0)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    F, b, H, _, n = oracle.normal_eqs(P, poses, [[0, 1], [0, 2], [1, 2]])
    assert n > 100
    np.testing.assert_allclose(H, H.T, atol=1e-13 * np.abs(H).max())
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= -1e-10 * ev.max()
    for k in range(3):
        tau = np.eye(3)[k]
        v = np.concatenate([np.r_[p[:9].reshape(3, 3).T @ tau, np.zeros(3)] for p in poses])
        assert np.linalg.norm(H @ v) <= 1e-10 * np.linalg.norm(H) * np.linalg.norm(v)
    for k in range(6):
        eta = np.eye(6)[k]
        vs = []
        for p in poses:
            R, t = p[:9].reshape(3, 3), p[9:]
            AdInv = np.block([[R.T, -R.T @ skew(t)], [np.zeros((3, 3)), R.T]])
            vs.append(AdInv @ eta)
        v = np.concatenate(vs)
        assert abs(b @ v) <= 1e-11 * np.abs(b).sum() * np.abs(v).max()


def test_noise_free_copy_has_zero_gradient():
    """Frame 2 is an exact rigid copy of frame 1; at the true poses both clouds
    coincide in the world and b vanishes (up to the FP32 storage of z)."""
    rng = np.random.default_rng(8)
    x = (rng.normal(size=(200, 3)) * 0.5).astype(np.float32)
    T2 = rand_pose(rng, 0.5, 0.5)
    R2, t2 = T2[:9].reshape(3, 3), T2[9:]
    z = ((x.astype(np.float64) - t2) @ R2).astype(np.float32)   # T2 z = x
    lab = rng.integers(0, 3, size=200).astype(np.uint16)
    P = oracle.Problem([x, z], [lab, lab.copy()], "class", 0.1)
    F, b, H, _, n = oracle.normal_eqs(P, np.stack([ident(), T2]), [[0, 1]])
    assert np.abs(b).max() <= 1e-6 * np.abs(np.diag(H)).max() * 0.3


def test_duplicate_edges_and_feature_scaling_leave_step_unchanged():
    """Listing an edge twice doubles F, b, H; scaling all features by s scales
    w by s^2.  With relative damping the Gauss-Newton step is unchanged."""
    rng = np.random.default_rng(9)
    P, pts, feats = dense_problem(rng, [80, 70], ell=0.3, cutoff=3.0)
    poses = np.stack([ident(), rand_pose(rng, 0.05, 0.05)])
    p1, l1 = oracle.gn(P, poses, [[0, 1]], 1)
    p2, l2 = oracle.gn(P, poses, [[0, 1], [0, 1]], 1)
    assert l2[0] == pytest.approx(2 * l1[0], rel=1e-13)
    np.testing.assert_allclose(p2, p1, atol=1e-13)
    P3 = oracle.Problem(pts, [f * 3.0 for f in feats], "dense", 0.3, 3.0)
    p3, l3 = oracle.gn(P3, poses, [[0, 1]], 1)
    assert l3[0] == pytest.approx(9 * l1[0], rel=1e-6)
    np.testing.assert_allclose(p3, p1, atol=1e-9)


# ----------------------------------------------------------------------------- solver pieces

def test_se3_exp_matches_matrix_exponential():
    rng = np.random.default_rng(10)
    for scale in (1e-9, 1e-5, 1e-3, 0.1, 1.0, 2.5):
        xi = rng.normal(size=6) * scale
        T = oracle.se3_exp(xi)
        ref = scipy.linalg.expm(wedge(xi))
        np.testing.assert_allclose(to44(T), ref, atol=1e-14)


def test_cholesky_solve_matches_numpy():
    rng = np.random.default_rng(11)
    for n in (1, 6, 42, 120):
        A = rng.normal(size=(n, n))
        A = A @ A.T + n * np.eye(n)
        b = rng.normal(size=n)
        np.testing.assert_allclose(oracle.cholesky_solve(A, b), np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky_solve(np.array([[1.0, 2.0], [2.0, 1.0]]), np.ones(2))


def weighted_kabsch(x, z, w):
    """Textbook weighted Procrustes: T minimising sum w |T z - x|^2."""
    cx = (w[:, None] * x).sum(0) / w.sum()
    cz = (w[:, None] * z).sum(0) / w.sum()
    Hc = ((z - cz) * w[:, None]).T @ (x - cx)
    U, S, Vt = np.linalg.svd(Hc)
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, cx - R @ cz


def test_gn_fixed_point_is_weighted_kabsch():
    """Points spaced far beyond the cutoff only see their own copy; the IRLS
    fixed point of Eq. (eq:irls_final) is then the weighted Procrustes
    solution with the final weights w_i = exp(-|T z_i - x_i|^2 / 2l^2)."""
    rng = np.random.default_rng(12)
    g = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(3), indexing="ij"), -1).reshape(-1, 3)
    x = (g * 2.0 + rng.normal(size=g.shape) * 0.05).astype(np.float32)
    T = rand_pose(rng, 0.05, 0.05)
    R, t = T[:9].reshape(3, 3), T[9:]
    z = (((x.astype(np.float64) - t) @ R) + rng.normal(size=x.shape) * 0.02).astype(np.float32)
    lab = np.zeros(len(x), np.uint16)
    ell = 0.1
    P = oracle.Problem([x, z], [lab, lab], "class", ell)
    poses, lpi = oracle.gn(P, np.stack([ident(), ident()]), [[0, 1]], 60, damping_rel=0.0)
    assert np.all(np.diff(lpi[-5:]) >= -1e-12)
    T2 = poses[1]
    R2, t2 = T2[:9].reshape(3, 3), T2[9:]
    xd, zd = x.astype(np.float64), z.astype(np.float64)
    r = zd @ R2.T + t2 - xd
    w = np.exp(-np.sum(r * r, 1) / (2 * ell ** 2))
    Rk, tk = weighted_kabsch(xd, zd, w)
    np.testing.assert_allclose(R2, Rk, atol=1e-9)
    np.testing.assert_allclose(t2, tk, atol=1e-9)


# ----------------------------------------------------------------------------- membership rule

def test_fp32_rule_brackets_the_fp64_definition():
    """The FP32 membership rule agrees with r^2 <= r_c^2 except within a
    relative band of 1e-5 around the cutoff (brute force, all pairs)."""
    rng = np.random.default_rng(13)
    pts = [(rng.normal(size=(400, 3)) * 0.4).astype(np.float32) for _ in range(2)]
    lab = [np.zeros(400, np.uint16)] * 2
    ell = 0.1
    P = oracle.Problem(pts, lab, "class", ell)
    poses = np.stack([rand_pose(rng, 0.3, 0.2), rand_pose(rng, 0.3, 0.2)])
    pr = oracle.pairs(P, poses, 0, 1)
    Wx = pts[0].astype(np.float64) @ poses[0][:9].reshape(3, 3).T + poses[0][9:]
    Wz = pts[1].astype(np.float64) @ poses[1][:9].reshape(3, 3).T + poses[1][9:]
    r2 = np.sum((Wx[:, None, :] - Wz[None, :, :]) ** 2, -1)
    rc2 = (3 * ell) ** 2
    inside = np.zeros_like(r2, dtype=bool)
    inside[pr[:, 0], pr[:, 1]] = True
    assert np.all(inside[r2 < rc2 * (1 - 1e-5)])
    assert not np.any(inside[r2 > rc2 * (1 + 1e-5)])
    assert len(pr) > 200
    # the listing is in (i, j) order without repeats
    key = pr[:, 0].astype(np.int64) * 1000 + pr[:, 1]
    assert np.all(np.diff(key) > 0)
    # and the rule is the one the loss uses in its FP32-rule mode
    _, _, _, _, n = oracle.normal_eqs(P, poses, [[0, 1]], oracle.MEMBER_FP32_RULE)
    assert n == len(pr)


def test_pairs_respect_labels():
    rng = np.random.default_rng(14)
    pts = [(rng.normal(size=(300, 3)) * 0.3).astype(np.float32) for _ in range(2)]
    lab = [rng.integers(0, 3, size=300).astype(np.uint16) for _ in range(2)]
    P = oracle.Problem(pts, lab, "class", 0.1)
    poses = np.stack([ident(), ident()])
    pr = oracle.pairs(P, poses, 0, 1)
    assert len(pr) > 0
    assert np.all(lab[0][pr[:, 0]] == lab[1][pr[:, 1]])
    Pall = oracle.Problem(pts, [np.zeros(300, np.uint16)] * 2, "class", 0.1)
    pa = oracle.pairs(Pall, poses, 0, 1)
    same = lab[0][pa[:, 0]] == lab[1][pa[:, 1]]
    np.testing.assert_array_equal(pa[same], pr)


def test_voxel_sort_properties():
    """Stable sort by cell key: a permutation, keys non-decreasing, ties by
    index, and each key decodes to the point's own cell floor(x * inv)."""
    rng = np.random.default_rng(15)
    x = (rng.normal(size=(5000, 3)) * 2.0).astype(np.float32)
    inv = 1.0 / (0.3 / 2)
    perm, keys, origin, dims = oracle.voxels(x, inv, margin=1)
    assert sorted(perm.tolist()) == list(range(5000))
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    same = np.diff(keys.astype(np.int64)) == 0
    assert np.all(np.diff(perm)[same] > 0)
    k = np.floor(x[perm].astype(np.float64) * inv).astype(np.int64)
    kx = keys % dims[0]
    ky = (keys // dims[0]) % dims[1]
    kz = keys // (dims[0] * dims[1])
    np.testing.assert_array_equal(np.stack([kx, ky, kz], 1) + origin, k)
    assert np.all(k.min(0) - origin == 1) and np.all(dims - (k.max(0) - origin) - 1 == 1)


def test_label_stacked_voxel_sort_properties():
    """With class ids the sort groups the points by id first: each key
    decodes to (id, cell) with z index id * NZ + kz, the points of one id are
    contiguous and in the unlabelled sort's order among themselves, and
    without labels (or with all ids 0) the keys are the unlabelled ones."""
    rng = np.random.default_rng(17)
    x = (rng.normal(size=(4000, 3)) * 1.5).astype(np.float32)
    lab = rng.integers(0, 7, size=4000).astype(np.uint16)
    inv = 1.0 / 0.25
    perm0, keys0, origin0, dims0 = oracle.voxels(x, inv)
    perm, keys, origin, dims = oracle.voxels(x, inv, labels=lab)
    np.testing.assert_array_equal(origin, origin0)
    np.testing.assert_array_equal(dims, dims0)
    assert sorted(perm.tolist()) == list(range(4000))
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    k = np.floor(x[perm].astype(np.float64) * inv).astype(np.int64) - origin
    kx = keys % dims[0]
    ky = (keys // dims[0]) % dims[1]
    kzl = keys.astype(np.int64) // (dims[0] * dims[1])
    np.testing.assert_array_equal(kx, k[:, 0])
    np.testing.assert_array_equal(ky, k[:, 1])
    np.testing.assert_array_equal(kzl % dims[2], k[:, 2])
    np.testing.assert_array_equal(kzl // dims[2], lab[perm])
    assert np.all(np.diff(lab[perm].astype(np.int64)) >= 0)
    rank0 = np.empty(4000, np.int64)
    rank0[perm0] = np.arange(4000)
    for L in range(7):
        sub = perm[lab[perm] == L]
        assert np.all(np.diff(rank0[sub]) > 0)
    perm_z, keys_z, _, _ = oracle.voxels(x, inv, labels=np.zeros(4000, np.uint16))
    np.testing.assert_array_equal(perm_z, perm0)
    np.testing.assert_array_equal(keys_z, keys0)


# ----------------------------------------------------------------------------- one Gauss-Newton step

def test_gn_step_is_the_damped_solve_with_right_update():
    """One oracle step (Sec. V-A) equals, rebuilt from its own normal
    equations with textbook routines: drop the fixed frame's rows and columns,
    add mu I with mu = damping_rel tr(H_red) / dim(H_red), solve with numpy,
    and move every other frame by T <- T expm(delta^) (right perturbation,
    scipy expm).  Frame 1 is the fixed one and the damping is large enough to
    matter; a left update, an undamped solve or the wrong fixed frame each
    miss the result by far more than the tolerance."""
    rng = np.random.default_rng(16)
    P, pts, feats = dense_problem(rng, [60, 50, 40], ell=0.3, cutoff=3.0)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    edges = [[0, 1], [0, 2], [1, 2]]
    fixed, damping = 1, 1e-2
    F, b, H, _, _ = oracle.normal_eqs(P, poses, edges)
    free = [0, 2]
    idx = np.concatenate([np.arange(6 * f, 6 * f + 6) for f in free])
    Hr, br = H[np.ix_(idx, idx)], b[idx]
    mu = damping * np.trace(Hr) / len(idx)

    def step(delta, right=True):
        out = poses.copy()
        for k, f in enumerate(free):
            E = scipy.linalg.expm(wedge(delta[6 * k:6 * k + 6]))
            out[f] = from44(to44(poses[f]) @ E if right else E @ to44(poses[f]))
        return out

    delta = np.linalg.solve(Hr + mu * np.eye(len(idx)), -br)
    expect = step(delta)
    got, lpi = oracle.gn(P, poses, edges, 1, fixed_frame=fixed, damping_rel=damping)
    assert lpi[0] == pytest.approx(F, rel=1e-14)
    assert lpi[1] == pytest.approx(oracle.loss(P, got, edges), rel=1e-14)
    np.testing.assert_array_equal(got[fixed], poses[fixed])
    np.testing.assert_allclose(got, expect, atol=1e-12)
    assert np.abs(delta).max() > 1e-3  # a real step
    # what a plausible mistake would give instead
    wrong = {
        "left update": step(delta, right=False),
        "undamped": step(np.linalg.solve(Hr, -br)),
    }
    for what, alt in wrong.items():
        assert np.abs(alt - got).max() > 1e-6, what
    other, _ = oracle.gn(P, poses, edges, 1, fixed_frame=0, damping_rel=damping)
    assert np.abs(other - got).max() > 1e-3


def test_gn_step_frame_without_pairs_stays():
    """A frame with no pair inside the radius gets delta = 0 (only the damping
    sees its rows); the other frames still move."""
    rng = np.random.default_rng(20)
    P, pts, feats = dense_problem(rng, [50, 40, 30], ell=0.3, cutoff=3.0)
    far = pts[2] + np.float32(100.0)
    P = oracle.Problem([pts[0], pts[1], far], feats, "dense", 0.3, 3.0)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    got, _ = oracle.gn(P, poses, [[0, 1], [0, 2]], 1, fixed_frame=0, damping_rel=1e-6)
    np.testing.assert_array_equal(got[2], poses[2])
    assert np.abs(got[1] - poses[1]).max() > 1e-4


def test_sigma_scales_the_loss_only():
    """F carries sigma^2 (Eq. (eq:kernel)); b and H are defined with the
    weights w = c k of Eq. (eq:irls_weight) and do not; the step is the same."""
    rng = np.random.default_rng(21)
    P1, pts, feats = dense_problem(rng, [60, 50, 40], ell=0.3, cutoff=3.0)
    P2 = oracle.Problem(pts, feats, "dense", 0.3, 3.0, 1.7)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(3)])
    edges = [[0, 1], [0, 2], [1, 2]]
    F1, b1, H1, Fe1, n1 = oracle.normal_eqs(P1, poses, edges)
    F2, b2, H2, Fe2, n2 = oracle.normal_eqs(P2, poses, edges)
    assert n1 == n2 > 0
    assert F2 == pytest.approx(1.7 ** 2 * F1, rel=1e-14)
    np.testing.assert_allclose(Fe2, 1.7 ** 2 * Fe1, rtol=1e-14)
    np.testing.assert_array_equal(b2, b1)
    np.testing.assert_array_equal(H2, H1)
    g1, _ = oracle.gn(P1, poses, edges, 2)
    g2, l2 = oracle.gn(P2, poses, edges, 2)
    np.testing.assert_array_equal(g2, g1)


def test_gradient_matches_central_differences_with_sigma():
    """grad_eps F = -(sigma^2/l^2) b with sigma = 1.7: central differences of
    the loss against b of the normal equations."""
    rng = np.random.default_rng(22)
    pts = [rng.normal(size=(n, 3)).astype(np.float32) * 0.6 for n in (30, 25)]
    feats = [rng.uniform(0.1, 1.0, size=(n, 4)).astype(np.float32) for n in (30, 25)]
    sigma, ell = 1.7, 0.4
    P = oracle.Problem(pts, feats, "dense", ell, 20.0, sigma)
    poses = np.stack([rand_pose(rng, 0.1, 0.1) for _ in range(2)])
    F, b, H, _, _ = oracle.normal_eqs(P, poses, [[0, 1]])
    h = 1e-6
    g = np.zeros(12)
    for m in range(2):
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = h
            pp, pm = poses.copy(), poses.copy()
            pp[m] = right_perturb(poses[m], xi)
            pm[m] = right_perturb(poses[m], -xi)
            g[6 * m + k] = (oracle.loss(P, pp, [[0, 1]]) - oracle.loss(P, pm, [[0, 1]])) / (2 * h)
    expect = -(sigma ** 2 / ell ** 2) * b
    np.testing.assert_allclose(g, expect, rtol=2e-6, atol=2e-6 * np.abs(expect).max())
