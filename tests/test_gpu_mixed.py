"""Dense features stored in bfloat16 / fp8 e4m3 (inner products on the matrix
cores, FP32 accumulation, Kahan-compensated FP32 sums of the normal-equation
terms) against the FP64 oracle.

Parity: the oracle is given the features rounded to the storage format (the
rounding is the documented input conversion), and the GPU must then match it
to the FP32 bar (1e-5 normwise; poses 1e-4 rad / 1e-4 m).  The error caused by
the rounding itself is measured against the oracle on the unrounded features
and printed per result (F, b, H, poses), with a loose bound from the formats'
precision."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from helpers import (REL_TOL, ROT_TOL, TRANS_TOL, bf16_round, e4m3_round, ident, normwise_rel,
                     pose_errors)

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]

ROUND = {"bf16": bf16_round, "fp8": e4m3_round}
# bound on the rounding error of F, b, H relative to the unrounded oracle (8 and 4 significant bits)
FORMAT_BOUND = {"bf16": 2e-2, "fp8": 1.5e-1}
# The fp8 matrix-core product does not round its 32-term sums like an FP32 chain: on random e4m3
# operands a 16x16x32 result deviates from the exact sum by up to ~2e-4 of sum |a_k b_k|, and few
# results equal the correctly rounded sum (test_matrix_core_inner_product_deviation measures it through
# the library and asserts this bar).  F, b and H are sums of w * c with c >= 0 after clamping, so their
# relative error is bounded by the same figure wherever sum |a_k b_k| is of the size of c (unit-vector
# features of one class); the bar for the fp8 matrix-core path is that bound.  The per-point walks
# (pass size 1) form c on the vector ALU: FP32 bar.
FP8_MFMA_TOL = 2.5e-4


def tolerance(kind, pass_points):
    return FP8_MFMA_TOL if (kind == "fp8" and pass_points != 1) else REL_TOL


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


SCENES = {
    "dense64_small": lambda: scenes.dense64(5, n_frames=3, n_points=3000, n_iter=3),
    "odometry_small": lambda: scenes.odometry(1, n_frames=4, n_points=3000, n_iter=3),
}


@pytest.fixture(scope="module", params=list(SCENES))
def scene(request):
    say(f"[scene] {request.param}")
    return request.param, SCENES[request.param]()


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("pass_points", [16, 1])
@pytest.mark.parametrize("hessian_fp32", [False, True])
def test_low_precision_normal_equations(rk, scene, kind, pass_points, hessian_fp32):
    name, p = scene
    rounded = [ROUND[kind](f) for f in p.feats]
    oq = oracle.Problem(p.points, rounded, "dense", p.ell, p.cutoff_factor)
    oF, ob, oH, _, on = oracle.normal_eqs(oq, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, pass_points=pass_points, hessian_fp32=hessian_fp32)
    ctx.build_neighbors(p.points, p.feats, kind)
    H, b, F, n = ctx.accumulate_normal_eqs(p.init_poses, p.edges)
    eF, eb, eH = abs(F - oF) / abs(oF), normwise_rel(b, ob), normwise_rel(H, oH)
    say(f"[{kind}/{pass_points}/{'fp32k' if hessian_fp32 else 'fp64'}] {name} vs oracle on rounded features: F {eF:.2e} b {eb:.2e} H {eH:.2e} "
        f"pairs {n}/{on}")
    assert abs(n - on) <= max(2, 1e-5 * on)  # c exactly 0 after clamping may differ in the last bit
    tol = tolerance(kind, pass_points)
    assert eF <= tol and eb <= tol and eH <= tol
    op = oracle.Problem.from_scene(p)
    rF, rb, rH, _, _ = oracle.normal_eqs(op, p.init_poses, p.edges, oracle.MEMBER_FP32_RULE)
    qF, qb, qH = abs(F - rF) / abs(rF), normwise_rel(b, rb), normwise_rel(H, rH)
    say(f"[{kind}/{pass_points}] {name} vs oracle on float32 features: F {qF:.2e} b {qb:.2e} H {qH:.2e}")
    assert max(qF, qb, qH) <= FORMAT_BOUND[kind]


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_low_precision_gauss_newton(rk, scene, kind):
    """Poses after Gauss-Newton steps with the library's default sweep choice."""
    name, p = scene
    rounded = [ROUND[kind](f) for f in p.feats]
    oq = oracle.Problem(p.points, rounded, "dense", p.ell, p.cutoff_factor)
    n_iter = 3
    oposes, olpi = oracle.gn(oq, p.init_poses, p.edges, n_iter, membership=oracle.MEMBER_FP32_RULE)
    ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor)
    ctx.build_neighbors(p.points, p.feats, kind)
    poses, lpi, ppi = ctx.gn_step(p.init_poses, p.edges, n_iter)
    rot, tr = pose_errors(poses, oposes)
    fposes, flpi = oracle.gn(oracle.Problem.from_scene(p), p.init_poses, p.edges, n_iter,
                             membership=oracle.MEMBER_FP32_RULE)
    frot, ftr = pose_errors(poses, fposes)
    say(f"[{kind}] {name} poses vs oracle on rounded features: rot {rot.max():.2e} trans {tr.max():.2e}; "
        f"vs float32 features: rot {frot.max():.2e} trans {ftr.max():.2e}")
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
    np.testing.assert_allclose(lpi, olpi, rtol=tolerance(kind, ctx.config()[1]))


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("pass_points", [16, 1])
def test_feature_rounding_is_exact(rk, kind, pass_points):
    """Each frame is one point at the origin with a one-dimensional feature;
    edge (k, 0) has F = c = round(v_k) * round(1) exactly (distance 0, kernel
    value 1), so the per-edge losses expose the stored values: ties, the
    subnormal range, saturation and signs."""
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 255.5, 257.0, 259.0, 0.3, 17.0, 19.0, 460.0, 1e4,
                     2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 0.015, -0.3, -19.0, 3.14159, 1e-3, 6.5e-5],
                    dtype=np.float32)
    pts = [np.zeros((1, 3), np.float32) for _ in range(len(vals) + 1)]
    feats = [np.ones((1, 1), np.float32)] + [np.array([[v]], np.float32) for v in vals]
    ctx = rk.Context(ell=0.1, clamp_negative_c=False, pass_points=pass_points)
    ctx.build_neighbors(pts, feats, kind)
    poses = np.stack([ident()] * len(pts))
    edges = [[k + 1, 0] for k in range(len(vals))]
    F, Fe, n = ctx.eval_loss(poses, edges)
    want = ROUND[kind](vals).astype(np.float64)
    np.testing.assert_array_equal(Fe, want)


@pytest.mark.parametrize("kind,bound", [("fp8", FP8_MFMA_TOL), ("bf16", 2e-6)])
def test_matrix_core_inner_product_deviation(rk, kind, bound):
    """The inner products of the tiled sweep as the matrix cores compute them, one pair at a time:
    frames 2k and 2k+1 hold one point each at the same place, so edge (2k, 2k+1) has exactly one pair
    with d = 0 and w = c exp(0) = c, and its loss is the FP32 matrix-core inner product of the two
    stored rows (negative values not clamped).  Against the exact sum of the products of the rounded
    operands (FP64, exact for these formats), the deviation relative to sum |a_k b_k| stays within the
    bound the fp8 parity bar uses (bf16: within FP32 accumulation of exact products)."""
    rng = np.random.default_rng(31)
    n_pairs, D = 128, 64
    worst, exact_count, total = 0.0, 0, 0
    for batch in range(4):
        # operands like the dense64 features (unit vectors around class means) and plain uniform ones
        if batch % 2 == 0:
            f = rng.normal(size=(2 * n_pairs, D))
            f /= np.linalg.norm(f, axis=1, keepdims=True)
        else:
            f = rng.uniform(-1.0, 1.0, size=(2 * n_pairs, D))
        f = ROUND[kind](f.astype(np.float32))
        pts = [np.zeros((1, 3), np.float32) for _ in range(2 * n_pairs)]
        feats = [f[k:k + 1] for k in range(2 * n_pairs)]
        edges = np.array([(2 * k, 2 * k + 1) for k in range(n_pairs)], dtype=np.int32)
        poses = np.stack([ident()] * (2 * n_pairs))
        ctx = rk.Context(ell=0.1, clamp_negative_c=False, cell_subdiv=1, pass_points=16)
        ctx.build_neighbors(pts, feats, kind)
        F, Fe, npairs = ctx.eval_loss(poses, edges)
        ctx.close()
        a, b = f[0::2].astype(np.float64), f[1::2].astype(np.float64)
        exact = (a * b).sum(1)
        scale = np.abs(a * b).sum(1)
        dev = np.abs(Fe - exact) / scale
        nz = exact != 0
        assert npairs == np.count_nonzero(Fe)  # pairs with c != 0
        worst = max(worst, float(dev.max()))
        exact_count += int(np.count_nonzero(Fe[nz] == exact[nz].astype(np.float32)))
        total += int(nz.sum())
    say(f"[mfma] {kind}: largest deviation {worst:.3g} of sum |a_k b_k| over {4 * n_pairs} inner products; "
        f"{exact_count} of {total} equal the correctly rounded sum")
    assert worst <= bound
