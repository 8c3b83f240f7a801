"""Class-id frames in label-stacked voxel grids against the FP64 oracle.

With class ids (l(x) one-hot, so c_ij = [l_i == l_j]) the build stacks one
layer of each frame's z extent per id, the binning segments and sweep passes
follow the source frame's layers, and every walk visits only the layer of its
source's id.  The pair set and the sums must not change: voxel keys against
the oracle's label-stacked sort, pair lists and per-source pair counts bit
for bit, F, b and H within 1e-5 normwise, for the stacked layout, for frames
whose ids are too large to stack (one id 65535: the keys would not fit 32
bits), for sparse ids (many empty layers), for a target frame that lacks some
of the source's ids, and for a batch that mixes stacked and unstacked
problems.
"""
import sys

import numpy as np
import pytest

import oracle
import scenes
from helpers import REL_TOL, assert_blocks_close, inv_cell, label_stacked

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


def variant(name):
    """two_view (3,000 points per frame, 10 ids, r_c = 0.3 m in a 20 m cube) with its ids rewritten."""
    p = scenes.two_view(11, n_points=3000)
    lab = [f.copy() for f in p.feats]
    if name == "large_id":      # 67^3 cells x 65,536 layers do not fit 32-bit keys: not stacked
        lab[1][17] = 65535
    elif name == "sparse_ids":  # ids 0, 11, ..., 88: 89 layers, most of them empty (stacked with 1-r_c cells)
        lab = [(f * 11).astype(np.uint16) for f in lab]
    elif name == "missing_ids":  # frame 1 carries ids 0..4 only: sources of ids 5..9 have no layer there
        lab[1] = (lab[1] % 5).astype(np.uint16)
    p.feats = lab
    p.recipe += f" ids={name}"
    return p


VARIANTS = ["stacked", "large_id", "sparse_ids", "missing_ids"]



@pytest.mark.parametrize("name", VARIANTS)
def test_voxels_and_pairs(rk, name):
    p = variant(name)
    op = oracle.Problem.from_scene(p)
    poses = p.gt_poses
    for subdiv, pp in ((1, 16), (2, 8), (2, 16), (1, 1), (1, 32)):
        say(f"[labels] {name} subdiv {subdiv} pass {pp}")
        ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, cell_subdiv=subdiv, pass_points=pp)
        ctx.build_neighbors(p.points, p.feats, p.feat_kind)
        inv = inv_cell(p.ell, p.cutoff_factor, subdiv)
        vox = [ctx.export_voxels(f, len(p.points[f])) for f in range(p.K)]
        stacked = label_stacked(p.feats, [v[3] for v in vox])
        # the variants cover both outcomes: sparse ids stack with cells of one r_c only
        assert stacked == (name != "large_id" and not (name == "sparse_ids" and subdiv > 1))
        say(f"[labels] {name} subdiv {subdiv}: stacked {stacked}")
        for f in range(p.K):
            perm, keys, org, dims, layers = vox[f]
            assert layers == (int(p.feats[f].max()) + 1 if stacked else 0)
            operm, okeys, oorg, odims = oracle.voxels(p.points[f], inv, labels=p.feats[f] if stacked else None)
            np.testing.assert_array_equal(org, oorg)
            np.testing.assert_array_equal(dims, odims)
            np.testing.assert_array_equal(keys, okeys)
            np.testing.assert_array_equal(perm, operm)
        for (m, n) in ((0, 1), (1, 0)):
            ref = oracle.pairs(op, poses, m, n)
            assert len(ref) > 0
            np.testing.assert_array_equal(ctx.export_pairs(poses, m, n), ref)
            # per-source counts from the kernel that sums (tiled sweeps of 8, 16 and 32 points, per-point walks)
            got = ctx.export_source_counts(poses, m, n, len(p.points[m]))
            np.testing.assert_array_equal(got, np.bincount(ref[:, 0], minlength=len(p.points[m])))
        edges = [[0, 1], [1, 0]]
        H, b, F, npairs = ctx.accumulate_normal_eqs(poses, edges)
        oF, ob, oH, _, onp = oracle.normal_eqs(op, poses, edges, oracle.MEMBER_FP32_RULE)
        assert npairs == onp
        assert abs(F - oF) <= REL_TOL * abs(oF)
        assert_blocks_close(b, ob, 6, what=f"{name} b")
        assert_blocks_close(H, oH, 6, what=f"{name} H")
        lF, _, lnp = ctx.eval_loss(poses, edges)
        assert lnp == onp and abs(lF - oF) <= REL_TOL * abs(oF)
        ctx.close()


def test_batch_mixing_stacked_and_unstacked(rk):
    """Two class-id requests served together, one stacked and one not (an id of 65535): every sweep of the
    batch then tests the ids, and each request's poses, losses and pair counts equal those it gets alone
    (where the stacked one skips the test)."""
    reqs = [variant("stacked"), variant("large_id"), variant("missing_ids")]
    for p in reqs:
        p.n_iter = 3

    def submit(srv, p):
        return srv.submit(p.points, p.feats, p.init_poses, p.edges, p.ell, p.n_iter)

    with rk.Server(feat_kind="class", D=0, max_active=8, lanes=1, pass_points=16) as srv:
        alone = [srv.wait(submit(srv, p), timeout=120) for p in reqs]
        tickets = [submit(srv, p) for p in reqs]
        mix = [srv.wait(t, timeout=120) for t in tickets]
        st = srv.stats()
    say(f"[labels] server stats {st}")
    assert st["failed"] == 0 and st["max_active"] >= 2
    for p, a, m in zip(reqs, alone, mix):
        np.testing.assert_array_equal(a[0], m[0])
        np.testing.assert_array_equal(a[1][:-1], m[1][:-1])
        np.testing.assert_array_equal(a[2], m[2])
        op = oracle.Problem.from_scene(p)
        _, olpi = oracle.gn(op, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
        np.testing.assert_allclose(a[1], olpi, rtol=REL_TOL)
