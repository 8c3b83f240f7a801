"""Request loop (continuous batching) through the C ABI: each request's
result is the same alone and in a mix of overlapping requests, equals the
single-problem context's, and matches the FP64 oracle within the pose and
loss tolerances; admission by memory footprint and argument checks."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from helpers import REL_TOL, ROT_TOL, TRANS_TOL, bf16_round, pose_errors

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rk():
    from paper_2403_01254_amd import rkhsba
    rkhsba.lib()
    return rkhsba


@pytest.fixture(scope="module")
def requests():
    # mixed frame counts, point counts and length scales (0.08 m and 0.3 m)
    return [scenes.request(s, k_range=(2, 5), n_range=(1500, 4000), n_iter=3) for s in range(5)]


def submit(srv, p):
    return srv.submit(p.points, p.feats, p.init_poses, p.edges, p.ell, p.n_iter)


@pytest.mark.parametrize("lanes,split_work,lane1_max,lane1_order",
                         [(1, 5e8, 1, 1), (2, 5e8, 1, 1), (2, 5e8, 0, 1), (2, 1.0, 1, 1), (2, 1.0, 1, 0)])
def test_alone_and_in_mix_agree(rk, requests, lanes, split_work, lane1_max, lane1_order):
    # plus one request with frames large enough for several entries per finalisation thread (with two
    # lanes it is the only one above the entry split and runs in the second lane, beside the others; with
    # a work split of 1 every request built in lane 0 moves to lane 1 and is built again there, where it
    # waits built ahead and starts in the order of its service estimate (lane1_order 1) or of arrival)
    requests = requests + [scenes.request(7, k_range=(3, 3), n_range=(40000, 60000), n_iter=2)]
    say(f"[server] lanes {lanes} work split {split_work} lane-1 limit {lane1_max} order {lane1_order}: " +
        "; ".join(p.recipe[:60] for p in requests))
    with rk.Server(feat_kind="dense", D=20, max_active=8, lanes=lanes, lane_split_entries=60000,
                   lane_split_work=split_work, lane1_max_active=lane1_max, lane1_order=lane1_order) as srv:
        alone = [srv.wait(submit(srv, p), timeout=120) for p in requests]
        assert srv.stats()["max_active"] == 1
        tickets = [submit(srv, p) for p in requests]       # all in flight together
        mix = [srv.wait(t, timeout=120) for t in tickets]
        st = srv.stats()
        say(f"[server] stats {st}")
        assert st["completed"] == 2 * len(requests) and st["failed"] == 0
        if not (lanes == 2 and split_work <= 1.0 and lane1_max == 1):  # else all run one by one in lane 1
            assert st["max_active"] >= 2
    for p, a, m in zip(requests, alone, mix):
        np.testing.assert_array_equal(a[0], m[0])          # poses
        np.testing.assert_array_equal(a[1][:-1], m[1][:-1])  # loss entering each step
        np.testing.assert_allclose(a[1][-1], m[1][-1], rtol=1e-6)
        np.testing.assert_array_equal(a[2], m[2])          # pair counts


def test_large_systems_alone_and_batched_agree(rk):
    """Requests of 24 frames (138 unknowns: the blocked Cholesky solve, beyond the in-LDS one), served alone
    and together: each system is factored by a workgroup of its own either way, so the poses agree bit for
    bit, and the first request's poses meet the oracle's."""
    reqs = [scenes.request(s, k_range=(24, 24), n_range=(600, 900), n_iter=3) for s in (31, 32)]
    say("[server] large systems: " + "; ".join(p.recipe[:50] for p in reqs))
    with rk.Server(feat_kind="dense", D=20, max_active=8, lanes=1) as srv:
        alone = [srv.wait(submit(srv, p), timeout=120) for p in reqs]
        tickets = [submit(srv, p) for p in reqs]
        both = [srv.wait(t, timeout=120) for t in tickets]
        assert srv.stats()["max_active"] == 2
    for p, a, m in zip(reqs, alone, both):
        np.testing.assert_array_equal(a[0], m[0])
        np.testing.assert_array_equal(a[1], m[1])
    op = oracle.Problem.from_scene(reqs[0], search="cells")
    oposes, _ = oracle.gn(op, reqs[0].init_poses, reqs[0].edges, reqs[0].n_iter, membership=oracle.MEMBER_FP32_RULE)
    rot, tr = pose_errors(alone[0][0], oposes)
    assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL


def test_served_matches_context_and_oracle(rk, requests):
    """Each served solve against the same solve on a context and against the oracle.  The context keeps its
    first iteration's binning of the source points for the later ones, the server bins every batch
    iteration afresh: the passes, and with them the FP32 summation order, differ after the first step, so the
    two agree to rounding (poses within 1e-6, pair counts within 1e-6 relative), not bit for bit."""
    with rk.Server(feat_kind="dense", D=20, max_active=8) as srv:
        tickets = [submit(srv, p) for p in requests]
        served = [srv.wait(t, timeout=120) for t in tickets]
    for p, (poses, lpi, ppi, lat, qs) in zip(requests, served):
        ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, cell_subdiv=0)
        ctx.build_neighbors(p.points, p.feats, p.feat_kind)
        cposes, clpi, cppi = ctx.gn_step(p.init_poses, p.edges, p.n_iter)
        rot_c, tr_c = pose_errors(poses, cposes)
        assert rot_c.max() <= 1e-6 and tr_c.max() <= 1e-6
        np.testing.assert_allclose(ppi, cppi, rtol=1e-6)
        np.testing.assert_allclose(lpi, clpi, rtol=1e-6)
        op = oracle.Problem.from_scene(p)
        oposes, olpi = oracle.gn(op, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
        rot, tr = pose_errors(poses, oposes)
        say(f"[server] {p.recipe[:50]}: latency {lat * 1e3:.1f} ms (queued {qs * 1e3:.1f}), rot {rot.max():.2g} "
            f"trans {tr.max():.2g}")
        assert rot.max() <= ROT_TOL and tr.max() <= TRANS_TOL
        np.testing.assert_allclose(lpi, olpi, rtol=REL_TOL)


@pytest.mark.parametrize("lanes,lane1_order", [(1, 1), (2, 1), (2, 0)])
def test_single_request_lane_matches_context(rk, requests, lanes, lane1_order):
    """A lane that runs one request at a time keeps the binning order of the request's first iteration, as
    the context's gn_step does: the served poses, loss and pair-count histories equal the context's bit for
    bit.  With two lanes and no entry split every request goes to lane 1, which builds waiting requests
    ahead and, with lane1_order 1, starts them out of arrival order: the results are the same."""
    with rk.Server(feat_kind="dense", D=20, max_active=1 if lanes == 1 else 8, lanes=lanes, lane_split_entries=0,
                   lane1_order=lane1_order) as srv:
        tickets = [submit(srv, p) for p in requests]
        served = [srv.wait(t, timeout=120) for t in tickets]
        st = srv.stats()
        assert st["max_active"] == 1 and st["completed"] == len(requests) and st["queued"] == 0
    for p, (poses, lpi, ppi, _, _) in zip(requests, served):
        ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, cell_subdiv=0)
        ctx.build_neighbors(p.points, p.feats, p.feat_kind)
        cposes, clpi, cppi = ctx.gn_step(p.init_poses, p.edges, p.n_iter)
        ctx.close()
        say(f"[server] one at a time: {p.recipe[:50]}")
        np.testing.assert_array_equal(poses, cposes)
        np.testing.assert_array_equal(lpi, clpi)
        np.testing.assert_array_equal(ppi, cppi)


def test_admission_by_footprint(rk, requests):
    """With a budget smaller than any request, requests run one at a time
    (a request is always admitted when nothing is active), with the same
    results."""
    with rk.Server(feat_kind="dense", D=20, max_active=8) as srv:
        ref = [srv.wait(submit(srv, p), timeout=120) for p in requests[:3]]
    with rk.Server(feat_kind="dense", D=20, max_active=8, hbm_budget_bytes=1) as srv:
        tickets = [submit(srv, p) for p in requests[:3]]
        got = [srv.wait(t, timeout=120) for t in tickets]
        st = srv.stats()
    assert st["max_active"] == 1 and st["completed"] == 3
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a[0], b[0])
        assert b[4] >= 0.0


def test_admission_by_work(rk, requests):
    """A lane admits the request at the head of its queue only while the active requests' entries plus its own
    stay within the work limit: with a limit of one entry, requests run one at a time (an idle lane always
    admits), with the same results; with a larger limit, never more requests than the limit can hold."""
    with rk.Server(feat_kind="dense", D=20, max_active=8) as srv:
        ref = [srv.wait(submit(srv, p), timeout=120) for p in requests]
    entries = sorted(sum(len(p.points[m]) for m, _ in p.edges) for p in requests)
    limit2 = entries[-1] + entries[-2]
    most2 = max(k for k in range(1, len(entries) + 1) if k == 1 or sum(entries[:k]) <= limit2)
    for limit, most in ((1, 1), (limit2, most2)):
        with rk.Server(feat_kind="dense", D=20, max_active=8, lane_work_entries=limit) as srv:
            tickets = [submit(srv, p) for p in requests]
            got = [srv.wait(t, timeout=120) for t in tickets]
            st = srv.stats()
        say(f"[server] work limit {limit}: max_active {st['max_active']}, {st['batch_iterations']} batch iterations")
        assert 1 <= st["max_active"] <= most and st["completed"] == len(requests)
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[2], b[2])


def test_invalid_requests(rk, requests):
    p = requests[0]
    with rk.Server(feat_kind="dense", D=20) as srv:
        with pytest.raises(rk.RkhsbaError) as e:
            srv.submit(p.points, p.feats, p.init_poses, [[0, 0]], p.ell, 2)
        assert e.value.code == rk.EINVAL
        with pytest.raises(rk.RkhsbaError) as e:
            srv.submit(p.points, [f[:, :10] for f in p.feats], p.init_poses, p.edges, p.ell, 2)
        assert e.value.code == rk.EINVAL
        with pytest.raises(rk.RkhsbaError) as e:
            srv.submit(p.points, p.feats, p.init_poses, p.edges, -1.0, 2)
        assert e.value.code == rk.EINVAL
        # the server still works after rejected submissions
        poses, lpi, ppi, lat, qs = srv.wait(submit(srv, p), timeout=120)
        assert np.all(np.isfinite(poses))
    for bad in (0, 3):
        with pytest.raises(rk.RkhsbaError):
            rk.Server(feat_kind="dense", D=20, lanes=bad)
    with pytest.raises(rk.RkhsbaError):
        rk.Server(feat_kind="dense", D=20, lane_work_entries=-1)


def test_served_forms_against_oracle(rk):
    """The pose accuracy of each served form on requests of the serving benchmark's generator (10
    Gauss-Newton steps, 20-class soft labels, ell 0.08 or 0.3 m), against the FP64 oracle run on the
    FP32 features (cell-list search, FP32 membership rule): one request at a time in FP32, the batched
    FP32 server (two lanes), and the batched server with bfloat16 features.  The FP32 forms meet the
    pose tolerance; the bfloat16 form's error, which comes from rounding the features, is printed and
    held to 5e-3, and against the oracle run on the same features rounded to bfloat16 (nearest even,
    as the library stores them) the bfloat16 form meets the pose tolerance."""
    reqs = [scenes.request(s, k_range=(2, 6), n_range=(4000, 15000), n_iter=10) for s in range(2000, 2006)]
    one = []
    for p in reqs:
        ctx = rk.Context(ell=p.ell, cutoff_factor=p.cutoff_factor, cell_subdiv=0)
        ctx.build_neighbors(p.points, p.feats, p.feat_kind)
        one.append(ctx.gn_step(p.init_poses, p.edges, p.n_iter)[0])
        ctx.close()
    served = {}
    for kind in ("dense", "bf16"):
        with rk.Server(feat_kind=kind, D=20, max_active=8, lanes=2, lane_work_entries=8_000_000) as srv:
            tickets = [submit(srv, p) for p in reqs]
            served[kind] = [srv.wait(t, timeout=120)[0] for t in tickets]
    rounded = "batched, bf16 (oracle on bf16-rounded features)"
    worst = {"one at a time, f32": [0.0, 0.0], "batched, f32": [0.0, 0.0], "batched, bf16": [0.0, 0.0],
             rounded: [0.0, 0.0]}
    for i, p in enumerate(reqs):
        op = oracle.Problem.from_scene(p, search="cells")
        oposes, _ = oracle.gn(op, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
        opr = oracle.Problem(p.points, [bf16_round(f) for f in p.feats], p.feat_kind, p.ell, p.cutoff_factor,
                             search="cells")
        rposes, _ = oracle.gn(opr, p.init_poses, p.edges, p.n_iter, membership=oracle.MEMBER_FP32_RULE)
        for name, poses, ref in (("one at a time, f32", one[i], oposes), ("batched, f32", served["dense"][i], oposes),
                                 ("batched, bf16", served["bf16"][i], oposes), (rounded, served["bf16"][i], rposes)):
            rot, tr = pose_errors(poses, ref)
            worst[name][0] = max(worst[name][0], rot.max())
            worst[name][1] = max(worst[name][1], tr.max())
    for name, (r, t) in worst.items():
        say(f"[served-vs-oracle] {name}: largest rotation error {r:.3g} rad, translation error {t:.3g} m "
            f"over {len(reqs)} requests")
    for name in ("one at a time, f32", "batched, f32", rounded):
        assert worst[name][0] <= ROT_TOL and worst[name][1] <= TRANS_TOL
    assert worst["batched, bf16"][0] <= 5e-3 and worst["batched, bf16"][1] <= 5e-3
