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
    ang = np.degrees(np.arccos(np.clip((np.trace(R, axis1=1, axis2=2) - 1) / 2, -1, 1)))
    classes = {a: int(np.sum(np.abs(ang - a) < 1e-6)) for a in (0, 72, 120, 144, 180)}
    assert classes == {0: 1, 72: 12, 120: 20, 144: 12, 180: 15}  # 1 + 15 + 20 + 24 (Sec. IV-A)


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
