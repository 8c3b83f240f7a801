"""Oracle for frame-to-frame tracking and the keyframe alignment (Sec. III-A,
Sec. IV-A, Sec. VI-C) -- TEST INFRASTRUCTURE ONLY.

Tracking is gradient ascent on F of one edge (m fixed, n moving) with the
step-length rule of the library's documented reading: move along the
normalised gradient grad F = -(sigma^2/ell^2) b_n by s, accept when F
increases (s *= 1.5), otherwise halve s and retry; stop after max_iter
accepted steps or when s < step_min.
"""
from __future__ import annotations

import numpy as np

import oracle


def _compose(T, xi):
    E = oracle.se3_exp(xi)
    R = T[:9].reshape(3, 3)
    t = T[9:]
    Re = E[:9].reshape(3, 3)
    te = E[9:]
    return np.concatenate([(R @ Re).reshape(9), R @ te + t])


def track(prob, poses, m, n, max_iter, step0, step_min, membership=oracle.MEMBER_FP64):
    P = np.array(poses, dtype=np.float64, copy=True)

    def value_and_b(Q):
        F, b, _, _, _ = oracle.normal_eqs(prob, Q, [[m, n]], membership)
        return F, b[6 * n:6 * n + 6]

    F, bn = value_and_b(P)
    s = step0
    it = 0
    while it < max_iter and s >= step_min:
        g = -(prob.sigma ** 2 / prob.ell ** 2) * bn
        gn = np.linalg.norm(g)
        if not gn > 0:
            break
        accepted = False
        while s >= step_min:
            Q = P.copy()
            Q[n] = _compose(P[n], s * g / gn)
            Fc = oracle.normal_eqs(prob, Q, [[m, n]], membership)[0]
            if Fc > F:
                P = Q
                s *= 1.5
                accepted = True
                break
            s *= 0.5
        if not accepted:
            break
        F, bn = value_and_b(P)
        it += 1
    return P, it, F


def cosine(prob, poses, m, n, membership=oracle.MEMBER_FP64):
    """<f_m, f_n> / sqrt(<f_m, f_m> <f_n, f_n>) with the truncated inner products."""
    F, _ = oracle.edge_sums(prob, poses, [[m, n], [m, m], [n, n]], membership)
    return F[0] / np.sqrt(F[1] * F[2]) if F[1] > 0 and F[2] > 0 else 0.0
