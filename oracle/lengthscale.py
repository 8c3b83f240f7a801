"""Oracle for the lengthscale outer loop (Sec. V-C) -- TEST INFRASTRUCTURE ONLY.

The RKHS distance of an edge (m, n) is d = <f_m, f_m> + <f_n, f_n> - 2 <f_m, f_n>
(Eq. (eq:dist_rkhs)), each inner product the truncated double sum of
Eq. (eq:double_sum) with the kernel of Eq. (eq:kernel); d_H sums it over the
edges of the graph.  Because d/d ell of exp(-r^2 / 2 ell^2) is
exp(-r^2 / 2 ell^2) r^2 / ell^3, the derivative of every inner product is
sigma^2 W / ell^3 with W = sum c exp(-r^2/2 ell^2) r^2 over its pairs (the
truncation radius moving with ell is not differentiated).

Outer loop (the paper fixes only its elements -- the direction from the
derivative of d_H, a fixed percentage step, inner Gauss-Newton loops at the
current ell, and a stop when the objective stops increasing; the rest is this
repository's reading):
  1. run `inner_iter` Gauss-Newton steps at ell;
  2. compute d_H and g = d d_H / d ell at the new poses; the elasticity
     eta = -ell g / d_H is near 2 when the frames are aligned below the
     current scale (d_H then comes from the residual spread) and near 0 when a
     gross misalignment dominates; eta >= `elasticity` shrinks ell by the step
     (the scale is resolved: refine), otherwise ell grows by it;
  3. clamp ell to [ell_min, ell_max]; stop when the clamped update leaves ell
     unchanged and the inner loop raised F by no more than tol |F|, or after
     max_outer outer iterations.
"""
from __future__ import annotations

import numpy as np

import oracle


def distance_and_derivative(make_problem, ell, poses, edges, membership):
    """d_H and d d_H / d ell at (ell, poses)."""
    prob = make_problem(ell)
    edges = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    frames = sorted(set(edges.reshape(-1).tolist()))
    Fc, Wc = oracle.edge_sums(prob, poses, edges, membership)
    Fs, Ws = oracle.edge_sums(prob, poses, [[f, f] for f in frames], membership)
    S = dict(zip(frames, Fs))
    SW = dict(zip(frames, Ws))
    s2 = prob.sigma ** 2
    d = sum(S[m] + S[n] - 2.0 * F for (m, n), F in zip(edges.tolist(), Fc))
    g = s2 / ell ** 3 * sum(SW[m] + SW[n] - 2.0 * W for (m, n), W in zip(edges.tolist(), Wc))
    return d, g


def gn_lengthscale(make_problem, poses, edges, ell_init, ell_min, ell_max, step=0.1, elasticity=1.0, tol=1e-6,
                   inner_iter=5, max_outer=30, fixed_frame=0, damping_rel=1e-10, membership=oracle.MEMBER_FP64):
    """Returns (poses, trace) with trace rows (ell, F_start, F_end, d_H, g)."""
    poses = np.array(poses, dtype=np.float64, copy=True)
    ell = min(max(ell_init, ell_min), ell_max)
    trace = []
    for _ in range(max_outer):
        prob = make_problem(ell)
        poses, lpi = oracle.gn(prob, poses, edges, inner_iter, fixed_frame, damping_rel, membership)
        d, g = distance_and_derivative(make_problem, ell, poses, edges, membership)
        trace.append((ell, lpi[0], lpi[-1], d, g))
        eta = -ell * g / d if d > 0 else 0.0
        new = ell * (1.0 - step) if eta >= elasticity else ell * (1.0 + step)
        new = min(max(new, ell_min), ell_max)
        if new == ell and lpi[-1] - lpi[0] <= tol * abs(lpi[0]):
            break
        ell = new
    return poses, np.array(trace)
