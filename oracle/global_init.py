"""Oracle for the global rotation initialisation (Sec. IV-A) -- TEST
INFRASTRUCTURE ONLY.

The rotation group of the icosahedron is built from its description in
Sec. IV-A: the identity, a half-turn about each of the 15 axes through
midpoints of opposite edges, turns by 2pi/3 and 4pi/3 about each of the 10
axes through centres of opposite faces, and turns by 2pi k/5 (k = 1..4) about
each of the 6 axes through opposite vertices.  The icosahedron is the one with
vertices (0, +-1, +-g), (+-1, +-g, 0), (+-g, 0, +-1), g the golden ratio.

The search scores each candidate rotation of frame n (about the centroid of
its points) by F of the edge (m, n) -- the pose-dependent term of the RKHS
distance, Eq. (eq:dist_rkhs) -- and keeps the largest.
"""
from __future__ import annotations

import itertools

import numpy as np


def _axis_angle(axis, angle):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def icosahedron_vertices():
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1, s2 in itertools.product((1.0, -1.0), repeat=2):
        v += [(0.0, s1, s2 * g), (s1, s2 * g, 0.0), (s2 * g, 0.0, s1)]
    return np.array(v)


def icosahedral_rotations():
    """The 60 rotations, (60, 3, 3), grouped as identity, edge, face and vertex turns."""
    V = icosahedron_vertices()
    n = len(V)
    adj = [[abs(np.linalg.norm(V[i] - V[j]) - 2.0) < 1e-9 for j in range(n)] for i in range(n)]
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if adj[i][j]]
    faces = [(i, j, k) for i, j, k in itertools.combinations(range(n), 3) if adj[i][j] and adj[j][k] and adj[i][k]]

    def half(axes):  # one direction per pair of opposite axes
        out = []
        for a in axes:
            a = a / np.linalg.norm(a)
            if not any(abs(abs(a @ b) - 1.0) < 1e-9 for b in out):
                out.append(a)
        return out

    vertex_axes = half([V[i] for i in range(n)])
    edge_axes = half([(V[i] + V[j]) / 2.0 for i, j in edges])
    face_axes = half([(V[i] + V[j] + V[k]) / 3.0 for i, j, k in faces])
    assert (len(vertex_axes), len(edge_axes), len(face_axes)) == (6, 15, 10)
    R = [np.eye(3)]
    R += [_axis_angle(a, np.pi) for a in edge_axes]
    R += [_axis_angle(a, t) for a in face_axes for t in (2 * np.pi / 3, 4 * np.pi / 3)]
    R += [_axis_angle(a, 2 * np.pi * k / 5) for a in vertex_axes for k in range(1, 5)]
    return np.array(R)


def candidate_pose(T_n, R_k, c):
    """T_n G_k with G_k(x) = R_k (x - c) + c, poses as [R (row-major) | t]."""
    Rn = np.asarray(T_n[:9]).reshape(3, 3)
    tn = np.asarray(T_n[9:])
    R = Rn @ R_k
    t = Rn @ (c - R_k @ c) + tn
    return np.concatenate([R.reshape(9), t])


def rotation_search(loss_fn, points_n, poses, m, n, rotations=None):
    """Scores F_k of edge (m, n) for every candidate and the index of the largest.
    loss_fn(poses, edges) evaluates F (the oracle's normal_eqs)."""
    R = icosahedral_rotations() if rotations is None else np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3)
    c = np.asarray(points_n, dtype=np.float64).mean(axis=0)
    scores = np.zeros(len(R))
    for k, Rk in enumerate(R):
        P = np.array(poses, dtype=np.float64, copy=True)
        P[n] = candidate_pose(P[n], Rk, c)
        scores[k] = loss_fn(P, [[m, n]])
    return scores, int(np.argmax(scores)), R
