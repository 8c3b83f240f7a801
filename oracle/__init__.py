"""FP64 CPU oracle for the RKHS-BA hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is a plain C restatement of the
paper's definitions (arXiv 2403.01254, Sec. III and Sec. V-A), loaded
through ctypes: brute force over all point pairs, or an independent
cell-list search over the same pairs.  It shares no code with the GPU
library.

Every function here follows a passage of the paper; see ``rkhs_oracle.c``
for the per-function citations.  Pins live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rkhs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MEMBER_FP64 = 0
MEMBER_FP32_RULE = 1
SEARCH = {"brute": 0, "cells": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int),
        ("n_points", ctypes.POINTER(ctypes.c_int64)),
        ("xyz", ctypes.POINTER(ctypes.c_void_p)),
        ("feat_kind", ctypes.c_int),
        ("D", ctypes.c_int),
        ("feats", ctypes.POINTER(ctypes.c_void_p)),
        ("ell", ctypes.c_double),
        ("cutoff_factor", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("clamp_negative_c", ctypes.c_int),
        ("top_k", ctypes.c_int),
        ("search", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_normal_eqs.argtypes = [P, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp, dp, dp,
                                        ctypes.POINTER(ctypes.c_int64)]
        L.oracle_gn.argtypes = [P, dp, ctypes.c_int, ip, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.c_int, dp, dp]
        L.oracle_edge_sums.argtypes = [P, dp, ctypes.c_int, ip, ctypes.c_int, dp, dp]
        L.oracle_pairs.argtypes = [P, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ip]
        L.oracle_pairs.restype = ctypes.c_int64
        L.oracle_voxels.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                    ip, ctypes.POINTER(ctypes.c_uint32), ip, ip]
        L.oracle_se3_exp.argtypes = [dp, dp]
        L.oracle_cholesky_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        _lib = L
    return _lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


class Problem:
    """Frames, features and kernel parameters in the layout the C oracle reads.

    points: list of (N_m, 3) float32; feats: list of (N_m,) uint16 class ids or
    (N_m, D) float32 rows; ell, cutoff_factor, sigma as in Eq. (eq:kernel).
    search: "brute" (every point pair, the definition) or "cells" (the targets
    of the 27 world-coordinate cells around each source point: the same pairs,
    summed in another order)."""

    def __init__(self, points, feats, feat_kind, ell, cutoff_factor=3.0, sigma=1.0, clamp_negative_c=True,
                 top_k=0, search="brute"):
        self.points = [np.ascontiguousarray(p, dtype=np.float32).reshape(-1, 3) for p in points]
        if feat_kind == "class":
            self.feats = [np.ascontiguousarray(f, dtype=np.uint16).reshape(-1) for f in feats]
            D = 0
        else:
            self.feats = [np.ascontiguousarray(f, dtype=np.float32) for f in feats]
            D = int(self.feats[0].shape[1])
        self.feat_kind = feat_kind
        self.ell, self.cutoff_factor, self.sigma = float(ell), float(cutoff_factor), float(sigma)
        self.K = len(self.points)
        self._n = np.array([len(p) for p in self.points], dtype=np.int64)
        self._xyz = (ctypes.c_void_p * self.K)(*[p.ctypes.data for p in self.points])
        self._f = (ctypes.c_void_p * self.K)(*[f.ctypes.data for f in self.feats])
        self.c = _Problem(self.K, _ptr(self._n, ctypes.c_int64), self._xyz, 0 if feat_kind == "class" else 1, D,
                          self._f, float(ell), float(cutoff_factor), float(sigma), int(bool(clamp_negative_c)),
                          int(top_k), SEARCH[search])
        self.top_k = int(top_k)
        self.search = search

    @classmethod
    def from_scene(cls, p, **kw):
        return cls(p.points, p.feats, p.feat_kind, p.ell, p.cutoff_factor, **kw)

    def with_search(self, search):
        """The same frames and parameters with another neighbour search."""
        return Problem(self.points, self.feats, self.feat_kind, self.ell, self.cutoff_factor, self.sigma,
                       bool(self.c.clamp_negative_c), self.top_k, search)


def _edges(edges):
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


def normal_eqs(prob: Problem, poses, edges, membership=MEMBER_FP64):
    """F, b (6K), H (6K x 6K), per-edge F and the in-cutoff c != 0 pair count."""
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(prob.K, 12)
    e = _edges(edges)
    K = prob.K
    F = ctypes.c_double()
    b = np.zeros(6 * K)
    H = np.zeros((6 * K, 6 * K))
    Fe = np.zeros(max(len(e), 1))
    npairs = ctypes.c_int64()
    rc = lib().oracle_normal_eqs(ctypes.byref(prob.c), _ptr(poses), len(e), _ptr(e, ctypes.c_int32), membership,
                                 ctypes.byref(F), _ptr(b), _ptr(H), _ptr(Fe), ctypes.byref(npairs))
    if rc != 0:
        raise ValueError(f"oracle_normal_eqs failed ({rc})")
    return F.value, b, H, Fe[:len(e)], npairs.value


def loss(prob: Problem, poses, edges, membership=MEMBER_FP64):
    return normal_eqs(prob, poses, edges, membership)[0]


def gn(prob: Problem, poses, edges, n_iter, fixed_frame=0, damping_rel=1e-10, membership=MEMBER_FP64,
       trace=False):
    """n_iter Gauss-Newton/IRLS steps (Sec. V-A); returns (poses, F per iteration), and with trace=True
    also the poses entering each step and after the last ((n_iter + 1, K, 12))."""
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(prob.K, 12).copy()
    e = _edges(edges)
    lpi = np.zeros(n_iter + 1)
    tr = np.zeros((n_iter + 1, prob.K, 12)) if trace else None
    rc = lib().oracle_gn(ctypes.byref(prob.c), _ptr(poses), len(e), _ptr(e, ctypes.c_int32), int(n_iter),
                         int(fixed_frame), float(damping_rel), membership, _ptr(lpi),
                         _ptr(tr) if trace else ctypes.cast(None, ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError(f"oracle_gn failed ({rc})")
    return (poses, lpi, tr) if trace else (poses, lpi)


def edge_sums(prob: Problem, poses, edges, membership=MEMBER_FP64):
    """Per-edge F and W = sum w |u|^2 (self-pairs (m, m) allowed)."""
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(prob.K, 12)
    e = _edges(edges)
    Fe = np.zeros(max(len(e), 1))
    We = np.zeros(max(len(e), 1))
    rc = lib().oracle_edge_sums(ctypes.byref(prob.c), _ptr(poses), len(e), _ptr(e, ctypes.c_int32), membership,
                                _ptr(Fe), _ptr(We))
    if rc != 0:
        raise ValueError("oracle_edge_sums failed")
    return Fe[:len(e)], We[:len(e)]


def pairs(prob: Problem, poses, m, n):
    """In-cutoff pairs (i, j) of edge (m, n) under the FP32 membership rule, (i, j) order."""
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(prob.K, 12)
    L = lib()
    total = L.oracle_pairs(ctypes.byref(prob.c), _ptr(poses), int(m), int(n), 0,
                           ctypes.cast(None, ctypes.POINTER(ctypes.c_int32)))
    if total < 0:
        raise ValueError("oracle_pairs failed")
    out = np.zeros((max(total, 1), 2), dtype=np.int32)
    L.oracle_pairs(ctypes.byref(prob.c), _ptr(poses), int(m), int(n), total, _ptr(out, ctypes.c_int32))
    return out[:total]


def voxels(xyz, inv_cell, margin=0, labels=None):
    """Stable voxel sort of one frame: (perm, keys, origin, dims); with class
    ids (labels) the label-stacked keys (one layer of the z extent per id)."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float32).reshape(-1, 3)
    N = len(xyz)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.uint16).reshape(N)
    perm = np.zeros(N, dtype=np.int32)
    keys = np.zeros(N, dtype=np.uint32)
    origin = np.zeros(3, dtype=np.int32)
    dims = np.zeros(3, dtype=np.int32)
    rc = lib().oracle_voxels(xyz.ctypes.data, None if lab is None else lab.ctypes.data, N, float(inv_cell),
                             int(margin), _ptr(perm, ctypes.c_int32),
                             _ptr(keys, ctypes.c_uint32), _ptr(origin, ctypes.c_int32), _ptr(dims, ctypes.c_int32))
    if rc != 0:
        raise ValueError("oracle_voxels failed")
    return perm, keys, origin, dims


def se3_exp(xi):
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(6)
    T = np.zeros(12)
    lib().oracle_se3_exp(_ptr(xi), _ptr(T))
    return T


def cholesky_solve(A, b):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(len(b))
    rc = lib().oracle_cholesky_solve(len(b), _ptr(A), _ptr(b), _ptr(x))
    if rc != 0:
        raise np.linalg.LinAlgError(f"oracle Cholesky failed ({rc})")
    return x
