"""Shared test helpers: tolerances, pose errors, library availability."""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# Relative tolerance of FP32 loss, gradient and Gauss-Newton matrix against the
# FP64 oracle, and the pose tolerance after Gauss-Newton steps.
REL_TOL = 1e-5
ROT_TOL = 1e-4   # rad
TRANS_TOL = 1e-4  # m


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def inv_cell(ell, cutoff_factor, subdiv):
    """Cell size formula of the voxel structure: edge r_c / cell_subdiv, inverse in FP64."""
    rc = cutoff_factor * ell
    cell = rc / subdiv
    return 1.0 / cell


def normwise_rel(x_hat, x):
    x_hat = np.asarray(x_hat, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    den = np.linalg.norm(x)
    return np.linalg.norm(x_hat - x) / den if den > 0 else np.linalg.norm(x_hat)


def assert_blocks_close(x_hat, x, block, rel=REL_TOL, floor=1e-2, what=""):
    """Normwise relative error over the whole array and per block (6-vectors of b,
    6x6 blocks of H); blocks much smaller than the largest (below `floor` of it)
    are held to rel * floor * largest instead (cancellation, near-empty blocks)."""
    x_hat = np.asarray(x_hat, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    tot = normwise_rel(x_hat, x)
    assert tot <= rel, f"{what}: normwise relative error {tot:.3g} > {rel}"
    if x.ndim == 1:
        blocks = [(slice(i, i + block),) for i in range(0, len(x), block)]
    else:
        blocks = [(slice(i, i + block), slice(j, j + block)) for i in range(0, x.shape[0], block)
                  for j in range(0, x.shape[1], block)]
    norms = [np.linalg.norm(x[s]) for s in blocks]
    big = max(norms) if norms else 0.0
    for s, nrm in zip(blocks, norms):
        err = np.linalg.norm(x_hat[s] - x[s])
        lim = rel * max(nrm, floor * big)
        assert err <= lim + 1e-300, f"{what}: block {s} error {err:.3g} > {lim:.3g} (block norm {nrm:.3g})"


def pose_errors(P_hat, P):
    """Per-frame rotation angle |log(R_hat^T R)| and translation distance."""
    P_hat = np.asarray(P_hat).reshape(-1, 12)
    P = np.asarray(P).reshape(-1, 12)
    rot, tr = [], []
    for a, b in zip(P_hat, P):
        Ra, Rb = a[:9].reshape(3, 3), b[:9].reshape(3, 3)
        rot.append(np.linalg.norm(Rotation.from_matrix(Ra.T @ Rb).as_rotvec()))
        tr.append(np.linalg.norm(a[9:] - b[9:]))
    return np.array(rot), np.array(tr)


def ident():
    return np.concatenate([np.eye(3).reshape(9), np.zeros(3)])


def _round_to_grid(x, exp_floor, mant_bits, max_abs):
    """Round to nearest (ties to even) on a binary floating grid with `mant_bits`
    fraction bits, exponents clamped below at `exp_floor` (subnormal step
    2^(exp_floor - mant_bits)), saturating at max_abs.  Done in float64, where
    every step is exact for float32 inputs."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    e = np.maximum(np.floor(np.log2(np.abs(x[nz]))), exp_floor)
    ulp = np.exp2(e - mant_bits)
    out[nz] = np.round(x[nz] / ulp) * ulp          # numpy rounds halves to even
    return np.clip(out, -max_abs, max_abs)


def bf16_round(x):
    """float32 -> bfloat16 (8 significant bits), nearest even, as float32."""
    return _round_to_grid(x, -126, 7, 3.3895313892515355e38).astype(np.float32)


def e4m3_round(x):
    """float32 -> OCP fp8 e4m3 (bias 7: normal exponents -6..8, 3 fraction bits,
    subnormal step 2^-9), nearest even, saturating at 448, as float32."""
    return _round_to_grid(x, -6, 3, 448.0).astype(np.float32)


def scene_digest(points, feats, poses, edges):
    """SHA-256 of a workload's inputs (points, features, initial poses, edges), so that stored
    expected values are only compared on the inputs they were computed from."""
    import hashlib
    h = hashlib.sha256()
    for a in list(points) + list(feats) + [poses, edges]:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode() + str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def label_stacked(class_ids, dims):
    """Whether a build stacks the class ids of its frames into label layers (the documented rule): every
    frame's cells x (largest id + 1) fit 32-bit keys and the stacked cell-row tables hold at most 16 rows
    per point + 2^20.  class_ids: per frame; dims: per frame, the cell grid's extent (x, y, z)."""
    layers = [int(f.max()) + 1 for f in class_ids]
    fits = all(int(np.prod(np.asarray(d, dtype=np.int64))) * L < 2**32 - 1 for d, L in zip(dims, layers))
    rows = sum(int(d[1]) * int(d[2]) * L for d, L in zip(dims, layers))
    n = sum(len(f) for f in class_ids)
    return fits and rows < 2**31 and rows <= 16 * n + 2**20
