"""Seeded synthetic inputs shaped like the paper's RGB-D and LiDAR workloads.

This module only synthesises inputs: point clouds in frame-local coordinates,
per-point pose-invariant features, ground-truth and initial poses and the
frame-pair graph.  It holds none of the method's arithmetic (no kernel, no
loss, no Jacobian, no solver); rotations are built with scipy's Rotation so
that neither the oracle nor the GPU path is used to make its own inputs.

Workloads (sizes follow the paper's experiments, stand-ins for datasets that
are not available here):

* ``two_view``    - 2 frames x 5,000 points of a plane/box scene, the second a
                    noisy rigid copy of the first (the paper's registration
                    experiments of Sec. VI-A/B use noisy rigid copies).
* ``odometry``    - 8 depth-camera views x 30,000 points along a trajectory,
                    20-class soft labels concatenated with RGB (Sec. VI-C
                    sliding-window semantic BA, Sec. III-A label tensors).
* ``lidar``       - 64 spinning-LiDAR frames x 100,000 points around a street
                    loop with 20% outliers and 10% flipped one-hot labels,
                    6-nearest-pose graph (Sec. VI-D LiDAR global mapping).
* ``dense64``     - as ``odometry`` with 64-dim unit-vector features.
* ``request``     - one serving request of 2-16 frames (random mix of the
                    two-view and odometry styles).

Poses are K x 12 float64 rows ``[R (row-major 3x3) | t]`` mapping local to
world coordinates.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Problem", "two_view", "odometry", "lidar", "dense64", "request",
    "make", "pose_from_rt", "pose_rt", "compose", "invert", "transform",
]


@dataclasses.dataclass
class Problem:
    name: str
    points: list            # K arrays (N_m, 3) float32, frame-local coordinates
    feat_kind: str          # "class" (uint16 ids, one-hot) or "dense" (float32 rows)
    feats: list             # K arrays: (N_m,) uint16 or (N_m, D) float32
    D: int                  # feature dimension (number of classes for "class")
    gt_poses: np.ndarray    # (K, 12) float64
    init_poses: np.ndarray  # (K, 12) float64
    edges: np.ndarray       # (E, 2) int32, (source m, target n)
    ell: float
    cutoff_factor: float = 3.0
    n_iter: int = 10
    fixed_frame: int = 0
    recipe: str = ""

    @property
    def K(self) -> int:
        return len(self.points)

    @property
    def n_points(self) -> np.ndarray:
        return np.array([len(p) for p in self.points], dtype=np.int64)


# ----------------------------------------------------------------------------- poses

def pose_from_rt(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    out = np.empty(12, dtype=np.float64)
    out[:9] = np.asarray(R, dtype=np.float64).reshape(9)
    out[9:] = np.asarray(t, dtype=np.float64).reshape(3)
    return out


def pose_rt(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    return p[:9].reshape(3, 3), p[9:12].copy()


def compose(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    Ra, ta = pose_rt(a)
    Rb, tb = pose_rt(b)
    return pose_from_rt(Ra @ Rb, Ra @ tb + ta)


def invert(a: np.ndarray) -> np.ndarray:
    R, t = pose_rt(a)
    return pose_from_rt(R.T, -R.T @ t)


def transform(p: np.ndarray, pts: np.ndarray) -> np.ndarray:
    R, t = pose_rt(p)
    return np.asarray(pts, dtype=np.float64) @ R.T + t


def _rot(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    return Rotation.from_rotvec(axis * angle).as_matrix()


def _unit(rng: np.random.Generator, n: int | None = None) -> np.ndarray:
    v = rng.normal(size=(3,) if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _perturb(rng: np.random.Generator, pose: np.ndarray, sigma_t: float, sigma_deg: float) -> np.ndarray:
    """Initial guess: ground truth with N(0, sigma_t) per translation axis and
    a rotation of N(0, sigma_deg) degrees about a uniform random axis."""
    R, t = pose_rt(pose)
    dR = _rot(_unit(rng), math.radians(rng.normal() * sigma_deg))
    return pose_from_rt(R @ dR, t + rng.normal(size=3) * sigma_t)


# ----------------------------------------------------------------------------- plane/box scene

@dataclasses.dataclass
class _Scene:
    plane_n: np.ndarray      # (P, 3) unit normals, plane n.x = d
    plane_d: np.ndarray      # (P,)
    box_c: np.ndarray        # (B, 3) centres
    box_h: np.ndarray        # (B, 3) half sizes
    box_R: np.ndarray        # (B, 3, 3) box->world rotations
    cube: float              # planes are clipped to [-cube, cube]^3
    n_prim: int


def _make_scene(rng: np.random.Generator, n_planes=10, n_boxes=5, cube=10.0, walls=False) -> _Scene:
    n = _unit(rng, n_planes)
    d = rng.uniform(-8.0, 8.0, size=n_planes)
    if walls:  # the six faces of the cube, so that a camera inside always sees a surface
        wn = np.concatenate([np.eye(3), -np.eye(3)])
        n = np.concatenate([n, wn])
        d = np.concatenate([d, np.full(6, cube)])
    c = rng.uniform(-8.0, 8.0, size=(n_boxes, 3))
    h = rng.uniform(0.5, 4.0, size=(n_boxes, 3)) / 2
    R = np.stack([_rot([0, 0, 1], rng.uniform(0, 2 * math.pi)) for _ in range(n_boxes)])
    return _Scene(n, d, c, h, R, cube, len(n) + n_boxes)


def _plane_basis(n: np.ndarray):
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(n, a)
    u /= np.linalg.norm(u)
    return u, np.cross(n, u)


def _sample_plane(rng, n, d, cube, count):
    u, v = _plane_basis(n)
    half = cube * math.sqrt(3.0)
    out = []
    got = 0
    while got < count:
        m = max(4 * (count - got), 1024)
        ab = rng.uniform(-half, half, size=(m, 2))
        p = d * n + ab[:, :1] * u + ab[:, 1:] * v
        p = p[np.all(np.abs(p) <= cube, axis=1)]
        out.append(p)
        got += len(p)
    return np.concatenate(out)[:count]


def _plane_area(rng, n, d, cube, samples=200_000):
    u, v = _plane_basis(n)
    half = cube * math.sqrt(3.0)
    ab = rng.uniform(-half, half, size=(samples, 2))
    p = d * n + ab[:, :1] * u + ab[:, 1:] * v
    return np.mean(np.all(np.abs(p) <= cube, axis=1)) * (2 * half) ** 2


def _sample_box(rng, c, h, R, count):
    areas = np.array([h[1] * h[2], h[1] * h[2], h[0] * h[2], h[0] * h[2], h[0] * h[1], h[0] * h[1]])
    face = rng.choice(6, size=count, p=areas / areas.sum())
    uv = rng.uniform(-1.0, 1.0, size=(count, 3))
    axis = face // 2
    sign = np.where(face % 2 == 0, 1.0, -1.0)
    uv[np.arange(count), axis] = sign
    return (uv * h) @ R.T + c


def _surface_sample(rng, scene: _Scene, count):
    """Area-weighted uniform sample of the scene's surfaces; returns points and primitive ids."""
    P = len(scene.plane_n)
    areas = [_plane_area(rng, scene.plane_n[i], scene.plane_d[i], scene.cube) for i in range(P)]
    for b in range(len(scene.box_c)):
        h = scene.box_h[b]
        areas.append(8 * (h[0] * h[1] + h[1] * h[2] + h[0] * h[2]))
    areas = np.array(areas)
    prim = rng.choice(len(areas), size=count, p=areas / areas.sum())
    pts = np.empty((count, 3))
    for k in range(len(areas)):
        idx = np.nonzero(prim == k)[0]
        if len(idx) == 0:
            continue
        if k < P:
            pts[idx] = _sample_plane(rng, scene.plane_n[k], scene.plane_d[k], scene.cube, len(idx))
        else:
            b = k - P
            pts[idx] = _sample_box(rng, scene.box_c[b], scene.box_h[b], scene.box_R[b], len(idx))
    return pts, prim


def _cast(scene: _Scene, o: np.ndarray, dirs: np.ndarray, max_range: float):
    """First hit of rays o + t*dirs against the scene; returns (t, primitive id), t=inf on miss."""
    n_rays = len(dirs)
    best_t = np.full(n_rays, np.inf)
    best_p = np.full(n_rays, -1, dtype=np.int64)
    eps = 1e-9
    for k in range(len(scene.plane_n)):
        nd = dirs @ scene.plane_n[k]
        with np.errstate(divide="ignore", invalid="ignore"):
            t = (scene.plane_d[k] - o @ scene.plane_n[k]) / nd
        ok = (np.abs(nd) > 1e-12) & (t > 1e-6) & (t < best_t)
        hit = o + np.where(ok, t, 0.0)[:, None] * dirs
        ok &= np.all(np.abs(hit) <= scene.cube + eps, axis=1)
        best_t = np.where(ok, t, best_t)
        best_p = np.where(ok, k, best_p)
    P = len(scene.plane_n)
    for b in range(len(scene.box_c)):
        R = scene.box_R[b]
        lo = (o - scene.box_c[b]) @ R
        ld = dirs @ R
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / ld
            t1 = (-scene.box_h[b] - lo) * inv
            t2 = (scene.box_h[b] - lo) * inv
        tmin = np.nanmax(np.minimum(t1, t2), axis=1)
        tmax = np.nanmin(np.maximum(t1, t2), axis=1)
        t = np.where(tmin > 1e-6, tmin, tmax)
        ok = (tmax >= tmin) & (t > 1e-6) & (t < best_t)
        best_t = np.where(ok, t, best_t)
        best_p = np.where(ok, P + b, best_p)
    best_t = np.where(best_t <= max_range, best_t, np.inf)
    return best_t, best_p


def _depth_view(rng, scene, pose, n_pts, fov_h=60.0, fov_v=45.0, grid=(200, 150), max_range=8.0, max_rounds=60,
                min_range=0.0):
    """Jittered depth-camera ray grid (x forward, y left, z up) from a camera pose;
    misses are re-drawn inside the field of view until n_pts hits are collected.  Hits nearer than
    min_range count as misses (a depth camera's minimum range)."""
    R, t = pose_rt(pose)
    gw, gh = grid
    hits_t, hits_d, hits_p = [], [], []
    got = 0
    for rnd in range(max_rounds):
        if rnd == 0:
            i, j = np.meshgrid(np.arange(gw), np.arange(gh), indexing="ij")
            a = np.radians(-fov_h / 2 + (i.ravel() + rng.uniform(size=i.size)) * fov_h / gw)
            e = np.radians(-fov_v / 2 + (j.ravel() + rng.uniform(size=j.size)) * fov_v / gh)
        else:
            m = max(2 * (n_pts - got), 256)
            a = np.radians(rng.uniform(-fov_h / 2, fov_h / 2, size=m))
            e = np.radians(rng.uniform(-fov_v / 2, fov_v / 2, size=m))
        d_loc = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], axis=1)
        d_w = d_loc @ R.T
        tt, pp = _cast(scene, t, d_w, max_range)
        ok = np.isfinite(tt) & (tt >= min_range)
        hits_t.append(tt[ok]); hits_d.append(d_loc[ok]); hits_p.append(pp[ok])
        got += int(ok.sum())
        if got >= n_pts:
            break
    if got < n_pts:
        return None
    tt = np.concatenate(hits_t)[:n_pts]
    dd = np.concatenate(hits_d)[:n_pts]
    pp = np.concatenate(hits_p)[:n_pts]
    return (tt[:, None] * dd), pp


def _dirichlet_rgb_feats(rng, prim, n_prim, n_classes=20, alpha=0.3, rgb_sigma=0.05):
    lab = rng.dirichlet(np.full(n_classes, alpha), size=n_prim)
    rgb = rng.uniform(0.0, 1.0, size=(n_prim, 3))
    def feats(prim_ids, rng2):
        c = np.clip(rgb[prim_ids] + rng2.normal(scale=rgb_sigma, size=(len(prim_ids), 3)), 0.0, 1.0)
        return np.concatenate([lab[prim_ids], c], axis=1).astype(np.float32)
    return feats


def _unit64_feats(rng, n_prim, n_classes=20, dim=64, sigma=0.1):
    means = rng.normal(size=(n_classes, dim))
    means /= np.linalg.norm(means, axis=1, keepdims=True)
    cls = rng.integers(0, n_classes, size=n_prim)
    def feats(prim_ids, rng2):
        f = means[cls[prim_ids]] + rng2.normal(scale=sigma, size=(len(prim_ids), dim))
        f /= np.linalg.norm(f, axis=1, keepdims=True)
        return f.astype(np.float32)
    return feats


# ----------------------------------------------------------------------------- workloads

def two_view(seed: int = 0, n_points: int = 5000, n_classes: int = 10, ell: float = 0.1,
             n_iter: int = 10, noise: float = 0.01, max_angle_deg: float = 10.0,
             max_trans: float = 0.3) -> Problem:
    """Plane/box scene in a 20 m cube; frame 2 is a noisy rigid copy of frame 1."""
    rng = np.random.default_rng(seed)
    scene = _make_scene(rng)
    x, prim = _surface_sample(rng, scene, n_points)
    cls = rng.integers(0, n_classes, size=scene.n_prim)
    G_R = _rot(_unit(rng), math.radians(rng.uniform(0.0, max_angle_deg)))
    G_t = _unit(rng) * rng.uniform(0.0, max_trans)
    z = x @ G_R.T + G_t + rng.normal(scale=noise, size=x.shape)
    G = pose_from_rt(G_R, G_t)
    gt = np.stack([pose_from_rt(np.eye(3), np.zeros(3)), invert(G)])
    init = np.stack([pose_from_rt(np.eye(3), np.zeros(3))] * 2)
    lab = cls[prim].astype(np.uint16)
    return Problem(
        name="two_view", points=[x.astype(np.float32), z.astype(np.float32)], feat_kind="class",
        feats=[lab.copy(), lab.copy()], D=n_classes, gt_poses=gt, init_poses=init,
        edges=np.array([[0, 1]], dtype=np.int32), ell=ell, n_iter=n_iter,
        recipe=f"two_view seed={seed} N={n_points} classes={n_classes} ell={ell}")


def _trajectory(rng, n_frames, step=0.2, step_deg=5.0, box=4.0):
    p = rng.uniform(-box, box, size=3)
    R = Rotation.random(random_state=int(rng.integers(1 << 31))).as_matrix()
    poses = [pose_from_rt(R, p)]
    for _ in range(n_frames - 1):
        fwd = R[:, 0]
        d = fwd + 0.5 * rng.normal(size=3)
        d /= np.linalg.norm(d)
        p = p + step * d
        R = R @ _rot(_unit(rng), math.radians(step_deg))
        poses.append(pose_from_rt(R, p))
    return np.stack(poses)


def _odometry_like(seed, n_frames, n_points, feat_builder, ell, n_iter, name, sigma_t=0.02, sigma_deg=1.0):
    rng = np.random.default_rng(seed)
    scene = _make_scene(rng, walls=True)
    feats_of = feat_builder(rng, scene.n_prim)
    for _attempt in range(50):
        gt = _trajectory(rng, n_frames)
        views = [_depth_view(rng, scene, gt[k], n_points) for k in range(n_frames)]
        if all(v is not None for v in views):
            break
    else:  # pragma: no cover - the room walls make this unreachable in practice
        raise RuntimeError("could not place a trajectory with enough surface hits")
    pts = [v[0].astype(np.float32) for v in views]
    feats = [feats_of(v[1], rng) for v in views]
    init = np.stack([gt[0]] + [_perturb(rng, gt[k], sigma_t, sigma_deg) for k in range(1, n_frames)])
    edges = np.array([(i, j) for i in range(n_frames) for j in range(i + 1, n_frames)], dtype=np.int32)
    D = feats[0].shape[1]
    return Problem(name=name, points=pts, feat_kind="dense", feats=feats, D=D, gt_poses=gt,
                   init_poses=init, edges=edges, ell=ell, n_iter=n_iter,
                   recipe=f"{name} seed={seed} K={n_frames} N={n_points} D={D} ell={ell}")


def odometry(seed: int = 0, n_frames: int = 8, n_points: int = 30000, ell: float = 0.08, n_iter: int = 15) -> Problem:
    """Depth-camera sliding window: 20-class Dirichlet(0.3) soft label (+) RGB features, D=23."""
    return _odometry_like(seed, n_frames, n_points,
                          lambda rng, n_prim: _dirichlet_rgb_feats(rng, None, n_prim),
                          ell, n_iter, "odometry")


def dense64(seed: int = 0, n_frames: int = 8, n_points: int = 30000, ell: float = 0.08, n_iter: int = 15) -> Problem:
    """As odometry, with 64-dim unit-vector features (per-class mean + N(0, 0.1) jitter)."""
    return _odometry_like(seed, n_frames, n_points,
                          lambda rng, n_prim: _unit64_feats(rng, n_prim),
                          ell, n_iter, "dense64")


# ----------------------------------------------------------------------------- LiDAR street loop

class _Street:
    """Rounded-rectangle loop of 200 m centreline with facades at +-10 m, ground z=0,
    parked cars (boxes) and poles (vertical cylinders)."""

    def __init__(self, rng, n_cars=40, n_poles=30, n_classes=20):
        self.r = 14.0
        self.a, self.b = 36.0, 20.0          # straight lengths; 2a + 2b + 2*pi*r ~= 200 m
        self.length = 2 * self.a + 2 * self.b + 2 * math.pi * self.r
        self.fac_h = 15.0
        s_car = rng.uniform(0, self.length, size=n_cars)
        lat_car = rng.choice([-1.0, 1.0], size=n_cars) * rng.uniform(3.0, 7.0, size=n_cars)
        self.car_c, self.car_R = [], []
        for s, lat in zip(s_car, lat_car):
            p, tang = self.at(s)
            nrm = np.array([-tang[1], tang[0]])
            c2 = p + lat * nrm
            self.car_c.append(np.array([c2[0], c2[1], 0.75]))
            self.car_R.append(_rot([0, 0, 1], math.atan2(tang[1], tang[0])))
        self.car_c = np.array(self.car_c)
        self.car_R = np.array(self.car_R)
        self.car_h = np.array([2.25, 0.9, 0.75])
        s_pole = rng.uniform(0, self.length, size=n_poles)
        lat_pole = rng.choice([-1.0, 1.0], size=n_poles) * 8.5
        self.pole_c = np.array([self.at(s)[0] + l * np.array([-self.at(s)[1][1], self.at(s)[1][0]])
                                for s, l in zip(s_pole, lat_pole)])
        self.pole_r, self.pole_h = 0.15, 6.0
        # primitive ids: 0 ground, 1 inner facade, 2 outer facade, 3.. cars, then poles
        self.n_prim = 3 + n_cars + n_poles
        self.cls = rng.integers(0, n_classes, size=self.n_prim)

    def at(self, s):
        """Centreline point and unit tangent at arc length s (counter-clockwise)."""
        a, b, r = self.a, self.b, self.r
        s = s % self.length
        q = math.pi * r / 2
        segs = [("L", np.array([-a / 2, -b / 2 - r]), np.array([1.0, 0.0]), a),
                ("A", np.array([a / 2, -b / 2]), -math.pi / 2, q),
                ("L", np.array([a / 2 + r, -b / 2]), np.array([0.0, 1.0]), b),
                ("A", np.array([a / 2, b / 2]), 0.0, q),
                ("L", np.array([a / 2, b / 2 + r]), np.array([-1.0, 0.0]), a),
                ("A", np.array([-a / 2, b / 2]), math.pi / 2, q),
                ("L", np.array([-a / 2 - r, b / 2]), np.array([0.0, -1.0]), b),
                ("A", np.array([-a / 2, -b / 2]), math.pi, q)]
        for kind, p0, d, ln in segs:
            if s <= ln:
                if kind == "L":
                    return p0 + s * d, d
                ang = d + s / r
                return p0 + r * np.array([math.cos(ang), math.sin(ang)]), np.array([-math.sin(ang), math.cos(ang)])
            s -= ln
        return self.at(0.0)

    def _facade_hits(self, o, d, offset):
        """2-D intersection of rays with the offset loop (rounded rectangle of corner radius r+offset)."""
        a, b = self.a, self.b
        rho = self.r + offset
        best = np.full(len(d), np.inf)
        dh = d[:, :2]
        oh = o[:2]
        lines = [(1, -(b / 2 + rho), 0, -a / 2, a / 2), (1, b / 2 + rho, 0, -a / 2, a / 2),
                 (0, a / 2 + rho, 1, -b / 2, b / 2), (0, -(a / 2 + rho), 1, -b / 2, b / 2)]
        for ax, val, other, lo, hi in lines:
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (val - oh[ax]) / dh[:, ax]
            w = oh[other] + t * dh[:, other]
            z = o[2] + t * d[:, 2]
            ok = np.isfinite(t) & (t > 1e-6) & (w >= lo) & (w <= hi) & (z >= 0) & (z <= self.fac_h)
            best = np.where(ok & (t < best), t, best)
        for cx, cy in [(a / 2, -b / 2), (a / 2, b / 2), (-a / 2, b / 2), (-a / 2, -b / 2)]:
            c = np.array([cx, cy])
            oc = oh - c
            A = np.sum(dh * dh, axis=1)
            B = 2 * dh @ oc
            C = oc @ oc - rho * rho
            disc = B * B - 4 * A * C
            sq = np.sqrt(np.maximum(disc, 0.0))
            for sgn in (-1.0, 1.0):
                with np.errstate(divide="ignore", invalid="ignore"):
                    t = (-B + sgn * sq) / (2 * A)
                hx = oh[0] + t * dh[:, 0] - cx
                hy = oh[1] + t * dh[:, 1] - cy
                z = o[2] + t * d[:, 2]
                ok = (disc >= 0) & (A > 1e-18) & (t > 1e-6) & (hx * np.sign(cx) >= 0) & (hy * np.sign(cy) >= 0) \
                    & (z >= 0) & (z <= self.fac_h)
                best = np.where(ok & (t < best), t, best)
        return best

    def cast(self, o, d, max_range):
        n = len(d)
        best_t = np.full(n, np.inf)
        best_p = np.full(n, -1, dtype=np.int64)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = -o[2] / d[:, 2]
        ok = (d[:, 2] < -1e-12) & (t > 1e-6)
        best_t = np.where(ok, t, best_t); best_p = np.where(ok, 0, best_p)
        for pid, off in ((1, -10.0), (2, 10.0)):
            t = self._facade_hits(o, d, off)
            ok = t < best_t
            best_t = np.where(ok, t, best_t); best_p = np.where(ok, pid, best_p)
        near = np.linalg.norm(self.car_c[:, :2] - o[:2], axis=1) < max_range + 5
        for k in np.nonzero(near)[0]:
            R = self.car_R[k]
            lo = (o - self.car_c[k]) @ R
            ld = d @ R
            with np.errstate(divide="ignore", invalid="ignore"):
                inv = 1.0 / ld
                t1 = (-self.car_h - lo) * inv
                t2 = (self.car_h - lo) * inv
            tmin = np.nanmax(np.minimum(t1, t2), axis=1)
            tmax = np.nanmin(np.maximum(t1, t2), axis=1)
            ok = (tmax >= tmin) & (tmin > 1e-6) & (tmin < best_t)
            best_t = np.where(ok, tmin, best_t); best_p = np.where(ok, 3 + k, best_p)
        near = np.linalg.norm(self.pole_c - o[:2], axis=1) < max_range + 1
        dh = d[:, :2]
        A = np.sum(dh * dh, axis=1)
        for k in np.nonzero(near)[0]:
            oc = o[:2] - self.pole_c[k]
            B = 2 * dh @ oc
            C = oc @ oc - self.pole_r ** 2
            disc = B * B - 4 * A * C
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (-B - np.sqrt(np.maximum(disc, 0.0))) / (2 * A)
            z = o[2] + t * d[:, 2]
            ok = (disc >= 0) & (A > 1e-18) & (t > 1e-6) & (z >= 0) & (z <= self.pole_h) & (t < best_t)
            best_t = np.where(ok, t, best_t); best_p = np.where(ok, 3 + len(self.car_c) + k, best_p)
        best_t = np.where(best_t <= max_range, best_t, np.inf)
        return best_t, best_p


def lidar(seed: int = 0, n_frames: int = 64, n_points: int = 100_000, ell: float = 0.3, n_iter: int = 10,
          n_beams: int = 64, n_azimuth: int = 1563, max_range: float = 50.0, outlier_frac: float = 0.2,
          flip_frac: float = 0.1, n_classes: int = 20, n_neighbours: int = 6, spacing: float | None = None) -> Problem:
    """Spinning 64-beam LiDAR around a 200 m street loop; 20% outliers, 10% flipped labels,
    each frame paired with its n_neighbours nearest poses (directed edges).  Poses are evenly
    spaced over the loop, or `spacing` metres apart along it."""
    rng = np.random.default_rng(seed)
    st = _Street(rng, n_classes=n_classes)
    gt = []
    for k in range(n_frames):
        p, tang = st.at(k * (st.length / n_frames if spacing is None else spacing))
        R = _rot([0, 0, 1], math.atan2(tang[1], tang[0]))
        gt.append(pose_from_rt(R, np.array([p[0], p[1], 1.8])))
    gt = np.stack(gt)
    elev = np.radians(np.linspace(-15.0, 15.0, n_beams))
    pts, feats = [], []
    for k in range(n_frames):
        R, t = pose_rt(gt[k])
        hits, prims, got = [], [], 0
        for rnd in range(200):
            if rnd == 0:
                e, a = np.meshgrid(elev, np.arange(n_azimuth) * 2 * math.pi / n_azimuth, indexing="ij")
                e, a = e.ravel(), a.ravel()
            else:
                m = max(2 * (n_points - got), 1024)
                e = elev[rng.integers(0, n_beams, size=m)]
                a = rng.uniform(0, 2 * math.pi, size=m)
            d_loc = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], axis=1)
            tt, pp = st.cast(t, d_loc @ R.T, max_range)
            ok = np.isfinite(tt)
            hits.append(tt[ok, None] * d_loc[ok]); prims.append(pp[ok]); got += int(ok.sum())
            if got >= n_points:
                break
        x = np.concatenate(hits)[:n_points]
        pr = np.concatenate(prims)[:n_points]
        lab = st.cls[pr].copy()
        flip = rng.random(n_points) < flip_frac
        lab[flip] = rng.integers(0, n_classes, size=int(flip.sum()))
        n_out = int(round(outlier_frac * n_points))
        oi = rng.choice(n_points, size=n_out, replace=False)
        u = _unit(rng, n_out) * (max_range * rng.random(n_out) ** (1.0 / 3.0))[:, None]
        x[oi] = u
        lab[oi] = rng.integers(0, n_classes, size=n_out)
        pts.append(x.astype(np.float32))
        feats.append(lab.astype(np.uint16))
    init = np.stack([gt[0]] + [_perturb(rng, gt[k], 0.05, 0.5) for k in range(1, n_frames)])
    pos = gt[:, 9:12]
    edges = []
    for i in range(n_frames):
        dist = np.linalg.norm(pos - pos[i], axis=1)
        dist[i] = np.inf
        for j in np.argsort(dist, kind="stable")[:n_neighbours]:
            edges.append((i, int(j)))
    return Problem(name="lidar", points=pts, feat_kind="class", feats=feats, D=n_classes, gt_poses=gt,
                   init_poses=init, edges=np.array(edges, dtype=np.int32), ell=ell, n_iter=n_iter,
                   recipe=f"lidar seed={seed} K={n_frames} N={n_points} ell={ell} outliers={outlier_frac}")


# ----------------------------------------------------------------------------- serving requests

def request(seed: int, k_range=(2, 16), n_range=(5000, 120_000), ells=(0.08, 0.3), n_classes=20,
            n_iter: int = 10, point_scale: float = 1.0) -> Problem:
    """One solve request: K ~ U{2..16} frames, N_m log-uniform points per frame, either K noisy
    rigid copies of a plane/box sample or a depth-camera trajectory (p = 1/2), with 20-class
    Dirichlet soft labels (D = 20); all i<j pairs."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(k_range[0], k_range[1] + 1))
    ell = float(rng.choice(ells))
    lo, hi = math.log(n_range[0]), math.log(n_range[1])
    Ns = [max(16, int(round(math.exp(rng.uniform(lo, hi)) * point_scale))) for _ in range(K)]
    style = "copies" if rng.random() < 0.5 else "trajectory"
    scene = _make_scene(rng, walls=(style == "trajectory"))
    lab = rng.dirichlet(np.full(n_classes, 0.3), size=scene.n_prim)
    if style == "copies":
        x, prim = _surface_sample(rng, scene, max(Ns))
        gt, pts, feats = [pose_from_rt(np.eye(3), np.zeros(3))], [], []
        for k in range(K):
            sel = rng.choice(len(x), size=Ns[k], replace=False) if k else np.arange(Ns[0])
            if k == 0:
                z = x[sel]
            else:
                G_R = _rot(_unit(rng), math.radians(rng.uniform(0, 10)))
                G_t = _unit(rng) * rng.uniform(0, 0.3)
                z = x[sel] @ G_R.T + G_t + rng.normal(scale=0.01, size=(len(sel), 3))
                gt.append(invert(pose_from_rt(G_R, G_t)))
            pts.append(z.astype(np.float32))
            feats.append(lab[prim[sel]].astype(np.float32))
        gt = np.stack(gt)
        init = np.stack([gt[0]] + [_perturb(rng, gt[k], 0.02, 1.0) for k in range(1, K)])
    else:
        for _attempt in range(50):
            gt = _trajectory(rng, K)
            views = [_depth_view(rng, scene, gt[k], Ns[k], min_range=0.3) for k in range(K)]
            if all(v is not None for v in views):
                break
        pts = [v[0].astype(np.float32) for v in views]
        feats = [lab[v[1]].astype(np.float32) for v in views]
        init = np.stack([gt[0]] + [_perturb(rng, gt[k], 0.02, 1.0) for k in range(1, K)])
    edges = np.array([(i, j) for i in range(K) for j in range(i + 1, K)], dtype=np.int32)
    return Problem(name=f"request{seed}", points=pts, feat_kind="dense", feats=feats, D=n_classes,
                   gt_poses=gt, init_poses=init, edges=edges, ell=ell, n_iter=n_iter,
                   recipe=f"request seed={seed} style={style} K={K} N={Ns} ell={ell}")


def make(name: str, seed: int = 0, **kw) -> Problem:
    return {"two_view": two_view, "odometry": odometry, "lidar": lidar, "dense64": dense64}[name](seed=seed, **kw)
