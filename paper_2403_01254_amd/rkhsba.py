"""Thin ctypes binding of the rkhsba C ABI (include/rkhsba.h).

Argument marshalling only: every step of the hot path runs in the HIP
library ``_lib/librkhsba.so``.  Importing this module without the built
library raises, so nothing can silently fall back to a CPU path.

Host inputs are numpy arrays; device inputs are torch CUDA tensors (their
``data_ptr()`` is passed with ``is_device=1``).  PyTorch is only used for
device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librkhsba.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTPD, ESTATE, EBUSY = 0, -1, -2, -3, -4, -5, -6
FEAT_CLASS_ID, FEAT_DENSE_F32, FEAT_DENSE_BF16, FEAT_DENSE_FP8 = 0, 1, 2, 3
_FEAT_NAMES = {"class": FEAT_CLASS_ID, "dense": FEAT_DENSE_F32, "bf16": FEAT_DENSE_BF16, "fp8": FEAT_DENSE_FP8}


class RkhsbaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rkhsba error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("ell", ctypes.c_double),
        ("cutoff_factor", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("damping_rel", ctypes.c_double),
        ("fixed_frame", ctypes.c_int),
        ("clamp_negative_c", ctypes.c_int),
        ("device", ctypes.c_int),
        ("cell_subdiv", ctypes.c_int),
        ("pass_points", ctypes.c_int),
        ("moment_path", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("hessian_fp32", ctypes.c_int),
        ("top_k", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("feat_kind", ctypes.c_int),
        ("D", ctypes.c_int),
        ("max_active", ctypes.c_int),
        ("hbm_budget_bytes", ctypes.c_int64),
        ("pass_points", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("hessian_fp32", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("lanes", ctypes.c_int),
        ("lane_split_entries", ctypes.c_int64),
        ("lane_work_entries", ctypes.c_int64),
        ("lane1_max_active", ctypes.c_int),
        ("lane_split_work", ctypes.c_double),
        ("lane0_weight", ctypes.c_double),
        ("lane1_order", ctypes.c_int),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int),
        ("n_points", ctypes.POINTER(ctypes.c_int64)),
        ("xyz", ctypes.POINTER(ctypes.c_void_p)),
        ("feats", ctypes.POINTER(ctypes.c_void_p)),
        ("is_device", ctypes.c_int),
        ("feat_kind", ctypes.c_int),
        ("D", ctypes.c_int),
        ("poses", ctypes.POINTER(ctypes.c_double)),
        ("E", ctypes.c_int),
        ("edges", ctypes.POINTER(ctypes.c_int32)),
        ("ell", ctypes.c_double),
        ("cutoff_factor", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("damping_rel", ctypes.c_double),
        ("fixed_frame", ctypes.c_int),
        ("clamp_negative_c", ctypes.c_int),
        ("cell_subdiv", ctypes.c_int),
        ("n_iter", ctypes.c_int),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "queued", "batch_iterations",
                                               "max_active", "peak_device_bytes", "pair_evals")]


class EllSchedule(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("ell_init", "ell_min", "ell_max", "step", "elasticity", "tol")] + \
               [("inner_iter", ctypes.c_int), ("max_outer", ctypes.c_int)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"rkhsba HIP library not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.rkhsba_default_options.argtypes = [ctypes.POINTER(Options)]
        L.rkhsba_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Options)]
        L.rkhsba_destroy.argtypes = [vp]
        L.rkhsba_last_error.argtypes = [vp]
        L.rkhsba_last_error.restype = ctypes.c_char_p
        L.rkhsba_build_neighbors.argtypes = [vp, ctypes.c_int, _i64p, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(vp), ctypes.c_int]
        L.rkhsba_eval_loss.argtypes = [vp, _dp, ctypes.c_int, _i32p, _dp, _dp, _i64p]
        L.rkhsba_eval_loss_noalloc.argtypes = [vp, _dp, ctypes.c_int, _i32p, _dp, _dp, _i64p]
        L.rkhsba_accumulate_normal_eqs.argtypes = [vp, _dp, ctypes.c_int, _i32p, _dp, _dp, _dp, _i64p]
        L.rkhsba_gn_step.argtypes = [vp, _dp, ctypes.c_int, _i32p, ctypes.c_int, _dp, _i64p]
        L.rkhsba_export_pairs.argtypes = [vp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p, _i64p]
        L.rkhsba_export_voxels.argtypes = [vp, ctypes.c_int, _i32p, ctypes.POINTER(ctypes.c_uint32), _i32p, _i32p,
                                           _i32p]
        L.rkhsba_export_source_counts.argtypes = [vp, _dp, ctypes.c_int, ctypes.c_int, _i64p]
        L.rkhsba_autotune.argtypes = [vp, ctypes.c_int, _i64p, ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(vp), ctypes.c_int, _dp, ctypes.c_int, _i32p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _dp]
        L.rkhsba_get_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _dp]
        L.rkhsba_server_default_options.argtypes = [ctypes.POINTER(ServerOptions)]
        L.rkhsba_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ServerOptions)]
        L.rkhsba_server_destroy.argtypes = [vp]
        L.rkhsba_server_submit.argtypes = [vp, ctypes.POINTER(Request), _i64p]
        L.rkhsba_server_wait.argtypes = [vp, ctypes.c_int64, ctypes.c_double, _dp, _dp, _i64p, _dp, _dp]
        L.rkhsba_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.rkhsba_server_last_error.argtypes = [vp]
        L.rkhsba_server_last_error.restype = ctypes.c_char_p
        L.rkhsba_ell_gradient.argtypes = [vp, _dp, ctypes.c_int, _i32p, _dp, _dp]
        L.rkhsba_default_ell_schedule.argtypes = [ctypes.POINTER(EllSchedule), ctypes.c_double]
        L.rkhsba_default_ell_schedule.restype = None
        L.rkhsba_gn_lengthscale.argtypes = [vp, _dp, ctypes.c_int, _i32p, ctypes.POINTER(EllSchedule),
                                            ctypes.POINTER(ctypes.c_int), _dp]
        L.rkhsba_track.argtypes = [vp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.POINTER(ctypes.c_int), _dp]
        L.rkhsba_cosine.argtypes = [vp, _dp, ctypes.c_int, ctypes.c_int, _dp]
        L.rkhsba_icosahedral_rotations.argtypes = [_dp]
        L.rkhsba_icosahedral_rotations.restype = None
        L.rkhsba_rotation_search.argtypes = [vp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                             ctypes.POINTER(ctypes.c_int), _dp]
        L.rkhsba_profile_enable.argtypes = [vp, ctypes.c_int]
        L.rkhsba_profile_read.argtypes = [vp, ctypes.c_int, _dp, _i64p, ctypes.c_int]
        _lib = L
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def default_options() -> Options:
    o = Options()
    lib().rkhsba_default_options(ctypes.byref(o))
    return o


class Context:
    """One rkhsba context (one stream, one set of resident frames)."""

    def __init__(self, ell: float, cutoff_factor: float = 3.0, sigma: float = 1.0, damping_rel: float = 1e-10,
                 fixed_frame: int = 0, clamp_negative_c: bool = True, device: int = 0, cell_subdiv: int = 0,
                 pass_points: int = 0, moment_path: int = 0, use_graphs: bool = True, hessian_fp32: bool = False,
                 top_k: int = 0, stream=None):
        o = default_options()
        o.ell, o.cutoff_factor, o.sigma, o.damping_rel = ell, cutoff_factor, sigma, damping_rel
        o.fixed_frame, o.clamp_negative_c, o.device = fixed_frame, int(bool(clamp_negative_c)), device
        o.cell_subdiv, o.pass_points, o.moment_path = cell_subdiv, pass_points, moment_path
        o.use_graphs = int(bool(use_graphs))
        o.hessian_fp32 = int(bool(hessian_fp32))
        o.top_k = int(top_k)
        o.stream = ctypes.c_void_p(int(stream)) if stream else None
        self._h = ctypes.c_void_p()
        rc = lib().rkhsba_create(ctypes.byref(self._h), ctypes.byref(o))
        if rc != OK:
            raise RkhsbaError(rc, "rkhsba_create failed")
        self.K = 0
        self.opts = o

    def close(self):
        if self._h:
            lib().rkhsba_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise RkhsbaError(rc, lib().rkhsba_last_error(self._h).decode())

    @staticmethod
    def _frames(points, feats, feat_kind):
        """Marshals K clouds (numpy host arrays or device tensors) for the C ABI."""
        kind = _FEAT_NAMES[feat_kind] if isinstance(feat_kind, str) else int(feat_kind)
        K = len(points)
        on_device = not isinstance(points[0], np.ndarray)
        keep = []
        if on_device:
            n = np.array([int(p.shape[0]) for p in points], dtype=np.int64)
            xp = [p.data_ptr() for p in points]
            fp = [f.data_ptr() for f in feats]
            D = 0 if kind == FEAT_CLASS_ID else int(feats[0].shape[1])
        else:
            pts = [np.ascontiguousarray(p, dtype=np.float32).reshape(-1, 3) for p in points]
            if kind == FEAT_CLASS_ID:
                fs = [np.ascontiguousarray(f, dtype=np.uint16).reshape(-1) for f in feats]
                D = 0
            else:
                fs = [np.ascontiguousarray(f, dtype=np.float32) for f in feats]
                D = int(fs[0].shape[1])
            keep = [pts, fs]
            n = np.array([len(p) for p in pts], dtype=np.int64)
            xp = [p.ctypes.data for p in pts]
            fp = [f.ctypes.data for f in fs]
        xarr = (ctypes.c_void_p * K)(*xp)
        farr = (ctypes.c_void_p * K)(*fp)
        return K, kind, D, n, xarr, farr, int(on_device), keep

    # -- rkhsba_build_neighbors
    def build_neighbors(self, points, feats, feat_kind="class"):
        """points: K arrays (N,3) float32 (numpy) or CUDA tensors; feats: K arrays of uint16 class
        ids (N,) or float32 rows (N, D)."""
        K, kind, D, n, xarr, farr, dev, keep = self._frames(points, feats, feat_kind)
        rc = lib().rkhsba_build_neighbors(self._h, K, _p(n, ctypes.c_int64), xarr, kind, D, farr, dev)
        del keep
        self._check(rc)
        self.K = K

    # -- rkhsba_autotune
    def autotune(self, points, feats, feat_kind, poses, edges, trials=2):
        """Times every (cell size, sweep size) pair on these frames and leaves the context
        built with the fastest.  Returns (cell_subdiv, pass_points, ms per evaluation)."""
        K, kind, D, n, xarr, farr, dev, keep = self._frames(points, feats, feat_kind)
        self.K = K
        p, e = self._poses(poses), self._edges(edges)
        S, P, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        rc = lib().rkhsba_autotune(self._h, K, _p(n, ctypes.c_int64), xarr, kind, D, farr, dev, _p(p), len(e),
                                   _p(e, ctypes.c_int32), trials, ctypes.byref(S), ctypes.byref(P), ctypes.byref(ms))
        del keep
        self._check(rc)
        return S.value, P.value, ms.value

    # -- rkhsba_get_config
    def config(self):
        """(cell_subdiv, pass_points, points per occupied r_c-cube) of the resident frames."""
        S, P, occ = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(lib().rkhsba_get_config(self._h, ctypes.byref(S), ctypes.byref(P), ctypes.byref(occ)))
        return S.value, P.value, occ.value

    def _poses(self, poses):
        return np.ascontiguousarray(poses, dtype=np.float64).reshape(self.K, 12)

    @staticmethod
    def _edges(edges):
        return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))

    # -- rkhsba_eval_loss
    def eval_loss(self, poses, edges):
        p, e = self._poses(poses), self._edges(edges)
        F = ctypes.c_double()
        Fe = np.zeros(len(e))
        npairs = ctypes.c_int64()
        self._check(lib().rkhsba_eval_loss(self._h, _p(p), len(e), _p(e, ctypes.c_int32), ctypes.byref(F), _p(Fe),
                                           ctypes.byref(npairs)))
        return F.value, Fe, npairs.value

    # -- rkhsba_eval_loss_noalloc
    def eval_loss_noalloc(self, poses, edges):
        """As eval_loss, with no device allocation (the library's static scratch)."""
        p, e = self._poses(poses), self._edges(edges)
        F = ctypes.c_double()
        Fe = np.zeros(len(e))
        npairs = ctypes.c_int64()
        self._check(lib().rkhsba_eval_loss_noalloc(self._h, _p(p), len(e), _p(e, ctypes.c_int32), ctypes.byref(F),
                                                   _p(Fe), ctypes.byref(npairs)))
        return F.value, Fe, npairs.value

    # -- rkhsba_accumulate_normal_eqs
    def accumulate_normal_eqs(self, poses, edges):
        p, e = self._poses(poses), self._edges(edges)
        n = 6 * self.K
        H = np.zeros((n, n))
        b = np.zeros(n)
        F = ctypes.c_double()
        npairs = ctypes.c_int64()
        self._check(lib().rkhsba_accumulate_normal_eqs(self._h, _p(p), len(e), _p(e, ctypes.c_int32), _p(H), _p(b),
                                                       ctypes.byref(F), ctypes.byref(npairs)))
        return H, b, F.value, npairs.value

    # -- rkhsba_gn_step
    def gn_step(self, poses, edges, n_iter):
        p, e = self._poses(poses).copy(), self._edges(edges)
        lpi = np.zeros(n_iter + 1)
        ppi = np.zeros(n_iter + 1, dtype=np.int64)
        self._check(lib().rkhsba_gn_step(self._h, _p(p), len(e), _p(e, ctypes.c_int32), int(n_iter), _p(lpi),
                                         _p(ppi, ctypes.c_int64)))
        return p, lpi, ppi

    # -- rkhsba_export_pairs
    def export_pairs(self, poses, m, n):
        p = self._poses(poses)
        total = ctypes.c_int64()
        null = ctypes.cast(None, _i32p)
        self._check(lib().rkhsba_export_pairs(self._h, _p(p), int(m), int(n), 0, null, ctypes.byref(total)))
        out = np.zeros((max(total.value, 1), 2), dtype=np.int32)
        self._check(lib().rkhsba_export_pairs(self._h, _p(p), int(m), int(n), total.value, _p(out, ctypes.c_int32),
                                              ctypes.byref(total)))
        return out[:total.value]

    # -- rkhsba_export_source_counts
    def export_source_counts(self, poses, m, n, n_points):
        """Pair count of every source point of edge (m, n), from the sweep that sums the pairs."""
        p = self._poses(poses)
        out = np.zeros(int(n_points), dtype=np.int64)
        self._check(lib().rkhsba_export_source_counts(self._h, _p(p), int(m), int(n), _p(out, ctypes.c_int64)))
        return out

    # -- rkhsba_export_voxels
    def export_voxels(self, frame, n_points):
        perm = np.zeros(n_points, dtype=np.int32)
        keys = np.zeros(n_points, dtype=np.uint32)
        org = np.zeros(3, dtype=np.int32)
        dims = np.zeros(3, dtype=np.int32)
        layers = np.zeros(1, dtype=np.int32)
        self._check(lib().rkhsba_export_voxels(self._h, int(frame), _p(perm, ctypes.c_int32),
                                               _p(keys, ctypes.c_uint32), _p(org, ctypes.c_int32),
                                               _p(dims, ctypes.c_int32), _p(layers, ctypes.c_int32)))
        return perm, keys, org, dims, int(layers[0])


    # -- rkhsba_ell_gradient
    def ell_gradient(self, poses, edges):
        """(d_H, d d_H / d ell) at the poses and the context's lengthscale."""
        p, e = self._poses(poses), self._edges(edges)
        d, g = ctypes.c_double(), ctypes.c_double()
        self._check(lib().rkhsba_ell_gradient(self._h, _p(p), len(e), _p(e, ctypes.c_int32), ctypes.byref(d),
                                              ctypes.byref(g)))
        return d.value, g.value

    # -- rkhsba_gn_lengthscale
    def gn_lengthscale(self, poses, edges, **schedule):
        """Inner-outer loop; schedule fields as rkhsba_ell_schedule (defaults from the context's ell).
        Returns (poses, trace rows (ell, F_start, F_end, d_H, g))."""
        sc = EllSchedule()
        lib().rkhsba_default_ell_schedule(ctypes.byref(sc), self.opts.ell)
        for k, v in schedule.items():
            setattr(sc, k, v)
        p = self._poses(poses).copy()
        e = self._edges(edges)
        trace = np.zeros((sc.max_outer, 5))
        n = ctypes.c_int()
        self._check(lib().rkhsba_gn_lengthscale(self._h, _p(p), len(e), _p(e, ctypes.c_int32), ctypes.byref(sc),
                                                ctypes.byref(n), _p(trace)))
        return p, trace[:n.value]

    # -- rkhsba_track / rkhsba_cosine
    def track(self, poses, m, n, max_iter=100, step0=None, step_min=None):
        """Gradient-ascent registration of frame n to frame m.  Returns (poses, accepted steps, F)."""
        p = self._poses(poses).copy()
        s0 = self.opts.ell if step0 is None else step0
        smin = 1e-4 * s0 if step_min is None else step_min
        it, F = ctypes.c_int(), ctypes.c_double()
        self._check(lib().rkhsba_track(self._h, _p(p), int(m), int(n), int(max_iter), float(s0), float(smin),
                                       ctypes.byref(it), ctypes.byref(F)))
        return p, it.value, F.value

    def cosine(self, poses, m, n):
        p = self._poses(poses)
        v = ctypes.c_double()
        self._check(lib().rkhsba_cosine(self._h, _p(p), int(m), int(n), ctypes.byref(v)))
        return v.value

    # -- rkhsba_rotation_search
    def rotation_search(self, poses, m, n, rotations=None):
        """Scores of candidate rotations of frame n about its centroid against frame m.
        Returns (scores, best index, best pose (12,))."""
        p = self._poses(poses)
        if rotations is None:
            nr, rp = 60, None
            rot = None
        else:
            rot = np.ascontiguousarray(rotations, dtype=np.float64).reshape(-1, 9)
            nr, rp = len(rot), _p(rot)
        scores = np.zeros(nr)
        best = ctypes.c_int()
        bp = np.zeros(12)
        self._check(lib().rkhsba_rotation_search(self._h, _p(p), int(m), int(n), 0 if rot is None else nr, rp,
                                                 _p(scores), ctypes.byref(best), _p(bp)))
        return scores, best.value, bp

    # -- rkhsba_profile_enable / rkhsba_profile_read
    def profile_enable(self, on=True):
        self._check(lib().rkhsba_profile_enable(self._h, int(bool(on))))

    def profile_read(self, stage, reset=False):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().rkhsba_profile_read(self._h, int(stage), ctypes.byref(ms), ctypes.byref(n), int(reset)))
        return ms.value, n.value


class Server:
    """Request loop with continuous batching (rkhsba_server_*): submit() queues a whole
    solve and returns a ticket at once; wait() returns its result."""

    def __init__(self, feat_kind="class", D=0, max_active=64, hbm_budget_bytes=0, device=0, pass_points=0,
                 use_graphs=True, hessian_fp32=False, stream=None, lanes=1, lane_split_entries=2_000_000,
                 lane_work_entries=0, lane1_max_active=1, lane_split_work=5e8, lane0_weight=0.25,
                 lane1_order=1):
        o = ServerOptions()
        lib().rkhsba_server_default_options(ctypes.byref(o))
        o.device = device
        o.feat_kind = _FEAT_NAMES[feat_kind] if isinstance(feat_kind, str) else int(feat_kind)
        o.D, o.max_active, o.hbm_budget_bytes = D, max_active, hbm_budget_bytes
        o.pass_points, o.use_graphs = pass_points, int(bool(use_graphs))
        o.hessian_fp32 = int(bool(hessian_fp32))
        o.stream = ctypes.c_void_p(int(stream)) if stream else None
        o.lanes, o.lane_split_entries = int(lanes), int(lane_split_entries)
        o.lane_work_entries = int(lane_work_entries)
        o.lane1_max_active = int(lane1_max_active)
        o.lane_split_work = float(lane_split_work)
        o.lane0_weight = float(lane0_weight)
        o.lane1_order = int(lane1_order)
        self.opts = o
        self._h = ctypes.c_void_p()
        rc = lib().rkhsba_server_create(ctypes.byref(self._h), ctypes.byref(o))
        if rc != OK:
            raise RkhsbaError(rc, "rkhsba_server_create failed")
        self._keep = {}

    def close(self):
        if self._h:
            lib().rkhsba_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, points, feats, poses, edges, ell, n_iter, cutoff_factor=3.0, sigma=1.0, damping_rel=1e-10,
               fixed_frame=0, clamp_negative_c=True, cell_subdiv=0):
        """points/feats as for Context.build_neighbors (host arrays or device tensors, kept
        alive here until wait()).  Returns the ticket."""
        K, kind, D, n, xarr, farr, dev, keep = Context._frames(points, feats, self.opts.feat_kind)
        p = np.ascontiguousarray(poses, dtype=np.float64).reshape(K, 12)
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        r = Request()
        r.K, r.n_points, r.xyz, r.feats, r.is_device = K, _p(n, ctypes.c_int64), xarr, farr, dev
        r.feat_kind, r.D = kind, D
        r.poses, r.E, r.edges = _p(p), len(e), _p(e, ctypes.c_int32)
        r.ell, r.cutoff_factor, r.sigma, r.damping_rel = ell, cutoff_factor, sigma, damping_rel
        r.fixed_frame, r.clamp_negative_c, r.cell_subdiv, r.n_iter = fixed_frame, int(bool(clamp_negative_c)), \
            cell_subdiv, n_iter
        t = ctypes.c_int64()
        rc = lib().rkhsba_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if rc != OK:
            raise RkhsbaError(rc, "rkhsba_server_submit rejected the request")
        self._keep[t.value] = (keep, n, xarr, farr, points, feats, K, n_iter)
        return t.value

    def wait(self, ticket, timeout=-1.0, with_status=False):
        """(poses (K,12), loss per evaluation, pairs per evaluation, latency s, queued s); with_status: the same
        plus the request's status, and RKHSBA_ENOTPD (a non-positive Cholesky pivot, outputs still written) is
        returned instead of raised."""
        keep = self._keep[ticket]
        K, n_iter = keep[6], keep[7]
        poses = np.zeros((K, 12))
        lpi = np.zeros(n_iter + 1)
        ppi = np.zeros(n_iter + 1, dtype=np.int64)
        lat, qs = ctypes.c_double(), ctypes.c_double()
        rc = lib().rkhsba_server_wait(self._h, ticket, float(timeout), _p(poses), _p(lpi), _p(ppi, ctypes.c_int64),
                                      ctypes.byref(lat), ctypes.byref(qs))
        if rc == EBUSY:
            raise TimeoutError(f"request {ticket} not finished within {timeout} s")
        del self._keep[ticket]
        if rc != OK and not (with_status and rc == ENOTPD):
            raise RkhsbaError(rc, lib().rkhsba_server_last_error(self._h).decode())
        if with_status:
            return poses, lpi, ppi, lat.value, qs.value, rc
        return poses, lpi, ppi, lat.value, qs.value

    def stats(self):
        st = ServerStats()
        rc = lib().rkhsba_server_stats_get(self._h, ctypes.byref(st))
        if rc != OK:
            raise RkhsbaError(rc, "rkhsba_server_stats_get failed")
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}


def icosahedral_rotations():
    """The library's 60 icosahedral rotations, (60, 3, 3)."""
    out = np.zeros(60 * 9)
    lib().rkhsba_icosahedral_rotations(_p(out))
    return out.reshape(60, 3, 3)


PROF_BUILD, PROF_BIN, PROF_PAIRS, PROF_PAIRS_LOSS, PROF_FINALIZE, PROF_SOLVE = range(6)
PROF_NAMES = ["build", "bin+sort", "pairs", "pairs(loss)", "finalize", "solve"]


# ABI names, for callers that prefer the C spelling.
def rkhsba_create(**kw) -> Context:
    return Context(**kw)


def rkhsba_build_neighbors(ctx: Context, points, feats, feat_kind="class"):
    return ctx.build_neighbors(points, feats, feat_kind)


def rkhsba_eval_loss(ctx: Context, poses, edges):
    return ctx.eval_loss(poses, edges)


def rkhsba_eval_loss_noalloc(ctx: Context, poses, edges):
    return ctx.eval_loss_noalloc(poses, edges)


def rkhsba_accumulate_normal_eqs(ctx: Context, poses, edges):
    return ctx.accumulate_normal_eqs(poses, edges)


def rkhsba_gn_step(ctx: Context, poses, edges, n_iter):
    return ctx.gn_step(poses, edges, n_iter)


def rkhsba_export_pairs(ctx: Context, poses, m, n):
    return ctx.export_pairs(poses, m, n)


def rkhsba_export_source_counts(ctx: Context, poses, m, n, n_points):
    return ctx.export_source_counts(poses, m, n, n_points)


def rkhsba_export_voxels(ctx: Context, frame, n_points):
    return ctx.export_voxels(frame, n_points)
