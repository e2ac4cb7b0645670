"""ctypes wrapper of the FP64 reference renderer in ``oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg.  Inputs are converted to float64 exactly
(float32 -> float64 is exact), so the reference sees the very same scene the
GPU path sees.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

from . import build as _build

_lib = None


class _Scene(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int), ("F", ctypes.c_int), ("C", ctypes.c_int), ("S", ctypes.c_int),
        ("K", ctypes.c_int), ("W", ctypes.c_int), ("H", ctypes.c_int),
        ("verts", ctypes.c_void_p), ("faces", ctypes.c_void_p), ("attrs", ctypes.c_void_p),
        ("model", ctypes.c_void_p), ("model_sub", ctypes.c_void_p), ("view", ctypes.c_void_p),
        ("tan_half_fov", ctypes.c_double), ("delta", ctypes.c_double), ("eps_cutoff", ctypes.c_double),
        ("solver", ctypes.c_int), ("motion", ctypes.c_int), ("distance", ctypes.c_int),
        ("stop_grad_sigma", ctypes.c_int), ("adj_wmin", ctypes.c_double), ("nthreads", ctypes.c_int),
        ("row_begin", ctypes.c_int), ("row_end", ctypes.c_int), ("row_step", ctypes.c_int),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_render.restype = ctypes.c_int
        L.orc_render.argtypes = [ctypes.POINTER(_Scene)] + [ctypes.c_void_p] * 10
        L.orc_decisions_new.restype = ctypes.c_void_p
        L.orc_decisions_free.argtypes = [ctypes.c_void_p]
        L.orc_keyframes.argtypes = [ctypes.POINTER(_Scene), ctypes.c_void_p]
        L.orc_fast_coeffs.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_double] * 2 + [ctypes.c_void_p] * 4
        L.orc_closest_point.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.orc_schedule_export.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 3
        L.orc_sizeof_scene.restype = ctypes.c_int
        assert L.orc_sizeof_scene() == ctypes.sizeof(_Scene), "scene struct layout mismatch"
        _lib = L
    return _lib


class _Bounds(ctypes.Structure):
    _fields_ = [("image_lo", ctypes.c_void_p), ("image_hi", ctypes.c_void_p), ("slack_kf", ctypes.c_void_p),
                ("slack_verts", ctypes.c_void_p), ("slack_attrs", ctypes.c_void_p)]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Decisions:
    """Opaque record of every discrete decision of one render (winner per
    (pixel, sub-frame), contributing background faces with their edge and
    clamp state), replayed to evaluate the frozen-decision surrogate."""

    def __init__(self):
        self.ptr = lib().orc_decisions_new()

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_decisions_free(self.ptr)
            self.ptr = None


@dataclasses.dataclass
class Result:
    image: np.ndarray                  # [C+1, H, W] float64
    flags: Optional[np.ndarray]        # [H, W] int32: guard-band sub-frames per pixel
    counters: Optional[dict]
    grad_verts: Optional[np.ndarray]   # [V, 3]
    grad_attrs: Optional[np.ndarray]   # [V, C]
    grad_kf: Optional[np.ndarray]      # [S+1, V, 2]
    decisions: Optional[Decisions]
    # guard band (bounds=True): range of the image over the decisions a
    # float32 evaluation could take the other way, and per-component bounds
    # on how far those decisions can move the gradient
    image_lo: Optional[np.ndarray] = None      # [C+1, H, W]
    image_hi: Optional[np.ndarray] = None
    slack_verts: Optional[np.ndarray] = None   # [V, 3]
    slack_attrs: Optional[np.ndarray] = None   # [V, C]
    slack_kf: Optional[np.ndarray] = None      # [S+1, V, 2]


COUNTER_NAMES = ["bbox_pairs", "cover_pairs", "fg_pixsub", "bg_pixsub", "bg_pairs",
                 "setup_triples", "flagged_pixsub", "skipped_pairs", "alt_value_pixsub",
                 "alt_pixsub", "unbounded_pixsub", "bg_pairs_live"]


def schedule(k: int, K: int, S: int):
    s = ctypes.c_int()
    tau = ctypes.c_double()
    X = ctypes.c_int()
    lib().orc_schedule_export(k, K, S, ctypes.byref(s), ctypes.byref(tau), ctypes.byref(X))
    return s.value, tau.value, X.value


def _subframe_times(K: int) -> np.ndarray:
    # t_k = k/(K-1) (Sec. 3.2); a single sub-frame sits at t = 0
    return np.zeros(1) if K == 1 else np.arange(K, dtype=np.float64) / (K - 1)


def _scene_struct(sc, keep: list, **kw) -> _Scene:
    verts = np.ascontiguousarray(sc.verts, np.float64)
    faces = np.ascontiguousarray(sc.faces, np.int32)
    attrs = np.ascontiguousarray(sc.attrs, np.float64)
    model = np.ascontiguousarray(np.asarray(sc.keyframe_model, np.float32), np.float64)
    view = np.ascontiguousarray(np.asarray(sc.view, np.float32), np.float64)
    keep += [verts, faces, attrs, model, view]
    st = _Scene()
    st.V, st.F, st.C = len(verts), len(faces), attrs.shape[1]
    st.S, st.K, st.W, st.H = sc.num_segments, sc.num_subframes, sc.width, sc.height
    st.verts, st.faces, st.attrs = _p(verts), _p(faces), _p(attrs)
    st.model, st.view = _p(model), _p(view)
    # the GPU receives tan(half fov) as a float32; use that same value
    st.tan_half_fov = float(np.float32(sc.tan_half_fov))
    st.model_sub = None
    if kw.get("motion") == 1:
        sub = np.stack([sc.motion.matrix(t) for t in _subframe_times(sc.num_subframes)])
        sub = np.ascontiguousarray(sub, np.float64)
        keep.append(sub)
        st.model_sub = _p(sub)
    for k, v in kw.items():
        setattr(st, k, v)
    return st


def render(sc, *, solver: str = "naive", motion: str = "segment", distance: str = "keyframe",
           delta: float = 1e-4, eps_cutoff: float = 1e-8, grad_image: Optional[np.ndarray] = None,
           flags: bool = False, counters: bool = False, rows=None, nthreads: int = 0,
           record: bool = False, replay: Optional[Decisions] = None,
           stop_grad_sigma: bool = False, bounds: bool = False, adj_wmin: float = 0.0) -> Result:
    """Render ``sc`` (a workloads.Scene) in FP64.

    solver: "naive" (per-sub-frame 3x3 solve) or "fast" (App. B coefficients)
    motion: "segment" (linear between keyframes) or "exact" (project M(t_k) P0)
    distance: "keyframe" (eq 13) or "exact" (eq 12)
    rows: None (all) or (begin, end, step) to render a subset of pixel rows
    grad_image: dL/dI [C+1, H, W]; returns dL/d(verts, attrs, keyframes)
    bounds: also return the guard band's image range and gradient bounds
    adj_wmin: leave out of the adjoint the background terms whose derivative
        weight prod_{m != j}(1 - A_m) A_j is below this, and the (pixel,
        sub-frame)s whose bound on those weights is (0: exact adjoint)
    """
    keep: list = []
    rb, re, rs = (0, 0, 1) if rows is None else rows
    st = _scene_struct(sc, keep, solver={"naive": 0, "fast": 1}[solver],
                       motion={"segment": 0, "exact": 1}[motion],
                       distance={"keyframe": 0, "exact": 1}[distance],
                       delta=float(np.float32(delta)), eps_cutoff=float(eps_cutoff),
                       stop_grad_sigma=int(stop_grad_sigma), adj_wmin=float(adj_wmin), nthreads=int(nthreads),
                       row_begin=rb, row_end=re, row_step=rs)
    C, H, W, V, S = st.C, st.H, st.W, st.V, st.S
    image = np.zeros((C + 1, H, W), np.float64)
    fl = np.zeros((H, W), np.int32) if flags else None
    cnt = np.zeros(len(COUNTER_NAMES), np.float64) if counters else None
    gi = gv = ga = gk = None
    if grad_image is not None:
        gi = np.ascontiguousarray(grad_image, np.float64).reshape(C + 1, H, W)
        gv = np.zeros((V, 3), np.float64)
        ga = np.zeros((V, C), np.float64)
        gk = np.zeros((S + 1, V, 2), np.float64)
    dec = Decisions() if record else None
    bd = None
    lo = hi = sv = sa = sk = None
    if bounds:
        lo, hi = np.zeros_like(image), np.zeros_like(image)
        if grad_image is not None:
            sv, sa, sk = np.zeros((V, 3)), np.zeros((V, C)), np.zeros((S + 1, V, 2))
        bd = _Bounds(_p(lo), _p(hi), _p(sk), _p(sv), _p(sa))
    rc = lib().orc_render(ctypes.byref(st), _p(image), _p(fl), _p(cnt), _p(gi), _p(gk), _p(gv), _p(ga),
                          dec.ptr if dec else None, replay.ptr if replay else None,
                          ctypes.byref(bd) if bd is not None else None)
    if rc != 0:
        raise ValueError(f"oracle render rejected its arguments (code {rc})")
    cd = dict(zip(COUNTER_NAMES, cnt.tolist())) if cnt is not None else None
    return Result(image, fl, cd, gv, ga, gk, dec, lo, hi, sv, sa, sk)


def keyframes(sc) -> np.ndarray:
    """[S+1, V, 3] keyframe (x_ndc, y_ndc, camera depth) in FP64."""
    keep: list = []
    st = _scene_struct(sc, keep)
    out = np.zeros((sc.num_segments + 1, len(sc.verts), 3), np.float64)
    lib().orc_keyframes(ctypes.byref(st), _p(out))
    return out


def fast_coeffs(x0, y0, x1, y1, u, v):
    """App. B coefficients (A1, A2, A3 as 3-vectors, a = (a1, a2, a3))."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x0, y0, x1, y1)]
    outs = [np.zeros(3) for _ in range(4)]
    lib().orc_fast_coeffs(*[_p(a) for a in arrs], float(u), float(v), *[_p(o) for o in outs])
    return tuple(outs)


def closest_point(tri, q):
    """Barycentric weights of the closest point of triangle tri [3,2] to q
    by the three clamped edge projections of App. B."""
    t = np.ascontiguousarray(tri, np.float64).reshape(3, 2)
    w = np.zeros(3)
    lib().orc_closest_point(_p(t), float(q[0]), float(q[1]), _p(w))
    return w
