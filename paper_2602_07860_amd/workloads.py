"""Seeded synthetic inputs: meshes, per-vertex attributes, camera and motion.

This module holds no rendering arithmetic.  It only builds the inputs that the
renderer and its FP64 reference both consume:

* geodesic spheres (an icosahedron whose faces are split into nu^2 triangles,
  vertices pushed to the unit sphere), optionally displaced radially;
* per-vertex RGB drawn uniformly in [0, 1];
* a look-at perspective camera (eye on +z looking at the origin, camera Z axis
  pointing into the scene) given as a world->camera 3x4 matrix plus the tangent
  of the half field of view (the paper's perspective model, App. I "Camera");
* rigid motions P(t) = R(t) P0 + T(t) over the exposure t in [0, 1]
  (App. I "Motion Parameters", App. L.1 for the parabolic path), sampled at the
  keyframe times t_s = s/S into the [S+1][3][4] matrices the renderer takes.

The standard workloads are built by :func:`make_workload` and :func:`make_batch`.  Every random
quantity comes from ``numpy.random.default_rng(seed)`` in a fixed draw order so
that the same seed gives the same arrays on every machine.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

__all__ = [
    "Motion", "Scene", "geodesic_sphere", "look_at_view", "make_workload",
    "make_target", "make_batch", "plain_start", "square_scene", "single_triangle_scene",
    "SMALL", "MEDIUM", "LARGE", "BATCH", "WORKLOAD_NAMES",
]

# ---------------------------------------------------------------- geometry


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def geodesic_sphere(nu: int):
    """Unit geodesic sphere of frequency ``nu``: 10 nu^2 + 2 vertices, 20 nu^2 faces.

    nu = 2^n reproduces the usual "icosphere subdivided n times" (nu=4: 162 V /
    320 F, nu=32: 10242 V / 20480 F, nu=64: 40962 V / 81920 F).  Faces are
    counter-clockwise seen from outside.  Returns (verts float64 [V,3],
    faces int32 [F,3]).
    """
    if nu < 1:
        raise ValueError("nu must be >= 1")
    iv, ifc = _icosahedron()
    index = {}
    verts: List[np.ndarray] = []

    def vid(weights):
        # canonical key: icosahedron vertex ids with non-zero integer weights
        key = tuple(sorted((int(a), int(w)) for a, w in weights if w != 0))
        got = index.get(key)
        if got is None:
            pos = np.zeros(3)
            for a, w in key:
                pos += iv[a] * (w / nu)
            pos /= np.linalg.norm(pos)
            got = len(verts)
            index[key] = got
            verts.append(pos)
        return got

    faces = []
    for a, b, c in ifc:
        grid = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                grid[(i, j)] = vid(((a, nu - i - j), (b, i), (c, j)))
        for i in range(nu):
            for j in range(nu - i):
                faces.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < nu - 1:
                    faces.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int32)


def look_at_view(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World->camera 3x4 matrix.  Camera axes: X right, Y up, Z from the eye
    towards the target, so visible points have Z > 0 (SoftRas convention, which
    the paper follows for its camera in App. I)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    upv = np.asarray(up, np.float64)
    x = np.cross(z, upv)
    if np.linalg.norm(x) < 1e-12:
        x = np.cross(z, np.array([0.0, 0.0, 1.0]))
    x /= np.linalg.norm(x)
    y = np.cross(x, z)
    r = np.stack([x, y, z])
    t = -r @ eye
    return np.concatenate([r, t[:, None]], axis=1)


def _rodrigues(axis, angle):
    k = np.asarray(axis, np.float64)
    k = k / np.linalg.norm(k)
    kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) * math.cos(angle) + math.sin(angle) * kx + (1 - math.cos(angle)) * np.outer(k, k)


# ------------------------------------------------------------------ motion


@dataclasses.dataclass
class Motion:
    """Rigid motion over the exposure.  ``matrix(t)`` is the 3x4 transform that
    takes a rest vertex P0 to P(t) = R(t) P0 + T(t).

    kind:
      * "translate": R = I, T(t) = (t - 0.5) * trans (centred straight path)
      * "rotate":    R = rotation about ``axis`` by 2*pi*revs*t, T = (t-0.5)*trans
      * "parabolic": App. L.1 path: R_y(pi t) as printed there, then
                     T(t) = (s, -4 s^2 + 0.5, s) with s = 0.5 - t
    """
    kind: str = "translate"
    trans: tuple = (0.0, 0.0, 0.0)
    axis: tuple = (0.0, 1.0, 0.0)
    revs: float = 0.0

    def matrix(self, t: float) -> np.ndarray:
        m = np.zeros((3, 4))
        if self.kind == "parabolic":
            th = math.pi * t
            c, s_ = math.cos(th), math.sin(th)
            # x_rot = x c + z s ; z_rot = -x s + z c  (App. L.1)
            m[:, :3] = np.array([[c, 0, s_], [0, 1, 0], [-s_, 0, c]])
            s = 0.5 - t
            m[:, 3] = (s, -4.0 * s * s + 0.5, s)
            return m
        if self.kind == "rotate" and self.revs != 0.0:
            m[:, :3] = _rodrigues(self.axis, 2.0 * math.pi * self.revs * t)
        else:
            m[:, :3] = np.eye(3)
        m[:, 3] = (t - 0.5) * np.asarray(self.trans, np.float64)
        return m

    def keyframes(self, num_segments: int) -> np.ndarray:
        """[S+1][3][4] transforms at t_s = s/S."""
        s = num_segments
        return np.stack([self.matrix(i / s) for i in range(s + 1)])


# ------------------------------------------------------------------- scene


@dataclasses.dataclass
class Scene:
    verts: np.ndarray        # float32 [V,3] rest positions (world)
    faces: np.ndarray        # int32   [F,3]
    attrs: np.ndarray        # float32 [V,C] per-vertex attributes (RGB)
    motion: Motion
    num_segments: int        # S
    view: np.ndarray         # float32 [3,4] world->camera
    tan_half_fov: float
    width: int
    height: int
    num_subframes: int       # K
    name: str = ""

    @property
    def keyframe_model(self) -> np.ndarray:
        """float32 [S+1][3][4] keyframe transforms at t_s = s/S."""
        return self.motion.keyframes(self.num_segments).astype(np.float32)

    def with_(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


DEFAULT_EYE_DIST = 4.0
DEFAULT_FOV_DEG = 40.0
# Named workloads (mesh, resolution, sub-frames, motion).
SMALL = "ico2-64px-k16-translate40"              # 162 V / 320 F
MEDIUM = "ico5-256px-k64-rotate3"                # 10242 V / 20480 F
LARGE = "ico6-1024px-k512-rotate5-translate200"  # 40962 V / 81920 F
BATCH = "batch32-mixed"
WORKLOAD_NAMES = [SMALL, MEDIUM, LARGE, BATCH]


def _camera(eye_dist=DEFAULT_EYE_DIST, fov_deg=DEFAULT_FOV_DEG):
    view = look_at_view((0.0, 0.0, eye_dist))
    return view.astype(np.float32), math.tan(math.radians(fov_deg) / 2.0)


def px_to_world_x(px: float, width: int, depth: float, tan_half_fov: float) -> float:
    """World distance parallel to the image plane at camera depth ``depth`` that
    spans ``px`` pixels of an image ``width`` pixels wide (NDC spans 2 units)."""
    return px * (2.0 / width) * depth * tan_half_fov


def _multi_octave(unit: np.ndarray, rng) -> np.ndarray:
    r = np.ones(len(unit))
    for o in range(4):
        amp = 0.04 * 2.0 ** (-o)
        acc = np.zeros(len(unit))
        for _ in range(8):
            k = rng.normal(size=3)
            k /= np.linalg.norm(k)
            ph = rng.uniform(0.0, 2.0 * math.pi)
            acc += np.sin(3.0 * 2.0 ** o * (unit @ k) + ph)
        r += amp * acc / math.sqrt(8.0)
    return r


def displaced_sphere(nu: int, seed: int, sigma: float = 0.02, octaves: bool = False):
    """Geodesic sphere with radial displacement and U[0,1] RGB.  Draw order
    from default_rng(seed): displacement first, then colours, so the same seed
    always gives the same mesh and colours."""
    v, f = geodesic_sphere(nu)
    rng = np.random.default_rng(seed)
    if octaves:
        r = _multi_octave(v, rng)
    elif sigma > 0:
        r = 1.0 + sigma * rng.normal(size=len(v))
    else:
        r = np.ones(len(v))
    cols = rng.uniform(0.0, 1.0, size=(len(v), 3))
    return (v * r[:, None]).astype(np.float32), f, cols.astype(np.float32), rng


def make_workload(name: str, seed: Optional[int] = None, **overrides) -> Scene:
    """The named synthetic single-scene workloads.

    SMALL : nu=4 sphere (162 V / 320 F), 64x64, K=16, +x translation over
            40 px, S=1.  Colours seed 0.
    MEDIUM: nu=32 sphere (10242 V / 20480 F), r = 1 + 0.02 N(0,1), 256x256,
            K=64, 3 revolutions about a random axis, S = 12 per revolution = 36.
            Seed 1 (its shape-recovery target uses seed 2).
    LARGE : nu=64 sphere (40962 V / 81920 F) with multi-octave displacement,
            1024x1024, K=512, 5 revolutions plus a 200 px translation, S = 60.
            Seed 4.
    """
    view, tanf = _camera()
    if name == SMALL:
        v, f, c, _ = displaced_sphere(4, 0 if seed is None else seed, sigma=0.0)
        dx = px_to_world_x(40, 64, DEFAULT_EYE_DIST, tanf)
        sc = Scene(v, f, c, Motion("translate", trans=(dx, 0.0, 0.0)), 1, view, tanf,
                   64, 64, 16, name)
    elif name == MEDIUM:
        v, f, c, rng = displaced_sphere(32, 1 if seed is None else seed, sigma=0.02)
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        sc = Scene(v, f, c, Motion("rotate", axis=tuple(axis), revs=3.0), 36, view, tanf,
                   256, 256, 64, name)
    elif name == LARGE:
        v, f, c, rng = displaced_sphere(64, 4 if seed is None else seed, octaves=True)
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        dx = px_to_world_x(200, 1024, DEFAULT_EYE_DIST, tanf)
        sc = Scene(v, f, c, Motion("rotate", axis=tuple(axis), revs=5.0, trans=(dx, 0.0, 0.0)),
                   60, view, tanf, 1024, 1024, 512, name)
    else:
        raise ValueError(f"unknown single-scene workload {name!r}")
    return sc.with_(**overrides) if overrides else sc


def make_target(sc: Scene, seed: int) -> Scene:
    """Same motion/camera as ``sc`` with a second seeded displacement and
    colours (the shape-recovery target)."""
    nu = int(round(math.sqrt(len(sc.faces) / 20)))
    octaves = sc.name == LARGE
    v, f, c, _ = displaced_sphere(nu, seed, sigma=0.02, octaves=octaves)
    assert np.array_equal(f, sc.faces)
    return sc.with_(verts=v, attrs=c)


def plain_start(sc: Scene, grey: float = 0.5) -> Scene:
    """Start of a shape-recovery loop toward ``sc``: the undisplaced geodesic
    sphere of the same frequency (same faces, unit radius) with every vertex
    attribute set to ``grey``, under the same motion and camera."""
    nu = int(round(math.sqrt(len(sc.faces) / 20)))
    v, f = geodesic_sphere(nu)
    assert np.array_equal(f, sc.faces)
    return sc.with_(verts=v.astype(np.float32), attrs=np.full_like(sc.attrs, grey, dtype=np.float32),
                    name=sc.name + "-plain-start")


def make_batch(seed: int = 3, n: int = 32) -> List[Scene]:
    """32 instances: F* log-uniform in [1e3, 4e4] -> nu = max(7, round(sqrt(F*/20))),
    r = 1 + 0.02 N(0,1), resolution from {128, 256, 512}^2, K ~ U{32..256},
    half translation (random in-plane direction, 20-80 % of the width) and half
    rotation (random axis, revs ~ U[1, 5], S = 12 ceil(revs))."""
    view, tanf = _camera()
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        fstar = math.exp(rng.uniform(math.log(1e3), math.log(4e4)))
        nu = max(7, int(round(math.sqrt(fstar / 20.0))))
        res = int(rng.choice([128, 256, 512]))
        k = int(rng.integers(32, 257))
        translate = bool(rng.uniform() < 0.5)
        inst_seed = int(rng.integers(0, 2 ** 31 - 1))
        v, f, c, irng = displaced_sphere(nu, inst_seed, sigma=0.02)
        if translate:
            ang = rng.uniform(0, 2 * math.pi)
            frac = rng.uniform(0.2, 0.8)
            d = px_to_world_x(frac * res, res, DEFAULT_EYE_DIST, tanf)
            mo = Motion("translate", trans=(d * math.cos(ang), d * math.sin(ang), 0.0))
            s = 1
        else:
            axis = rng.normal(size=3)
            axis /= np.linalg.norm(axis)
            revs = rng.uniform(1.0, 5.0)
            mo = Motion("rotate", axis=tuple(axis), revs=revs)
            s = 12 * int(math.ceil(revs))
        out.append(Scene(v, f, c, mo, s, view, tanf, res, res, k, f"batch-inst{b}"))
    return out


SWEEP_EYE_DIST = 2.232       # App. I camera distance
SWEEP_FOV_DEG = 60.0         # App. I half field of view 30 degrees


def make_sweep(seed: int = 50, n: int = 50, num_subframes: int = 50) -> List[Scene]:
    """Stand-in for the speed comparison's models (Sec. 4.2: 50 models of
    5536 faces on average, 128x128 front view, linear translation): n
    geodesic spheres nu = 17 (5780 faces) with r = 1 + 0.02 N(0,1) and U[0,1]
    colours, scaled so that the largest vertex norm is 1 and rotated about
    the x axis by an angle from U[-90, 90] degrees (App. I object
    initialisation), moving as x(t) = x0 + (0.5 - t) (App. I translation),
    seen from distance 2.232 with a 30-degree half field of view; K
    sub-frames, one linear segment."""
    view, tanf = _camera(SWEEP_EYE_DIST, SWEEP_FOV_DEG)
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        v, f, c, _ = displaced_sphere(17, int(rng.integers(0, 2 ** 31 - 1)), sigma=0.02)
        v = v.astype(np.float64) / np.linalg.norm(v, axis=1).max()
        a = math.radians(rng.uniform(-90.0, 90.0))
        rx = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
        v = (v @ rx.T).astype(np.float32)
        out.append(Scene(v, f, c, Motion("translate", trans=(-1.0, 0.0, 0.0)), 1, view, tanf, 128, 128,
                         num_subframes, f"sweep-model{b}"))
    return out


def uv_sphere(rings: int = 30, segments: int = 45, radius: float = 1.0):
    """Closed latitude-longitude sphere: two poles plus `rings` rings of
    `segments` vertices; 30 x 45 gives 1352 vertices and 2700 faces, the size
    of the paper's deformation template (App. J).  Faces wind outward."""
    v = [(0.0, 0.0, radius)]
    for i in range(1, rings + 1):
        th = math.pi * i / (rings + 1)
        for j in range(segments):
            ph = 2.0 * math.pi * j / segments
            v.append((radius * math.sin(th) * math.cos(ph), radius * math.sin(th) * math.sin(ph),
                      radius * math.cos(th)))
    v.append((0.0, 0.0, -radius))
    south = len(v) - 1
    ring = lambda i, j: 1 + (i - 1) * segments + (j % segments)
    f = []
    for j in range(segments):
        f.append((0, ring(1, j), ring(1, j + 1)))
        f.append((south, ring(rings, j + 1), ring(rings, j)))
    for i in range(1, rings):
        for j in range(segments):
            a, b, c, d = ring(i, j), ring(i, j + 1), ring(i + 1, j), ring(i + 1, j + 1)
            f.append((a, c, d))
            f.append((a, d, b))
    return np.asarray(v, np.float32), np.asarray(f, np.int32)


MULTIVIEW_ELEVATIONS = (-60.0, -30.0, 0.0, 30.0, 60.0)                      # App. I
MULTIVIEW_AZIMUTHS = (-315.0, -270.0, -225.0, -180.0, -135.0, -90.0, -45.0, 0.0)


def multiview_cameras(dist: float = SWEEP_EYE_DIST):
    """The 40 viewpoints of the translational recovery (App. I): eye at
    d (cos phi cos theta, cos phi sin theta, sin phi) for the 5 elevations phi
    and 8 azimuths theta, looking at the origin.  Reading: the elevation is
    measured towards +z, so +z is the up direction of every view."""
    out = []
    for ph in MULTIVIEW_ELEVATIONS:
        for th in MULTIVIEW_AZIMUTHS:
            a, b = math.radians(ph), math.radians(th)
            eye = (dist * math.cos(a) * math.cos(b), dist * math.cos(a) * math.sin(b), dist * math.sin(a))
            out.append(look_at_view(eye, up=(0.0, 0.0, 1.0)).astype(np.float32))
    return out


def make_multiview(seed: int = 60, num_subframes: int = 64, res: int = 128):
    """Translational recovery set-up (Sec. 5.1, App. I-J): the target is a
    multi-octave displaced nu=17 sphere with U[0,1] colours (stand-in for a
    ShapeNet object), scaled to largest vertex norm 1 and rotated about x by
    U[-90, 90] degrees, moving as x(t) = x0 + (0.5 - t), seen from the 40
    viewpoints at res x res with K sub-frames; the template is the 1352-vertex
    sphere of radius 0.6 with grey colours.  Returns (target Scene, template
    Scene, list of 40 view matrices); the Scenes carry the first view."""
    view0, tanf = _camera(SWEEP_EYE_DIST, SWEEP_FOV_DEG)
    v, f, c, rng = displaced_sphere(17, seed, octaves=True)
    v = v.astype(np.float64) / np.linalg.norm(v, axis=1).max()
    a = math.radians(rng.uniform(-90.0, 90.0))
    rx = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    v = (v @ rx.T).astype(np.float32)
    views = multiview_cameras()
    mo = Motion("translate", trans=(-1.0, 0.0, 0.0))
    target = Scene(v, f, c, mo, 1, views[0], tanf, res, res, num_subframes, "multiview-target")
    tv, tf = uv_sphere(radius=0.6)
    template = Scene(tv, tf, np.full((len(tv), 3), 0.5, np.float32), mo, 1, views[0], tanf, res, res,
                     num_subframes, "multiview-template")
    return target, template, views


def subframe_times(K: int) -> np.ndarray:
    """t_k = k/(K-1) (Sec. 3.2); a single sub-frame sits at t = 0."""
    return np.zeros(1) if K == 1 else np.arange(K, dtype=np.float64) / (K - 1)


# ------------------------------------------------------- small test scenes


def square_scene(center_px=(0.0, 0.0), half_px=8.0, depth=4.0, shift_px=10.0,
                 width=64, height=64, k=16, color=(0.25, 0.5, 0.75), segments=1,
                 fov_deg=DEFAULT_FOV_DEG) -> Scene:
    """Flat-coloured square (two triangles) facing the camera at camera depth
    ``depth``, translating parallel to the image plane by ``shift_px`` pixels
    along +x over the exposure.  ``center_px`` offsets the square's centre (in
    pixels, +y up) from the image centre at t = 0.5."""
    view, tanf = _camera(DEFAULT_EYE_DIST, fov_deg)
    to_w = lambda p: px_to_world_x(p, width, depth, tanf)
    z = DEFAULT_EYE_DIST - depth
    cx, cy, h = to_w(center_px[0]), to_w(center_px[1]) * width / height, to_w(half_px)
    hy = h * width / height
    v = np.array([[cx - h, cy - hy, z], [cx + h, cy - hy, z], [cx + h, cy + hy, z],
                  [cx - h, cy + hy, z]], np.float32)
    f = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    c = np.tile(np.asarray(color, np.float32), (4, 1))
    mo = Motion("translate", trans=(to_w(shift_px), 0.0, 0.0))
    return Scene(v, f, c, mo, segments, view, tanf, width, height, k, "square")


def single_triangle_scene(verts_world, colors=None, width=32, height=32, k=1,
                          motion: Optional[Motion] = None, segments=1) -> Scene:
    view, tanf = _camera()
    v = np.asarray(verts_world, np.float32).reshape(3, 3)
    c = np.eye(3, dtype=np.float32) if colors is None else np.asarray(colors, np.float32)
    return Scene(v, np.array([[0, 1, 2]], np.int32), c, motion or Motion("translate"),
                 segments, view, tanf, width, height, k, "triangle")
