"""Pins of the oracle's guard band and of the pair counters that feed the
roofline figures, against quantities computed here from scratch (pinhole
projection, barycentrics, textbook point-triangle distances, brute-force
counting) rather than by the oracle."""
import math

import numpy as np

import oracle
from paper_2602_07860_amd import workloads as wl

DELTA = 1e-4
DMAX = DELTA * math.log(1e8)      # A = exp(-d/delta) >= 1e-8


def _project(sc):
    """[S+1, V, 2] keyframe positions in normalized image coordinates: camera
    transform of the keyframe model, x = X/(Z tan a), y = Y/(Z tan a)."""
    model = np.asarray(sc.keyframe_model, np.float32).astype(np.float64)
    view = np.asarray(sc.view, np.float32).astype(np.float64)
    P = sc.verts.astype(np.float64)
    tanf = float(np.float32(sc.tan_half_fov))
    out = []
    for M in model:
        w = P @ M[:, :3].T + M[:, 3]
        c = w @ view[:, :3].T + view[:, 3]
        out.append(np.stack([c[:, 0] / (c[:, 2] * tanf), c[:, 1] / (c[:, 2] * tanf)], 1))
    return np.array(out)


def _centres(W, H):
    return (2 * np.arange(W) + 1 - W) / W, (H - 2 * np.arange(H) - 1) / H


def _seg_dist2(p, a, b):
    e = b - a
    t = np.clip(np.dot(p - a, e) / np.dot(e, e), 0.0, 1.0)
    q = a + t * e
    return float(np.dot(p - q, p - q))


def _bary(p, T):
    (x0, y0), (x1, y1), (x2, y2) = T
    D = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
    w1 = ((p[0] - x0) * (y2 - y0) - (x2 - x0) * (p[1] - y0)) / D
    w2 = ((x1 - x0) * (p[1] - y0) - (p[0] - x0) * (y1 - y0)) / D
    return np.array([1 - w1 - w2, w1, w2])


def _brute_counts(sc):
    """Counters of a single-segment scene translating parallel to the image
    plane, where the keyframe closest point (eq 13) is the textbook one."""
    assert sc.num_segments == 1
    kf = _project(sc)
    W, H, K = sc.width, sc.height, sc.num_subframes
    us, vs = _centres(W, H)
    ts = np.zeros(1) if K == 1 else np.arange(K) / (K - 1)
    n = dict(bbox_pairs=0, cover_pairs=0, fg_pixsub=0, bg_pairs=0, setup_triples=0)
    seen = set()
    for k, t in enumerate(ts):
        pos = (1 - t) * kf[0] + t * kf[1]
        tris = [pos[f] for f in sc.faces]
        for r, v in enumerate(vs):
            for c, u in enumerate(us):
                p = np.array([u, v])
                cov = 0
                for fi, T in enumerate(tris):
                    if T[:, 0].min() <= u <= T[:, 0].max() and T[:, 1].min() <= v <= T[:, 1].max():
                        n["bbox_pairs"] += 1
                        seen.add((r, c, fi))
                    cov += int(_bary(p, T).min() >= 0)
                n["cover_pairs"] += cov
                if cov:
                    n["fg_pixsub"] += 1
                    continue
                for T in tris:
                    d = min(_seg_dist2(p, T[i], T[(i + 1) % 3]) for i in range(3))
                    n["bg_pairs"] += int(d <= DMAX)
    n["setup_triples"] = len(seen)
    return n


def test_counters_match_brute_force_single_triangle():
    base = wl.square_scene(center_px=(-3.1, 4.6), half_px=6.3, depth=4.0, shift_px=17.4,
                           width=40, height=32, k=9)
    sc = base.with_(faces=base.faces[:1])
    want = _brute_counts(sc)
    got = oracle.render(sc, counters=True).counters
    for k, v in want.items():
        assert got[k] == v, (k, got[k], v)


def test_counters_match_brute_force_two_triangles():
    sc = wl.square_scene(center_px=(2.2, -1.7), half_px=5.1, depth=4.0, shift_px=-11.3,
                         width=36, height=30, k=7)
    want = _brute_counts(sc)
    got = oracle.render(sc, counters=True).counters
    for k, v in want.items():
        assert got[k] == v, (k, got[k], v)
    assert want["bg_pairs"] > 0 and want["fg_pixsub"] > 0


# ---------------------------------------------------------------- guard band

W = H = 64
COL, ROW = 40, 20
L_EDGE, GAP = 0.06, 0.02          # edge (0,1) length, pixel's distance below it
ULP = 2.0 ** -25                  # float32 spacing of world x in [0.25, 0.5)
# a rotation about the vertical axis foreshortens the triangle on screen, so
# the keyframe triangle F(X) is not similar to F(tau): the eq 13 closest point
# differs from the exact one and its clamp changes the frozen-decision
# gradient.  K = 3, S = 1: sub-frame 1 sits at tau = 1/2 with X = 0.
MOTION = wl.Motion("rotate", axis=(0.0, 1.0, 0.0), revs=0.04)


def _clamp_scene(sigma):
    """Triangle with edge (0,1) horizontal, GAP above the centre p of pixel
    (ROW, COL), placed so that at sub-frame 1 the point q = F(X) w(tau) of
    eq 13 projects onto that edge of F(X) at parameter ~sigma; returns the
    scene and that parameter computed here from the float32 world vertices."""
    u0, v0 = _centres(W, H)[0][COL], _centres(W, H)[1][ROW]
    tanf = float(np.float32(np.tan(np.radians(20.0))))
    s = 4.0 * tanf                  # world units per normalized unit at depth 4
    p = np.array([u0, v0])

    def make(ax, shift_ulps):
        xs = np.array([ax, ax + L_EDGE, ax + 0.5 * L_EDGE]) * s
        ys = np.array([v0 + GAP, v0 + GAP, v0 + GAP + 0.1]) * s
        xs = np.float32(xs) + np.float32(shift_ulps * ULP)
        tri = np.stack([xs, np.float32(ys), np.zeros(3, np.float32)], 1)
        sc = wl.single_triangle_scene(tri, width=W, height=H, k=3, motion=MOTION, segments=1)
        kf = _project(sc)
        Ft, FX = 0.5 * (kf[0] + kf[1]), kf[0]
        q = _bary(p, Ft) @ FX
        e = FX[1] - FX[0]
        return sc, float(np.dot(q - FX[0], e) / np.dot(e, e))

    # solve for the x position (the parameter is affine in it), then step
    # the float32 vertices by single ulps towards the target
    ax = u0 - sigma * L_EDGE
    for h in (1e-3, 1e-5, 1e-6):
        s0, s1 = make(ax, 0)[1], make(ax + h, 0)[1]
        ax += (sigma - s0) * h / (s1 - s0)
    return min((make(ax, k) for k in range(-16, 17)), key=lambda x: abs(x[1] - sigma))


def _alpha_grad(sc):
    G = np.zeros((4, H, W))
    G[3, ROW, COL] = 1.0
    return oracle.render(sc, grad_image=G, bounds=True, flags=True)


def test_guard_band_pins_clamp_decision_of_closest_point():
    # at sub-frame 1, q projects onto edge (0,1) of F(X) at a parameter within
    # float32 rounding distance of 0: clamped (sigma < 0) and unclamped
    # (sigma > 0) give different frozen-decision gradients; the band must
    # flag both sides and its bound must cover the jump.  At sigma = +-0.01
    # nothing is flagged and the gradient is continuous.
    sp, sig_p = _clamp_scene(3e-7)
    sm, sig_m = _clamp_scene(-3e-7)
    assert 0 < sig_p < 8e-7 and -8e-7 < sig_m < 0, (sig_p, sig_m)
    rp, rm = _alpha_grad(sp), _alpha_grad(sm)
    assert rp.flags[ROW, COL] & 2 and rm.flags[ROW, COL] & 2
    # alpha is continuous across the clamp: no value alternative
    assert rp.image_hi[3, ROW, COL] == rp.image_lo[3, ROW, COL]
    jump = np.abs(rp.grad_verts - rm.grad_verts)
    gmax = np.abs(rp.grad_verts).max()
    assert jump.max() > 1e-3 * gmax, (jump.max(), gmax)
    # a step of the same size on one side moves the gradient 100x less
    same = np.abs(_alpha_grad(_clamp_scene(9e-7)[0]).grad_verts - rp.grad_verts)
    assert same.max() < 1e-2 * jump.max(), (same.max(), jump.max())
    tol = 1e-4 * np.abs(rp.grad_verts).max()
    assert np.all(rp.slack_verts >= jump - tol) and np.all(rm.slack_verts >= jump - tol)
    for sig in (1e-2, -1e-2):
        so, s_o = _clamp_scene(sig)
        ro = _alpha_grad(so)
        assert abs(s_o - sig) < 1e-4
        assert ro.flags[ROW, COL] == 0 and ro.slack_verts.max() == 0.0
    # on one side of the band the gradient is continuous
    g1 = _alpha_grad(_clamp_scene(1e-2)[0]).grad_verts
    g2 = _alpha_grad(_clamp_scene(1.1e-2)[0]).grad_verts
    assert np.abs(g1 - g2).max() < 0.05 * np.abs(g1).max()


def test_guard_band_range_of_a_pixel_centre_on_the_outline():
    # a square whose outline passes through a column of pixel centres: the
    # inclusive coverage test puts those centres in the foreground (colour c,
    # alpha 1); the other choice is the background with d = 0 (rgb 0, alpha
    # 1 - (1 - 1) = 1).  The range is [0, c] in rgb and exactly 1 in alpha.
    sc = wl.square_scene(half_px=3.5, shift_px=0.0, width=16, height=16, k=1)
    r = oracle.render(sc, bounds=True, flags=True)
    kf = _project(sc)[0]
    us, vs = _centres(16, 16)
    on = [(ri, ci) for ri, v in enumerate(vs) for ci, u in enumerate(us)
          if (np.isclose(u, kf[:, 0].min()) or np.isclose(u, kf[:, 0].max()))
          and kf[:, 1].min() + 1e-9 < v < kf[:, 1].max() - 1e-9]
    assert on
    col = sc.attrs[0].astype(np.float64)
    for ri, ci in on:
        assert r.flags[ri, ci] & 2
        np.testing.assert_allclose(r.image_lo[:3, ri, ci], 0.0, atol=1e-12)
        np.testing.assert_allclose(r.image_hi[:3, ri, ci], col, rtol=1e-6)
        np.testing.assert_allclose([r.image_lo[3, ri, ci], r.image_hi[3, ri, ci]], 1.0, atol=1e-12)
    # everywhere else the range is the value itself
    mask = np.ones((16, 16), bool)
    for ri, ci in on:
        mask[ri, ci] = False
    sharp = r.flags == 0
    assert np.array_equal(r.image_lo[:, sharp], r.image[:, sharp])
    assert np.array_equal(r.image_hi[:, sharp], r.image[:, sharp])
