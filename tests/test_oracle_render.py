"""Pins of the oracle's rendering against closed forms and invariants that do
not come from the oracle itself (pinhole geometry, counting, textbook
distances, linear algebra, convergence orders)."""
import math

import numpy as np
import pytest

import oracle
from paper_2602_07860_amd import workloads as wl

DELTA = 1e-4


def _ndc_centres(W, H):
    """Pixel centres, row 0 at the top (reading of SoftRas' convention)."""
    u = (2 * np.arange(W) + 1 - W) / W
    v = (H - 2 * np.arange(H) - 1) / H
    return u, v


def test_full_field_of_view_square_covers_expected_columns():
    # A square spanning +-(1 - 1.5/W) of the half field of view at its depth
    # must cover exactly columns/rows 1 .. W-2 (pinhole: x_ndc = X / (Z tan a)).
    W = H = 32
    depth = 3.0
    sc = wl.square_scene(half_px=W / 2 - 0.75, depth=depth, shift_px=0.0, width=W, height=H, k=1)
    r = oracle.render(sc)
    cov = r.image[3] > 0.999999
    want = np.zeros((H, W), bool)
    want[1:H - 1, 1:W - 1] = True
    assert np.array_equal(cov, want)
    np.testing.assert_allclose(r.image[:3, 1:H - 1, 1:W - 1],
                               np.broadcast_to(np.array([0.25, 0.5, 0.75])[:, None, None], (3, H - 2, W - 2)),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("K,S", [(16, 1), (9, 1), (23, 3), (2, 1), (1, 1)])
def test_translating_square_box_filter_count(K, S):
    # Flat square translating parallel to the image plane: each foreground
    # sub-frame gives exactly the flat colour, so RGB = c * #{k: centre inside
    # at t_k} / K with t_k = k/(K-1) (Sec. 3.2) and a linear path.
    W, H = 48, 40
    half, shift, cx, cy = 6.3, 17.4, -3.1, 4.6      # pixels; edges avoid pixel centres
    sc = wl.square_scene(center_px=(cx, cy), half_px=half, depth=4.0, shift_px=shift,
                         width=W, height=H, k=K, segments=S)
    r = oracle.render(sc)
    u, v = _ndc_centres(W, H)
    ts = np.zeros(1) if K == 1 else np.arange(K) / (K - 1)
    count = np.zeros((H, W))
    for t in ts:
        xl = (cx - half + (t - 0.5) * shift) * 2.0 / W
        xr = (cx + half + (t - 0.5) * shift) * 2.0 / W
        yb = (cy - half) * 2.0 / H
        yt = (cy + half) * 2.0 / H
        count += ((u[None, :] >= xl) & (u[None, :] <= xr) & (v[:, None] >= yb) & (v[:, None] <= yt))
    col = np.array([0.25, 0.5, 0.75])
    np.testing.assert_allclose(r.image[:3], col[:, None, None] * count[None] / K, rtol=0, atol=1e-6)
    # alpha: 1 for covered sub-frames; background ones add a soft term
    assert np.all(r.image[3] >= count / K - 1e-12)
    # the square sits above the centre: rows near the top are covered
    rows = np.where(count.sum(1) > 0)[0]
    assert rows.mean() < H / 2


def test_box_filter_converges_to_trapezoid():
    W, H = 32, 8
    half, shift = 4.3, 9.0
    err = []
    for K in (8, 32, 128):
        sc = wl.square_scene(half_px=half, shift_px=shift, width=W, height=H, k=K)
        r = oracle.render(sc)
        u, _ = _ndc_centres(W, H)
        x = u * W / 2.0   # pixels from the centre
        # fraction of t in [0, 1] with |x - (t - 0.5) shift| <= half
        lo = np.clip((x - half) / shift + 0.5, 0, 1)
        hi = np.clip((x + half) / shift + 0.5, 0, 1)
        frac = hi - lo
        err.append(np.abs(r.image[0, H // 2] / 0.25 - frac).max())
    assert err[0] <= 1.0 / 8 + 1e-9 and err[1] <= 1.0 / 32 + 1e-9 and err[2] <= 1.0 / 128 + 1e-9


def test_zero_motion_equals_static_frame():
    sc = wl.make_workload(wl.SMALL)
    still = sc.with_(motion=wl.Motion("translate"), num_segments=3, num_subframes=7)
    one = still.with_(num_subframes=1, num_segments=1)
    a = oracle.render(still).image
    b = oracle.render(one).image
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


def test_fast_solver_equals_naive_solve():
    rng = np.random.default_rng(5)
    for trial in range(3):
        v = rng.normal(size=(12, 3)).astype(np.float32) * 0.6
        f = rng.integers(0, 12, size=(10, 3)).astype(np.int32)
        f = f[(f[:, 0] != f[:, 1]) & (f[:, 1] != f[:, 2]) & (f[:, 0] != f[:, 2])]
        c = rng.uniform(size=(12, 3)).astype(np.float32)
        axis = tuple(rng.normal(size=3))
        sc = wl.Scene(v, f, c, wl.Motion("rotate", axis=axis, revs=0.7, trans=(0.8, -0.3, 0.2)),
                      5, *wl._camera(), 40, 40, 23, "random")
        a = oracle.render(sc, solver="naive").image
        b = oracle.render(sc, solver="fast").image
        assert np.abs(a - b).max() <= 1e-12


def test_linear_path_is_independent_of_segment_count():
    # A straight path cut into more segments is the same piecewise-linear path.
    base = wl.square_scene(half_px=5.2, shift_px=13.1, width=32, height=32, k=21)
    a = oracle.render(base.with_(num_segments=1)).image
    b = oracle.render(base.with_(num_segments=4)).image
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_segment_linear_equals_exact_projection_for_in_plane_translation():
    # (the sub-frame transforms are exact while the keyframe transforms are
    #  float32 inputs: the soft alpha sees that 1e-8 rounding, amplified by
    #  at most 2 r exp(-r^2/delta)/delta < 86)
    sc = wl.square_scene(half_px=5.2, shift_px=13.1, width=32, height=32, k=17)
    a = oracle.render(sc, motion="segment").image
    b = oracle.render(sc, motion="exact").image
    np.testing.assert_allclose(a[:3], b[:3], rtol=0, atol=1e-12)
    np.testing.assert_allclose(a[3], b[3], rtol=0, atol=2e-6)


def test_keyframe_distance_exact_for_translation_and_at_keyframes():
    # eq 13 approximates F(t) by F(0)/F(1); for a rigid screen translation the
    # closest point in F(X) maps onto the closest point in F(t) (exact), and at
    # keyframe sub-frames (tau in {0, 1}) it is exact for any motion.
    sc = wl.square_scene(half_px=5.2, shift_px=13.1, width=32, height=32, k=17)
    a = oracle.render(sc, distance="keyframe").image
    b = oracle.render(sc, distance="exact").image
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    rot = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, 0.2), revs=1.0),
                           num_segments=6, num_subframes=7, width=40, height=40)
    a = oracle.render(rot, distance="keyframe").image
    b = oracle.render(rot, distance="exact").image
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)
    # between keyframes the two differ (the approximation is not vacuous)
    rot2 = rot.with_(num_subframes=13)
    a = oracle.render(rot2, distance="keyframe").image
    b = oracle.render(rot2, distance="exact").image
    assert np.abs(a - b).max() > 1e-6


def _proj(sc, P):
    view = np.asarray(sc.view, np.float64)
    Xc = P @ view[:, :3].T + view[:, 3]
    t = float(np.float32(sc.tan_half_fov))
    return Xc[:, 0] / (Xc[:, 2] * t), Xc[:, 1] / (Xc[:, 2] * t)


def _seg_dist2(p, a, b):
    e = b - a
    t = np.clip(np.dot(p - a, e) / np.dot(e, e), 0, 1)
    return float(np.sum((p - (a + t * e)) ** 2))


def test_single_static_triangle_closed_forms():
    # Foreground: colour = barycentric interpolation (eq 9) by a 3x3 solve.
    # Background: alpha = 1 - (1 - A) = exp(-d / delta) with d the squared
    # distance to the triangle (eqs 10-12, exact at a keyframe).
    W = H = 40
    P = np.array([[-0.5, -0.4, 0.3], [0.6, -0.2, 0.0], [-0.1, 0.55, -0.2]], np.float32)
    sc = wl.single_triangle_scene(P, width=W, height=H, k=1)
    r = oracle.render(sc, eps_cutoff=0.0)
    x, y = _proj(sc, P.astype(np.float64))
    u, v = _ndc_centres(W, H)
    M = np.array([x, y, np.ones(3)])
    tri = np.stack([x, y], 1)
    nfg = nbg = 0
    for rr in range(H):
        for cc in range(W):
            w = np.linalg.solve(M, [u[cc], v[rr], 1.0])
            if w.min() >= 1e-9:
                np.testing.assert_allclose(r.image[:3, rr, cc], w, atol=1e-12)
                assert r.image[3, rr, cc] == 1.0
                nfg += 1
            elif w.min() < -1e-9:
                p = np.array([u[cc], v[rr]])
                d = min(_seg_dist2(p, tri[i], tri[(i + 1) % 3]) for i in range(3))
                np.testing.assert_allclose(r.image[3, rr, cc], math.exp(-d / float(np.float32(DELTA))),
                                           rtol=1e-9, atol=1e-15)
                assert np.all(r.image[:3, rr, cc] == 0)
                nbg += 1
    assert nfg > 20 and nbg > 20


def test_two_triangles_background_product_and_depth_order():
    W = H = 80
    T1 = np.array([[-0.8, -0.3, 0.0], [-0.2, -0.3, 0.0], [-0.5, 0.3, 0.0]], np.float32)
    T2 = T1 + np.array([0.62, 0.0, 0.0], np.float32)
    v = np.concatenate([T1, T2])
    sc = wl.Scene(v, np.array([[0, 1, 2], [3, 4, 5]], np.int32),
                  np.concatenate([np.tile([1, 0, 0], (3, 1)), np.tile([0, 1, 0], (3, 1))]).astype(np.float32),
                  wl.Motion("translate"), 1, *wl._camera(), W, H, 1, "two")
    r = oracle.render(sc, eps_cutoff=0.0)
    x, y = _proj(sc, v.astype(np.float64))
    u, vv = _ndc_centres(W, H)
    checked = 0
    for rr in range(H):
        for cc in range(W):
            p = np.array([u[cc], vv[rr]])
            inside = []
            A = []
            for f in range(2):
                M = np.array([x[3 * f:3 * f + 3], y[3 * f:3 * f + 3], np.ones(3)])
                w = np.linalg.solve(M, [p[0], p[1], 1.0])
                inside.append(w.min() >= 0)
                tri = np.stack([x[3 * f:3 * f + 3], y[3 * f:3 * f + 3]], 1)
                d = min(_seg_dist2(p, tri[i], tri[(i + 1) % 3]) for i in range(3))
                A.append(math.exp(-d / float(np.float32(DELTA))))
            if not any(inside) and min(A) > 1e-3:
                np.testing.assert_allclose(r.image[3, rr, cc], 1 - (1 - A[0]) * (1 - A[1]), rtol=1e-9)
                checked += 1
    assert checked >= 2
    # depth order: move the second triangle in front of the first, overlapping
    T3 = T1 + np.array([0.15, 0.05, 0.5], np.float32)   # nearer the eye at z = 4
    v2 = np.concatenate([T1, T3])
    sc2 = sc.with_(verts=v2)
    r2 = oracle.render(sc2)
    both = (r2.image[3] == 1.0) & (r2.image[1] > 0.999) & (r2.image[0] < 1e-9)
    assert both.sum() > 10      # the nearer (green) face wins where they overlap
    # identical coincident faces: the lower face index wins
    sc3 = sc.with_(verts=np.concatenate([T1, T1]))
    r3 = oracle.render(sc3)
    fg = r3.image[3] == 1.0
    assert fg.sum() > 10 and np.all(r3.image[0][fg] > 0.999) and np.all(r3.image[1][fg] < 1e-12)


def test_cutoff_truncation_is_below_tolerance():
    sc = wl.make_workload(wl.SMALL)
    a = oracle.render(sc, eps_cutoff=1e-8).image
    b = oracle.render(sc, eps_cutoff=0.0).image
    assert np.abs(a - b).max() <= 1e-6 * np.abs(b).max()


def test_segment_count_convergence_is_second_order():
    # Piecewise-linear keyframe motion approaches the exact rotation as O(1/S^2)
    # (App. D trend): compare to per-sub-frame exact projection.
    base = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.2, 1.0, 0.1), revs=1.0),
                            width=48, height=48, num_subframes=97)
    errs = []
    for S in (4, 8, 16):
        sc = base.with_(num_segments=S)
        a = oracle.render(sc, motion="segment", distance="exact").image
        b = oracle.render(sc, motion="exact", distance="exact").image
        errs.append(np.abs(a - b).mean())
    assert errs[1] < 0.45 * errs[0] and errs[2] < 0.45 * errs[1]


def test_counters_and_invariants_on_small_workload():
    sc = wl.make_workload(wl.SMALL)
    r = oracle.render(sc, flags=True, counters=True)
    c = r.counters
    n = sc.width * sc.height * sc.num_subframes
    assert c["fg_pixsub"] + c["bg_pixsub"] == n
    assert c["cover_pairs"] >= c["fg_pixsub"]
    assert c["bbox_pairs"] >= c["cover_pairs"]
    # a closed surface: every foreground pixel-subframe is covered by an even
    # number of faces (front and back), >= 2
    assert c["cover_pairs"] >= 2 * c["fg_pixsub"]
    assert ((r.flags & 1) > 0).sum() <= 0.01 * sc.width * sc.height
    assert (r.flags > 0).sum() <= 0.03 * sc.width * sc.height
    assert 0.0 <= r.image.min() and r.image[3].max() <= 1.0


def test_guard_band_flags_edge_on_pixel_centres():
    # an edge passing exactly through a column of pixel centres at a sub-frame
    W = H = 16
    sc = wl.square_scene(half_px=3.5, shift_px=0.0, width=W, height=H, k=1)
    r = oracle.render(sc, flags=True)
    assert r.flags.sum() > 0
    # (offset so that neither the outline nor the shared diagonal meets a centre;
    #  a centre on the diagonal is ambiguous: both faces sit on their edge)
    sc2 = wl.square_scene(center_px=(0.0, 0.25), half_px=3.3, shift_px=0.0, width=W, height=H, k=1)
    r2 = oracle.render(sc2, flags=True)
    assert (r2.flags & 1).sum() == 0


def test_exact_mode_is_the_mean_of_still_frames():
    # the oracle's exact-motion, exact-distance mode (project M(t_k) P0 per
    # sub-frame, closest point in the sub-frame's own triangle, eq 12) equals
    # the mean of K separate still renders, each a single keyframe at
    # M(t_k) where the keyframe closest point (eq 13) is the exact one
    class Still:
        def __init__(self, m):
            self.m = np.asarray(m, np.float64)

        def matrix(self, t):
            return self.m

        def keyframes(self, num_segments):
            return np.stack([self.m] * (num_segments + 1))

    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.6,
                                                     trans=(0.3, 0.0, 0.0)),
                          num_segments=4, num_subframes=7, width=40, height=36)
    ex = oracle.render(sc, motion="exact", distance="exact").image
    acc = np.zeros_like(ex)
    for t in wl.subframe_times(sc.num_subframes):
        acc += oracle.render(sc.with_(motion=Still(sc.motion.matrix(t)), num_segments=1, num_subframes=1)).image
    # (the still frames take their transform rounded to float32, the exact
    # mode in double: positions differ by ~1e-7 relative)
    np.testing.assert_allclose(acc / sc.num_subframes, ex, rtol=0, atol=2e-6)
