"""Edge cases of the HIP path against the FP64 oracle (forward and adjoint):
channel counts 1, 2 and 4 (the maximum); a mesh whose motion keeps it
outside the image (every list empty, image and gradients zero); degenerate
faces (a repeated vertex, three collinear vertices) mixed into a mesh; and
exact depth ties (every face duplicated on its own copy of the vertices: the
lower face index wins, so the copies receive no colour gradient)."""
import numpy as np
import pytest

from paper_2602_07860_amd import workloads as wl

from gpu_common import (assert_grad_parity, assert_image_parity, gpu_backward, gpu_forward, reference, rel_l2,
                        say)

pytestmark = pytest.mark.gpu


def _rot():
    return wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.8, trans=(0.3, 0.0, 0.0)),
                            num_segments=10, num_subframes=41, width=48, height=40)


def _parity(sc, label, seed=0):
    G = np.random.default_rng(seed).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
    og = reference(sc, G)
    img, state, st = gpu_forward(sc)
    assert_image_parity(img, og, label=label)
    gv, ga = gpu_backward(st, state, G)
    assert_grad_parity(gv, og.grad_verts, og.slack_verts, label=f"{label} verts")
    assert_grad_parity(ga, og.grad_attrs, og.slack_attrs, label=f"{label} attrs")
    return img, gv, ga, og


@pytest.mark.parametrize("C", [1, 2, 4])
def test_channel_counts(C):
    sc = _rot()
    a = np.random.default_rng(70 + C).uniform(size=(len(sc.verts), C)).astype(np.float32)
    sc = sc.with_(attrs=a, name=f"rot-C{C}")
    say(f"case: small rotation with {C} channels")
    img, _, _, _ = _parity(sc, f"C={C}", seed=C)
    assert img.shape == (C + 1, sc.height, sc.width)


def test_mesh_outside_the_image():
    sc = wl.make_workload(wl.SMALL)
    sc = sc.with_(motion=wl.Motion("translate", trans=(3.0, 0.0, 0.0)),
                  verts=(sc.verts + np.array([6.0, 0.0, 0.0], np.float32)).astype(np.float32), name="outside")
    say("case: mesh outside the image at every sub-frame")
    img, gv, ga, og = _parity(sc, "outside")
    assert not np.any(og.image) and not np.any(img)
    assert not np.any(gv) and not np.any(ga)


def test_degenerate_faces():
    sc = _rot()
    f = sc.faces.copy()
    v = sc.verts.copy()
    a = sc.attrs.copy()
    # a repeated vertex, and three collinear vertices (the midpoint of an edge
    # added as a new vertex)
    rep = np.array([[f[0, 0], f[0, 0], f[0, 1]], [f[5, 1], f[5, 2], f[5, 2]]], np.int32)
    mid = 0.5 * (v[f[9, 0]] + v[f[9, 1]])
    v = np.concatenate([v, mid[None]]).astype(np.float32)
    a = np.concatenate([a, a[f[9, 0]][None]]).astype(np.float32)
    col = np.array([[f[9, 0], len(v) - 1, f[9, 1]]], np.int32)
    sc = sc.with_(verts=v, attrs=a, faces=np.concatenate([f[:20], rep, col, f[20:]]).astype(np.int32), name="degenerate")
    say(f"case: small rotation with {len(rep) + 1} degenerate faces")
    _parity(sc, "degenerate", seed=9)


def test_exact_depth_ties_go_to_the_lower_face_index():
    sc = _rot()
    V = len(sc.verts)
    v = np.concatenate([sc.verts, sc.verts]).astype(np.float32)
    a = np.concatenate([sc.attrs, sc.attrs]).astype(np.float32)
    f = np.concatenate([sc.faces, sc.faces + V]).astype(np.int32)
    tie = sc.with_(verts=v, attrs=a, faces=f, name="ties")
    say("case: every face duplicated on a copy of its vertices")
    img, gv, ga, og = _parity(tie, "ties", seed=11)
    # the copies (higher face indices) never win a pixel: their attribute
    # gradient is zero on the GPU as in the oracle
    assert not np.any(ga[V:]) and not np.any(og.grad_attrs[V:])
    # and the colour channels are the single mesh's (coverage is the same;
    # alpha differs where the background counts both copies' factors)
    single, _, _ = gpu_forward(sc)
    C = sc.attrs.shape[1]
    d = float(np.abs(img[:C] - single[:C]).max() / np.abs(single[:C]).max())
    say(f"  colour vs the single mesh: {d:.2e}")
    assert d <= 1e-5
