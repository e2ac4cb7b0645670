"""Deterministic mode (RB_FLAG_DETERMINISTIC) through the C ABI: two runs of
the same forward and adjoint give bitwise-equal images and gradients, the
results keep parity with the FP64 oracle, and they agree with the default
mode to float rounding.  Cases: the medium workload (narrow halo, several
background tasks per list in the default mode), the wide-halo build (items
grouped by pixel) and a batch of instances of different sizes."""
import numpy as np
import pytest
import torch

from paper_2602_07860_amd import batch as BT
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

from gpu_common import (assert_grad_parity, assert_image_parity, gpu_backward, gpu_forward, reference, rel_l2,
                        say)

pytestmark = pytest.mark.gpu


def _wide():
    return wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.5, trans=(0.4, 0.1, 0.0)),
                            num_segments=6, num_subframes=13, width=640, height=640)


def _run(sc, G, **kw):
    img, state, st = gpu_forward(sc, **kw)
    gv, ga = gpu_backward(st, state, G)
    return img, gv, ga


@pytest.mark.parametrize("which", ["medium", "wide"])
def test_two_runs_bitwise_equal_and_oracle_parity(which):
    sc = wl.make_workload(wl.MEDIUM) if which == "medium" else _wide()
    say(f"case: deterministic {which} {sc.width}x{sc.height} K={sc.num_subframes}")
    G = np.random.default_rng(21).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
    a = _run(sc, G, deterministic=True)
    b = _run(sc, G, deterministic=True)
    for x, y, name in zip(a, b, ("image", "grad_verts", "grad_attrs")):
        same = np.array_equal(x.view(np.uint64), y.view(np.uint64))
        say(f"  {name}: bitwise equal {same}")
        assert same, name
    # the default mode agrees to float rounding (its sums run in another order)
    d = _run(sc, G)
    d2 = _run(sc, G)
    say("  default mode, two runs bitwise equal: "
        + ", ".join(f"{n} {np.array_equal(x.view(np.uint64), y.view(np.uint64))}"
                    for x, y, n in zip(d, d2, ("image", "grad_verts", "grad_attrs"))))
    scale = np.abs(d[0]).max()
    di = float(np.abs(a[0] - d[0]).max() / scale)
    dv, da = rel_l2(a[1], d[1]), rel_l2(a[2], d[2])
    say(f"  vs default mode: image max rel {di:.2e}, grad verts rel-L2 {dv:.2e}, attrs {da:.2e}")
    assert di <= 1e-6 and dv <= 1e-5 and da <= 1e-5
    # and parity with the oracle holds
    og = reference(sc, G)
    assert_image_parity(a[0], og, label=f"det {which}")
    assert_grad_parity(a[1], og.grad_verts, og.slack_verts, label=f"det {which} verts")
    assert_grad_parity(a[2], og.grad_attrs, og.slack_attrs, label=f"det {which} attrs")


def test_batch_two_runs_bitwise_equal():
    scs = [wl.make_workload(wl.MEDIUM),
           wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.1, 0.8, 0.5), revs=0.6, trans=(0.5, 0.2, 0.0)),
                            num_segments=5, num_subframes=23, width=61, height=37),
           wl.make_workload(wl.SMALL)]
    say(f"case: deterministic batch of {len(scs)}")
    Gs = [np.random.default_rng(30 + i).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
          for i, sc in enumerate(scs)]

    def once():
        sts = [R.scene_tensors(sc, "cuda") for sc in scs]
        r = BT.BatchRenderer(sts, R.RenderOptions(0, deterministic=True))
        r.fit()
        imgs = [im.clone() for im in r.forward()]
        for g, G in zip(r.grad_images, Gs):
            g.copy_(torch.as_tensor(G, dtype=torch.float32))
        r.backward()
        torch.cuda.synchronize()
        return ([x.cpu().numpy() for x in imgs], [x.cpu().numpy() for x in r.grad_verts],
                [x.cpu().numpy() for x in r.grad_attrs])

    a, b = once(), once()
    for xs, ys, name in zip(a, b, ("image", "grad_verts", "grad_attrs")):
        for i, (x, y) in enumerate(zip(xs, ys)):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (name, i)
    say("  two batch runs bitwise equal")
    # each instance agrees with its own deterministic single render (the
    # batch runs the kernel build for its longest chunk)
    for i, sc in enumerate(scs):
        img, gv, ga = _run(sc, Gs[i], deterministic=True)
        di = float(np.abs(img - a[0][i]).max() / np.abs(img).max())
        dv, da = rel_l2(a[1][i].astype(np.float64), gv), rel_l2(a[2][i].astype(np.float64), ga)
        say(f"  instance {i} vs single: image {di:.2e}, verts {dv:.2e}, attrs {da:.2e}")
        assert di <= 1e-6 and dv <= 1e-5 and da <= 1e-5


@pytest.mark.parametrize("solver,tile_w", [("recompute", 0), ("fast", 16), ("recompute", 4)])
def test_deterministic_with_other_solver_and_tiles(solver, tile_w):
    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.8, trans=(0.3, 0.0, 0.0)),
                          num_segments=10, num_subframes=41, width=48, height=40)
    say(f"case: deterministic small rotation solver={solver} tile_w={tile_w}")
    G = np.random.default_rng(23).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
    a = _run(sc, G, deterministic=True, solver=solver, tile_w=tile_w)
    b = _run(sc, G, deterministic=True, solver=solver, tile_w=tile_w)
    for x, y, name in zip(a, b, ("image", "grad_verts", "grad_attrs")):
        assert np.array_equal(x.view(np.uint64), y.view(np.uint64)), name
    og = reference(sc, G)
    assert_image_parity(a[0], og, label=f"det {solver} tile{tile_w}")
    assert_grad_parity(a[1], og.grad_verts, og.slack_verts, label=f"det {solver} tile{tile_w} verts")
    assert_grad_parity(a[2], og.grad_attrs, og.slack_attrs, label=f"det {solver} tile{tile_w} attrs")
