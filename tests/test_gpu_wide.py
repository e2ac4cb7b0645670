"""Element-wise parity of the wide-halo builds: at 640x640 the background
halo spans 13.7 pixels (>= 12), so the background forward groups items by
pixel in per-lane runs and the background adjoint uses runs of 8 at 4 waves
per SIMD.  A small translating and rotating mesh keeps the FP64 oracle fast
while faces reach hundreds of pixels of background."""
import numpy as np
import pytest

import oracle
from paper_2602_07860_amd import workloads as wl

from gpu_common import GRAD_RTOL, assert_image_parity, gpu_backward, gpu_forward, rel_l2, say

pytestmark = pytest.mark.gpu


def test_wide_halo_forward_and_adjoint():
    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.5, trans=(0.4, 0.1, 0.0)),
                          num_segments=6, num_subframes=13, width=640, height=640)
    say(f"case: wide halo 640x640 K={sc.num_subframes} S={sc.num_segments}")
    ref = oracle.render(sc, flags=True)
    G = np.random.default_rng(5).normal(size=ref.image.shape)
    G[:, ref.flags != 0] = 0.0
    og = oracle.render(sc, grad_image=G)
    for solver in ("fast", "recompute"):
        img, state, st = gpu_forward(sc, solver=solver)
        assert_image_parity(img, ref.image, ref.flags, label=f"wide/{solver}")
        gv, ga = gpu_backward(st, state, G)
        ev, ea = rel_l2(gv, og.grad_verts), rel_l2(ga, og.grad_attrs)
        say(f"  {solver}: grad rel-L2 verts {ev:.2e} attrs {ea:.2e}")
        assert ev <= GRAD_RTOL and ea <= GRAD_RTOL


def test_wide_halo_batch_of_two_matches_oracle():
    # every instance wide: the batched launch takes the wide builds, with the
    # background adjoint's per-instance task counters
    import torch
    from paper_2602_07860_amd import batch as BT
    from paper_2602_07860_amd import render as R
    scs = [wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.5, trans=(0.4, 0.1, 0.0)),
                            num_segments=6, num_subframes=13, width=640, height=640),
           wl.make_workload(wl.SMALL, motion=wl.Motion("translate", trans=(0.3, -0.2, 0.0)),
                            num_segments=3, num_subframes=9, width=704, height=600)]
    say("case: batch of two wide-halo instances")
    refs = [oracle.render(sc, flags=True) for sc in scs]
    Gs = []
    for i, ref in enumerate(refs):
        G = np.random.default_rng(20 + i).normal(size=ref.image.shape)
        G[:, ref.flags != 0] = 0.0
        Gs.append(G)
    ogs = [oracle.render(sc, grad_image=G) for sc, G in zip(scs, Gs)]
    r = BT.BatchRenderer([R.scene_tensors(sc, "cuda") for sc in scs], R.RenderOptions(0))
    r.fit()
    imgs = [im.double().cpu().numpy() for im in r.forward()]
    for g, G in zip(r.grad_images, Gs):
        g.copy_(torch.as_tensor(G, dtype=torch.float32))
    r.backward()
    torch.cuda.synchronize()
    for i in range(len(scs)):
        assert_image_parity(imgs[i], refs[i].image, refs[i].flags, label=f"wide batch {i}")
        ev = rel_l2(r.grad_verts[i].double().cpu().numpy(), ogs[i].grad_verts)
        ea = rel_l2(r.grad_attrs[i].double().cpu().numpy(), ogs[i].grad_attrs)
        say(f"  instance {i}: grad rel-L2 verts {ev:.2e} attrs {ea:.2e}")
        assert ev <= GRAD_RTOL and ea <= GRAD_RTOL
