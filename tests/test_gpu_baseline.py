"""The paper-style baseline (K independent static renders of the exactly
moved mesh, averaged; paper_2602_07860_amd/baseline.py) through the batched C
ABI, against the FP64 oracle: its image against the oracle's exact-motion,
exact-distance mode (eq 12) on every pixel, and its gradient against the sum
of the oracle's adjoints of the K still frames."""
import numpy as np
import pytest

import oracle
from paper_2602_07860_amd import baseline
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

from gpu_common import assert_grad_parity, assert_image_parity, say

pytestmark = pytest.mark.gpu


class _Still:
    """A motion that holds one rigid transform for the whole exposure."""

    def __init__(self, m):
        self.m = np.asarray(m, np.float64)

    def matrix(self, t):
        return self.m

    def keyframes(self, num_segments):
        return np.stack([self.m] * (num_segments + 1))


@pytest.mark.parametrize("case", ["translate", "rotate"])
def test_static_frames_match_oracle(case):
    import torch
    if case == "translate":
        sc = wl.make_workload(wl.SMALL, num_subframes=9)
    else:
        sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.6,
                                                         trans=(0.3, 0.0, 0.0)),
                              num_segments=4, num_subframes=12, width=48, height=40)
    K = sc.num_subframes
    say(f"case: static-frames baseline {case} K={K}")
    ref = oracle.render(sc, motion="exact", distance="exact", bounds=True)
    st = R.scene_tensors(sc, "cuda")
    b = baseline.for_scene(st, sc.motion, K)
    b.fit()
    img = b.forward().double().cpu().numpy()
    assert_image_parity(img, ref, label=f"baseline/{case}")
    G = np.random.default_rng(41).normal(size=ref.image.shape)
    gv, ga = b.backward(torch.as_tensor(G, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    ogv = np.zeros((len(sc.verts), 3))
    oga = np.zeros((len(sc.verts), 3))
    sv, sa = np.zeros_like(ogv), np.zeros_like(oga)
    for t in wl.subframe_times(K):
        still = sc.with_(motion=_Still(sc.motion.matrix(t)), num_segments=1, num_subframes=1)
        r = oracle.render(still, grad_image=G / K, bounds=True)
        ogv += r.grad_verts
        oga += r.grad_attrs
        sv += r.slack_verts
        sa += r.slack_attrs
    assert_grad_parity(gv.double().cpu().numpy(), ogv, sv, label=f"baseline/{case} verts")
    assert_grad_parity(ga.double().cpu().numpy(), oga, sa, label=f"baseline/{case} attrs")
