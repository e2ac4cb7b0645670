"""Parabolic rotation + translation (App. L.1): every vertex is rotated by
pi t about the y axis and then moved along the parabola
T(t) = (s, -4 s^2 + 0.5, s), s = 0.5 - t.  The motion is cut into S = 6
linear segments (12 per full revolution, the paper's rotation rule, for a
half revolution).  Forward and adjoint of the HIP path through the C ABI
against the FP64 oracle on the 64^2 and 256^2 meshes, every pixel compared
and carrying an upstream gradient."""
import numpy as np
import pytest

from paper_2602_07860_amd import workloads as wl

from gpu_common import (assert_band_small, assert_grad_parity, assert_image_parity, gpu_backward, gpu_forward,
                        reference, say)

pytestmark = pytest.mark.gpu

PARABOLIC = wl.Motion("parabolic")


@pytest.mark.parametrize("name,K", [(wl.SMALL, 48), (wl.MEDIUM, 64)])
def test_parabolic_forward_and_adjoint(name, K):
    sc = wl.make_workload(name, motion=PARABOLIC, num_segments=6, num_subframes=K)
    say(f"case: parabolic {sc.name} {sc.width}^2 K={K} S=6")
    G = np.random.default_rng(31).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
    ref = reference(sc, G)
    assert_band_small(ref, "parabolic")
    for solver in ("fast", "recompute"):
        img, state, st = gpu_forward(sc, solver=solver)
        assert_image_parity(img, ref, label=f"parabolic/{solver}")
        gv, ga = gpu_backward(st, state, G)
        assert_grad_parity(gv, ref.grad_verts, ref.slack_verts, label=f"parabolic/{solver} verts")
        assert_grad_parity(ga, ref.grad_attrs, ref.slack_attrs, label=f"parabolic/{solver} attrs")
