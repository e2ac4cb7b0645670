"""Gradient parity of the HIP adjoint (through the C ABI) with the FP64
oracle's adjoint and with central finite differences of the oracle's
frozen-decision surrogate.  Bar: relative L2 error <= 1e-3, separately for
vertex positions and attributes, with an upstream gradient on every pixel.
Where a (pixel, sub-frame) has a decision within float32 rounding distance
of flipping (winner identity, coverage, the closest point's edge or clamp
state), the oracle bounds per component how far the other choice moves the
gradient, and the residual is shrunk by that bound before its norm is taken;
the raw residual is printed beside it."""
import numpy as np
import pytest

import oracle
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

from gpu_common import (GRAD_RTOL, assert_band_small, assert_grad_parity, gpu_backward, gpu_forward,
                        reference, rel_l2, say)

pytestmark = pytest.mark.gpu


def _grad_case(sc, solver="fast", chunk_len=4, seed=0):
    G = np.random.default_rng(seed).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
    og = reference(sc, G)
    assert_band_small(og, sc.name)
    img, state, st = gpu_forward(sc, solver=solver, chunk_len=chunk_len)
    gv, ga = gpu_backward(st, state, G)
    lab = f"{sc.name}/{solver}/T{chunk_len}"
    assert_grad_parity(gv, og.grad_verts, og.slack_verts, label=lab + " verts")
    assert_grad_parity(ga, og.grad_attrs, og.slack_attrs, label=lab + " attrs")


@pytest.mark.parametrize("solver", ["fast", "recompute"])
def test_small_translation_gradients(solver):
    sc = wl.make_workload(wl.SMALL)
    say(f"case: grad {sc.name} {solver}")
    _grad_case(sc, solver)


# segments of 4-5 sub-frames: chunk_len 1, 2, 4, 8 run the 1-, 2-, 3- and
# 8-sub-frame kernel builds
@pytest.mark.parametrize("chunk_len", [1, 2, 4, 8])
def test_small_rotation_gradients(chunk_len):
    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.8,
                                                     trans=(0.3, 0.0, 0.0)),
                          num_segments=10, num_subframes=41, width=48, height=40)
    say(f"case: grad small rotation chunk_len={chunk_len}")
    _grad_case(sc, "fast", chunk_len, seed=1)


def test_medium_gradients_vs_oracle():
    sc = wl.make_workload(wl.MEDIUM)
    say(f"case: grad {sc.name} full image")
    _grad_case(sc, "fast", 4, seed=2)


def test_medium_gradient_vs_frozen_fd_64_vertices():
    # central FD (eps = 1e-3 world units, two Richardson levels: eps, eps/2,
    # eps/4) of the oracle's frozen-decision surrogate along a random direction
    # per vertex, for 64 vertices drawn with seed 102 among those the loss
    # depends on.  The perturbed vertices go to the FP64 oracle unrounded.
    # Six pixel rows across the sphere (its projection spans rows 40-216), the
    # first one through its motion-blurred top silhouette, all with an
    # upstream gradient on every pixel.
    sc = wl.make_workload(wl.MEDIUM)
    rows = (40, 216, 32)
    say(f"case: FD {sc.name} rows {rows}")
    base = oracle.render(sc, rows=rows, record=True)
    G = np.zeros_like(base.image)
    G[:, rows[0]:rows[1]:rows[2]] = np.random.default_rng(7).normal(size=G[:, rows[0]:rows[1]:rows[2]].shape)
    live_rows = [r for r in range(*rows) if np.abs(base.image[:, r]).sum() > 0]
    assert len(live_rows) >= 4, live_rows
    og = reference(sc, G, rows=rows)
    img, state, st = gpu_forward(sc)
    gv, _ = gpu_backward(st, state, G)
    live = np.where(np.abs(og.grad_verts).sum(1) > 0)[0]
    rng = np.random.default_rng(102)
    picks = rng.choice(live, size=min(64, len(live)), replace=False)

    def loss(vi, d, h):
        v = sc.verts.astype(np.float64).copy()
        v[vi] += h * d
        r = oracle.render(sc.with_(verts=v), rows=rows, replay=base.decisions)
        return float(np.sum(G * r.image))

    fds, gpus, adj, slk = [], [], [], []
    eps = 1e-3
    for vi in picks:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        D = [(loss(vi, d, h) - loss(vi, d, -h)) / (2 * h) for h in (eps, eps / 2, eps / 4)]
        R1 = [(4 * D[1] - D[0]) / 3, (4 * D[2] - D[1]) / 3]
        fds.append((16 * R1[1] - R1[0]) / 15)
        gpus.append(float(gv[vi] @ d))
        adj.append(float(og.grad_verts[vi] @ d))
        slk.append(float(og.slack_verts[vi] @ np.abs(d)))
    fds, gpus, adj, slk = np.array(fds), np.array(gpus), np.array(adj), np.array(slk)
    e_or = rel_l2(adj, fds)
    say(f"FD over {len(picks)} vertices on live rows {live_rows}: oracle adjoint vs FD {e_or:.2e}")
    assert e_or <= 1e-4      # the FD itself is accurate
    assert_grad_parity(gpus, fds, slk, label="GPU vs FD")


def test_autograd_function_matches_adjoint():
    import torch
    sc = wl.make_workload(wl.SMALL)
    tgt = wl.make_workload(wl.SMALL, seed=5)
    st = R.scene_tensors(sc, "cuda")
    target = torch.as_tensor(oracle.render(tgt).image, dtype=torch.float32, device="cuda")
    verts = st.verts.clone().requires_grad_(True)
    attrs = st.attrs.clone().requires_grad_(True)
    opts = R.RenderOptions(sc.num_subframes)
    say("case: autograd L2 loss")
    img = R.render(verts, attrs, st.faces, st.model, st.camera, opts)
    loss = ((img - target) ** 2).sum()
    loss.backward()
    img2, state = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, opts)
    gv, ga = R.render_backward(st.verts, st.faces, st.attrs, st.model, state, 2.0 * (img2 - target))
    torch.cuda.synchronize()
    assert torch.allclose(verts.grad, gv, rtol=1e-4, atol=1e-6)
    assert torch.allclose(attrs.grad, ga, rtol=1e-4, atol=1e-6)
    assert float(loss.detach()) > 0
