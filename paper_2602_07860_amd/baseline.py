"""Paper-style baseline: the motion blur as K independent static renders.

Sub-frame k places the mesh with the exact rigid motion M(t_k) at
t_k = k/(K-1) (no segment-linear keyframes), renders it as a still image
(a single keyframe, so the closest point of eqs 13-14 is the exact
per-frame one of eq 12) and the K images are averaged with weight 1/K: the
"render K frames and average" scheme the paper's speed comparison measures
the fast solver against (Sec. 4.2).  Its backward sends dL/dI / K into every
frame and sums the frames' gradients.  All K frames go through one batched
launch sequence of the same HIP library (rb_render_blur_batched); this
module only arranges arguments and sums outputs.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

from .batch import BatchRenderer
from .render import RenderOptions, SceneTensors


class StaticFrames:
    """BASE-B renderer of one scene (verts [V,3], faces, attrs [V,C] device
    tensors; motion_matrices: K rigid 3x4 transforms M(t_k); camera)."""

    def __init__(self, verts: torch.Tensor, faces: torch.Tensor, attrs: torch.Tensor,
                 motion_matrices: Sequence[np.ndarray], camera, opts: RenderOptions = None):
        m = np.asarray(motion_matrices, np.float32).reshape(-1, 1, 3, 4)
        self.K = m.shape[0]
        # frame k: one segment whose two keyframes are both M(t_k)
        self.models = torch.as_tensor(np.ascontiguousarray(np.repeat(m, 2, axis=1)), device=verts.device)
        scenes = [SceneTensors(verts, faces, attrs, self.models[k], camera, 1) for k in range(self.K)]
        o = opts or RenderOptions(0)
        self.r = BatchRenderer(scenes, RenderOptions(0, delta=o.delta, eps_cutoff=o.eps_cutoff, solver=o.solver,
                                                     chunk_len=1, slice_len=o.slice_len))
        self.image = torch.empty_like(self.r.images[0])
        self.grad_verts = torch.empty_like(verts)
        self.grad_attrs = torch.empty_like(attrs)

    def fit(self) -> None:
        self.r.fit()

    def forward(self) -> torch.Tensor:
        self.r.forward()
        torch.sum(torch.stack(self.r.images), dim=0, out=self.image)
        self.image.mul_(1.0 / self.K)
        return self.image

    def backward(self, grad_image: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        for g in self.r.grad_images:
            torch.mul(grad_image, 1.0 / self.K, out=g)
        self.r.backward()
        torch.sum(torch.stack(self.r.grad_verts), dim=0, out=self.grad_verts)
        torch.sum(torch.stack(self.r.grad_attrs), dim=0, out=self.grad_attrs)
        return self.grad_verts, self.grad_attrs


def for_scene(st: SceneTensors, motion, num_subframes: int, opts: RenderOptions = None) -> StaticFrames:
    """BASE-B of a workloads.Motion over K sub-frames for scene tensors st."""
    from .workloads import subframe_times
    mats = [motion.matrix(t) for t in subframe_times(num_subframes)]
    return StaticFrames(st.verts, st.faces, st.attrs, mats, st.camera, opts)
