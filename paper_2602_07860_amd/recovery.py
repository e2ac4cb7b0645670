"""Multi-view translational shape recovery (Sec. 5.1, App. G and J).

A template mesh (vertex offsets delta from its rest positions, per-vertex
colours) is fitted to motion-blurred RGBA images of a target from 40
viewpoints: each iteration renders a batch of 16 views through one batched
launch sequence of the HIP library, takes the L1 image loss
||I - I_hat||_1 + ||alpha - alpha_hat||_1, adds the smoothness loss
lambda_s sum_edges (cos theta + 1)^2 (theta the dihedral angle at the edge)
and the Laplacian loss lambda_L sum_v |delta_v - mean_{N(v)} delta|^2, and
takes an Adam step (lr 0.01, betas (0.5, 0.99), lambda_s = 3e-2,
lambda_L = 3e-4, App. J).  The renderer's gradient comes from its adjoint
kernels; the two regularizers are small mesh-sized terms differentiated by
PyTorch.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import torch

from .batch import BatchRenderer
from .render import RenderOptions, SceneTensors, make_camera

LAMBDA_S = 3e-2
LAMBDA_L = 3e-4


def edge_faces(faces: np.ndarray) -> np.ndarray:
    """[E, 4] (a, b, c, d) per interior edge (a, b): c and d are the third
    vertices of its two faces, (a, b, c) wound like its face."""
    seen = {}
    out = []
    for f in faces:
        for i in range(3):
            a, b, c = int(f[i]), int(f[(i + 1) % 3]), int(f[(i + 2) % 3])
            key = (min(a, b), max(a, b))
            if key in seen:
                a0, b0, c0 = seen.pop(key)
                out.append((a0, b0, c0, c))
            else:
                seen[key] = (a, b, c)
    return np.asarray(out, np.int64)


def neighbours(faces: np.ndarray, V: int):
    """Sparse row-normalized adjacency [V, V] (mean over the neighbours)."""
    e = set()
    for f in faces:
        for i in range(3):
            a, b = int(f[i]), int(f[(i + 1) % 3])
            e.add((a, b))
            e.add((b, a))
    idx = np.asarray(sorted(e), np.int64).T
    deg = np.bincount(idx[0], minlength=V).astype(np.float64)
    val = 1.0 / deg[idx[0]]
    return torch.sparse_coo_tensor(torch.as_tensor(idx), torch.as_tensor(val, dtype=torch.float32), (V, V))


def smoothness_loss(verts: torch.Tensor, ef: torch.Tensor) -> torch.Tensor:
    """sum over edges of (cos theta + 1)^2, theta the dihedral angle between
    the two faces at the edge (pi for a flat surface, so the term is 0)."""
    a, b, c, d = verts[ef[:, 0]], verts[ef[:, 1]], verts[ef[:, 2]], verts[ef[:, 3]]
    n1 = torch.cross(b - a, c - a, dim=1)
    n2 = torch.cross(a - b, d - b, dim=1)
    cos_n = (n1 * n2).sum(1) / (n1.norm(dim=1) * n2.norm(dim=1) + 1e-12)
    return ((1.0 - cos_n) ** 2).sum()        # cos theta = -cos(angle between the normals)


def laplacian_loss(delta: torch.Tensor, adj: torch.Tensor) -> torch.Tensor:
    """sum_v |delta_v - mean over the neighbours of delta|^2."""
    return ((delta - torch.sparse.mm(adj, delta)) ** 2).sum()


class MultiViewRecovery:
    """State of one recovery run: template, targets of all views, optimizer."""

    def __init__(self, template, views: Sequence[np.ndarray], targets: Sequence[torch.Tensor],
                 batch: int = 16, seed: int = 0, device="cuda", opts: RenderOptions = None):
        dev = torch.device(device)
        self.rest = torch.as_tensor(template.verts, device=dev)
        self.faces = torch.as_tensor(template.faces, device=dev)
        self.delta = torch.zeros_like(self.rest, requires_grad=True)
        self.colors = torch.as_tensor(template.attrs, device=dev).clone().requires_grad_(True)
        self.verts = self.rest.clone()               # rest + delta, read by the renderer
        self.attrs = self.colors.detach().clone()    # colours, read by the renderer
        self.model = torch.as_tensor(np.ascontiguousarray(template.keyframe_model, np.float32), device=dev)
        self.cams = [make_camera(v, template.tan_half_fov, template.width, template.height) for v in views]
        self.targets = list(targets)
        self.batch = batch
        self.K = template.num_subframes
        self.ef = torch.as_tensor(edge_faces(template.faces), device=dev)
        self.adj = neighbours(template.faces, len(template.verts)).to(dev)
        self.opt = torch.optim.Adam([self.delta, self.colors], lr=0.01, betas=(0.5, 0.99))
        self.rng = np.random.default_rng(seed)
        self.order: List[int] = []
        o = opts or RenderOptions(0)
        self.r = BatchRenderer([SceneTensors(self.verts, self.faces, self.attrs, self.model,
                                             self.cams[i], self.K) for i in range(batch)], o)
        self.last = {}

    def next_views(self) -> List[int]:
        """16 views per iteration, each of the 40 once per epoch (seeded order)."""
        if len(self.order) < self.batch:
            self.order += list(self.rng.permutation(len(self.cams)))
        out, self.order = self.order[:self.batch], self.order[self.batch:]
        return out

    def step(self, views: Sequence[int] = None) -> None:
        views = list(views) if views is not None else self.next_views()
        with torch.no_grad():
            torch.add(self.rest, self.delta, out=self.verts)
            self.attrs.copy_(self.colors)
        self.r.set_cameras([self.cams[v] for v in views])
        self.r.fit()                                  # forward (grows lists if a view needs it)
        image_loss = 0.0
        for i, v in enumerate(views):
            diff = self.r.images[i] - self.targets[v]
            torch.sign(diff, out=self.r.grad_images[i])   # d/dI of the L1 loss
            image_loss = image_loss + diff.abs().sum()
        self.r.backward()
        self.opt.zero_grad(set_to_none=True)
        reg = LAMBDA_S * smoothness_loss(self.rest + self.delta, self.ef) + LAMBDA_L * laplacian_loss(self.delta,
                                                                                                      self.adj)
        reg.backward()                                # gradients of the regularizers (delta only)
        with torch.no_grad():
            self.delta.grad += torch.stack(self.r.grad_verts).sum(0)
            self.colors.grad = torch.stack(self.r.grad_attrs).sum(0)
        self.opt.step()
        self.last = {"views": views, "image_loss": image_loss, "reg": reg.detach()}
