"""Pins of the recovery loop's regularizers (App. G) and mesh helpers against
closed forms: the dihedral-angle smoothness loss of a regular tetrahedron and
of a flat sheet, the Laplacian loss of a single displaced vertex, the
template's size and topology (App. J), and the 40 viewpoints (App. I)."""
import math

import numpy as np
import torch

from paper_2602_07860_amd import recovery as RC
from paper_2602_07860_amd import workloads as wl


def test_smoothness_of_tetrahedron_and_flat_sheet():
    # regular tetrahedron: every dihedral angle is arccos(1/3), so each of the
    # 6 edges adds (1/3 + 1)^2 = 16/9
    v = torch.tensor([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=torch.float64)
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    ef = torch.as_tensor(RC.edge_faces(f))
    assert len(ef) == 6
    assert abs(float(RC.smoothness_loss(v, ef)) - 6 * 16 / 9) < 1e-12
    # a flat square of two triangles: dihedral angle pi, loss 0
    sq = torch.tensor([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], dtype=torch.float64)
    ef2 = torch.as_tensor(RC.edge_faces(np.array([[0, 1, 2], [0, 2, 3]])))
    assert len(ef2) == 1 and float(RC.smoothness_loss(sq, ef2)) < 1e-20
    # folding the sheet by 90 degrees: cos(pi/2) + 1 = 1
    # rotate vertex 3 about the diagonal (0 -> 2) by 90 degrees out of the plane
    fold = sq.clone()
    axis = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    p3 = np.array([0.0, 1.0, 0.0])
    perp = p3 - axis * (p3 @ axis)
    fold[3] = torch.as_tensor(axis * (p3 @ axis) + np.cross(axis, perp), dtype=torch.float64)
    assert abs(float(RC.smoothness_loss(fold, ef2)) - 1.0) < 1e-12


def test_laplacian_of_one_displaced_vertex():
    v, f = wl.uv_sphere()
    V = len(v)
    adj = RC.neighbours(f, V)
    # neighbour counts straight from the faces
    nb = [set() for _ in range(V)]
    for a, b, c in f:
        nb[a] |= {b, c}
        nb[b] |= {a, c}
        nb[c] |= {a, b}
    assert float(RC.laplacian_loss(torch.zeros(V, 3), adj)) == 0.0
    k = 100
    d = torch.zeros(V, 3)
    d[k] = torch.tensor([0.3, -0.2, 0.1])
    want = float((d[k] ** 2).sum()) * (1.0 + sum(1.0 / len(nb[u]) ** 2 for u in nb[k]))
    assert abs(float(RC.laplacian_loss(d, adj)) - want) < 1e-6 * want


def test_template_and_viewpoints():
    v, f = wl.uv_sphere()
    assert v.shape == (1352, 3) and f.shape == (2700, 3)           # App. J template size
    e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), 1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert set(cnt.tolist()) == {2}                                  # closed, manifold
    assert len(RC.edge_faces(f)) == len(cnt)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert np.all((n * v[f].mean(1)).sum(1) > 0)                    # outward winding
    views = wl.multiview_cameras()
    assert len(views) == 40
    for m in views:
        R, t = m[:, :3].astype(np.float64), m[:, 3].astype(np.float64)
        eye = -R.T @ t
        assert abs(np.linalg.norm(eye) - 2.232) < 1e-5
        assert R[2] @ (-eye) > 0                                     # looks at the origin
