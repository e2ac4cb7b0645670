"""One iteration of the multi-view translational recovery loop
(paper_2602_07860_amd/recovery.py) on the GPU against the FP64 oracle: the
rendered views of the template on every pixel, and the renderer's share of
the vertex-offset and colour gradients (the adjoint of the L1 image loss
summed over the batch of views) against the sum of the oracle's adjoints of
the same views with the same upstream gradient."""
import numpy as np
import pytest

import oracle
from paper_2602_07860_amd import workloads as wl

from gpu_common import assert_grad_parity, assert_image_parity, say

pytestmark = pytest.mark.gpu


def test_recovery_step_matches_oracle():
    import torch
    from paper_2602_07860_amd import recovery as RC
    from paper_2602_07860_amd.batch import BatchRenderer
    from paper_2602_07860_amd.render import RenderOptions, SceneTensors, scene_tensors, make_camera
    target, template, views = wl.make_multiview(num_subframes=24, res=64)
    pick = [0, 13, 27]
    say(f"case: recovery step, views {pick}, 64x64, K=24")
    tt = scene_tensors(target, "cuda")
    cams = [make_camera(v, target.tan_half_fov, 64, 64) for v in views]
    tr = BatchRenderer([SceneTensors(tt.verts, tt.faces, tt.attrs, tt.model, cams[v], 24) for v in pick],
                       RenderOptions(0))
    tr.fit()
    targets = [None] * len(views)
    for i, v in enumerate(pick):
        targets[v] = tr.images[i].clone()
    run = RC.MultiViewRecovery(template, views, targets, batch=len(pick))
    run.step(pick)
    torch.cuda.synchronize()
    gv = torch.stack(run.r.grad_verts).sum(0).double().cpu().numpy()
    ga = torch.stack(run.r.grad_attrs).sum(0).double().cpu().numpy()
    ogv, oga = np.zeros_like(gv), np.zeros_like(ga)
    sv, sa = np.zeros_like(gv), np.zeros_like(ga)
    for i, v in enumerate(pick):
        sc = template.with_(view=views[v])
        G = run.r.grad_images[i].double().cpu().numpy()
        ref = oracle.render(sc, grad_image=G, bounds=True)
        assert_image_parity(run.r.images[i].double().cpu().numpy(), ref, label=f"recovery view {v}")
        ogv += ref.grad_verts
        oga += ref.grad_attrs
        sv += ref.slack_verts
        sa += ref.slack_attrs
    assert_grad_parity(gv, ogv, sv, label="recovery step verts")
    assert_grad_parity(ga, oga, sa, label="recovery step attrs")
    assert float(run.last["image_loss"]) > 0
