"""Parity of the 32-instance mixed batch (face counts 1280-36980, 128^2 to
512^2, K 37-251, half translation, half rotation) rendered in one launch
sequence through rb_render_blur_batched, forward and adjoint captured in one
graph and replayed, against the FP64 oracle on sampled rows of four
instances (tests/golden/batch_rows.npz, written by
tests/golden/make_batch_rows.py): the one with the most faces, the one with
the most sub-frames (a 512^2 rotation), a 256^2 one with 35280 faces and a
512^2 rotation with 20480 faces.  Every pixel of those rows is compared and
carries an upstream gradient; the other instances get none."""
import os

import numpy as np
import pytest

from paper_2602_07860_amd import workloads as wl

from gpu_common import MAX_ALT_PIXSUB, assert_grad_parity, assert_image_bounds, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_rows.npz")


def _dense(n, width, idx, vals):
    out = np.zeros((n, width))
    out[idx] = vals
    return out


def test_batch32_instances_on_sampled_rows():
    import torch
    from paper_2602_07860_amd import batch as BT
    from paper_2602_07860_amd import render as R
    gold = np.load(GOLD)
    names = gold["counter_names"].tolist()
    scenes = wl.make_batch(seed=3, n=32)
    say(f"case: batch32 graph replay, checked instances {gold['instances'].tolist()}")
    r = BT.BatchRenderer([R.scene_tensors(sc, "cuda") for sc in scenes], R.RenderOptions(0))
    r.fit()
    for g in r.grad_images:
        g.zero_()
    for i in gold["instances"].tolist():
        rows = gold[f"i{i}_rows"]
        G = np.zeros(tuple(r.grad_images[i].shape))
        G[:, rows, :] = np.random.default_rng(int(gold["grad_seed"]) + i).normal(size=(G.shape[0], len(rows), G.shape[2]))
        r.grad_images[i].copy_(torch.as_tensor(G, dtype=torch.float32))

    def body():
        r.forward()
        r.backward()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        body()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body()
    for t in r.images + r.grad_verts + r.grad_attrs:
        t.fill_(float("nan"))
    graph.replay()
    torch.cuda.synchronize()
    hs = r.headers()
    assert not any(h.error_bits for h in hs)
    for i in gold["instances"].tolist():
        p = f"i{i}_"
        cnt = dict(zip(names, gold[p + "counters"].tolist()))
        tot = cnt["fg_pixsub"] + cnt["bg_pixsub"]
        assert cnt["unbounded_pixsub"] == 0 and cnt["alt_pixsub"] <= MAX_ALT_PIXSUB * tot
        sc = scenes[i]
        say(f"  instance {i}: {len(sc.faces)} faces, {sc.width}^2, K {sc.num_subframes}, S {sc.num_segments}; "
            f"{100 * cnt['alt_pixsub'] / tot:.2f}% pixel-sub-frames with an alternative")
        img = r.images[i].double().cpu().numpy()
        assert np.all(np.isfinite(img))
        rows = gold[p + "rows"]
        assert_image_bounds(img[:, rows, :], gold[p + "image"].astype(np.float64),
                            gold[p + "image_lo"].astype(np.float64), gold[p + "image_hi"].astype(np.float64),
                            label=f"batch32 instance {i}")
        gv = r.grad_verts[i].double().cpu().numpy()
        ga = r.grad_attrs[i].double().cpu().numpy()
        V, C = gv.shape[0], ga.shape[1]
        assert_grad_parity(gv, _dense(V, 3, gold[p + "gv_idx"], gold[p + "gv"]),
                           _dense(V, 3, gold[p + "gv_idx"], gold[p + "sv"]), label=f"batch32 instance {i} verts")
        assert_grad_parity(ga, _dense(V, C, gold[p + "ga_idx"], gold[p + "ga"]),
                           _dense(V, C, gold[p + "ga_idx"], gold[p + "sa"]), label=f"batch32 instance {i} attrs")
