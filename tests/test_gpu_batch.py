"""Batched path (one launch sequence over many instances, graph capture,
autotuner) through the C ABI: every instance of a batch against its own
single-instance render and against the FP64 oracle; graph replays against the
eager step."""
import numpy as np
import pytest
import torch

from paper_2602_07860_amd import batch as BT
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

from gpu_common import assert_grad_parity, assert_image_parity, gpu_backward, gpu_forward, reference, rel_l2, say

pytestmark = pytest.mark.gpu


def _scenes():
    return [
        wl.make_workload(wl.SMALL),
        wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.8, trans=(0.3, 0.0, 0.0)),
                         num_segments=10, num_subframes=41, width=48, height=40),
        wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.1, 0.8, 0.5), revs=0.6, trans=(0.5, 0.2, 0.0)),
                         num_segments=5, num_subframes=23, width=61, height=37),
        wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.1, 0.8, 0.5), revs=0.6, trans=(0.5, 0.2, 0.0)),
                         num_segments=7, num_subframes=4, width=33, height=31),
    ]


@pytest.fixture(scope="module")
def case():
    scs = _scenes()
    Gs = [np.random.default_rng(10 + i).normal(size=(sc.attrs.shape[1] + 1, sc.height, sc.width))
          for i, sc in enumerate(scs)]
    ogs = [reference(sc, G) for sc, G in zip(scs, Gs)]
    return scs, ogs, Gs, ogs


@pytest.mark.parametrize("chunk_len,slice_len", [(4, 0), (8, 32), (1, 128)])
def test_batch_matches_single_and_oracle(case, chunk_len, slice_len):
    scs, refs, Gs, ogs = case
    say(f"case: batch of {len(scs)} chunk_len={chunk_len} slice_len={slice_len}")
    sts = [R.scene_tensors(sc, "cuda") for sc in scs]
    r = BT.BatchRenderer(sts, R.RenderOptions(0, chunk_len=chunk_len, slice_len=slice_len))
    r.fit()
    imgs = [im.double().cpu().numpy() for im in r.forward()]
    for g, G in zip(r.grad_images, Gs):
        g.copy_(torch.as_tensor(G, dtype=torch.float32))
    r.backward()
    torch.cuda.synchronize()
    for i, sc in enumerate(scs):
        single, state, st = gpu_forward(sc, chunk_len=chunk_len, slice_len=slice_len)
        scale = np.abs(single).max()
        d = np.abs(imgs[i] - single).max() / scale
        say(f"  instance {i}: batch vs single max rel {d:.2e}")
        assert d <= 1e-6
        assert_image_parity(imgs[i], refs[i], label=f"batch{i}")
        gv1, ga1 = gpu_backward(st, state, Gs[i])
        gv = r.grad_verts[i].double().cpu().numpy()
        ga = r.grad_attrs[i].double().cpu().numpy()
        e1, e2 = rel_l2(gv, gv1), rel_l2(ga, ga1)
        say(f"  instance {i}: grads batch vs single {e1:.2e} {e2:.2e}")
        assert e1 <= 1e-5 and e2 <= 1e-5
        assert_grad_parity(gv, ogs[i].grad_verts, ogs[i].slack_verts, label=f"batch{i} verts")
        assert_grad_parity(ga, ogs[i].grad_attrs, ogs[i].slack_attrs, label=f"batch{i} attrs")


def test_graph_replays_match_eager(case):
    scs, refs, Gs, ogs = case
    say("case: graph capture of the batched L2 step, 3 replays")
    sts = [R.scene_tensors(sc, "cuda") for sc in scs]
    targets = [torch.as_tensor(ref.image, dtype=torch.float32, device="cuda") * 0.9 for ref in refs]
    r = BT.BatchRenderer(sts, R.RenderOptions(0))
    r.fit()
    step = BT.L2Step(r, targets)
    step.eager()
    torch.cuda.synchronize()
    want_img = [im.clone() for im in r.images]
    want_gv = [g.clone() for g in r.grad_verts]
    want_ga = [g.clone() for g in r.grad_attrs]
    step.capture()
    for rep in range(3):
        for t in r.images + r.grad_verts + r.grad_attrs:
            t.fill_(float("nan"))          # eager work between replays
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        for i in range(len(scs)):
            di = (r.images[i] - want_img[i]).abs().max().item() / want_img[i].abs().max().item()
            dv = rel_l2(r.grad_verts[i].double().cpu().numpy(), want_gv[i].double().cpu().numpy())
            da = rel_l2(r.grad_attrs[i].double().cpu().numpy(), want_ga[i].double().cpu().numpy())
            say(f"  replay {rep} instance {i}: image {di:.2e} grads {dv:.2e} {da:.2e}")
            assert di <= 1e-6 and dv <= 1e-5 and da <= 1e-5


def test_autotuner_picks_a_valid_configuration(case):
    scs, refs, Gs, ogs = case
    say("case: autotuner on a batch of 4")
    sts = [R.scene_tensors(sc, "cuda") for sc in scs]
    targets = [torch.as_tensor(ref.image, dtype=torch.float32, device="cuda") for ref in refs]
    import os
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(), "autotune.json")
    timed = []

    def log(m):
        timed.append(m)
        say(m)

    T, SL, TW = BT.autotune(sts, targets, chunk_lens=(2, 4), slice_lens=(32, 64), reps=2, log=log, cache_path=cache)
    assert T in (2, 4) and SL in (32, 64) and TW in (8, 16, 4)
    # 2 x 2 (chunk, slice) pairs on 8 x 8 tiles, then the two other tile shapes
    assert len(timed) == 6
    assert BT.autotune(sts, targets, chunk_lens=(2, 4), slice_lens=(32, 64)) == (T, SL, TW)
    # a fresh process state reads the batch class from the file without timing
    BT._tuned.clear()
    timed.clear()
    assert BT.autotune(sts, targets, chunk_lens=(2, 4), slice_lens=(32, 64), log=log,
                       cache_path=cache) == (T, SL, TW)
    assert not timed
