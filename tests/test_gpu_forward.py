"""Forward parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: per channel and on every pixel, I_gpu within 1e-5 * max|I_oracle| of
the oracle's value, or of the range the oracle gives for the pixel where one
of its sub-frames has a decision within float32 rounding distance of
flipping (guard band)."""
import ctypes

import numpy as np
import pytest

from paper_2602_07860_amd import binding as B
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

from gpu_common import assert_band_small, assert_image_parity, gpu_forward, reference, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("solver", ["fast", "recompute"])
def test_small_translation_parity(solver):
    sc = wl.make_workload(wl.SMALL)
    say(f"case: {sc.name} solver={solver}")
    ref = reference(sc)
    assert_band_small(ref, sc.name)
    img, _, _ = gpu_forward(sc, solver=solver)
    assert_image_parity(img, ref, label=f"small/{solver}")


@pytest.mark.parametrize("chunk_len,slice_len", [(1, 1), (2, 3), (8, 1), (8, 2), (4, 5), (4, 64)])
def test_chunking_does_not_change_the_image(chunk_len, slice_len):
    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=1.0),
                          num_segments=12, num_subframes=37)
    say(f"case: small rotate chunk_len={chunk_len} slice_len={slice_len}")
    ref = reference(sc)
    img, _, _ = gpu_forward(sc, chunk_len=chunk_len, slice_len=slice_len)
    assert_image_parity(img, ref, label=f"chunk{chunk_len}x{slice_len}")


@pytest.mark.parametrize("W,H,K,S", [(61, 37, 23, 5), (13, 70, 1, 1), (40, 40, 2, 1), (33, 31, 4, 7)])
def test_ragged_sizes_and_degenerate_schedules(W, H, K, S):
    # image edges that cut tiles, a single sub-frame, two sub-frames, and more
    # segments than sub-frame gaps (empty segments)
    sc = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.1, 0.8, 0.5), revs=0.6,
                                                     trans=(0.5, 0.2, 0.0)),
                          num_segments=S, num_subframes=K, width=W, height=H)
    say(f"case: ragged W={W} H={H} K={K} S={S}")
    ref = reference(sc)
    for solver in ("fast", "recompute"):
        img, _, _ = gpu_forward(sc, solver=solver, chunk_len=2)
        assert_image_parity(img, ref, label=f"ragged{W}x{H}K{K}S{S}/{solver}")


def test_medium_workload_full_image():
    sc = wl.make_workload(wl.MEDIUM)
    say(f"case: {sc.name} full image vs oracle")
    ref = reference(sc)
    assert_band_small(ref, sc.name)
    fast, _, _ = gpu_forward(sc, solver="fast")
    rec, _, _ = gpu_forward(sc, solver="recompute")
    assert_image_parity(fast, ref, label="medium/fast")
    assert_image_parity(rec, ref, label="medium/recompute")
    # the two solvers compute the same barycentrics (away from decisions
    # within rounding distance of flipping)
    ok = np.all(ref.image_hi == ref.image_lo, axis=0)
    assert np.abs(fast - rec)[:, ok].max() <= 5e-6


def test_overflow_is_reported_and_retried():
    import torch
    sc = wl.make_workload(wl.SMALL)
    st = R.scene_tensors(sc, "cuda")
    say("case: list overflow with capacity 64")
    opts = R.RenderOptions(sc.num_subframes)
    o = opts.c_struct(64)
    V, F, C = len(sc.verts), len(sc.faces), 3
    motion = B.rb_motion(sc.num_segments, st.model.data_ptr())
    n = B.rb_workspace_size(V, F, C, motion, st.camera, o)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    img = torch.empty((4, sc.height, sc.width), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    assert B.rb_render_blur_fwd(st.verts.data_ptr(), V, st.faces.data_ptr(), F, st.attrs.data_ptr(), C, motion,
                                st.camera, o, img.data_ptr(), ws.data_ptr(), n, stream) == B.RB_OK
    h = B.rb_read_header(ws.data_ptr(), stream)
    assert h.error_bits & B.HDR_OVERFLOW and h.list_entries > 64
    assert torch.isnan(img).all()
    # the front end grows the capacity and renders correctly
    R._capacity.clear()
    ref = reference(sc)
    good, _, _ = gpu_forward(sc)
    assert_image_parity(good, ref, label="after-retry")


def test_device_checks_raise():
    sc = wl.make_workload(wl.SMALL)
    bad = sc.faces.copy()
    bad[5, 1] = len(sc.verts) + 10
    say("case: face index out of range")
    with pytest.raises(B.RenderError) as e:
        gpu_forward(sc.with_(faces=bad))
    assert e.value.status == B.RB_ERANGE
    say("case: vertex behind the camera")
    v = sc.verts.copy()
    v[0] = (0.0, 0.0, 5.0)     # eye at z = 4 looking towards -z
    with pytest.raises(B.RenderError) as e:
        gpu_forward(sc.with_(verts=v))
    assert e.value.status == B.RB_EBEHIND


def test_cpu_tensors_are_refused():
    import torch
    sc = wl.make_workload(wl.SMALL)
    st = R.scene_tensors(sc, "cpu")
    with pytest.raises(ValueError):
        R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, R.RenderOptions(16))
