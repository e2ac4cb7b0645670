"""rb_render_blur_fwd_static (the forward with a library-held workspace, for
callers that cannot allocate) against rb_render_blur_fwd with a caller
workspace, through the C ABI: two static calls in a row, the second with a
smaller input, each matching the workspace entry point's image; sizes beyond
the library-held array are refused before any launch."""
import numpy as np
import pytest

from paper_2602_07860_amd import binding as B
from paper_2602_07860_amd import render as R
from paper_2602_07860_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _args(sc, capacity=0):
    import torch
    st = R.scene_tensors(sc, "cuda")
    opts = R.RenderOptions(sc.num_subframes).c_struct(capacity)
    motion = B.rb_motion(sc.num_segments, st.model.data_ptr())
    img = torch.full((4, sc.height, sc.width), float("nan"), device="cuda")
    return st, opts, motion, img


def _with_workspace(sc):
    import torch
    st, opts, motion, img = _args(sc)
    V, F = len(sc.verts), len(sc.faces)
    n = B.rb_workspace_size(V, F, 3, motion, st.camera, opts)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert B.rb_render_blur_fwd(st.verts.data_ptr(), V, st.faces.data_ptr(), F, st.attrs.data_ptr(), 3, motion,
                                st.camera, opts, img.data_ptr(), ws.data_ptr(), n, s) == B.RB_OK
    torch.cuda.synchronize()
    return n, img.double().cpu().numpy()


def test_static_forward_matches_workspace_forward_on_two_calls():
    import torch
    big = wl.make_workload(wl.SMALL, motion=wl.Motion("rotate", axis=(0.3, 1.0, -0.2), revs=0.8,
                                                      trans=(0.3, 0.0, 0.0)),
                           num_segments=10, num_subframes=41, width=160, height=144)
    small = wl.make_workload(wl.SMALL)
    want = []
    for sc in (big, small):
        n, img = _with_workspace(sc)
        print(f"case: {sc.width}x{sc.height} K={sc.num_subframes}: workspace {n} bytes "
              f"(library-held {B.RB_STATIC_SCRATCH_BYTES})", flush=True)
        assert n <= B.RB_STATIC_SCRATCH_BYTES
        want.append(img)
    # two calls in a row on the same library-held array, the second smaller
    keep = []
    for sc in (big, small):
        st, opts, motion, img = _args(sc)
        s = torch.cuda.current_stream().cuda_stream
        assert B.rb_render_blur_fwd_static(st.verts.data_ptr(), len(sc.verts), st.faces.data_ptr(), len(sc.faces),
                                           st.attrs.data_ptr(), 3, motion, st.camera, opts, img.data_ptr(),
                                           s) == B.RB_OK
        keep.append((st, img))
    torch.cuda.synchronize()
    for (st, img), ref in zip(keep, want):
        got = img.double().cpu().numpy()
        assert np.all(np.isfinite(got))
        d = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"  static vs workspace forward {got.shape[2]}x{got.shape[1]}: max rel diff {d:.2e}", flush=True)
        assert d <= 1e-6


def test_static_forward_refuses_sizes_beyond_its_array():
    sc = wl.make_workload(wl.MEDIUM)
    st, opts, motion, img = _args(sc)
    n = B.rb_workspace_size(len(sc.verts), len(sc.faces), 3, motion, st.camera, opts)
    assert n > B.RB_STATIC_SCRATCH_BYTES
    assert B.rb_render_blur_fwd_static(st.verts.data_ptr(), len(sc.verts), st.faces.data_ptr(), len(sc.faces),
                                       st.attrs.data_ptr(), 3, motion, st.camera, opts, img.data_ptr(),
                                       None) == B.RB_EWORKSPACE
    assert B.rb_render_blur_fwd_static(0, len(sc.verts), st.faces.data_ptr(), len(sc.faces), st.attrs.data_ptr(),
                                       3, motion, st.camera, opts, img.data_ptr(), None) == B.RB_EINVAL
