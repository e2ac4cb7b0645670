"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
(via the PyTorch front end) and compare with the FP64 oracle."""
import sys

import numpy as np

import oracle
from paper_2602_07860_amd import render as R

IMAGE_RTOL = 1e-5      # per channel, relative to the channel's max |I|
GRAD_RTOL = 1e-3       # relative L2 over all vertices


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_forward(sc, solver="fast", chunk_len=4, slice_len=0, delta=1e-4, eps=1e-8):
    import torch
    st = R.scene_tensors(sc, "cuda")
    opts = R.RenderOptions(sc.num_subframes, delta=delta, eps_cutoff=eps, solver=solver,
                           chunk_len=chunk_len, slice_len=slice_len)
    img, state = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, opts)
    torch.cuda.synchronize()
    return img.double().cpu().numpy(), state, st


def gpu_backward(st, state, G):
    import torch
    g = torch.as_tensor(np.ascontiguousarray(G, np.float32), device="cuda")
    gv, ga = R.render_backward(st.verts, st.faces, st.attrs, st.model, state, g)
    torch.cuda.synchronize()
    return gv.double().cpu().numpy(), ga.double().cpu().numpy()


def image_errors(gpu, orc, flags, rows=None):
    """max over unflagged pixels of |gpu - orc| / max|orc| per channel."""
    if rows is not None:
        gpu = gpu[:, rows[0]:rows[1]:rows[2]]
        orc = orc[:, rows[0]:rows[1]:rows[2]]
        flags = flags[rows[0]:rows[1]:rows[2]]
    ok = (flags & 1) == 0          # bit 0: value within rounding distance of a flip
    errs = []
    for c in range(orc.shape[0]):
        scale = max(np.abs(orc[c]).max(), 1e-30)
        d = np.abs(gpu[c] - orc[c])[ok] / scale
        errs.append(float(d.max()) if d.size else 0.0)
    return errs, int((~ok).sum())


def assert_image_parity(gpu, orc, flags, rows=None, tol=IMAGE_RTOL, label=""):
    errs, nflag = image_errors(gpu, orc, flags, rows)
    say(f"[{label}] per-channel max rel err {['%.2e' % e for e in errs]}, flagged px {nflag}")
    assert np.all(np.isfinite(gpu)), "non-finite GPU image"
    assert max(errs) <= tol, (label, errs)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
