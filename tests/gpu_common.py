"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
(via the PyTorch front end) and compare with the FP64 oracle.

Every pixel and every gradient component is compared.  Where the oracle finds
a decision within float32 rounding distance of flipping (its guard band), it
also returns the range the pixel can take over the other choices, and a bound
on how far those choices (and the float32 error of ill-conditioned sliver
terms) can move each gradient component:
  image:    lo - tol*scale <= I_gpu <= hi + tol*scale on every pixel, per channel
            (lo == hi == I_oracle wherever no decision is ambiguous);
  gradient: the residual g_gpu - g_oracle, shrunk per component by that bound,
            has relative L2 norm <= tol.  The raw residual is printed beside it.
"""
import sys

import numpy as np

import oracle
from paper_2602_07860_amd import render as R

IMAGE_RTOL = 1e-5      # per channel, relative to the channel's max |I|
GRAD_RTOL = 1e-3       # relative L2 over all vertices
# the guard band must stay a small part of the work: pixel-sub-frames with an
# alternative decision, and pixels whose range is wider than the tolerance
MAX_ALT_PIXSUB = 0.05
MAX_WIDE_PIXELS = 0.05


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_forward(sc, solver="fast", chunk_len=4, slice_len=0, delta=1e-4, eps=1e-8, deterministic=False, tile_w=0):
    import torch
    st = R.scene_tensors(sc, "cuda")
    opts = R.RenderOptions(sc.num_subframes, delta=delta, eps_cutoff=eps, solver=solver,
                           chunk_len=chunk_len, slice_len=slice_len, deterministic=deterministic, tile_w=tile_w)
    img, state = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, opts)
    torch.cuda.synchronize()
    return img.double().cpu().numpy(), state, st


def gpu_backward(st, state, G):
    import torch
    g = torch.as_tensor(np.ascontiguousarray(G, np.float32), device="cuda")
    gv, ga = R.render_backward(st.verts, st.faces, st.attrs, st.model, state, g)
    torch.cuda.synchronize()
    return gv.double().cpu().numpy(), ga.double().cpu().numpy()


def reference(sc, G=None, rows=None):
    """The oracle's image (and adjoint of G) with the guard band's bounds."""
    return oracle.render(sc, grad_image=G, bounds=True, counters=True, rows=rows)


def image_check(gpu, image, lo, hi, tol=IMAGE_RTOL):
    """Per channel: the largest excursion of gpu outside [lo, hi], and the
    largest |gpu - image| on pixels without alternatives, both relative to
    the channel's max |image|; and the number of pixels whose range is wider
    than the tolerance."""
    out, exact, wide = [], [], 0
    for c in range(image.shape[0]):
        scale = max(np.abs(image[c]).max(), 1e-30)
        ex = np.maximum(np.maximum(lo[c] - gpu[c], gpu[c] - hi[c]), 0.0) / scale
        out.append(float(ex.max()) if ex.size else 0.0)
        sharp = hi[c] == lo[c]
        d = np.abs(gpu[c] - image[c])[sharp] / scale
        exact.append(float(d.max()) if d.size else 0.0)
        wide = max(wide, int(((hi[c] - lo[c]) > tol * scale).sum()))
    return out, exact, wide


def assert_image_parity(gpu, ref, tol=IMAGE_RTOL, label="", rows=None):
    image, lo, hi = ref.image, ref.image_lo, ref.image_hi
    if rows is not None:
        sl = slice(rows[0], rows[1], rows[2])
        gpu, image, lo, hi = gpu[:, sl], image[:, sl], lo[:, sl], hi[:, sl]
    assert_image_bounds(gpu, image, lo, hi, tol, label)


def assert_image_bounds(gpu, image, lo, hi, tol=IMAGE_RTOL, label=""):
    out, exact, wide = image_check(gpu, image, lo, hi, tol)
    touched = int((np.abs(image).sum(0) > 0).sum())
    say(f"[{label}] outside oracle range (rel) {['%.2e' % e for e in out]}; "
        f"|gpu - oracle| on pixels without alternatives {['%.2e' % e for e in exact]}; "
        f"pixels with a range wider than tol {wide} of {touched} touched")
    assert np.all(np.isfinite(gpu)), "non-finite GPU image"
    assert max(out) <= tol, (label, out)
    assert wide <= MAX_WIDE_PIXELS * max(touched, 1), (label, wide, touched)


def assert_grad_parity(g, ref, slack, tol=GRAD_RTOL, label=""):
    """Relative L2 of the residual shrunk by the oracle's per-component bound."""
    r = g - ref
    shrunk = np.sign(r) * np.maximum(np.abs(r) - slack, 0.0)
    n = max(float(np.linalg.norm(ref)), 1e-300)
    e_shr, e_raw = float(np.linalg.norm(shrunk)) / n, float(np.linalg.norm(r)) / n
    loose = float(np.linalg.norm(np.minimum(slack, np.abs(ref)))) / n
    say(f"[{label}] grad rel-L2 {e_shr:.2e} beyond the bound (raw {e_raw:.2e}; bound covers {loose:.2e} of |g|)")
    assert np.all(np.isfinite(g)), "non-finite GPU gradient"
    assert e_shr <= tol, (label, e_shr, e_raw)
    return e_shr, e_raw


def assert_band_small(ref, label=""):
    """The guard band covers few pixel-sub-frames and enumerates all of them."""
    c = ref.counters
    tot = max(c["fg_pixsub"] + c["bg_pixsub"], 1.0)
    say(f"[{label}] guard band: {c['alt_pixsub']:.0f} of {tot:.0f} pixel-sub-frames with an alternative "
        f"({100 * c['alt_pixsub'] / tot:.2f}%), {c['alt_value_pixsub']:.0f} with another value")
    assert c["unbounded_pixsub"] == 0
    assert c["alt_pixsub"] <= MAX_ALT_PIXSUB * tot


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
