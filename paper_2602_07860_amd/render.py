"""PyTorch front end of the HIP motion-blur rasterizer.

PyTorch supplies device memory, the current stream and autograd; every step of
the rendering (projection, binning, rasterization, adjoint) runs in the HIP
library through the C ABI (binding.py).  There is no CPU or PyTorch fallback:
without the built library, or with CPU tensors, calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import binding as B


@dataclasses.dataclass
class RenderOptions:
    num_subframes: int
    delta: float = 1e-4          # App. J
    eps_cutoff: float = 1e-8     # probabilities below this are dropped
    solver: str = "fast"         # "fast" (eq 8) or "recompute" (per sub-frame solve)
    chunk_len: int = 4           # sub-frames per work chunk (1, 2, 4, 8)
    slice_len: int = 0           # background-list entries per task (0: automatic)
    check: bool = True           # read the device header after each forward (one sync)
    deterministic: bool = False  # bitwise-reproducible results (RB_FLAG_DETERMINISTIC; slower)
    tile_w: int = 0              # tile width in pixels: 4, 8 or 16 (height 64 / tile_w); 0 = 8

    def c_struct(self, capacity: int) -> B.rb_options:
        o = B.rb_options()
        o.num_subframes = int(self.num_subframes)
        o.delta = float(self.delta)
        o.eps_cutoff = float(self.eps_cutoff)
        o.solver = {"fast": B.RB_SOLVER_FAST, "recompute": B.RB_SOLVER_RECOMPUTE}[self.solver]
        o.flags = B.RB_FLAG_DETERMINISTIC if self.deterministic else 0
        o.chunk_len = int(self.chunk_len)
        o.slice_len = int(self.slice_len)
        o.list_capacity = int(capacity)
        o.tile_w = int(self.tile_w)
        return o


def make_camera(view, tan_half_fov: float, width: int, height: int) -> B.rb_camera:
    c = B.rb_camera()
    v = np.asarray(view, np.float32).reshape(12)
    for i in range(12):
        c.view[i] = float(v[i])
    c.tan_half_fov = float(np.float32(tan_half_fov))
    c.width = int(width)
    c.height = int(height)
    return c


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_tensor(t: torch.Tensor, name: str, dtype) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the renderer has no CPU path)")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")


# bin-list capacity that the last call of the same shape needed
_capacity: Dict[tuple, int] = {}


@dataclasses.dataclass
class ForwardState:
    """What the backward needs from the forward: the workspace and its plan."""
    workspace: torch.Tensor
    ws_bytes: int
    options: B.rb_options
    motion: B.rb_motion
    camera: B.rb_camera


def render_forward(verts: torch.Tensor, faces: torch.Tensor, attrs: torch.Tensor, model: torch.Tensor,
                   camera: B.rb_camera, opts: RenderOptions) -> Tuple[torch.Tensor, ForwardState]:
    """image [C+1, H, W] (attributes premultiplied by coverage, alpha last)."""
    for t, n, d in ((verts, "verts", torch.float32), (faces, "faces", torch.int32),
                    (attrs, "attrs", torch.float32), (model, "keyframe_model", torch.float32)):
        _check_tensor(t, n, d)
    V, F, C = verts.shape[0], faces.shape[0], attrs.shape[1]
    S = model.shape[0] - 1
    motion = B.rb_motion(S, model.data_ptr())
    key = (V, F, C, S, opts.num_subframes, camera.width, camera.height, opts.chunk_len,
           opts.slice_len, opts.solver)
    cap = _capacity.get(key)
    known = cap is not None
    if cap is None:
        cap = max(1 << 20, 6 * F * (opts.num_subframes // max(1, opts.chunk_len) + S))
    stream = _stream_ptr(verts.device)
    for _ in range(4):
        o = opts.c_struct(cap)
        nbytes = B.rb_workspace_size(V, F, C, motion, camera, o)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=verts.device)
        image = torch.empty((C + 1, camera.height, camera.width), dtype=torch.float32, device=verts.device)
        st = B.rb_render_blur_fwd(verts.data_ptr(), V, faces.data_ptr(), F, attrs.data_ptr(), C,
                                  motion, camera, o, image.data_ptr(), ws.data_ptr(), nbytes, stream)
        if st != B.RB_OK:
            raise B.RenderError(st, "rb_render_blur_fwd")
        if known and not opts.check:
            break
        h = B.rb_read_header(ws.data_ptr(), stream)
        if h.error_bits & B.HDR_FACE_RANGE:
            raise B.RenderError(B.RB_ERANGE, "rb_render_blur_fwd")
        if h.error_bits & B.HDR_BEHIND:
            raise B.RenderError(B.RB_EBEHIND, "rb_render_blur_fwd")
        if h.error_bits & B.HDR_OVERFLOW:
            cap = int(h.list_entries * 1.25) + 4096
            known = False
            continue
        if not known:
            _capacity[key] = int(h.list_entries * 1.25) + 4096 if h.list_entries * 1.25 + 4096 > cap else cap
        break
    else:
        raise B.RenderError(B.RB_EOVERFLOW, "rb_render_blur_fwd")
    return image, ForwardState(ws, nbytes, o, motion, camera)


def render_backward(verts, faces, attrs, model, state: ForwardState, grad_image: torch.Tensor):
    grad_image = grad_image.contiguous().to(torch.float32)
    _check_tensor(grad_image, "grad_image", torch.float32)
    V, F, C = verts.shape[0], faces.shape[0], attrs.shape[1]
    gv = torch.empty((V, 3), dtype=torch.float32, device=verts.device)
    ga = torch.empty((V, C), dtype=torch.float32, device=verts.device)
    motion = B.rb_motion(model.shape[0] - 1, model.data_ptr())
    st = B.rb_render_blur_bwd(verts.data_ptr(), V, faces.data_ptr(), F, attrs.data_ptr(), C, motion,
                              state.camera, state.options, grad_image.data_ptr(), gv.data_ptr(),
                              ga.data_ptr(), state.workspace.data_ptr(), state.ws_bytes,
                              _stream_ptr(verts.device))
    if st != B.RB_OK:
        raise B.RenderError(st, "rb_render_blur_bwd")
    return gv, ga


class BlurRender(torch.autograd.Function):
    """Differentiable motion-blur render: (verts, attrs) -> image [C+1, H, W].

    Backward is the hand-written adjoint kernel (gradients through every
    sub-frame into the keyframes and the rest vertices, Sec. 3.3)."""

    @staticmethod
    def forward(ctx, verts, attrs, faces, model, camera, opts):
        image, state = render_forward(verts.detach().contiguous(), faces, attrs.detach().contiguous(),
                                      model, camera, opts)
        ctx.state = state
        ctx.save_for_backward(verts, attrs, faces, model)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        verts, attrs, faces, model = ctx.saved_tensors
        gv, ga = render_backward(verts.detach().contiguous(), faces, attrs.detach().contiguous(), model,
                                 ctx.state, grad_image)
        return gv, ga, None, None, None, None


def render(verts, attrs, faces, model, camera: B.rb_camera, opts: RenderOptions) -> torch.Tensor:
    return BlurRender.apply(verts, attrs, faces, model, camera, opts)


# ------------------------------------------------------------ scene helpers


@dataclasses.dataclass
class SceneTensors:
    verts: torch.Tensor
    faces: torch.Tensor
    attrs: torch.Tensor
    model: torch.Tensor
    camera: B.rb_camera
    num_subframes: int


def scene_tensors(sc, device="cuda") -> SceneTensors:
    """Device tensors of a workloads.Scene."""
    return SceneTensors(
        torch.as_tensor(np.ascontiguousarray(sc.verts, np.float32), device=device),
        torch.as_tensor(np.ascontiguousarray(sc.faces, np.int32), device=device),
        torch.as_tensor(np.ascontiguousarray(sc.attrs, np.float32), device=device),
        torch.as_tensor(np.ascontiguousarray(sc.keyframe_model, np.float32), device=device),
        make_camera(sc.view, sc.tan_half_fov, sc.width, sc.height),
        sc.num_subframes,
    )
