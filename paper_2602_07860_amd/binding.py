"""ctypes binding of the C ABI in include/motion_blur_raster.h (same names).

Argument marshalling only: every step of the rendering runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

from .build import LIB

RB_OK, RB_EINVAL, RB_ERANGE, RB_EWORKSPACE, RB_EBEHIND, RB_EOVERFLOW, RB_EDEVICE, RB_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
RB_SOLVER_FAST, RB_SOLVER_RECOMPUTE = 0, 1
RB_MAX_CHANNELS = 4
RB_MAX_FACES = 1 << 23
RB_MAX_CHUNK = 8
RB_STATIC_SCRATCH_BYTES = 64 << 20
HDR_FACE_RANGE, HDR_BEHIND, HDR_OVERFLOW, HDR_DET_RANGE = 1, 2, 4, 8
RB_FLAG_DETERMINISTIC = 1

RB_BATCH_FORWARD, RB_BATCH_BACKWARD = 0, 1

EXPORTED = ["rb_workspace_size", "rb_validate", "rb_render_blur_fwd", "rb_render_blur_fwd_static",
            "rb_render_blur_bwd",
            "rb_batch_workspace_size", "rb_render_blur_batched", "rb_batch_read_headers",
            "rb_read_header", "rb_profile_enable", "rb_profile_read", "rb_status_string"]


class rb_camera(ctypes.Structure):
    _fields_ = [("view", ctypes.c_float * 12), ("tan_half_fov", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class rb_motion(ctypes.Structure):
    _fields_ = [("num_segments", ctypes.c_int32), ("keyframe_model", ctypes.c_void_p)]


class rb_options(ctypes.Structure):
    _fields_ = [("num_subframes", ctypes.c_int32), ("delta", ctypes.c_float),
                ("eps_cutoff", ctypes.c_float), ("solver", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("chunk_len", ctypes.c_int32),
                ("slice_len", ctypes.c_int32), ("list_capacity", ctypes.c_int64),
                ("tile_w", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class rb_header(ctypes.Structure):
    _fields_ = [("error_bits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("list_entries", ctypes.c_int64), ("list_capacity", ctypes.c_int64)]


class rb_profile_stats(ctypes.Structure):
    _fields_ = [("project_ms", ctypes.c_double), ("bin_ms", ctypes.c_double),
                ("fg_ms", ctypes.c_double), ("bg_ms", ctypes.c_double),
                ("resolve_ms", ctypes.c_double), ("fg_bwd_ms", ctypes.c_double),
                ("bg_bwd_ms", ctypes.c_double), ("vertex_grad_ms", ctypes.c_double),
                ("fwd_calls", ctypes.c_int64), ("bwd_calls", ctypes.c_int64)]


class rb_instance(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("V", ctypes.c_int32),
                ("faces", ctypes.c_void_p), ("F", ctypes.c_int32),
                ("attrs", ctypes.c_void_p), ("C", ctypes.c_int32),
                ("motion", rb_motion), ("camera", rb_camera),
                ("num_subframes", ctypes.c_int32), ("list_capacity", ctypes.c_int64),
                ("image", ctypes.c_void_p), ("grad_image", ctypes.c_void_p),
                ("grad_verts", ctypes.c_void_p), ("grad_attrs", ctypes.c_void_p)]


class RenderError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {rb_status_string(status)} ({status})")


_lib = None


def library_path() -> str:
    return LIB


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"HIP library not built: {LIB} missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
        L.rb_workspace_size.restype = i32
        L.rb_workspace_size.argtypes = [i32, i32, i32, P(rb_motion), P(rb_camera), P(rb_options), P(sz)]
        L.rb_validate.restype = i32
        L.rb_validate.argtypes = [i32, i32, i32, P(rb_motion), P(rb_camera), P(rb_options), sz]
        L.rb_render_blur_fwd.restype = i32
        L.rb_render_blur_fwd.argtypes = [vp, i32, vp, i32, vp, i32, P(rb_motion), P(rb_camera),
                                         P(rb_options), vp, vp, sz, vp]
        L.rb_render_blur_fwd_static.restype = i32
        L.rb_render_blur_fwd_static.argtypes = [vp, i32, vp, i32, vp, i32, P(rb_motion), P(rb_camera),
                                                P(rb_options), vp, vp]
        L.rb_render_blur_bwd.restype = i32
        L.rb_render_blur_bwd.argtypes = [vp, i32, vp, i32, vp, i32, P(rb_motion), P(rb_camera),
                                         P(rb_options), vp, vp, vp, vp, sz, vp]
        L.rb_read_header.restype = i32
        L.rb_read_header.argtypes = [vp, P(rb_header), vp]
        L.rb_profile_enable.restype = i32
        L.rb_profile_enable.argtypes = [i32]
        L.rb_profile_read.restype = i32
        L.rb_profile_read.argtypes = [P(rb_profile_stats)]
        L.rb_status_string.restype = ctypes.c_char_p
        L.rb_status_string.argtypes = [i32]
        L.rb_batch_workspace_size.restype = i32
        L.rb_batch_workspace_size.argtypes = [P(rb_instance), i32, P(rb_options), P(sz)]
        L.rb_render_blur_batched.restype = i32
        L.rb_render_blur_batched.argtypes = [P(rb_instance), i32, P(rb_options), i32, vp, sz, vp]
        L.rb_batch_read_headers.restype = i32
        L.rb_batch_read_headers.argtypes = [P(rb_instance), i32, P(rb_options), vp, P(rb_header), vp]
        _lib = L
    return _lib


def rb_workspace_size(V, F, C, motion: rb_motion, camera: rb_camera, options: rb_options) -> int:
    out = ctypes.c_size_t()
    st = lib().rb_workspace_size(V, F, C, ctypes.byref(motion), ctypes.byref(camera),
                                 ctypes.byref(options), ctypes.byref(out))
    if st != RB_OK:
        raise RenderError(st, "rb_workspace_size")
    return out.value


def rb_validate(V, F, C, motion, camera, options, workspace_bytes) -> int:
    m = ctypes.byref(motion) if motion is not None else None
    c = ctypes.byref(camera) if camera is not None else None
    o = ctypes.byref(options) if options is not None else None
    return lib().rb_validate(V, F, C, m, c, o, workspace_bytes)


def rb_render_blur_fwd(verts, V, faces, F, attrs, C, motion, camera, options, image,
                       workspace, workspace_bytes, stream) -> int:
    return lib().rb_render_blur_fwd(verts, V, faces, F, attrs, C, ctypes.byref(motion),
                                    ctypes.byref(camera), ctypes.byref(options), image,
                                    workspace, workspace_bytes, stream)


def rb_render_blur_fwd_static(verts, V, faces, F, attrs, C, motion, camera, options, image, stream) -> int:
    return lib().rb_render_blur_fwd_static(verts, V, faces, F, attrs, C, ctypes.byref(motion),
                                           ctypes.byref(camera), ctypes.byref(options), image, stream)


def rb_render_blur_bwd(verts, V, faces, F, attrs, C, motion, camera, options, grad_image,
                       grad_verts, grad_attrs, workspace, workspace_bytes, stream) -> int:
    return lib().rb_render_blur_bwd(verts, V, faces, F, attrs, C, ctypes.byref(motion),
                                    ctypes.byref(camera), ctypes.byref(options), grad_image,
                                    grad_verts, grad_attrs, workspace, workspace_bytes, stream)


def rb_batch_workspace_size(instances, options: rb_options) -> int:
    arr = (rb_instance * len(instances))(*instances)
    out = ctypes.c_size_t()
    st = lib().rb_batch_workspace_size(arr, len(instances), ctypes.byref(options), ctypes.byref(out))
    if st != RB_OK:
        raise RenderError(st, "rb_batch_workspace_size")
    return out.value


def rb_render_blur_batched(instances, options: rb_options, mode: int, workspace, workspace_bytes,
                           stream) -> int:
    arr = (rb_instance * len(instances))(*instances)
    return lib().rb_render_blur_batched(arr, len(instances), ctypes.byref(options), mode, workspace,
                                        workspace_bytes, stream)


def rb_batch_read_headers(instances, options: rb_options, workspace, stream):
    arr = (rb_instance * len(instances))(*instances)
    out = (rb_header * len(instances))()
    st = lib().rb_batch_read_headers(arr, len(instances), ctypes.byref(options), workspace, out, stream)
    if st != RB_OK:
        raise RenderError(st, "rb_batch_read_headers")
    return list(out)


def rb_read_header(workspace, stream) -> rb_header:
    h = rb_header()
    st = lib().rb_read_header(workspace, ctypes.byref(h), stream)
    if st != RB_OK:
        raise RenderError(st, "rb_read_header")
    return h


def rb_profile_enable(enable: bool) -> None:
    st = lib().rb_profile_enable(1 if enable else 0)
    if st != RB_OK:
        raise RenderError(st, "rb_profile_enable")


def rb_profile_read() -> rb_profile_stats:
    s = rb_profile_stats()
    st = lib().rb_profile_read(ctypes.byref(s))
    if st != RB_OK:
        raise RenderError(st, "rb_profile_read")
    return s


def rb_status_string(status: int) -> str:
    try:
        return lib().rb_status_string(status).decode()
    except RuntimeError:
        return f"status {status}"
