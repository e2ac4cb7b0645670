"""Batched rendering: many meshes of uneven size, sub-frame count and
resolution through one sequence of launches of the HIP library (every kernel
covers all instances; the background passes are persistent kernels over the
tasks of all instances), optionally captured once in a hipGraph and replayed,
with the chunk length, the background slice length and the tile shape
chosen by a small autotuner that times the candidates on the batch itself.

Argument marshalling only: all rendering work runs in the library.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import binding as B
from .render import RenderOptions, SceneTensors, _check_tensor, _stream_ptr


def _initial_capacity(st: SceneTensors, chunk_len: int) -> int:
    F = st.faces.shape[0]
    S = st.model.shape[0] - 1
    return max(1 << 20, 6 * F * (st.num_subframes // max(1, chunk_len) + S))


class BatchRenderer:
    """Fixed batch of scenes with preallocated outputs.

    forward() writes self.images[i] ([C+1, H, W] per instance); backward()
    reads self.grad_images[i] and writes self.grad_verts[i] / self.grad_attrs[i].
    Both are pure launch sequences on the current stream (no host copies, no
    allocation), so they can be captured in a CUDA/HIP graph; fit() grows the
    bin-list capacities until a forward needs no more, which must happen
    before capture."""

    def __init__(self, scenes: Sequence[SceneTensors], opts: RenderOptions,
                 capacities: Optional[List[int]] = None):
        self.scenes = list(scenes)
        self.opts = opts
        dev = self.scenes[0].verts.device
        for st in self.scenes:
            for t, n, d in ((st.verts, "verts", torch.float32), (st.faces, "faces", torch.int32),
                            (st.attrs, "attrs", torch.float32), (st.model, "keyframe_model", torch.float32)):
                _check_tensor(t, n, d)
        self.images = [torch.empty((st.attrs.shape[1] + 1, st.camera.height, st.camera.width),
                                   dtype=torch.float32, device=dev) for st in self.scenes]
        self.grad_images = [torch.zeros_like(im) for im in self.images]
        self.grad_verts = [torch.empty_like(st.verts) for st in self.scenes]
        self.grad_attrs = [torch.empty_like(st.attrs) for st in self.scenes]
        self.caps = list(capacities) if capacities else [_initial_capacity(st, opts.chunk_len) for st in self.scenes]
        self._plan()

    def _instances(self) -> List[B.rb_instance]:
        out = []
        for i, st in enumerate(self.scenes):
            x = B.rb_instance()
            x.verts, x.V = st.verts.data_ptr(), st.verts.shape[0]
            x.faces, x.F = st.faces.data_ptr(), st.faces.shape[0]
            x.attrs, x.C = st.attrs.data_ptr(), st.attrs.shape[1]
            x.motion = B.rb_motion(st.model.shape[0] - 1, st.model.data_ptr())
            x.camera = st.camera
            x.num_subframes = st.num_subframes
            x.list_capacity = int(self.caps[i])
            x.image = self.images[i].data_ptr()
            x.grad_image = self.grad_images[i].data_ptr()
            x.grad_verts = self.grad_verts[i].data_ptr()
            x.grad_attrs = self.grad_attrs[i].data_ptr()
            out.append(x)
        return out

    def _plan(self) -> None:
        self.inst = self._instances()
        self.o = self.opts.c_struct(0)
        self.ws_bytes = B.rb_batch_workspace_size(self.inst, self.o)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.images[0].device)

    def set_cameras(self, cameras: Sequence[B.rb_camera]) -> None:
        """Give the instances new cameras of the same image sizes (host
        records only; the workspace is kept unless the plan needs more)."""
        for st, cam in zip(self.scenes, cameras):
            if (cam.width, cam.height) != (st.camera.width, st.camera.height):
                raise ValueError("set_cameras keeps every instance's image size")
            st.camera = cam
        self.inst = self._instances()
        need = B.rb_batch_workspace_size(self.inst, self.o)
        if need > self.ws_bytes:
            self.ws_bytes = need
            self.workspace = torch.empty(need, dtype=torch.uint8, device=self.images[0].device)

    def forward(self) -> List[torch.Tensor]:
        st = B.rb_render_blur_batched(self.inst, self.o, B.RB_BATCH_FORWARD, self.workspace.data_ptr(),
                                      self.ws_bytes, _stream_ptr(self.workspace.device))
        if st != B.RB_OK:
            raise B.RenderError(st, "rb_render_blur_batched(forward)")
        return self.images

    def backward(self) -> Tuple[List[torch.Tensor], List[torch.Tensor]]:
        st = B.rb_render_blur_batched(self.inst, self.o, B.RB_BATCH_BACKWARD, self.workspace.data_ptr(),
                                      self.ws_bytes, _stream_ptr(self.workspace.device))
        if st != B.RB_OK:
            raise B.RenderError(st, "rb_render_blur_batched(backward)")
        return self.grad_verts, self.grad_attrs

    def headers(self) -> List[B.rb_header]:
        return B.rb_batch_read_headers(self.inst, self.o, self.workspace.data_ptr(),
                                       _stream_ptr(self.workspace.device))

    def fit(self, max_rounds: int = 4) -> None:
        """Run the forward, grow every overflowing list capacity and re-plan
        until no instance overflows; raise on device-side argument errors."""
        for _ in range(max_rounds):
            self.forward()
            hs = self.headers()
            grow = False
            for i, h in enumerate(hs):
                if h.error_bits & B.HDR_FACE_RANGE:
                    raise B.RenderError(B.RB_ERANGE, f"instance {i}")
                if h.error_bits & B.HDR_BEHIND:
                    raise B.RenderError(B.RB_EBEHIND, f"instance {i}")
                if h.error_bits & B.HDR_OVERFLOW:
                    self.caps[i] = int(h.list_entries * 1.25) + 4096
                    grow = True
            if not grow:
                return
            self._plan()
        raise B.RenderError(B.RB_EOVERFLOW, "BatchRenderer.fit")


class L2Step:
    """One fwd + dL/dimage + bwd step of an L2 loss against fixed targets,
    eager or captured in a graph and replayed."""

    def __init__(self, renderer: BatchRenderer, targets: Sequence[torch.Tensor]):
        self.r = renderer
        self.targets = list(targets)
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def _body(self) -> None:
        imgs = self.r.forward()
        for g, im, tg in zip(self.r.grad_images, imgs, self.targets):
            torch.sub(im, tg, out=g)
            g.mul_(2.0)
        self.r.backward()

    def eager(self) -> None:
        self._body()

    def capture(self) -> None:
        # warm up on a side stream (required before capture), then capture
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._body()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._body()

    def replay(self) -> None:
        self.graph.replay()


# ---------------------------------------------------------------- autotuner

_tuned: Dict[tuple, Tuple[int, int]] = {}


def batch_signature(scenes: Sequence[SceneTensors], solver: str) -> tuple:
    return (solver,) + tuple((st.verts.shape[0], st.faces.shape[0], st.attrs.shape[1], st.model.shape[0],
                              st.num_subframes, st.camera.width, st.camera.height) for st in scenes)


def batch_class(scenes: Sequence[SceneTensors], solver: str) -> str:
    """Coarse class of a batch for the on-disk cache: solver, instance count,
    the count of each image size, and the total faces, the median sub-frame
    count and the median segment count rounded to powers of two."""
    import math
    res: Dict[str, int] = {}
    for st in scenes:
        k = f"{st.camera.width}x{st.camera.height}"
        res[k] = res.get(k, 0) + 1
    p2 = lambda x: int(round(math.log2(max(1, x))))
    faces = sum(int(st.faces.shape[0]) for st in scenes)
    ks = sorted(int(st.num_subframes) for st in scenes)
    ss = sorted(int(st.model.shape[0]) - 1 for st in scenes)
    return (f"{solver}|n{len(scenes)}|" + ",".join(f"{k}:{v}" for k, v in sorted(res.items()))
            + f"|F2^{p2(faces)}|K2^{p2(ks[len(ks) // 2])}|S2^{p2(ss[len(ss) // 2])}")


def _load_cache(path: str) -> Dict[str, list]:
    import json
    import os
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _store_cache(path: str, key: str, value: Tuple[int, ...]) -> None:
    import json
    import os
    data = _load_cache(path)
    data[key] = list(value)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(scenes: Sequence[SceneTensors], targets: Sequence[torch.Tensor], solver: str = "fast",
             chunk_lens=(1, 2, 4, 8), slice_lens=(32, 64, 128, 256), tile_ws=(8, 16, 4), reps: int = 3,
             log=None, cache_path: Optional[str] = None) -> Tuple[int, int, int]:
    """Chunk length, background slice length and tile width with the shortest
    fwd+bwd L2 step on this batch (each candidate timed with device events
    over `reps` eager steps after one warm-up that also sizes its lists):
    every (chunk, slice) pair on the first tile shape, then the other tile
    shapes at the best pair.  Results are remembered per batch signature in
    memory and, with cache_path, per batch class (batch_class) in a JSON file
    that later runs read instead of timing."""
    key = batch_signature(scenes, solver)
    if key in _tuned:
        return _tuned[key]
    if cache_path:
        hit = _load_cache(cache_path).get(batch_class(scenes, solver))
        if hit is not None and len(hit) == 3 and hit[0] in chunk_lens and hit[1] in slice_lens and hit[2] in tile_ws:
            _tuned[key] = (int(hit[0]), int(hit[1]), int(hit[2]))
            return _tuned[key]

    def time_one(T, SL, TW, caps):
        r = BatchRenderer(scenes, RenderOptions(0, solver=solver, chunk_len=T, slice_len=SL, tile_w=TW), caps)
        r.fit()
        step = L2Step(r, targets)
        step.eager()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step.eager()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if log:
            log(f"autotune T={T} SL={SL} tile={TW}x{64 // TW}: {ms:.3f} ms")
        return ms, r.caps

    best, best_ms = None, float("inf")
    TW0 = tile_ws[0]
    for T in chunk_lens:
        caps = None   # list sizes depend on the chunk length and the tiles
        for SL in slice_lens:
            ms, caps = time_one(T, SL, TW0, caps)
            if ms < best_ms:
                best, best_ms = (T, SL, TW0), ms
    for TW in tile_ws[1:]:
        ms, _ = time_one(best[0], best[1], TW, None)
        if ms < best_ms:
            best, best_ms = (best[0], best[1], TW), ms
    _tuned[key] = best
    if cache_path:
        _store_cache(cache_path, batch_class(scenes, solver), best)
    return best
