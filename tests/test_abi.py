"""Host-only tests of the C ABI: the library loads, exports every entry point
declared in include/*.h, its structs match the header's layout, and every
argument check returns its status code without touching a GPU."""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2602_07860_amd import binding as B
from paper_2602_07860_amd import build as pkg_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = glob.glob(os.path.join(ROOT, "include", "*.h"))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pkg_build.LIB):
        pkg_build.build()
    return B.lib()


def _declared_functions():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(rb_[A-Za-z0-9_]+)\s*\(", txt, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_binding_names():
    assert set(_declared_functions()) == set(B.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", pkg_build.LIB], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    for name in _declared_functions():
        assert name in exported, name
        assert getattr(L, name) is not None


def test_struct_layouts_match_the_header(tmp_path):
    fields = [("rb_camera", None), ("rb_motion", None), ("rb_options", None), ("rb_header", None),
              ("rb_profile_stats", None), ("rb_instance", None), ("rb_options", "list_capacity"), ("rb_options", "tile_w"),
              ("rb_motion", "keyframe_model"), ("rb_instance", "motion"), ("rb_instance", "camera"),
              ("rb_instance", "list_capacity"), ("rb_instance", "grad_attrs"),
              ("rb_profile_stats", "fwd_calls")]
    exprs = [f"sizeof({t})" if f is None else f"offsetof({t}, {f})" for t, f in fields]
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "motion_blur_raster.h"\n'
                   'int main(void){' + "".join(f'printf("%zu\\n", (size_t){e});' for e in exprs)
                   + ' return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(getattr(B, t)) if f is None else getattr(getattr(B, t), f).offset for t, f in fields]
    assert got == want


def _args(V=100, F=50, C=3, S=2, K=16, W=64, H=48):
    cam = B.rb_camera()
    for i, v in enumerate([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, -1, 4]):
        cam.view[i] = v
    cam.tan_half_fov = 0.36
    cam.width, cam.height = W, H
    mo = B.rb_motion(S, 0x1000)      # host-side checks only look at the pointer's presence
    op = B.rb_options()
    op.num_subframes, op.delta, op.eps_cutoff, op.solver = K, 1e-4, 1e-8, B.RB_SOLVER_FAST
    op.chunk_len, op.slice_len, op.list_capacity = 4, 0, 1 << 16
    return V, F, C, mo, cam, op


def test_workspace_size_and_validate_ok(L):
    V, F, C, mo, cam, op = _args()
    n = B.rb_workspace_size(V, F, C, mo, cam, op)
    assert n > 0
    assert B.rb_validate(V, F, C, mo, cam, op, n) == B.RB_OK
    assert B.rb_validate(V, F, C, mo, cam, op, n - 1) == B.RB_EWORKSPACE
    # capacity and sub-frame count both grow the workspace
    op2 = _args()[5]
    op2.list_capacity = 1 << 20
    assert B.rb_workspace_size(V, F, C, mo, cam, op2) > n


def test_deterministic_flag_adds_the_fixed_point_sums(L):
    # RB_FLAG_DETERMINISTIC keeps [S+1][V][2] keyframe and [V][C] attribute
    # gradient sums as 64-bit integers in the workspace; its background tasks
    # are whole lists, so the task array holds capacity / slice_len fewer
    V, F, C, mo, cam, op = _args()
    op.list_capacity, op.slice_len = 1 << 20, 64
    n = B.rb_workspace_size(V, F, C, mo, cam, op)
    op.flags = B.RB_FLAG_DETERMINISTIC
    nd = B.rb_workspace_size(V, F, C, mo, cam, op)
    need = ((mo.num_segments + 1) * V * 2 + V * C) * 8 - (1 << 20) // 64 * 8
    assert abs((nd - n) - need) < 512
    assert B.rb_validate(V, F, C, mo, cam, op, nd) == B.RB_OK
    assert B.rb_validate(V, F, C, mo, cam, op, nd - 1) == B.RB_EWORKSPACE


@pytest.mark.parametrize("mutate,code", [
    (lambda a: a.update(V=0), B.RB_EINVAL),
    (lambda a: a.update(F=-1), B.RB_EINVAL),
    (lambda a: a.update(C=0), B.RB_EINVAL),
    (lambda a: a.update(C=5), B.RB_EUNSUPPORTED),
    (lambda a: a.update(F=1 << 23), B.RB_EUNSUPPORTED),
    (lambda a: setattr(a["op"], "num_subframes", 0), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "delta", 0.0), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "delta", float("nan")), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "eps_cutoff", 0.0), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "eps_cutoff", 1.0), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "solver", 7), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "chunk_len", 3), B.RB_EUNSUPPORTED),
    (lambda a: setattr(a["op"], "chunk_len", 16), B.RB_EUNSUPPORTED),
    (lambda a: setattr(a["op"], "list_capacity", -5), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "flags", 2), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "tile_w", 3), B.RB_EUNSUPPORTED),
    (lambda a: setattr(a["op"], "tile_w", 32), B.RB_EUNSUPPORTED),
    (lambda a: setattr(a["op"], "tile_w", -8), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "reserved", 1), B.RB_EINVAL),
    (lambda a: setattr(a["op"], "flags", -1), B.RB_EINVAL),
    (lambda a: setattr(a["cam"], "width", 0), B.RB_EINVAL),
    (lambda a: setattr(a["cam"], "tan_half_fov", -1.0), B.RB_EINVAL),
    (lambda a: a["cam"].view.__setitem__(3, float("inf")), B.RB_EINVAL),
    (lambda a: setattr(a["mo"], "num_segments", 0), B.RB_EINVAL),
    (lambda a: setattr(a["mo"], "keyframe_model", None), B.RB_EINVAL),
])
def test_validate_rejects(L, mutate, code):
    V, F, C, mo, cam, op = _args()
    n = B.rb_workspace_size(V, F, C, mo, cam, op)
    a = dict(V=V, F=F, C=C, mo=mo, cam=cam, op=op)
    mutate(a)
    assert B.rb_validate(a["V"], a["F"], a["C"], a["mo"], a["cam"], a["op"], n) == code


def test_null_structs_and_pointers_rejected(L):
    V, F, C, mo, cam, op = _args()
    assert B.rb_validate(V, F, C, None, cam, op, 1 << 30) == B.RB_EINVAL
    assert B.rb_validate(V, F, C, mo, None, op, 1 << 30) == B.RB_EINVAL
    assert B.rb_validate(V, F, C, mo, cam, None, 1 << 30) == B.RB_EINVAL
    # null device pointers are refused before any launch
    st = B.rb_render_blur_fwd(None, V, None, F, None, C, mo, cam, op, None, None, 1 << 30, None)
    assert st == B.RB_EINVAL
    st = B.rb_render_blur_bwd(None, V, None, F, None, C, mo, cam, op, None, None, None, None, 1 << 30, None)
    assert st == B.RB_EINVAL
    h = B.rb_header()
    assert L.rb_read_header(None, ctypes.byref(h), None) == B.RB_EINVAL


def test_status_strings(L):
    for code in range(-7, 1):
        assert isinstance(B.rb_status_string(code), str) and B.rb_status_string(code)
    assert B.rb_status_string(-99) == "unknown status"


def test_chunk_schedule_covers_every_subframe_once():
    # the host and kernels share seg_first/chunk_info; mirror the integer
    # arithmetic here and check it against t_k = k/(K-1) segment membership
    def seg_first(s, K, S):
        if K <= 1:
            return 0 if s == 0 else 1
        if s <= 0:
            return 0
        return -(-s * (K - 1) // S)

    for K in (1, 2, 7, 16, 64, 513):
        for S in (1, 3, 36, 60):
            seen = []
            for s in range(S):
                lo = seg_first(s, K, S)
                hi = K if s == S - 1 else seg_first(s + 1, K, S)
                for k in range(lo, hi):
                    t = 0.0 if K == 1 else k / (K - 1)
                    assert min(int(np.floor(t * S + 1e-12)), S - 1) == s
                    seen.append(k)
            assert seen == list(range(K))
