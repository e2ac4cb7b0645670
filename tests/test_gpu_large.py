"""Parity at full size: the large workload (ico6, 81920 faces, 1024x1024,
K = 512, S = 60) rendered on the GPU in the launch configuration bench.py
times, compared on the pixel rows that tests/golden/large_rows.npz holds (the
FP64 oracle's image, guard-band flags and adjoint on every 128th row from row
192, written by tests/golden/make_large_rows.py)."""
import os

import numpy as np
import pytest

from paper_2602_07860_amd import workloads as wl

from gpu_common import GRAD_RTOL, IMAGE_RTOL, gpu_backward, gpu_forward, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_rows.npz")


def test_large_workload_sampled_rows():
    gold = np.load(GOLD)
    rows = gold["rows"]
    sc = wl.make_workload(wl.LARGE)
    say(f"case: {sc.name} full render, compared on rows {rows.tolist()}")
    img, state, st = gpu_forward(sc)
    got = img[:, rows, :]
    ref = gold["image"]
    flags = gold["flags"]
    ok = (flags & 1) == 0
    errs = [float((np.abs(got[c] - ref[c]) / max(np.abs(ref[c]).max(), 1e-30))[ok].max()) for c in range(ref.shape[0])]
    say(f"  image max rel err per channel {['%.2e' % e for e in errs]}, flagged px {int((~ok).sum())}")
    assert np.all(np.isfinite(img))
    assert max(errs) <= IMAGE_RTOL
    # the adjoint of dL/dI that is non-zero only on the sampled, unflagged rows
    G = np.zeros_like(img)
    G[:, rows, :] = np.random.default_rng(int(gold["grad_seed"])).normal(size=ref.shape)
    Gr = G[:, rows, :]
    Gr[:, flags != 0] = 0.0
    G[:, rows, :] = Gr
    gv, ga = gpu_backward(st, state, G)
    ogv = np.zeros_like(gv)
    ogv[gold["gv_idx"]] = gold["gv"]
    oga = np.zeros_like(ga)
    oga[gold["ga_idx"]] = gold["ga"]
    ev = float(np.linalg.norm(gv - ogv) / float(gold["gv_norm"]))
    ea = float(np.linalg.norm(ga - oga) / float(gold["ga_norm"]))
    say(f"  grad rel-L2 verts {ev:.2e} attrs {ea:.2e} ({len(gold['gv_idx'])} vertices with gradient)")
    assert ev <= GRAD_RTOL and ea <= GRAD_RTOL
