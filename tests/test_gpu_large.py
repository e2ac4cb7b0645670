"""Parity at full size: the large workload (ico6, 81920 faces, 1024x1024,
K = 512, S = 60) rendered on the GPU in the launch configuration bench.py
times, compared on the pixel rows that tests/golden/large_rows.npz holds (the
FP64 oracle's image with the guard band's range, and its adjoint with the
guard band's bounds, on every 32nd row, written by
tests/golden/make_large_rows.py).  Every pixel of those rows is compared and
carries an upstream gradient."""
import os

import numpy as np
import pytest

from paper_2602_07860_amd import workloads as wl

from gpu_common import (MAX_ALT_PIXSUB, assert_grad_parity, assert_image_bounds, gpu_backward, gpu_forward,
                        say)

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_rows.npz")


def _dense(n, width, idx, vals):
    out = np.zeros((n, width))
    out[idx] = vals
    return out


def test_large_workload_sampled_rows():
    gold = np.load(GOLD)
    rows = gold["rows"]
    cnt = dict(zip(gold["counter_names"].tolist(), gold["counters"].tolist()))
    tot = cnt["fg_pixsub"] + cnt["bg_pixsub"]
    say(f"guard band on the sampled rows: {cnt['alt_pixsub']:.0f} of {tot:.0f} pixel-sub-frames "
        f"({100 * cnt['alt_pixsub'] / tot:.2f}%) with an alternative")
    assert cnt["unbounded_pixsub"] == 0 and cnt["alt_pixsub"] <= MAX_ALT_PIXSUB * tot
    sc = wl.make_workload(wl.LARGE)
    say(f"case: {sc.name} full render, compared on {len(rows)} rows {rows[0]}..{rows[-1]}")
    img, state, st = gpu_forward(sc)
    assert np.all(np.isfinite(img))
    assert_image_bounds(img[:, rows, :], gold["image"].astype(np.float64), gold["image_lo"].astype(np.float64),
                        gold["image_hi"].astype(np.float64), label="large rows")
    # upstream gradient on every pixel of the sampled rows
    G = np.zeros_like(img)
    G[:, rows, :] = np.random.default_rng(int(gold["grad_seed"])).normal(size=(img.shape[0], len(rows), img.shape[2]))
    gv, ga = gpu_backward(st, state, G)
    V, C = gv.shape[0], ga.shape[1]
    assert_grad_parity(gv, _dense(V, 3, gold["gv_idx"], gold["gv"]), _dense(V, 3, gold["gv_idx"], gold["sv"]),
                       label="large rows verts")
    assert_grad_parity(ga, _dense(V, C, gold["ga_idx"], gold["ga"]), _dense(V, C, gold["ga_idx"], gold["sa"]),
                       label="large rows attrs")
