"""Writes large_rows.npz: the FP64 oracle's image, guard-band flags and
adjoint on sampled pixel rows of the large workload (ico6, 1024x1024, K=512,
S=60, 5 revolutions + 200 px translation), for the GPU parity test at full
size.  Calls only oracle/ and the seeded input generators; run it again after
any change to the oracle's arithmetic:

    python tests/golden/make_large_rows.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2602_07860_amd import workloads as wl  # noqa: E402

ROWS = (192, 1024, 128)      # rows 192, 320, ..., 960
GRAD_SEED = 77


def main():
    sc = wl.make_workload(wl.LARGE)
    t0 = time.time()
    ref = oracle.render(sc, flags=True, rows=ROWS)
    rows = np.arange(*ROWS)
    print(f"forward + flags on {len(rows)} rows: {time.time() - t0:.1f} s", flush=True)
    G = np.zeros_like(ref.image)
    g = np.random.default_rng(GRAD_SEED).normal(size=(ref.image.shape[0], len(rows), sc.width))
    G[:, rows, :] = g
    G[:, ref.flags != 0] = 0.0
    t0 = time.time()
    og = oracle.render(sc, grad_image=G, rows=ROWS)
    print(f"adjoint on the same rows: {time.time() - t0:.1f} s", flush=True)
    gv_idx = np.nonzero(np.abs(og.grad_verts).sum(1))[0]
    ga_idx = np.nonzero(np.abs(og.grad_attrs).sum(1))[0]
    np.savez_compressed(os.path.join(HERE, "large_rows.npz"), rows=rows, image=ref.image[:, rows, :],
                        flags=ref.flags[rows, :], grad_seed=GRAD_SEED,
                        gv_idx=gv_idx.astype(np.int32), gv=og.grad_verts[gv_idx].astype(np.float32),
                        ga_idx=ga_idx.astype(np.int32), ga=og.grad_attrs[ga_idx].astype(np.float32),
                        gv_norm=np.linalg.norm(og.grad_verts), ga_norm=np.linalg.norm(og.grad_attrs))
    print("wrote", os.path.join(HERE, "large_rows.npz"), len(gv_idx), "vertices with gradient", flush=True)


if __name__ == "__main__":
    main()
