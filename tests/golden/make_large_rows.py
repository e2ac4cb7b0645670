"""Writes large_rows.npz: the FP64 oracle's image with the guard band's range,
and its adjoint with the guard band's per-component bounds, on sampled pixel
rows of the large workload (ico6, 1024x1024, K=512, S=60, 5 revolutions +
200 px translation), for the GPU parity test at full size.  Calls only
oracle/ and the seeded input generators; run it again after any change to the
oracle's arithmetic:

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

ROWS = (16, 1024, 32)        # rows 16, 48, ..., 1008: every 32nd
GRAD_SEED = 77


def main():
    sc = wl.make_workload(wl.LARGE)
    rows = np.arange(*ROWS)
    G = np.zeros((sc.attrs.shape[1] + 1, sc.height, sc.width))
    G[:, rows, :] = np.random.default_rng(GRAD_SEED).normal(size=(G.shape[0], len(rows), sc.width))
    t0 = time.time()
    ref = oracle.render(sc, grad_image=G, rows=ROWS, bounds=True, counters=True)
    print(f"forward + adjoint with guard-band bounds on {len(rows)} rows: {time.time() - t0:.1f} s", flush=True)
    gv_idx = np.nonzero(np.abs(ref.grad_verts).sum(1) + ref.slack_verts.sum(1))[0]
    ga_idx = np.nonzero(np.abs(ref.grad_attrs).sum(1) + ref.slack_attrs.sum(1))[0]
    cnt = np.array([ref.counters[k] for k in oracle.COUNTER_NAMES])
    np.savez_compressed(os.path.join(HERE, "large_rows.npz"), rows=rows, grad_seed=GRAD_SEED,
                        image=ref.image[:, rows, :].astype(np.float32),
                        image_lo=ref.image_lo[:, rows, :].astype(np.float32),
                        image_hi=ref.image_hi[:, rows, :].astype(np.float32),
                        gv_idx=gv_idx.astype(np.int32), gv=ref.grad_verts[gv_idx].astype(np.float32),
                        sv=ref.slack_verts[gv_idx].astype(np.float32),
                        ga_idx=ga_idx.astype(np.int32), ga=ref.grad_attrs[ga_idx].astype(np.float32),
                        sa=ref.slack_attrs[ga_idx].astype(np.float32),
                        counters=cnt, counter_names=np.array(oracle.COUNTER_NAMES))
    print("wrote", os.path.join(HERE, "large_rows.npz"), len(gv_idx), "vertices with gradient", flush=True)


if __name__ == "__main__":
    main()
