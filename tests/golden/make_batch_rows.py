"""Writes batch_rows.npz: the FP64 oracle's image with the guard band's range,
and its adjoint with the guard band's per-component bounds, on sampled pixel
rows of four instances of the 32-instance mixed batch (seed 3): the one with
the most faces (36980, 128x128, translation), the one with the most
sub-frames (K = 251, 512x512, rotation), a 256x256 one with 35280 faces, and
a 512x512 rotation with 20480 faces.  Every 16th row of each (16 rows per
instance).  Calls only oracle/ and the seeded input generators:

    python tests/golden/make_batch_rows.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2602_07860_amd import workloads as wl  # noqa: E402

INSTANCES = (3, 11, 29, 7)
GRAD_SEED = 300


def rows_of(sc):
    step = sc.height // 16
    return (step // 2, sc.height, step)


def main():
    scenes = wl.make_batch(seed=3, n=32)
    out = {"instances": np.array(INSTANCES, np.int32)}
    for i in INSTANCES:
        sc = scenes[i]
        rows = rows_of(sc)
        ridx = np.arange(*rows)
        G = np.zeros((sc.attrs.shape[1] + 1, sc.height, sc.width))
        G[:, ridx, :] = np.random.default_rng(GRAD_SEED + i).normal(size=(G.shape[0], len(ridx), sc.width))
        t0 = time.time()
        ref = oracle.render(sc, grad_image=G, rows=rows, bounds=True, counters=True)
        print(f"instance {i} ({len(sc.faces)} faces, {sc.width}^2, K {sc.num_subframes}): "
              f"{len(ridx)} rows in {time.time() - t0:.1f} s", flush=True)
        gv_idx = np.nonzero(np.abs(ref.grad_verts).sum(1) + ref.slack_verts.sum(1))[0]
        ga_idx = np.nonzero(np.abs(ref.grad_attrs).sum(1) + ref.slack_attrs.sum(1))[0]
        p = f"i{i}_"
        out.update({p + "rows": ridx, p + "image": ref.image[:, ridx, :].astype(np.float32),
                    p + "image_lo": ref.image_lo[:, ridx, :].astype(np.float32),
                    p + "image_hi": ref.image_hi[:, ridx, :].astype(np.float32),
                    p + "gv_idx": gv_idx.astype(np.int32), p + "gv": ref.grad_verts[gv_idx].astype(np.float32),
                    p + "sv": ref.slack_verts[gv_idx].astype(np.float32),
                    p + "ga_idx": ga_idx.astype(np.int32), p + "ga": ref.grad_attrs[ga_idx].astype(np.float32),
                    p + "sa": ref.slack_attrs[ga_idx].astype(np.float32),
                    p + "counters": np.array([ref.counters[k] for k in oracle.COUNTER_NAMES])})
    out["grad_seed"] = GRAD_SEED
    out["counter_names"] = np.array(oracle.COUNTER_NAMES)
    np.savez_compressed(os.path.join(HERE, "batch_rows.npz"), **out)
    print("wrote", os.path.join(HERE, "batch_rows.npz"), flush=True)


if __name__ == "__main__":
    main()
