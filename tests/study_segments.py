"""Segment-count study (App. D "Segmentation Analysis"; the keyframe-distance
approximation of eq 13, Sec. 3.3).

The nu=32 sphere of the 256^2 workload (10242 V / 20480 F), K = 192
sub-frames, one revolution about its seeded axis, cut into S = 6, 12, 24 and
48 linear segments.  For each S:
  * GPU image (fast solver) against the continuous motion: the FP64 oracle's
    exact-motion, exact-distance render (every sub-frame projected from
    M(t_k), closest point in its own triangle, eq 12);
  * that error split into the segment-linear part (oracle, segments +
    exact distance, against the continuous motion) and the eq 13 part (the
    GPU's keyframe distance against the oracle's exact distance on the same
    segments);
  * GPU vertex-gradient error against the static-frames baseline (K still
    renders of the exactly moved mesh: the gradient of the continuous
    motion), both for the same upstream gradient dL/dI (the continuous
    motion's L2 residual against a second seeded displacement);
  * GPU ms per fwd+bwd step.
Needs a GPU (run from the repository root: python tests/study_segments.py);
prints a markdown table and one JSON line.  Test infrastructure: it calls
the oracle, so it is not part of the package.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2602_07860_amd import baseline  # noqa: E402
from paper_2602_07860_amd import render as R  # noqa: E402
from paper_2602_07860_amd import workloads as wl  # noqa: E402

SEGMENTS = (6, 12, 24, 48)
K = 192


def err(a, b):
    """mean and max |a - b| over pixels touched by either, relative to max|b|."""
    scale = np.abs(b).max()
    touched = (np.abs(a).sum(0) + np.abs(b).sum(0)) > 0
    d = np.abs(a - b)[:, touched] / scale
    return float(d.mean()), float(d.max())


def main():
    import torch
    base = wl.make_workload(wl.MEDIUM)
    sc0 = base.with_(motion=wl.Motion("rotate", axis=base.motion.axis, revs=1.0), num_subframes=K)
    tgt = wl.make_target(sc0, 2)
    t0 = time.time()
    exact = oracle.render(sc0, motion="exact", distance="exact").image
    print(f"oracle, continuous motion: {time.time() - t0:.1f} s", flush=True)
    st = R.scene_tensors(sc0, "cuda")
    tt = R.scene_tensors(tgt, "cuda")
    # reference gradient of the continuous motion: static frames
    tb = baseline.for_scene(tt, sc0.motion, K)
    tb.fit()
    target = tb.forward().clone()
    b = baseline.for_scene(st, sc0.motion, K)
    b.fit()
    img_b = b.forward()
    G = (2.0 * (img_b - target)).clone()
    gv_b, _ = b.backward(G)
    gv_b = gv_b.double().cpu().numpy()
    del b, tb
    rows = []
    for S in SEGMENTS:
        sc = sc0.with_(num_segments=S)
        t0 = time.time()
        seg = oracle.render(sc, distance="exact").image
        print(f"oracle, S={S} segments, exact distance: {time.time() - t0:.1f} s", flush=True)
        st = R.scene_tensors(sc, "cuda")
        o = R.RenderOptions(K)
        img, state = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, o)
        gv, _ = R.render_backward(st.verts, st.faces, st.attrs, st.model, state, G)
        o.check = False
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            im2, s2 = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, o)
            R.render_backward(st.verts, st.faces, st.attrs, st.model, s2, G)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        g = img.double().cpu().numpy()
        gvn = gv.double().cpu().numpy()
        row = {"S": S, "per_rev": S, "gpu_vs_continuous": err(g, exact), "segments_only": err(seg, exact),
               "eq13_only": err(g, seg),
               "grad_vs_continuous": float(np.linalg.norm(gvn - gv_b) / np.linalg.norm(gv_b)),
               "ms_per_step": round(ms, 3)}
        rows.append(row)
        print(json.dumps(row), flush=True)
    print()
    print("| S (per revolution) | image vs continuous motion: mean / max | segments only | eq 13 only "
          "| vertex gradient vs continuous (rel L2) | GPU fwd+bwd ms |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        f = lambda x: f"{x[0]:.2e} / {x[1]:.2e}"
        print(f"| {r['S']} | {f(r['gpu_vs_continuous'])} | {f(r['segments_only'])} | {f(r['eq13_only'])} "
              f"| {r['grad_vs_continuous']:.3f} | {r['ms_per_step']:.3f} |")
    print(json.dumps({"study": "segments", "K": K, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
