#!/usr/bin/env python3
"""Throughput benchmark of the motion-blur rasterizer: pixel-sub-frames per
second of one forward + backward step.

Workload (default): nu=32 geodesic sphere (10242 V / 20480 F) displaced by
0.02 N(0,1), per-vertex RGB, 256x256, K = 64 sub-frames, 3 revolutions about a
seeded axis cut into S = 36 linear segments; L2 loss against the render of a
second seeded displacement.  One step = forward render + dL/dI + adjoint into
vertex positions and colours.  Inputs are resident in GPU memory before the
timed region.  The step is timed for the fast solver (eq 8) and for the
per-sub-frame recompute (eqs 1-3) on the same GPU.

Prints ONE JSON line (rank 0).  Extra objects: "roofline" for the dominant
kernel (algorithmic FLOPs from the FP64 reference's exact pair counters,
divided by the kernel's average duration measured with HIP events on its
stream), and "cpu_baseline": the FP64 reference renderer timed on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pixel-subframes/sec fwd+bwd, fast solver vs per-subframe recompute"
KERNEL_NAMES = {"fg": "k_fg", "bg": "k_bg", "fg_bwd": "k_fg_bwd", "bg_bwd": "k_bg_bwd"}
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (packed); 78.6 without packing
PEAK_HBM_GBS = 8000.0

# Algorithmic FLOPs per counted unit (FMA = 2), per kernel:
#   foreground pass: 18 per bbox pair, +6 per covering pair, 24 per
#     (pixel, face, segment) coefficient setup, 20 per foreground pixel-sub-frame;
#   background pass: 75 per contributing background pair, 2 per background
#     pixel-sub-frame;
#   foreground adjoint: 18 + 90 per foreground pixel-sub-frame (recomputed
#     barycentrics + adjoint);
#   background adjoint: 75 + 75 per contributing background pair.
KERNEL_COEF = {
    "fg": {"bbox_pairs": 18, "cover_pairs": 6, "setup_triples": 24, "fg_pixsub": 20},
    "bg": {"bg_pairs": 75, "bg_pixsub": 2},
    "fg_bwd": {"fg_pixsub": 108},
    "bg_bwd": {"bg_pairs": 150},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def flops(counters, coef):
    return float(sum(coef[k] * counters[k] for k in coef))


def kernel_ms(prof):
    f, b = max(1, prof.fwd_calls), max(1, prof.bwd_calls)
    return {"project": prof.project_ms / f, "bin": prof.bin_ms / f, "fg": prof.fg_ms / f, "bg": prof.bg_ms / f,
            "resolve": prof.resolve_ms / f, "fg_bwd": prof.fg_bwd_ms / b, "bg_bwd": prof.bg_bwd_ms / b,
            "vertex_grad": prof.vertex_grad_ms / b}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk-len", type=int, default=4)
    ap.add_argument("--slice-len", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_07860_amd import binding as B
    from paper_2602_07860_amd import render as R
    from paper_2602_07860_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    sc = wl.make_workload(wl.MEDIUM)
    tg = wl.make_target(sc, 2)
    st = R.scene_tensors(sc, dev)
    tt = R.scene_tensors(tg, dev)
    H, W, K = sc.height, sc.width, sc.num_subframes
    units = H * W * K

    def opts(solver, check=True):
        return R.RenderOptions(K, solver=solver, chunk_len=args.chunk_len,
                               slice_len=args.slice_len, check=check)

    target, _ = R.render_forward(tt.verts, tt.faces, tt.attrs, tt.model, tt.camera, opts("fast"))

    def step(o):
        img, state = R.render_forward(st.verts, st.faces, st.attrs, st.model, st.camera, o)
        g = 2.0 * (img - target)
        gv, ga = R.render_backward(st.verts, st.faces, st.attrs, st.model, state, g)
        return img, gv, ga, state

    results = {}
    for solver in ("fast", "recompute"):
        o = opts(solver, check=True)
        for _ in range(max(1, args.warmup)):
            step(o)
            o = opts(solver, check=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            img, gv, ga, state = step(o)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        h = B.rb_read_header(state.workspace.data_ptr(), torch.cuda.current_stream().cuda_stream)
        if h.error_bits:
            raise RuntimeError(f"device header reports error bits {h.error_bits}")
        if not (torch.isfinite(img).all() and torch.isfinite(gv).all() and torch.isfinite(ga).all()):
            raise RuntimeError("non-finite output")
        # per-kernel durations: a second timed pass with phase events on the stream
        B.rb_profile_enable(True)
        for _ in range(args.steps):
            step(o)
        torch.cuda.synchronize()
        prof = B.rb_profile_read()
        B.rb_profile_enable(False)
        results[solver] = dict(ms=ms, value=units / (ms * 1e-3), prof=prof)
        km = kernel_ms(prof)
        results[solver]["kernel_ms"] = km
        log(f"{solver}: {ms:.3f} ms/step  {units / (ms * 1e-3):.3e} px-sub/s  "
            + " ".join(f"{k} {v:.3f}" for k, v in km.items()) + " ms")

    # ---- FP64 reference on the host: CPU baseline and exact pair counters
    cpu = None
    counters = None
    if not args.no_cpu_baseline:
        import oracle
        nth = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        G = np.random.default_rng(0).normal(size=(4, H, W))
        t0 = time.perf_counter()
        ref = oracle.render(sc, grad_image=G, counters=True, nthreads=nth)
        dt = time.perf_counter() - t0
        counters = ref.counters
        cpu = {"value": units / dt, "unit": "pixel-subframes/s", "cores": nth, "kind": "oracle",
               "sample": f"full workload, forward + backward, {H}x{W}x{K} pixel-sub-frames, "
                         f"FP64, {nth} OpenMP threads, {dt:.1f} s"}
        log(f"cpu oracle: {dt:.2f} s with {nth} threads; counters {counters}")

    fast = results["fast"]
    km = fast["kernel_ms"]
    roof = None
    if counters is not None:
        # dominant kernel: the longest of the four raster kernels
        name = max(KERNEL_COEF, key=lambda k: km[k])
        fl, ms = flops(counters, KERNEL_COEF[name]), km[name]
        ach = fl / (ms * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": KERNEL_NAMES[name], "achieved": round(ach, 4), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 6), "traffic": None,
                "flop_per_launch": fl, "avg_launch_ms": round(ms, 5),
                "all_kernels": {KERNEL_NAMES[k]: {"ms": round(km[k], 5),
                                                  "tflops": round(flops(counters, KERNEL_COEF[k]) / (km[k] * 1e-3) / 1e12, 4)}
                                for k in KERNEL_COEF}}
    out = {
        "metric": METRIC,
        "value": round(fast["value"], 1),
        "unit": "pixel-subframes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fast["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.name} fwd+bwd L2", "vertices": int(len(sc.verts)),
                   "faces": int(len(sc.faces)), "resolution": f"{W}x{H}", "subframes": K,
                   "segments": sc.num_segments, "solver": "fast", "chunk_len": args.chunk_len},
        "recompute": {"value": round(results["recompute"]["value"], 1),
                      "ms_per_step": round(results["recompute"]["ms"], 4)},
        "fast_over_recompute": round(fast["value"] / results["recompute"]["value"], 4),
        "kernel_ms": {k: round(v, 5) for k, v in km.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
