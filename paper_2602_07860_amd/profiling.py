"""Helpers for the rocprofv3 measurements quoted next to the benchmark.

  python -m paper_2602_07860_amd.profiling copy
      a plain 1 GiB device-to-device copy, three times: the reference that
      scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes;
  python -m paper_2602_07860_amd.profiling traffic --kernel K --workload W \\
          [--match NAME] --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --out FILE
      combine `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs of the
      benchmark (DIR holds the run's counter_collection.csv) and of the copy
      into HBM bytes per launch of kernel K, and record them in FILE (JSON,
      keyed "K@W") with a hash of the kernel sources and launch plan, so that
      the benchmark reports the figure only while the kernels are the ones
      measured.

Nothing here runs on the rendering path.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

COPY_BYTES = 1 << 30
SOURCES = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
           for f in ("rb_kernels.hip", "rb_api.cpp", "rb_internal.h")]


def source_hash() -> str:
    """Hash of the kernel sources and of the host plan that sets their launch
    parameters."""
    h = hashlib.sha256()
    for p in SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_mean(run_dir: str, counter: str, kernel_substr: str) -> float:
    """Mean per-dispatch value (KiB for the size counters) of `counter` over
    the dispatches whose kernel name contains kernel_substr."""
    vals = []
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
                    vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} samples for {kernel_substr!r} under {run_dir}")
    return sum(vals) / len(vals)


def lookup(path: str, kernel: str, workload: str):
    """Per-launch HBM bytes of `kernel` on `workload` recorded in `path`, or
    None when absent or measured on other kernel sources."""
    try:
        with open(path) as f:
            rec = json.load(f).get(f"{kernel}@{workload}")
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != source_hash():
        return None
    return rec["bytes_per_launch"]


def _copy() -> None:
    import torch
    x = torch.ones(COPY_BYTES // 4, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {COPY_BYTES} bytes x3", flush=True)


def _traffic(a) -> None:
    match = a.match or a.kernel
    fetch_kib = _counter_mean(a.fetch, "FETCH_SIZE", match)
    write_kib = _counter_mean(a.write, "WRITE_SIZE", match)
    # the copy reads and writes COPY_BYTES per dispatch
    cf = COPY_BYTES / (_counter_mean(a.copy_fetch, "FETCH_SIZE", a.copy_kernel) * 1024)
    cw = COPY_BYTES / (_counter_mean(a.copy_write, "WRITE_SIZE", a.copy_kernel) * 1024)
    rec = {"match": match, "fetch_kib": fetch_kib, "write_kib": write_kib, "fetch_scale": round(cf, 4), "write_scale": round(cw, 4),
           "bytes_per_launch": fetch_kib * 1024 * cf + write_kib * 1024 * cw, "source_sha256": source_hash()}
    data = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            data = json.load(f)
    data[f"{a.kernel}@{a.workload}"] = rec
    with open(a.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(rec))


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--match", default="", help="substring of the profiled kernel names (default: --kernel)")
    t.add_argument("--workload", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "copy":
        _copy()
    else:
        _traffic(a)


if __name__ == "__main__":
    main()
