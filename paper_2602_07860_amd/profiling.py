"""Helpers for the rocprofv3 measurements quoted next to the benchmark.

  python -m paper_2602_07860_amd.profiling copy
      a plain 1 GiB device-to-device copy, three times: the reference that
      scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes;
  python -m paper_2602_07860_amd.profiling summary DB [--title T] [--command C]
      per-kernel table (calls, average and total milliseconds, share) of a
      `rocprofv3 --kernel-trace --stats` run whose results database is DB;
  python -m paper_2602_07860_amd.profiling counters CSV [--title T] [--command C]
      per-kernel mean of every counter of a `rocprofv3 --pmc ... --output-format
      csv` run (CSV = its counter_collection.csv), with the kernels' register,
      scratch and LDS sizes;
  python -m paper_2602_07860_amd.profiling derived --a CSV --b CSV --fetch DIR --write DIR \\
          --copy-fetch DIR --copy-write DIR [--title T]
      per kernel, from the two counter runs (A: SQ_INSTS_VALU,
      SQ_THREAD_CYCLES_VALU, SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT; B: SQ_INSTS_SALU,
      SQ_INSTS_VMEM_RD, SQ_INSTS_VMEM_WR, SQ_WAIT_ANY, SQ_ACTIVE_INST_ANY) and the
      traffic runs: the share of active lanes in VALU instructions, LDS bank
      conflict cycles per LDS instruction, the VALU share of issued
      instructions, the share of wave cycles spent waiting, and HBM GB read
      and written per launch;
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


def code_text(src: str) -> str:
    """C++ source without its comments and with whitespace collapsed, so that
    an edit of the comments alone does not count as a change of the code."""
    out, i, n = [], 0, len(src)
    while i < n:
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif src[i] == '"':
            j = i + 1
            while j < n and src[j] != '"':
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(src[i])
            i += 1
    return " ".join("".join(out).split())


def source_hash(texts=None) -> str:
    """Hash of the code (comments left out) of the kernel sources and of the
    host plan that sets their launch parameters."""
    h = hashlib.sha256()
    if texts is None:
        texts = []
        for p in SOURCES:
            with open(p) as f:
                texts.append(f.read())
    for t in texts:
        h.update(code_text(t).encode())
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


def _summary(a) -> None:
    import sqlite3
    db = sqlite3.connect(a.db)
    per: dict = {}
    for name, start, end in db.execute("select name, start, end from kernels order by start"):
        per.setdefault(name, []).append(end - start)
    rows = []
    for name, d in per.items():
        d = d[a.skip:]
        if a.count > 0:
            d = d[:a.count]
        if d:
            rows.append((name, len(d), sum(d) / len(d), sum(d)))
    rows.sort(key=lambda r: -r[3])
    tot = sum(r[3] for r in rows) or 1
    out = ["# rocprofv3 kernel trace summary" + (f": {a.title}" if a.title else "")]
    if a.command:
        out.append(f"# command (from the repository root on the GPU box): {a.command}")
    if a.skip or a.count:
        out.append(f"# per kernel: its dispatches {a.skip + 1}.." + (f"{a.skip + a.count}" if a.count else "last")
                   + " in time order")
    out.append("# durations in milliseconds (avg per dispatch, total), share of total kernel time")
    out.append("")
    out.append(f"{'kernel':<72}{'calls':>7}{'avg_ms':>11}{'total_ms':>12}{'share%':>8}")
    for name, n, avg, total in rows[:a.top]:
        nm = name if len(name) <= 70 else name[:68] + ".."
        out.append(f"{nm:<72}{n:>7}{avg / 1e6:>11.3f}{total / 1e6:>12.1f}{100.0 * total / tot:>8.2f}")
    print("\n".join(out))


def _counters(a) -> None:
    agg: dict = {}
    meta: dict = {}
    with open(a.csv) as fh:
        for r in csv.DictReader(fh):
            k = r["Kernel_Name"]
            agg.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            meta[k] = (r["VGPR_Count"], r["Accum_VGPR_Count"], r["SGPR_Count"], r["Scratch_Size"], r["LDS_Block_Size"])
    names = sorted({c for d in agg.values() for c in d})
    out = ["# rocprofv3 counters, mean per dispatch" + (f": {a.title}" if a.title else "")]
    if a.command:
        out.append(f"# command (from the repository root on the GPU box): {a.command}")
    out.append("# vgpr/agpr/sgpr as rocprofv3 reports them (allocation granules), scratch bytes per lane, LDS bytes")
    out.append("")
    out.append(f"{'kernel':<48}{'n':>4}" + "".join(f"{c.replace('SQ_', ''):>22}" for c in names)
               + "   vgpr/agpr/sgpr/scratch/lds")
    order = sorted(agg, key=lambda k: -max(sum(v) / len(v) for v in agg[k].values()))
    for k in order[:a.top]:
        d = agg[k]
        n = max(len(v) for v in d.values())
        nm = k if len(k) <= 46 else k[:44] + ".."
        out.append(f"{nm:<48}{n:>4}" + "".join(f"{(sum(d[c]) / len(d[c])) if c in d else float('nan'):>22.6g}"
                                               for c in names) + "   " + "/".join(meta[k]))
    print("\n".join(out))


def _means(path: str) -> dict:
    """{kernel: {counter: mean per dispatch}} of one counter_collection.csv
    (or of every such file under a directory)."""
    files = [path] if os.path.isfile(path) else glob.glob(os.path.join(path, "**", "*counter_collection.csv"),
                                                          recursive=True)
    agg: dict = {}
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                agg.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}


def _derived(a) -> None:
    A, Bc = _means(a.a), _means(a.b)
    fe, wr = _means(a.fetch), _means(a.write)
    cf = COPY_BYTES / (_counter_mean(a.copy_fetch, "FETCH_SIZE", a.copy_kernel) * 1024)
    cw = COPY_BYTES / (_counter_mean(a.copy_write, "WRITE_SIZE", a.copy_kernel) * 1024)
    out = ["# derived per-dispatch figures" + (f": {a.title}" if a.title else ""),
           "# active lanes = SQ_THREAD_CYCLES_VALU / (64 SQ_INSTS_VALU); LDS conflict cycles per LDS instruction;",
           "# VALU share = SQ_INSTS_VALU / (VALU + SALU + LDS + VMEM instructions); waiting = SQ_WAIT_ANY /",
           "# (SQ_WAIT_ANY + SQ_ACTIVE_INST_ANY); HBM GB per launch from FETCH_SIZE and WRITE_SIZE (KiB per",
           f"# dispatch) scaled by a 1 GiB device copy (x{cf:.3f} and x{cw:.3f})",
           "",
           f"{'kernel':<34}{'active lanes':>13}{'LDS confl/ins':>14}{'VALU share':>11}{'waiting':>9}{'fetch GB':>10}{'write GB':>10}"]
    rows = []
    for k, d in A.items():
        if "rb::" not in k or "SQ_INSTS_VALU" not in d or k not in Bc:
            continue
        b = Bc[k]
        valu = d["SQ_INSTS_VALU"]
        lanes = d["SQ_THREAD_CYCLES_VALU"] / (64.0 * valu) if valu else float("nan")
        lds = d.get("SQ_INSTS_LDS", 0.0)
        confl = d.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds if lds else 0.0
        tot = valu + b.get("SQ_INSTS_SALU", 0.0) + lds + b.get("SQ_INSTS_VMEM_RD", 0.0) + b.get("SQ_INSTS_VMEM_WR", 0.0)
        wait = b.get("SQ_WAIT_ANY", 0.0) / max(b.get("SQ_WAIT_ANY", 0.0) + b.get("SQ_ACTIVE_INST_ANY", 0.0), 1.0)
        f = fe.get(k, {}).get("FETCH_SIZE", float("nan")) * 1024 * cf / 1e9
        w = wr.get(k, {}).get("WRITE_SIZE", float("nan")) * 1024 * cw / 1e9
        name = k.split("(")[0].replace("void ", "")
        rows.append((valu, f"{name:<34}{lanes:>13.3f}{confl:>14.3f}{valu / tot:>11.3f}{wait:>9.3f}{f:>10.2f}{w:>10.2f}"))
    out += [r for _, r in sorted(rows, key=lambda x: -x[0])]
    print("\n".join(out))


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
    sm = sub.add_parser("summary")
    sm.add_argument("db")
    sm.add_argument("--title", default="")
    sm.add_argument("--command", default="")
    sm.add_argument("--top", type=int, default=24)
    sm.add_argument("--skip", type=int, default=0, help="skip each kernel's first N dispatches")
    sm.add_argument("--count", type=int, default=0, help="then keep N dispatches (0: all)")
    cn = sub.add_parser("counters")
    cn.add_argument("csv")
    cn.add_argument("--title", default="")
    cn.add_argument("--command", default="")
    cn.add_argument("--top", type=int, default=16)
    dv = sub.add_parser("derived")
    for k in ("a", "b", "fetch", "write", "copy_fetch", "copy_write"):
        dv.add_argument("--" + k.replace("_", "-"), required=True)
    dv.add_argument("--copy-kernel", default="copyBuffer")
    dv.add_argument("--title", default="")
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
    elif a.cmd == "summary":
        _summary(a)
    elif a.cmd == "counters":
        _counters(a)
    elif a.cmd == "derived":
        _derived(a)
    else:
        _traffic(a)


if __name__ == "__main__":
    main()
