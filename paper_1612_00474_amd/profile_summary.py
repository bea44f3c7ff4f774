"""Summaries of rocprofv3 output for `profiles/` (markdown tables plus machine-readable blocks).

    python -m paper_1612_00474_amd.profile_summary valu PASS1_DIR PASS2_DIR TRACE_DIR N
    python -m paper_1612_00474_amd.profile_summary hbm FETCH_DIR WRITE_DIR
    python -m paper_1612_00474_amd.profile_summary trace TRACE_DIR [TOP]

The directories are rocprofv3 `-d` output directories of `profile_kernels` (valu, hbm) or of any
run (trace).  Counter values are averaged per dispatch over the dispatches after the profiling
driver's calibration copy (the copy kernel with the largest grid).  `valu` needs pass 1 with
SQ_INSTS_VALU, the FP32 FMA/MUL/ADD/TRANS counters and GRBM_GUI_ACTIVE, pass 2 with the FP64 ones,
and a kernel trace of the same driver for the durations; `hbm` scales FETCH_SIZE and WRITE_SIZE
by what they read for the calibration copy of known size.  The machine-readable blocks (kernel,
value per launch, pair-kernel source hash) are what `bench.py` reads back.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import statistics
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
CALIB = "copyBuffer"
PAIR_SOURCES = ("matvec.hip", "multi.hip", "pair_common.h", "pair_tensor.h")


def kernel_source_hash() -> str:
    """sha256[:16] of the pair-kernel sources with comments and blank lines removed (so that
    editing a comment does not void recorded counters)."""
    h = hashlib.sha256()
    for name in PAIR_SOURCES:
        with open(os.path.join(PKG, "csrc", name)) as f:
            for line in f:
                code = re.sub(r"//.*$", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("rpb::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    i = name.find("(")
    return name[:i] if i > 0 else name


def _rows(d: str, pattern: str):
    out = []
    for f in glob.glob(os.path.join(d, "**", pattern), recursive=True):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def per_kernel(d: str):
    """{kernel: {counter: mean per dispatch, "_dispatches": count}} over the dispatches after
    the calibration copy, and the calibration copy's own counter values."""
    rs = _rows(d, "*counter_collection.csv")
    key = "Dispatch_Id" if rs and "Dispatch_Id" in rs[0] else "Correlation_Id"
    calib_id, grid = None, -1
    for r in rs:
        if CALIB in r["Kernel_Name"] and int(r["Grid_Size"]) > grid:
            calib_id, grid = int(r[key]), int(r["Grid_Size"])
    vals = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    calib = defaultdict(float)
    for r in rs:
        did = int(r[key])
        if did == calib_id:
            calib[r["Counter_Name"]] += float(r["Counter_Value"])
        elif calib_id is None or did > calib_id:
            vals[short(r["Kernel_Name"])][r["Counter_Name"]][did] += float(r["Counter_Value"])
    out = {}
    for k, cs in vals.items():
        out[k] = {}
        for c, by in cs.items():
            out[k][c] = sum(by.values()) / len(by)
            out[k]["_dispatches"] = len(by)
    return out, dict(calib)


def durations(d: str):
    out = {}
    for r in _rows(d, "*kernel_stats.csv"):
        out[short(r["Name"])] = (float(r["AverageNs"]), int(r["Calls"]))
    return out


F32 = ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
       "SQ_INSTS_VALU_TRANS_F32")
F64 = ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
       "SQ_INSTS_VALU_TRANS_F64")


def issued_flops(c, names) -> float:
    """Lane operations of wave instructions: FMA = 2; MUL, ADD and transcendental = 1."""
    return 64 * (2 * c.get(names[0], 0) + c.get(names[1], 0) + c.get(names[2], 0)
                 + c.get(names[3], 0))


def valu(p1_dir, p2_dir, trace_dir, n):
    p1, _ = per_kernel(p1_dir)
    p2, _ = per_kernel(p2_dir)
    dur = durations(trace_dir)
    h = kernel_source_hash()
    pairs = n * (n + 1) / 2.0
    print("| kernel | ms | clock (GHz) | VALU instr / launch | VALU instr per unordered pair "
          "| FP32 FMA | FP32 MUL | FP32 ADD | FP32 TRANS | FP64 FMA | FP64 MUL | FP64 ADD | "
          "FP64 TRANS | issued flop / launch | issued TFLOP/s |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    block = []
    for k in sorted(p1):
        if not k.startswith("pair_kernel"):
            continue
        c = dict(p1[k])
        c.update(p2.get(k, {}))
        ms = dur.get(k, (0, 0))[0] / 1e6
        clk = c.get("GRBM_GUI_ACTIVE", 0) / 8 / (ms * 1e-3) / 1e9 if ms else 0.0
        v = c.get("SQ_INSTS_VALU", 0)
        fl = issued_flops(c, F32) + issued_flops(c, F64)
        print(f"| `{k}` | {ms:.3f} | {clk:.2f} | {v:.4g} | {v * 64 / pairs:.1f} | "
              + " | ".join(f"{c.get(x, 0):.4g}" for x in F32 + F64)
              + f" | {fl:.4g} | {fl / (ms * 1e-3) / 1e12 if ms else 0:.1f} |")
        block.append(f"{k}\t{fl:.6e}\t{h}")
    print("\nMachine-readable (kernel, issued flop per launch, pair-kernel source hash):\n\n```")
    print("\n".join(block))
    print("```")


def hbm(fetch_dir, write_dir, copy_kib=512 * 1024):
    fe, cf = per_kernel(fetch_dir)
    wr, cw = per_kernel(write_dir)
    h = kernel_source_hash()
    sf = copy_kib / cf["FETCH_SIZE"] if cf.get("FETCH_SIZE") else 1.0
    sw = copy_kib / cw["WRITE_SIZE"] if cw.get("WRITE_SIZE") else 1.0
    print(f"Calibration copy of {copy_kib} KiB: FETCH_SIZE reads {cf.get('FETCH_SIZE')} KiB "
          f"(scale {sf:.4f}), WRITE_SIZE reads {cw.get('WRITE_SIZE')} KiB (scale {sw:.4f}).\n")
    print("| kernel | launches | FETCH_SIZE (KiB/launch) | WRITE_SIZE (KiB/launch) | "
          "HBM bytes/launch (scaled) |")
    print("|---|---:|---:|---:|---:|")
    block = []
    for k in sorted(set(fe) | set(wr)):
        if CALIB in k:
            continue
        f = fe.get(k, {}).get("FETCH_SIZE", 0)
        w = wr.get(k, {}).get("WRITE_SIZE", 0)
        b = (f * sf + w * sw) * 1024
        print(f"| `{k}` | {fe.get(k, {}).get('_dispatches', 0)} | {f:.1f} | {w:.1f} | {b:.4e} |")
        block.append(f"{k}\t{b:.6e}\t{h}")
    print("\nMachine-readable (kernel, HBM bytes per launch, pair-kernel source hash):\n\n```")
    print("\n".join(block))
    print("```")


def trace(trace_dir, top=25):
    rows = _rows(trace_dir, "*kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"Total kernel time {tot / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} "
          "launches.\n")
    print("| kernel | calls | avg (us) | min (us) | max (us) | % of GPU time |")
    print("|---|---:|---:|---:|---:|---:|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        print(f"| `{short(r['Name'])}` | {int(r['Calls'])} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
              f"{100.0 * float(r['TotalDurationNs']) / tot:.2f} |")
    # kernel time per stream, and how much of it ran beside kernels of another stream
    trace_rows = _rows(trace_dir, "*kernel_trace.csv")
    per_stream = defaultdict(float)
    spans = []
    for r in trace_rows:
        s0, s1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        per_stream[r.get("Stream_Id", "0")] += (s1 - s0) / 1e6
        spans.append((s0, s1))
    if len(per_stream) > 1:
        spans.sort()
        busy, cur0, cur1 = 0, None, None
        for s0, s1 in spans:
            if cur1 is None or s0 > cur1:
                if cur1 is not None:
                    busy += cur1 - cur0
                cur0, cur1 = s0, s1
            else:
                cur1 = max(cur1, s1)
        busy += cur1 - cur0
        total = sum(per_stream.values())
        print("\nKernel time per stream (ms): "
              + ", ".join(f"stream {k}: {v:.2f}" for k, v in sorted(per_stream.items()))
              + f"; time with at least one kernel running {busy / 1e6:.2f} ms, so "
              f"{total - busy / 1e6:.2f} ms of kernel time ran beside another kernel.")
    # pair kernels: launches that did work apart from those that found a stop flag set
    by = defaultdict(list)
    for r in trace_rows:
        k = short(r["Kernel_Name"])
        if k.startswith("pair_kernel"):
            by[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    if not by:
        return
    print("\nPair kernels, launches that did work apart from launches that returned at once "
          "(under 5 % of the median duration: an iteration enqueued past a Lanczos stop):\n")
    print("| kernel | launches that did work | avg (us) | min (us) | max (us) | "
          "launches that returned at once | their avg (us) |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for k in sorted(by, key=lambda k: -sum(by[k])):
        d = by[k]
        med = statistics.median(d)
        work = [x for x in d if x >= 0.05 * med]
        idle = [x for x in d if x < 0.05 * med]
        print(f"| `{k}` | {len(work)} | {statistics.mean(work):.1f} | {min(work):.1f} | "
              f"{max(work):.1f} | {len(idle)} | "
              f"{(statistics.mean(idle) if idle else 0.0):.1f} |")


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    mode = argv[1]
    if mode == "valu":
        valu(argv[2], argv[3], argv[4], int(argv[5]))
    elif mode == "hbm":
        hbm(argv[2], argv[3])
    elif mode == "trace":
        trace(argv[2], int(argv[3]) if len(argv) > 3 else 25)
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
