"""Summarize rocprofv3 CSV output for one kernel into a short text file.

Usage (after a kernel-trace run and two counter runs of the same command):
  python -m paper_1908_02464_amd.rocprof_summary --kernel fused3d_kernel \
      --trace DIR_TRACE --fetch DIR_FETCH --write DIR_WRITE \
      --command "the rocprofv3 command line" --out profiles/NAME.txt

FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for the device copy of one 655360 KiB state array in the same
runs (bench.py --copy-calibration), so the reported traffic is in bytes.
With --valu DIR (a run with the SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64,
SQ_INSTS_VALU and SQ_WAVES counters) the FP64 operations per dispatch are
added: 64 lanes x (2 FMA + ADD + MUL + TRANS) wave instructions, i.e. every
lane counted (inactive lanes of a partial wave included).
The summary records a hash of the kernel sources (their code without
comments) so that stale counter numbers are recognised.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics

PKG = os.path.dirname(os.path.abspath(__file__))
COPY_KIB = 655360.0  # one 256^3 x 5 FP64 state array


# Sources and compile flags that determine the fused 3D stage kernel.
FUSED_FILES = ("wl2_device.hpp", "wl2_lface.hpp", "wl2_fused.hpp", "wl2_fused_launch.hpp",
               "wl2_fused3d.hip")


_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/|\s+', re.S)


def code_text(src: str) -> str:
    """C++ source without its comments, runs of white space as one blank
    (string and character literals kept as written): what the compiler
    sees, so that a comment edit does not mark a profile stale."""
    def keep(m):
        t = m.group(0)
        return t if t[0] in "\"'" else "\0"
    return re.sub("\0+", " ", _TOKENS.sub(keep, src)).strip()


def source_hash(files=FUSED_FILES, unit="wl2_fused3d.hip") -> str:
    from .build import compile_flags
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(PKG, "csrc", name), encoding="utf-8") as fh:
            h.update(name.encode())
            h.update(code_text(fh.read()).encode())
    h.update(" ".join(compile_flags(unit)).encode())
    return h.hexdigest()[:16]


def _rows(d, pattern):
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise FileNotFoundError(f"{pattern} under {d}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def trace_stats(d, kernel, last=0):
    """Per kernel name: calls and durations from the stats file, or with
    last > 0 from the last `last` dispatches of the trace file."""
    out = {}
    if last:
        rows = _rows(d, "*kernel_trace.csv")
        by = {}
        for r in rows:
            if kernel in r["Kernel_Name"]:
                by.setdefault(r["Kernel_Name"], []).append(
                    (int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for name, v in by.items():
            dur = [x[1] for x in sorted(v)[-last:]]
            out[name] = {"calls": len(dur), "avg_ns": statistics.mean(dur), "min_ns": min(dur),
                         "max_ns": max(dur), "of_calls": len(v)}
        return out
    rows = _rows(d, "*kernel_stats.csv")
    for r in rows:
        if kernel in r["Name"]:
            out[r["Name"]] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                              "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                              "pct": float(r["Percentage"])}
    return out


LAST = 0  # > 0: counters of the kernel's last LAST dispatches only


def counter(d, kernel, name):
    rows = _rows(d, "*counter_collection.csv")
    sel = [r for r in rows if kernel in r["Kernel_Name"] and r["Counter_Name"] == name]
    if LAST:
        sel = sorted(sel, key=lambda r: int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0))[-LAST:]
    vals = [float(r["Counter_Value"]) for r in sel]
    cal = [float(r["Counter_Value"]) for r in rows
           if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == name
           and int(r["Grid_Size"]) > 1000]
    return vals, cal


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--valu")
    ap.add_argument("--command", required=True)
    ap.add_argument("--pmc", nargs="*", default=[],
                    help="further counter runs: every counter found for the kernel, per dispatch")
    ap.add_argument("--last", type=int, default=0,
                    help="use only the kernel's last N dispatches (trace and counters)")
    ap.add_argument("--workload", default="3D Euler turbulence 256^3 periodic, FP64")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    global LAST
    LAST = a.last
    info = {"kernel": a.kernel, "workload": a.workload, "command": a.command,
            "source_hash": source_hash(), "trace": trace_stats(a.trace, a.kernel, a.last)}
    if a.last:
        info["dispatches_used"] = f"last {a.last} of the kernel"
    if a.fetch and a.write:
        fv, fc = counter(a.fetch, a.kernel, "FETCH_SIZE")
        wv, wc = counter(a.write, a.kernel, "WRITE_SIZE")
        ff = COPY_KIB / statistics.mean(fc) if fc else None
        wf = COPY_KIB / statistics.mean(wc) if wc else None
        info["counters"] = {
            "FETCH_SIZE_KiB_per_dispatch": statistics.mean(fv),
            "WRITE_SIZE_KiB_per_dispatch": statistics.mean(wv),
            "dispatches": len(fv),
            "copy_calibration": {"FETCH_SIZE_KiB": statistics.mean(fc) if fc else None,
                                 "WRITE_SIZE_KiB": statistics.mean(wc) if wc else None,
                                 "true_KiB": COPY_KIB, "fetch_factor": ff, "write_factor": wf},
        }
        if ff and wf:
            info["traffic_bytes_per_launch"] = (statistics.mean(fv) * ff +
                                                statistics.mean(wv) * wf) * 1024.0
    if a.valu:
        v = {}
        for name in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                     "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_VALU", "SQ_WAVES"):
            vals, _ = counter(a.valu, a.kernel, name)
            if vals:
                v[name + "_per_dispatch"] = statistics.mean(vals)
        info["valu"] = v
        need = ("SQ_INSTS_VALU_ADD_F64_per_dispatch", "SQ_INSTS_VALU_MUL_F64_per_dispatch",
                "SQ_INSTS_VALU_FMA_F64_per_dispatch", "SQ_INSTS_VALU_TRANS_F64_per_dispatch")
        if all(k in v for k in need):
            info["fp64_flops_per_launch"] = 64.0 * (2.0 * v[need[2]] + v[need[0]] + v[need[1]] +
                                                    v[need[3]])
    if a.pmc:
        extra = {}
        for d in a.pmc:
            names = sorted({r["Counter_Name"] for r in _rows(d, "*counter_collection.csv")})
            for name in names:
                vals, _ = counter(d, a.kernel, name)
                if vals:
                    extra[name + "_per_dispatch"] = statistics.mean(vals)
        info["pmc"] = extra
    lines = ["# rocprofv3 summary: " + a.kernel, "",
             "command: " + a.command, "",
             "```json", json.dumps(info, indent=1), "```", ""]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
