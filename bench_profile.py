#!/usr/bin/env python
"""Summaries of rocprofv3 output for profiles/ (run on the host after a
profiled GPU run; reads rocprofv3's files, runs nothing on the GPU).

  trace DB [--kernel NAME ...] [--command CMD]
      Markdown summary of a `rocprofv3 --kernel-trace --stats` results
      database: the top kernels by total time, then per named kernel its
      launches, average / min / max duration and resources.
  traffic --fetch CSV --write CSV --kernel NAME --workload W --calib-mib MIB
          [--out JSON]
      HBM bytes per launch of one kernel from two counter runs
      (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`, CSV output) of the same
      command, each counter scaled by what it reads for the plain copy of
      MIB MiB of float64 (an elementwise negation, 8 bytes read and 8
      written per element) that `bench.py --calibrate-copy MIB` runs first.
      The JSON carries the hash of the kernel's sources (bench.py reports it
      only while they are unchanged).
  hbm --fetch CSV --write CSV --kernel NAME ... --calib-mib MIB
      The same calibration for several kernels: bytes read and written,
      summed durations and GB/s.
  mfma CSV --kernel NAME ...
      BF16 MFMA flops and MFMA-busy fraction from a counter run of
      SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE.
  valu CSV --kernel NAME ...
      VALU and LDS busy fractions and the FP64 share of the VALU
      instructions from one counter run (see valu_table).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sqlite3
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def trace_summary(db: str, kernels, command: str | None) -> str:
    c = sqlite3.connect(db)
    out = []
    if command:
        out += [f"Command: `{command}`", ""]
    out += ["| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in list(c.execute(
            "select name, total_calls, total_duration, average, percentage from top_kernels"))[:16]:
        short = n if len(n) < 100 else n[:97] + "..."
        out.append(f"| `{short}` | {calls} | {tot / 1e3:.3f} | {avg:.1f} | {pct:.1f} |")
    for k in kernels:
        out += ["", f"`{k}` launches (durations from the trace, ns -> us):", "",
                "| blocks | threads | launches | average us | min us | max us | VGPRs | "
                "scratch B/lane | LDS B |", "|---|---|---|---|---|---|---|---|---|"]
        q = ("select grid_x/workgroup_x, workgroup_x, count(*), avg(duration), min(duration), "
             "max(duration), max(vgpr_count), max(scratch_size), max(lds_size) from kernels "
             "where name like ? group by grid_x/workgroup_x, workgroup_x order by 1")
        for b, t, n, avg, mn, mx, vg, sc, lds in c.execute(q, (f"%{k}%",)):
            out.append(f"| {b} | {t} | {n} | {avg / 1e3:.1f} | {mn / 1e3:.1f} | {mx / 1e3:.1f} "
                       f"| {vg} | {sc} | {lds} |")
    return "\n".join(out) + "\n"


def _counters(path: str):
    """{dispatch id: (kernel name, {counter: value summed over instances})}."""
    files = [path] if os.path.isfile(path) else sorted(
        glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no counter_collection.csv under {path}")
    disp = defaultdict(lambda: ["", defaultdict(float)])
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                d = disp[(f, row["Dispatch_Id"])]
                d[0] = row["Kernel_Name"]
                d[1][row["Counter_Name"]] += float(row["Counter_Value"])
    return list(disp.values())


def traffic(fetch_csv: str, write_csv: str, kernel: str, workload: str, calib_mib: int) -> dict:
    from bench import f_kernel_hash
    calib_bytes = calib_mib * (1 << 20)
    res = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _counters(path)
        # the calibration copy: bench.py's elementwise negation (torch's
        # neg kernel), the only one of the run
        cal = next(v[name] for k, v in rows if "neg_kernel" in k and name in v)
        ker = [v[name] for k, v in rows if kernel in k and name in v]
        if not ker:
            raise SystemExit(f"no dispatch of {kernel} in {path}")
        kib = sum(ker) / len(ker)
        factor = calib_bytes / (cal * 1024.0)
        res[name] = {"kib_per_launch": kib, "launches": len(ker), "calibration_kib": cal,
                     "bytes_per_kib": factor * 1024.0, "bytes_per_launch": kib * 1024.0 * factor}
    return {"kernel": kernel, "workload": workload, "source_sha256": f_kernel_hash(),
            "calibration": f"{calib_mib} MiB float64 copy, {calib_bytes} B read and written",
            "counters": res,
            "hbm_bytes_per_launch": res["FETCH_SIZE"]["bytes_per_launch"] +
            res["WRITE_SIZE"]["bytes_per_launch"]}


def _dispatches(path: str):
    """[(kernel name, {counter: value}, duration ns)] per dispatch."""
    files = [path] if os.path.isfile(path) else sorted(
        glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    disp = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (f, row["Dispatch_Id"])
                if key not in disp:
                    disp[key] = [row["Kernel_Name"], defaultdict(float),
                                 int(row["End_Timestamp"]) - int(row["Start_Timestamp"])]
                disp[key][1][row["Counter_Name"]] += float(row["Counter_Value"])
    return list(disp.values())


def hbm_table(fetch_csv: str, write_csv: str, kernels, calib_mib: int) -> str:
    """Per kernel: launches, calibrated HBM bytes read / written, summed
    duration (counter runs serialise dispatches) and GB/s."""
    calib_bytes = calib_mib * (1 << 20)
    tot = defaultdict(lambda: [0, 0.0, 0.0, 0])
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _dispatches(path)
        cal = next(c[name] for k, c, _ in rows if "neg_kernel" in k)
        scale = calib_bytes / cal  # bytes per counter unit
        for k, c, dur in rows:
            for want in kernels:
                if want in k:
                    t = tot[want]
                    if name == "FETCH_SIZE":
                        t[0] += 1
                        t[1] += c[name] * scale
                        t[3] += dur
                    else:
                        t[2] += c[name] * scale
    out = ["| kernel | launches | read GB | written GB | summed duration ms | GB/s |",
           "|---|---|---|---|---|---|"]
    for k, (n, rd, wr, dur) in tot.items():
        out.append(f"| `{k}` | {n} | {rd / 1e9:.3f} | {wr / 1e9:.3f} | {dur / 1e6:.3f} | "
                   f"{(rd + wr) / max(dur, 1):.1f} |")
    return "\n".join(out) + "\n"


def mfma_table(path: str, kernels, simds: int = 1024, xcds: int = 8) -> str:
    """Per kernel: BF16 MFMA flops (SQ_INSTS_VALU_MFMA_MOPS_BF16 x 512), the
    MFMA-busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (GPU-active cycles x SIMDs)
    (rocprofv3 reports GRBM_GUI_ACTIVE summed over the 8 XCDs, so the active
    cycles are that sum / 8), and flops / duration."""
    rows = _dispatches(path)
    tot = defaultdict(lambda: [0, 0.0, 0.0, 0.0, 0])
    for k, c, dur in rows:
        for want in kernels:
            if want in k:
                t = tot[want]
                t[0] += 1
                t[1] += c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) * 512
                t[2] += c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
                t[3] += c.get("GRBM_GUI_ACTIVE", 0.0)
                t[4] += dur
    out = ["| kernel | launches | BF16 MFMA TFLOP | MFMA busy | TFLOP/s over the summed duration |",
           "|---|---|---|---|---|"]
    for k, (n, fl, busy, act, dur) in tot.items():
        frac = busy / (act / xcds * simds) if act else float("nan")
        out.append(f"| `{k}` | {n} | {fl / 1e12:.4f} | {frac:.4f} | "
                   f"{fl / max(dur, 1) / 1e3:.2f} |")
    return "\n".join(out) + "\n"


def valu_table(path: str, kernels, cus: int = 256, xcds: int = 8) -> str:
    """Per kernel, from SQ_ACTIVE_INST_VALU, SQ_INSTS_VALU, SQ_INSTS_VALU_{FMA,
    MUL,ADD}_F64, SQ_INSTS_LDS, SQ_LDS_IDX_ACTIVE, SQ_WAVE_CYCLES and
    GRBM_GUI_ACTIVE: VALU busy (rocprof's VALUBusy: active VALU cycles per CU
    over the GPU-active cycles; GRBM_GUI_ACTIVE comes summed over the XCDs),
    LDS busy (LdsUtil, likewise), FP64 share of the VALU instructions, and
    VALU instructions per wave-cycle."""
    rows = _dispatches(path)
    tot = defaultdict(lambda: defaultdict(float))
    for k, c, dur in rows:
        for want in kernels:
            if want in k:
                t = tot[want]
                t["n"] += 1
                for name, v in c.items():
                    t[name] += v
    out = ["| kernel | launches | VALU busy | LDS busy | FP64 share of VALU instructions | "
           "VALU instructions per wave quad-cycle |", "|---|---|---|---|---|---|"]
    for k, t in tot.items():
        act = t["GRBM_GUI_ACTIVE"] / xcds
        f64 = t["SQ_INSTS_VALU_FMA_F64"] + t["SQ_INSTS_VALU_MUL_F64"] + t["SQ_INSTS_VALU_ADD_F64"]
        out.append(f"| `{k}` | {int(t['n'])} | {t['SQ_ACTIVE_INST_VALU'] / cus / act:.3f} | "
                   f"{t['SQ_LDS_IDX_ACTIVE'] / cus / act:.3f} | "
                   f"{f64 / max(t['SQ_INSTS_VALU'], 1):.3f} | "
                   f"{t['SQ_INSTS_VALU'] / max(t['SQ_WAVE_CYCLES'], 1):.3f} |")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--kernel", action="append", default=[])
    t.add_argument("--command")
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--kernel", required=True)
    f.add_argument("--workload", required=True)
    f.add_argument("--calib-mib", type=int, required=True)
    f.add_argument("--out")
    h = sub.add_parser("hbm")
    h.add_argument("--fetch", required=True)
    h.add_argument("--write", required=True)
    h.add_argument("--kernel", action="append", required=True)
    h.add_argument("--calib-mib", type=int, required=True)
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("--kernel", action="append", required=True)
    v = sub.add_parser("valu")
    v.add_argument("csv")
    v.add_argument("--kernel", action="append", required=True)
    a = ap.parse_args()
    if a.cmd == "valu":
        sys.stdout.write(valu_table(a.csv, a.kernel))
        return
    if a.cmd == "trace":
        sys.stdout.write(trace_summary(a.db, a.kernel, a.command))
    elif a.cmd == "hbm":
        sys.stdout.write(hbm_table(a.fetch, a.write, a.kernel, a.calib_mib))
    elif a.cmd == "mfma":
        sys.stdout.write(mfma_table(a.csv, a.kernel))
    else:
        r = traffic(a.fetch, a.write, a.kernel, a.workload, a.calib_mib)
        s = json.dumps(r, indent=1)
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(s + "\n")
        print(s)


if __name__ == "__main__":
    main()
