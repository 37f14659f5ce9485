"""Occupancy, VALU and LDS shares of the ERI kernels from two rocprofv3
counter passes.

Usage (two passes of one build, each ``rocprofv3 --pmc ... --output-format
csv -d DIR -- python3 bench.py ...``):

    pass 1: SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY
            SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_WAIT_INST_LDS SQ_INSTS_VALU
    pass 2: SQ_LDS_IDX_ACTIVE SQ_LDS_BANK_CONFLICT SQ_LDS_DATA_FIFO_FULL
            SQ_LDS_CMD_FIFO_FULL SQ_INSTS_LDS_LOAD_BANDWIDTH
            SQ_INSTS_LDS_STORE_BANDWIDTH SQ_LDS_ADDR_CONFLICT SQ_WAVE_CYCLES
            GRBM_GUI_ACTIVE

    python -m paper_2009_03555_amd.sqcounters DIR1 DIR2

Normalisation.  Each counter is summed over its hardware instances (the
rows rocprofv3 gives for a dispatch): SQ counters over the shader engines,
GRBM_GUI_ACTIVE over the XCDs, whose count (and the SIMD and compute-unit
counts) come from the pass's agent_info.csv.  GUI_ACTIVE / XCDs is the
launch's length in cycles (C); SQ counters count in units of 4 cycles.
* waves/SIMD = SQ_WAVE_CYCLES x 4 / (C x SIMDs)
* VALU busy = SQ_ACTIVE_INST_VALU x 4 / (C x SIMDs), the share of SIMD
  cycles issuing a vector ALU instruction
* LDS wait = SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES, the share of wave time spent
  waiting for LDS results
* LDS busy = SQ_LDS_IDX_ACTIVE / (C x compute units)
* bank conflicts = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE
ms is the dispatch's end minus start timestamp.  Pass 2 repeats
SQ_WAVE_CYCLES, and its GRBM_GUI_ACTIVE serves both passes.  Each kernel
is averaged over its launches, and the output is a markdown table, longest
kernel first.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
from collections import defaultdict

from paper_2009_03555_amd.counters import class_label, _CLASS


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def topology(d):
    """(XCDs, SIMDs, compute units) of the GPU agent of a pass"""
    files = glob.glob(os.path.join(d, "**", "*agent_info.csv"), recursive=True)
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Agent_Type") == "GPU":
                    return int(r["Num_Xcc"]), int(r["Simd_Count"]), int(r["Cu_Count"])
    return 8, 1024, 256  # MI355X


def per_dispatch(d):
    """{dispatch id: (kernel name, ns, {counter: sum over its rows})}"""
    acc = defaultdict(lambda: defaultdict(float))
    meta = {}
    for r in _rows(d):
        k = int(r["Dispatch_Id"])
        ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) if r.get("End_Timestamp") else 0
        meta[k] = (r["Kernel_Name"], ns)
        acc[k][r["Counter_Name"]] += float(r["Counter_Value"])
    return {k: (meta[k][0], meta[k][1], dict(cs)) for k, cs in acc.items()}


def kernel_table(d1, d2):
    """per ERI class kernel: averaged shares over its launches"""
    a, b = per_dispatch(d1), per_dispatch(d2)
    nxcc, nsimd, ncu = topology(d2)
    out = defaultdict(lambda: defaultdict(list))
    for k, (name, ns, c2) in b.items():
        m = _CLASS.search(name)
        if not m or k not in a:
            continue
        c1 = a[k][2]
        cyc = c2.get("GRBM_GUI_ACTIVE", 0.0) / nxcc
        if cyc <= 0:
            continue
        lab = class_label(int(m.group(1)), int(m.group(2)))
        kind = "lane" if "lane" in name else ("coop" if "coop" in name else "one-lane")
        if "float" in name.split(">")[0]:
            kind += " FP32"
        wc = c1.get("SQ_WAVE_CYCLES", 0.0)
        o = out[(lab, kind)]
        o["ms"].append(ns / 1e6 if ns else cyc / 2.4e6)
        o["waves"].append(wc * 4 / (cyc * nsimd))
        o["valu"].append(c1.get("SQ_ACTIVE_INST_VALU", 0.0) * 4 / (cyc * nsimd))
        o["ldswait"].append(c1.get("SQ_WAIT_INST_LDS", 0.0) / wc if wc else 0.0)
        lds = c2.get("SQ_LDS_IDX_ACTIVE", 0.0)
        o["ldsbusy"].append(lds / (cyc * ncu))
        o["bank"].append(c2.get("SQ_LDS_BANK_CONFLICT", 0.0) / lds if lds else 0.0)
    return {k: {f: sum(v) / len(v) for f, v in o.items()} for k, o in out.items()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("pass1")
    ap.add_argument("pass2")
    a = ap.parse_args(argv)
    t = kernel_table(a.pass1, a.pass2)
    print("| class | kernel | ms | waves/SIMD | VALU busy | LDS wait | LDS busy | bank conflicts |")
    print("|---|---|---:|---:|---:|---:|---:|---:|")
    for (lab, kind), v in sorted(t.items(), key=lambda kv: -kv[1]["ms"]):
        print(f"| {lab.replace('|', chr(92) + '|')} | {kind} | {v['ms']:.0f} | {v['waves']:.2f} | "
              f"{100 * v['valu']:.0f}% | {100 * v['ldswait']:.0f}% | {100 * v['ldsbusy']:.0f}% | "
              f"{100 * v['bank']:.1f}% |")


if __name__ == "__main__":
    main()
