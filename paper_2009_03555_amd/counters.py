"""HBM traffic of the ERI kernels from two rocprofv3 counter passes.

Usage (after the two passes of ``bench.py ... --copy-gib 1``, one with
``rocprofv3 --pmc FETCH_SIZE`` and one with ``--pmc WRITE_SIZE``):

    python -m paper_2009_03555_amd.counters FETCH_DIR WRITE_DIR \\
        --workload diamond64 --out profiles/traffic.json

Each pass's counter CSV (``*counter_collection.csv`` under the directory)
gives FETCH_SIZE / WRITE_SIZE in KiB per dispatch.  The reference dispatch
is the plain device-to-device copy of ``--copy-gib`` GiB that bench.py runs
first (the largest dispatch whose kernel name contains "copy"): what the
counter reads for it, against the bytes it really moves, is the scale
factor applied to every other dispatch.  Per ERI class kernel (one launch
per class and build) the scaled bytes are averaged over its launches and
written with the hash of the kernel sources (bench.py reports them only
while the sources are unchanged).  Prints a markdown table.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def per_dispatch(d, counter):
    """{dispatch id: (kernel name, grid size, summed counter value)}"""
    out = {}
    for r in _rows(d):
        if r.get("Counter_Name") != counter:
            continue
        k = int(r["Dispatch_Id"])
        name, grid, v = out.get(k, (r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0), 0.0))
        out[k] = (name, grid, v + float(r["Counter_Value"]))
    return out


_CLASS = re.compile(r"eri_(?:digest|lane|coop)_kernel<(\d), (\d), (\d)")


def class_label(cb, ck):
    pc = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    a, b = pc[cb]
    c, d = pc[ck]
    return f"({'spd'[a]}{'spd'[b]}|{'spd'[c]}{'spd'[d]})"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--workload", default="diamond64")
    ap.add_argument("--copy-gib", type=float, default=1.0)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    from bench import kernel_hash  # the same hash bench.py checks
    f = per_dispatch(args.fetch_dir, "FETCH_SIZE")
    w = per_dispatch(args.write_dir, "WRITE_SIZE")
    ref = float(args.copy_gib) * (1 << 30)

    def copy_of(disp):
        c = [(v, name) for (name, grid, v) in disp.values() if "copy" in name.lower()]
        if not c:
            raise SystemExit("no reference copy dispatch found")
        return max(c)

    fv, fname = copy_of(f)
    wv, wname = copy_of(w)
    rf, rw = fv * 1024 / ref, wv * 1024 / ref
    print(f"reference copy: FETCH_SIZE {fv:.1f} KiB ({fname}), WRITE_SIZE {wv:.1f} KiB ({wname}) for "
          f"{ref / 1024:.1f} KiB each way: factors {rf:.3f} (reads), {rw:.3f} (writes)")
    acc = defaultdict(lambda: {"fetch": [], "write": [], "kernel": ""})
    for disp, key in ((f, "fetch"), (w, "write")):
        for name, grid, v in disp.values():
            m = _CLASS.search(name)
            if not m:
                continue
            lab = class_label(int(m.group(1)), int(m.group(2)))
            acc[lab][key].append(v)
            acc[lab]["kernel"] = re.sub(r"^.*?(eri_\w+_kernel<[^>]*>).*$", r"\1", name)
    h = kernel_hash()
    tab = {}
    for lab, a in acc.items():
        if not a["fetch"] or not a["write"]:
            continue
        fk = sum(a["fetch"]) / len(a["fetch"])
        wk = sum(a["write"]) / len(a["write"])
        rb, wb = fk * 1024 / rf, wk * 1024 / rw
        tab[lab] = {"bytes_per_launch": rb + wb, "read_bytes": rb, "write_bytes": wb, "fetch_kib_raw": fk,
                    "write_kib_raw": wk, "copy_read_factor": rf, "copy_write_factor": rw,
                    "launches": len(a["fetch"]), "kernel": a["kernel"], "kernel_hash": h}
    old = {}
    if os.path.exists(args.out):
        try:
            old = json.load(open(args.out))
        except ValueError:
            old = {}
    old[args.workload] = tab
    with open(args.out, "w") as fh:
        json.dump(old, fh, indent=1)
    print("| class | kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled read GB | scaled write GB |")
    print("|---|---|---:|---:|---:|---:|")
    for lab, t in sorted(tab.items(), key=lambda x: -x[1]["bytes_per_launch"]):
        print(f"| {lab.replace('|', chr(92) + '|')} | `{t['kernel']}` | {t['fetch_kib_raw']:.1f} | "
              f"{t['write_kib_raw']:.1f} | {t['read_bytes'] / 1e9:.2f} | {t['write_bytes'] / 1e9:.2f} |")


if __name__ == "__main__":
    main()
