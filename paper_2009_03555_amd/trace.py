"""Kernel-time summary and launch gaps of an exchange build from a rocprofv3
kernel trace.

Usage (after ``rocprofv3 --kernel-trace --stats --output-format csv -d DIR
-- python3 bench.py ...``):

    python -m paper_2009_03555_amd.trace DIR [--top 25]

Reads ``*kernel_trace.csv`` under DIR and prints markdown:

* per kernel name: dispatches, total and average duration, share of all
  kernel time (the same figures as rocprofv3's own stats);
* the last build in the trace, from the last density kernel (the first
  kernel of a build) to the finalisation kernel after it: its wall span,
  the time covered by at least one kernel, the uncovered time between
  launches (what a single persistent launch could at most remove) and the
  largest gaps with the kernels on either side.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
from collections import defaultdict


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {d}")
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise SystemExit(f"none of the columns {names} in the kernel trace")


def dispatches(d):
    """[(start ns, end ns, kernel name)] sorted by start"""
    out = []
    cols = None
    for r in _rows(d):
        if cols is None:
            cols = (_col(r, "Start_Timestamp", "BeginNs", "Start"), _col(r, "End_Timestamp", "EndNs", "End"),
                    _col(r, "Kernel_Name", "KernelName", "Name"))
        out.append((int(r[cols[0]]), int(r[cols[1]]), r[cols[2]]))
    out.sort()
    return out


def short(name: str) -> str:
    """kernel name without its argument list"""
    m = re.match(r"(?:void )?([^(]*)", name)
    return (m.group(1) if m else name).strip()


def per_kernel(ds):
    acc = defaultdict(lambda: [0, 0])
    for s, e, n in ds:
        acc[short(n)][0] += 1
        acc[short(n)][1] += e - s
    return acc


def last_build(ds):
    """dispatches of the last build: from the last density kernel to the
    first finalisation kernel after it"""
    starts = [i for i, (_, _, n) in enumerate(ds) if "density_kernel" in n]
    if not starts:
        return []
    i0 = starts[-1]
    for j in range(i0, len(ds)):
        if "finalize_kernel" in ds[j][2]:
            return ds[i0:j + 1]
    return ds[i0:]


def covered(ds):
    """time covered by the union of the dispatch intervals"""
    tot, cur_s, cur_e = 0, None, None
    for s, e, _ in ds:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args(argv)
    ds = dispatches(a.dir)
    acc = per_kernel(ds)
    total = sum(v[1] for v in acc.values()) or 1
    print("| kernel | calls | total ms | avg ms | % |\n|---|---:|---:|---:|---:|")
    for name, (c, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])[: a.top]:
        print(f"| `{name}` | {c} | {t / 1e6:.3f} | {t / c / 1e6:.3f} | {100 * t / total:.2f} |")
    b = last_build(ds)
    if not b:
        return
    wall = b[-1][1] - b[0][0]
    cov = covered(b)
    busy = sum(e - s for s, e, _ in b)
    gaps = []
    end_so_far, prev = b[0][1], b[0]
    for d in b[1:]:
        if d[0] > end_so_far:
            gaps.append((d[0] - end_so_far, short(prev[2]), short(d[2])))
        if d[1] >= end_so_far:
            end_so_far, prev = d[1], d
    print(f"\nLast build in the trace: {len(b)} dispatches, wall {wall / 1e6:.3f} ms from the start of "
          f"the density kernel to the end of the finalisation kernel; kernels cover {cov / 1e6:.3f} ms "
          f"({100 * cov / wall:.3f}%), summed kernel time {busy / 1e6:.3f} ms; time with no kernel running "
          f"{(wall - cov) / 1e6:.3f} ms in {len(gaps)} gaps.")
    if gaps:
        print("\n| gap us | after | before |\n|---:|---|---|")
        for g, p, n in sorted(gaps, reverse=True)[:8]:
            print(f"| {g / 1e3:.1f} | `{p}` | `{n}` |")


if __name__ == "__main__":
    main()
