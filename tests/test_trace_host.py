"""Host logic of the kernel-trace summary (paper_2009_03555_amd.trace) on a
synthetic rocprofv3 kernel_trace.csv."""
import csv

from paper_2009_03555_amd import trace


def _write(tmp_path, rows):
    d = tmp_path / "prof"
    d.mkdir()
    with open(d / "x_kernel_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for n, s, e in rows:
            w.writerow(["KERNEL_DISPATCH", n, s, e])
    return str(d)


def test_last_build_gaps_and_cover(tmp_path, capsys):
    rows = [
        ("void hfx::density_kernel(a)", 0, 10),          # first build
        ("void hfx::finalize_kernel(a)", 20, 30),
        ("void hfx::density_kernel(a)", 100, 110),       # last build
        ("void hfx::screen_kernel(a)", 115, 140),        # gap 5 after density
        ("void hfx::eri_lane_kernel<4, 2>(a)", 140, 400),
        ("void hfx::eri_digest_kernel<1, 0>(a)", 390, 500),  # overlaps: no gap
        ("void hfx::finalize_kernel(a)", 520, 530),      # gap 20
    ]
    d = _write(tmp_path, rows)
    ds = trace.dispatches(d)
    b = trace.last_build(ds)
    assert [trace.short(n) for _, _, n in b][0] == "hfx::density_kernel"
    assert len(b) == 5 and b[-1][0] == 520
    assert trace.covered(b) == 10 + 25 + (500 - 140) + 10
    acc = trace.per_kernel(ds)
    assert acc["hfx::density_kernel"] == [2, 20]
    trace.main([d])
    out = capsys.readouterr().out
    assert "5 dispatches" in out and "in 2 gaps" in out
    assert "| 0.0 | `hfx::eri_digest_kernel<1, 0>` | `hfx::finalize_kernel` |" in out
