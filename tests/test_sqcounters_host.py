"""Arithmetic of the SQ counter summary (paper_2009_03555_amd.sqcounters)
on synthetic rocprofv3 counter_collection.csv files."""
import csv

from paper_2009_03555_amd import sqcounters


def _write(d, rows):
    d.mkdir()
    with open(d / "p_counter_collection.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)
    return str(d)


def test_shares_of_one_launch(tmp_path):
    name = "void hfx::eri_lane_kernel<4, 2, 1, true, double>(hfx::DevSys const*)"
    cyc = 2.4e6  # one millisecond at 2.4 GHz
    # MI355X: 8 XCDs, 1024 SIMDs, 256 compute units (no agent_info.csv);
    # counters summed over their instances, split here over two rows each
    p1 = []
    for v in (2 * cyc * 1024 / 4 * 0.4, 2 * cyc * 1024 / 4 * 0.6):   # 2 waves per SIMD
        p1.append((7, name, "SQ_WAVE_CYCLES", v))
    for v in (0.5 * cyc * 1024 / 4 * 0.5, 0.5 * cyc * 1024 / 4 * 0.5):  # VALU busy 50%
        p1.append((7, name, "SQ_ACTIVE_INST_VALU", v))
    p1.append((7, name, "SQ_WAIT_INST_LDS", 0.25 * 2 * cyc * 1024 / 4))  # a quarter of the wave time
    p2 = [(7, name, "GRBM_GUI_ACTIVE", 4 * cyc), (7, name, "GRBM_GUI_ACTIVE", 4 * cyc),
          (7, name, "SQ_LDS_IDX_ACTIVE", 0.6 * cyc * 256), (7, name, "SQ_LDS_BANK_CONFLICT", 0.03 * 0.6 * cyc * 256),
          (8, "void hfx::density_kernel(x)", "GRBM_GUI_ACTIVE", 10.0)]
    t = sqcounters.kernel_table(_write(tmp_path / "a", p1), _write(tmp_path / "b", p2))
    assert list(t) == [("(dp|pp)", "lane")]
    v = t[("(dp|pp)", "lane")]
    assert abs(v["ms"] - 1.0) < 1e-12
    assert abs(v["waves"] - 2.0) < 1e-12
    assert abs(v["valu"] - 0.5) < 1e-12
    assert abs(v["ldswait"] - 0.25) < 1e-12
    assert abs(v["ldsbusy"] - 0.6) < 1e-12
    assert abs(v["bank"] - 0.03) < 1e-12
