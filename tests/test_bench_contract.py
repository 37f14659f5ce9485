"""bench.py's output contract on the host: a stand-in for the library (a plan
whose builds only sleep) and for the device, so that the budget logic and the
JSON line are checked without a GPU.  One line on stdout, valid JSON, with
the fields the benchmark line needs (roofline and cpu_baseline included);
--gpus other than 1 exits with status 2."""
import json
import sys
import time

import numpy as np
import pytest
import torch

import bench
from paper_2009_03555_amd import hfx


class _FakePlan:
    def __init__(self, system, stream=None):
        self.n_blocks, self.nnz = 10, 10
        self.blocks = np.zeros((10, 5), dtype=np.int32)

    def schwarz(self):
        return np.zeros(10)

    def build_K(self, D, K, flags=0, info=False):
        time.sleep(0.01)
        if info:
            return {"n_quartets": 100, "n_quartets_class": [5] * 21, "n_prim_quartets": 1000,
                    "n_fp32_quartets": 3, "flops": 1e9, "ms_density": 0.1, "ms_screen": 0.1, "ms_eri": 10.0,
                    "ms_finalize": 0.1, "ms_total": 10.3, "ms_class": [10.0 / 21] * 21,
                    "flops_class": [1e9 / 21] * 21}

    def destroy(self):
        pass


@pytest.fixture
def fake_device(monkeypatch):
    monkeypatch.setattr(hfx, "Plan", _FakePlan)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "is_available", lambda: True)
    monkeypatch.setattr(torch.Tensor, "cuda", lambda self, *a, **k: self)
    import systems
    monkeypatch.setattr(systems, "density_blocks", lambda s, b, **k: [np.zeros(10)])
    monkeypatch.setattr(bench, "cpu_baseline", lambda s, sec: {
        "value": 5.0, "unit": "quartets/s", "cores": 8, "kind": "oracle", "sample": "stand-in"})


def test_one_json_line_with_the_contract_fields(fake_device, monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "3", "--warmup", "2", "--budget-s", "3600"])
    bench.main()
    out = capsys.readouterr().out.strip().split("\n")
    assert len(out) == 1
    d = json.loads(out[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["higher_is_better"] is True
    assert d["config"]["workload"]
    r = d["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 8 and c["full_build_s_extrapolated"] == 100 / 5.0
    assert d["mixed"]["steps"] >= 1 and "max_abs_dK_vs_fp64" in d["mixed"]


def test_more_than_one_gpu_is_refused(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
