"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/hfx.h, and rejects bad systems with
the documented status before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import systems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")


def _declared():
    src = open(os.path.join(ROOT, "include", "hfx.h")).read()
    return sorted(set(re.findall(r"\b(hfx_[A-Za-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert {"hfx_plan", "hfx_schwarz", "hfx_build_K", "hfx_build_K_multi", "hfx_pattern",
            "hfx_footprint", "hfx_export", "hfx_plan_destroy", "hfx_last_error"} <= set(names)
    L = hfx.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", hfx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hfx_[A-Za-z_]+)$", out, flags=re.M))
    assert set(names) <= exported


def _status_of(system):
    a = hfx._SystemArgs(system)
    dev = ctypes.c_size_t(0)
    per = ctypes.c_size_t(0)
    return hfx.lib().hfx_footprint(ctypes.byref(a.c), ctypes.byref(dev), ctypes.byref(per)), dev.value


def test_footprint_of_the_molecule():
    st, dev = _status_of(systems.molecule8())
    assert st == hfx.HFX_OK and dev > 0


@pytest.mark.parametrize("mutate,expected", [
    (lambda s: s.with_(shell_l=np.where(np.arange(s.n_shells) == 0, 3, s.shell_l).astype(np.int32)),
     hfx.HFX_ERR_UNSUPPORTED),
    (lambda s: s.with_(prim_exp=np.where(np.arange(len(s.prim_exp)) == 1, -1.0, s.prim_exp)),
     hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(prim_exp=np.where(np.arange(len(s.prim_exp)) == 1, np.nan, s.prim_exp)),
     hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(atom_xyz=np.where(np.arange(s.atom_xyz.size).reshape(-1, 3) == 4, np.inf, s.atom_xyz)),
     hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(lattice=np.zeros((3, 3)), pair_cutoff=5.0), hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(lattice=np.eye(3) * 10.0, pair_cutoff=0.0), hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(op="erfc", omega=0.0), hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(tau=-1.0), hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(shell_nprim=np.where(np.arange(s.n_shells) == 0, 9, s.shell_nprim).astype(np.int32),
                       prim_exp=np.concatenate([s.prim_exp, np.ones(6)]),
                       prim_coef=np.concatenate([s.prim_coef, np.ones(6)])), hfx.HFX_ERR_INVALID),
    (lambda s: s.with_(shell_atom=np.where(np.arange(s.n_shells) == 2, 99, s.shell_atom).astype(np.int32)),
     hfx.HFX_ERR_INVALID),
])
def test_invalid_systems_rejected(mutate, expected):
    st, _ = _status_of(mutate(systems.molecule8()))
    assert st == expected
    assert hfx.hfx_last_error()


def test_plan_rejects_before_device_work():
    s = systems.molecule8().with_(tau=-5.0)
    a = hfx._SystemArgs(s)
    h = ctypes.c_void_p(None)
    st = hfx.lib().hfx_plan(ctypes.byref(a.c), None, ctypes.byref(h))
    assert st == hfx.HFX_ERR_INVALID and not h.value


def test_null_and_bogus_handles():
    L = hfx.lib()
    assert L.hfx_plan_destroy(None) == hfx.HFX_ERR_STATE
    n = ctypes.c_int64(0)
    assert L.hfx_export(ctypes.c_void_p(12345), 0, None, ctypes.byref(n)) == hfx.HFX_ERR_STATE


def test_translation_range_checked_at_plan_time():
    # a cutoff long against the cell could need ket translations beyond the
    # 5-bit quartet encoding: refused when planning, never dropped silently
    s = systems.diamond_cell(n=(1, 1, 1), nprim=1, shells=(0,), r_cut=50.0)
    with pytest.raises(hfx.HfxError) as e:
        hfx.hfx_footprint(s)
    assert e.value.status == hfx.HFX_ERR_UNSUPPORTED
    assert "translations" in str(e.value)
    # the benchmark cell is far inside the range
    dev, per = hfx.hfx_footprint(systems.diamond_cell())
    assert dev > 0 and per == 8


def test_nao2gto_and_progress_symbols_are_host_callable():
    # the fit needs no device: it runs here
    r, R = systems.nao_radial(2, 1.1, 6.0)
    e, c, rms = hfx.nao2gto_fit(2, r, R, 4)
    assert np.all(np.diff(e) > 0) and rms < 0.05


def test_missing_library_raises_and_nothing_falls_back(monkeypatch):
    # the binding loads only the built library; without it every call fails
    # loudly (there is no CPU path to fall back to)
    from paper_2009_03555_amd import hfx as H
    monkeypatch.setattr(H, "_lib", None)
    monkeypatch.setattr(H, "LIB_PATH", "/nonexistent/libhfx.so")
    with pytest.raises(ImportError):
        H.lib()
    import systems
    with pytest.raises(ImportError):
        H.hfx_footprint(systems.molecule8())
