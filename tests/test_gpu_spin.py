"""GPU: collinear-spin builds (hfx_build_K_spin) - both spins' K from one
ERI evaluation - against the oracle's spin build (Eq. H-HFX per spin
density, block maxima the larger of the two spins'), 1e-10 in FP64 and
1e-7 in mixed precision; equal spin densities reproduce the unpolarised
build (1e-12)."""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dens(system, blocks, seed_shift=0):
    s = system.with_(seed=system.seed + seed_shift) if seed_shift else system
    vals = systems.density_blocks(s, np.asarray(blocks, dtype=np.int64))
    return np.concatenate([v.ravel() for v in vals])


def _tiny_cell(**kw):
    kw.setdefault("seed", 77)
    return systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, **kw)


@pytest.mark.parametrize("which", ["molecule8", "cell", "cell_mixed", "cell_chunked"])
def test_spin_build_against_oracle(which):
    if which == "molecule8":
        s = systems.molecule8()
    elif which == "cell_mixed":
        s = _tiny_cell(precision="mixed").with_(fp32_cutoff=1e-2)
    else:
        s = _tiny_cell()
    plan = hfx.Plan(s)
    if which == "cell_chunked":
        plan.set_list_limit(4096)
    Da = _dens(s, plan.blocks)
    Db = 0.4 * _dens(s, plan.blocks, seed_shift=17)
    da, db = torch.from_numpy(Da).to(DEV), torch.from_numpy(Db).to(DEV)
    ka, kb = torch.full_like(da, np.nan), torch.full_like(da, np.nan)
    info = plan.build_K_spin(da, db, ka, kb, flags=hfx.HFX_SYNC, info=True)
    if which == "cell_chunked":
        assert info["n_chunks"] >= 3
    o = oracle.Oracle(s)
    o.schwarz()
    ra, rb = o.build_K_spin(Da, Db)
    tol = 1e-10 if s.precision == "fp64" else 1e-7
    assert np.max(np.abs(ka.cpu().numpy() - ra)) <= tol
    assert np.max(np.abs(kb.cpu().numpy() - rb)) <= tol
    # the unpolarised build of the same plan is unaffected
    k1 = torch.full_like(da, np.nan)
    plan.build_K(da, k1, flags=hfx.HFX_SYNC)
    o.set_density(Da)
    r1, _ = o.build_K()
    assert np.max(np.abs(k1.cpu().numpy() - r1)) <= tol
    plan.destroy()


def test_equal_spins_equal_the_unpolarised_build_and_graphs_replay():
    s = _tiny_cell()
    plan = hfx.Plan(s)
    D = torch.from_numpy(_dens(s, plan.blocks)).to(DEV)
    k = torch.zeros_like(D)
    i1 = plan.build_K(D, k, flags=hfx.HFX_SYNC, info=True)
    ref = k.cpu().numpy()
    ka, kb = torch.full_like(D, np.nan), torch.full_like(D, np.nan)
    i2 = plan.build_K_spin(D, D, ka, kb, flags=hfx.HFX_SYNC, info=True)
    assert i2["n_quartets"] == i1["n_quartets"] and i2["n_prim_quartets"] == i1["n_prim_quartets"]
    assert i2["flops"] > i1["flops"]
    scale = max(1.0, float(np.max(np.abs(ref))))
    for kk in (ka, kb):
        assert np.max(np.abs(kk.cpu().numpy() - ref)) <= 1e-12 * scale
    # graph replays of the spin build, with eager work between them
    for r in range(3):
        ka.fill_(np.nan)
        kb.fill_(np.nan)
        plan.build_K_spin(D, D, ka, kb, flags=hfx.HFX_GRAPH)
        plan.build_K(D, k, flags=hfx.HFX_SYNC)
        for kk in (ka, kb):
            assert np.max(np.abs(kk.cpu().numpy() - ref)) <= 1e-12 * scale, r
    plan.destroy()
