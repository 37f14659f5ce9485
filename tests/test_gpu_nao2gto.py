"""GPU: a basis of GTO contractions fitted to synthetic numerical atomic
orbitals (NAO2GTO, hfx_nao2gto_fit) feeds the exchange build like any other
basis: K of a small cluster and of a small periodic cell on that basis
equals the oracle (1e-10)."""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _fitted_element(seed, shells, n_gto):
    """(shell l list, exponents, raw coefficients) of one element whose
    shells are GTO fits of seeded numerical radial functions."""
    ls, ex, co = [], [], []
    for (l, z, rc) in systems.nao_basis(seed, shells):
        r, R = systems.nao_radial(l, z, rc)
        e, c, rms = hfx.nao2gto_fit(l, r, R, n_gto)
        assert rms < 0.05
        ls.append(l)
        ex.append(e)
        co.append(c)
    return ls, ex, co


def _system(base, n_gto):
    ls, ex, co = _fitted_element(21, (0, 0, 1, 1, 2), n_gto)
    nat = base.n_atoms
    return base.with_(shell_atom=np.repeat(np.arange(nat, dtype=np.int32), len(ls)),
                      shell_l=np.tile(np.array(ls, dtype=np.int32), nat),
                      shell_nprim=np.full(nat * len(ls), n_gto, dtype=np.int32),
                      prim_exp=np.tile(np.concatenate(ex), nat), prim_coef=np.tile(np.concatenate(co), nat),
                      name=base.name + "_nao2gto")


@pytest.mark.parametrize("which", ["cluster", "cell"])
def test_fitted_basis_build_against_oracle(which):
    if which == "cluster":
        s = _system(systems.random_cluster(4, seed=91, nprim=1), 3)
    else:
        s = _system(systems.diamond_cell(n=(1, 1, 1), nprim=1, shells=(0,), r_cut=4.6, seed=92), 2)
    plan = hfx.Plan(s)
    vals = systems.density_blocks(s, plan.blocks.astype(np.int64))
    D = np.concatenate([v.ravel() for v in vals])
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.full_like(Dd, np.nan)
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    o = oracle.Oracle(s)
    o.set_density(D)
    Kref, _ = o.build_K()
    err = np.max(np.abs(Kd.cpu().numpy() - Kref))
    print(f"{which}: {s.n_shells} fitted shells, {info['n_quartets']} quartets, max|dK| = {err:.3e}")
    assert err <= 1e-10
    plan.destroy()
