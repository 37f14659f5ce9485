"""GPU: k-space assembly of the exchange Hamiltonian (hfx_kspace) against
the oracle's plain Bloch sum, on seeded symmetric K in the pattern layout
(the density recipe, so no input comes from the HIP path), HSE06 fraction
1/4: every element within 1e-13 of max|H|."""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _K(system, blocks):
    vals = systems.density_blocks(system, np.asarray(blocks, dtype=np.int64))
    return np.concatenate([v.ravel() for v in vals])


@pytest.mark.parametrize("which", ["cell", "cell_cartesian_d", "diamond64", "molecule"])
def test_kspace_against_oracle(which):
    if which == "molecule":
        s = systems.molecule8()
        kp = np.zeros((1, 3))
    else:
        if which == "diamond64":
            s = systems.diamond_cell()
        else:
            s = systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, seed=79,
                                        spherical_d=(which == "cell"))
        rec = 2 * np.pi * np.linalg.inv(np.asarray(s.lattice)).T
        rng = np.random.default_rng(3)
        kp = np.concatenate([np.zeros((1, 3)), 0.5 * rec[:1], rng.uniform(-0.5, 0.5, size=(3, 3)) @ rec])
    plan = hfx.Plan(s)
    K = _K(s, plan.blocks)
    Kd = torch.from_numpy(K).to(DEV)
    nbf = int(sum(systems.nfunc(int(l), s.spherical_d) for l in s.shell_l))
    H = torch.full((len(kp), nbf, nbf, 2), np.nan, dtype=torch.float64, device=DEV)
    plan.kspace(Kd, kp, 0.25, H)
    Hg = H.cpu().numpy()
    Hg = Hg[..., 0] + 1j * Hg[..., 1]
    Ho = oracle.kspace(s, plan.blocks, plan.offsets, K, kp, 0.25)
    err = np.max(np.abs(Hg - Ho))
    print(f"{which}: {len(kp)} k-points, nbf {nbf}, max|dH| = {err:.3e}, max|H| = {np.max(np.abs(Ho)):.3e}")
    assert err <= 1e-13 * np.max(np.abs(Ho))
    plan.destroy()


def test_kspace_rejects_bad_arguments():
    s = systems.molecule8()
    plan = hfx.Plan(s)
    K = torch.zeros(plan.nnz, dtype=torch.float64, device=DEV)
    H = torch.zeros((1, 40, 40, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(hfx.HfxError):
        plan.kspace(K, np.array([[np.nan, 0, 0]]), 0.25, H)
    plan.destroy()
