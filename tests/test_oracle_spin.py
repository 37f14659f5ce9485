"""Pins of the oracle's collinear-spin build (Eq. H-HFX per spin density,
one screening predicate whose block maxima are the larger of the two
spins'): equal spins give the unpolarised K; a zero beta density gives the
unpolarised K of alpha and a zero K of beta; swapping the densities swaps
the results; without screening each spin's K is the plain sum of its own
density."""
import numpy as np
import pytest

import oracle
import systems


def _dens(system, blocks, seed_shift=0):
    s = system.with_(seed=system.seed + seed_shift) if seed_shift else system
    vals = systems.density_blocks(s, np.asarray(blocks, dtype=np.int64))
    return np.concatenate([v.ravel() for v in vals])


@pytest.fixture(scope="module")
def cell():
    s = systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, seed=77)
    o = oracle.Oracle(s)
    o.schwarz()
    return s, o


def test_equal_spins_give_the_unpolarised_K(cell):
    s, o = cell
    D = _dens(s, o.blocks)
    ka, kb = o.build_K_spin(D, D)
    o.set_density(D)
    k, _ = o.build_K()
    assert np.array_equal(ka, k) and np.array_equal(kb, k)


def test_zero_beta_and_swap(cell):
    s, o = cell
    Da = _dens(s, o.blocks)
    Db = 0.4 * _dens(s, o.blocks, seed_shift=17)
    ka, kb = o.build_K_spin(Da, np.zeros_like(Da))
    o.set_density(Da)
    k, _ = o.build_K()
    assert np.array_equal(ka, k)
    assert not np.any(kb)
    xa, xb = o.build_K_spin(Da, Db)
    ya, yb = o.build_K_spin(Db, Da)
    assert np.array_equal(xa, yb) and np.array_equal(xb, ya)
    # the shared predicate keeps at least what each spin's own keeps
    assert not np.array_equal(xa, xb)


def test_unscreened_spin_K_is_each_densitys_plain_sum():
    s = systems.molecule8().with_(tau=0.0)
    o = oracle.Oracle(s)
    o.schwarz()
    Da = _dens(s, o.blocks)
    Db = -0.7 * _dens(s, o.blocks, seed_shift=5)
    ka, kb = o.build_K_spin(Da, Db)
    for D, k in ((Da, ka), (Db, kb)):
        o.set_density(D)
        ref, _ = o.build_K(screened=False)
        assert np.allclose(k, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
