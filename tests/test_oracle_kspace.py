"""Pins of the oracle's k-space assembly of the exchange Hamiltonian
(Bloch sum of Eq. H-HFX with its -1/2, times the exact-exchange fraction):
one block's term and its phase; Hermiticity for a symmetric K; the
reciprocal-lattice relation H(k + b) = U^+ H(k) U, U = diag(exp(i b.r_mu));
band folding: the Gamma-point matrix of a 2x1x1 supercell has the
eigenvalues of the cell's H(0) and H(pi b_1) together."""
import numpy as np
import pytest

import oracle
import systems

ALPHA = 0.25  # HSE06


def _cell(seed=79):
    return systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, seed=seed)


def _pattern(s):
    o = oracle.Oracle(s)
    return o.blocks.astype(np.int64), o.offsets


def _sym_K(s, blocks):
    # a seeded K with K^G_{mu nu} = K^{-G}_{nu mu} (the density recipe has it)
    vals = systems.density_blocks(s, blocks)
    return np.concatenate([v.ravel() for v in vals])


def _rec(s):
    return 2 * np.pi * np.linalg.inv(np.asarray(s.lattice)).T  # rows b_i, b_i . a_j = 2 pi delta_ij


def test_one_block_term_and_its_phase():
    s = _cell()
    blocks, off = _pattern(s)
    b = int(np.flatnonzero((blocks[:, 0] != blocks[:, 1]) & np.any(blocks[:, 2:] != 0, axis=1))[0])
    I, J = int(blocks[b, 0]), int(blocks[b, 1])
    K = np.zeros(off[-1])
    K[off[b]] = 0.8  # element (0, 0) of block b
    k = np.array([[0.13, -0.27, 0.05]])
    H = oracle.kspace(s, blocks, off, K, k, ALPHA)
    nf = [systems.nfunc(int(l), s.spherical_d) for l in s.shell_l]
    fo = np.concatenate([[0], np.cumsum(nf)])
    xyz = np.asarray(s.atom_xyz)[np.asarray(s.shell_atom)]
    T = blocks[b, 2:] @ np.asarray(s.lattice)
    expect = -0.5 * ALPHA * 0.8 * np.exp(1j * k[0] @ (T + xyz[J] - xyz[I]))
    assert H[0, fo[I], fo[J]] == pytest.approx(expect, rel=1e-14)
    assert np.count_nonzero(H) == 1


def test_gamma_is_real_symmetric_sum_and_hermitian_elsewhere():
    s = _cell()
    blocks, off = _pattern(s)
    K = _sym_K(s, blocks)
    kp = np.array([[0.0, 0.0, 0.0], [0.21, 0.07, -0.33], [0.5, 0.5, 0.5]])
    H = oracle.kspace(s, blocks, off, K, kp, ALPHA)
    assert np.max(np.abs(H[0].imag)) == 0.0
    assert np.allclose(H[0].real, H[0].real.T, rtol=0, atol=1e-15)
    for h in H:
        assert np.allclose(h, h.conj().T, rtol=0, atol=1e-14)


def test_reciprocal_lattice_relation():
    s = _cell()
    blocks, off = _pattern(s)
    K = _sym_K(s, blocks)
    rec = _rec(s)
    k = np.array([0.11, -0.05, 0.19])
    nf = [systems.nfunc(int(l), s.spherical_d) for l in s.shell_l]
    r = np.repeat(np.asarray(s.atom_xyz)[np.asarray(s.shell_atom)], nf, axis=0)
    for j in range(3):
        H0 = oracle.kspace(s, blocks, off, K, k[None], ALPHA)[0]
        H1 = oracle.kspace(s, blocks, off, K, (k + rec[j])[None], ALPHA)[0]
        U = np.diag(np.exp(1j * (r @ rec[j])))
        assert np.allclose(H1, U.conj().T @ H0 @ U, rtol=0, atol=1e-13)
        # the relation is not the identity: the orbital positions enter
        assert np.max(np.abs(H1 - H0)) > 1e-3


def test_band_folding_of_a_supercell():
    s = _cell()
    sup = systems.diamond_cell(n=(2, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, seed=79)
    bs, os_ = _pattern(s)
    bb, ob = _pattern(sup)
    Ks = _sym_K(s, bs)
    # the supercell's K: the cell's block of the same pair of atoms at the
    # same separation (3 shells per atom, 8 atoms per conventional cell)
    skey = {tuple(int(v) for v in x): i for i, x in enumerate(bs)}

    def cellvec(shell):
        return np.array([(shell // 3) // 8, 0, 0])

    def small_shell(shell):
        return ((shell // 3) % 8) * 3 + shell % 3

    Kb = np.concatenate([
        Ks[os_[skey[(small_shell(I), small_shell(J), *map(int, cellvec(J) - cellvec(I) + np.array([n1, n2, n3]) * [2, 1, 1]))]]:
           os_[skey[(small_shell(I), small_shell(J), *map(int, cellvec(J) - cellvec(I) + np.array([n1, n2, n3]) * [2, 1, 1]))] + 1]]
        for (I, J, n1, n2, n3) in bb])
    Hs = oracle.kspace(sup, bb, ob, Kb, np.zeros((1, 3)), ALPHA)[0]
    rec = _rec(s)
    Hc = oracle.kspace(s, bs, os_, Ks, np.array([[0.0, 0.0, 0.0], 0.5 * rec[0]]), ALPHA)
    ev_sup = np.sort(np.linalg.eigvalsh(Hs))
    ev_cell = np.sort(np.concatenate([np.linalg.eigvalsh(Hc[0]), np.linalg.eigvalsh(Hc[1])]))
    assert np.allclose(ev_sup, ev_cell, rtol=0, atol=1e-12)
    # a wrong fold point does not reproduce them
    Hw = oracle.kspace(s, bs, os_, Ks, np.array([0.5 * rec[1]]), ALPHA)[0]
    ev_w = np.sort(np.concatenate([np.linalg.eigvalsh(Hc[0]), np.linalg.eigvalsh(Hw)]))
    assert np.max(np.abs(ev_sup - ev_w)) > 1e-6
