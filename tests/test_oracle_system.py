"""System-level pins of the oracle's exchange build (Eq. H-HFX without -1/2).

K symmetry, positivity of Tr(DK) (the kernels 1/r and erfc(omega r)/r are
positive definite), linearity in D, the screening error bound, and the
periodic / explicit-cluster equivalence that defines the lattice sums.
"""
import numpy as np
import pytest

import oracle
import systems


def _block_map(o):
    return {tuple(int(v) for v in b): i for i, b in enumerate(o.blocks)}


def _blk(o, K, i):
    return K[o.offsets[i]:o.offsets[i + 1]].reshape(
        systems.nfunc(int(o.system.shell_l[o.blocks[i, 0]]), o.system.spherical_d),
        systems.nfunc(int(o.system.shell_l[o.blocks[i, 1]]), o.system.spherical_d))


@pytest.fixture(scope="module")
def c1():
    s = systems.molecule8()
    o = oracle.Oracle(s)
    o.schwarz()
    D = o.density_from_system()
    o.set_density(D)
    K, n = o.build_K()
    Ku, nu = o.build_K(screened=False)
    return s, o, D, K, Ku, n, nu


@pytest.fixture(scope="module")
def tiny_cell():
    s = systems.diamond_cell(seed=77, n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6)
    o = oracle.Oracle(s)
    o.schwarz()
    D = o.density_from_system()
    o.set_density(D)
    Ku, _ = o.build_K(screened=False)
    K, _ = o.build_K()
    return s, o, D, K, Ku


def test_pattern_is_symmetric_and_complete(tiny_cell):
    s, o, *_ = tiny_cell
    keys = _block_map(o)
    for (I, J, a, b, c) in keys:
        assert (J, I, -a, -b, -c) in keys
    # every pair within the cutoff is present, nothing beyond it
    xyz, lat = s.atom_xyz, s.lattice
    for (I, J, a, b, c) in keys:
        r = xyz[s.shell_atom[I]] - xyz[s.shell_atom[J]] - np.array([a, b, c]) @ lat
        assert np.linalg.norm(r) <= s.pair_cutoff
    n_expected = 0
    for I in range(s.n_shells):
        for J in range(s.n_shells):
            for n in np.ndindex(7, 7, 7):
                nn = np.array(n) - 3
                r = xyz[s.shell_atom[I]] - xyz[s.shell_atom[J]] - nn @ lat
                n_expected += np.linalg.norm(r) <= s.pair_cutoff
    assert n_expected == len(keys)


def test_K_symmetric_molecule(c1):
    s, o, D, K, Ku, *_ = c1
    keys = _block_map(o)
    for (I, J, a, b, c), i in keys.items():
        j = keys[(J, I, 0, 0, 0)]
        assert np.allclose(_blk(o, K, i), _blk(o, K, j).T, rtol=0, atol=1e-13)


def test_K_symmetric_periodic(tiny_cell):
    s, o, D, K, Ku = tiny_cell
    keys = _block_map(o)
    for (I, J, a, b, c), i in keys.items():
        j = keys[(J, I, -a, -b, -c)]
        assert np.allclose(_blk(o, Ku, i), _blk(o, Ku, j).T, rtol=0, atol=1e-13)


def test_trace_DK_positive(c1, tiny_cell):
    for (o, D, Ku) in ((c1[1], c1[2], c1[4]), (tiny_cell[1], tiny_cell[2], tiny_cell[4])):
        # sum_{mu nu} D_{mu nu} K_{mu nu} = int int rho(r,r')^2 v(r - r') > 0
        assert float(np.dot(D, Ku)) > 0.0


def test_linear_in_density(c1):
    s, o, D, K, Ku, *_ = c1
    D2 = o.density_from_system(iteration=3) * 0.5 - D * 0.25
    o.set_density(D2)
    K2, _ = o.build_K(screened=False)
    o.set_density(1.5 * D - 2.0 * D2)
    K3, _ = o.build_K(screened=False)
    o.set_density(D)
    assert np.allclose(K3, 1.5 * Ku - 2.0 * K2, rtol=0, atol=1e-12)


def test_screening_error_bound(c1):
    s, o, D, K, Ku, n, nu = c1
    dropped = nu - n
    assert 0 < dropped
    # each dropped quartet moves one K element by at most nb*nd*tau (<= 9 tau here)
    assert np.max(np.abs(K - Ku)) <= dropped * 9 * s.tau
    # and the bound is not vacuous: screening does change K above rounding
    assert np.max(np.abs(K - Ku)) > 1e-14


def test_periodic_equals_explicit_cluster(tiny_cell):
    """Lattice sums of Eq. H-HFX equal a molecule made of the needed images."""
    s, o, D, K, Ku = tiny_cell
    rc = s.pair_cutoff
    xyz, lat = s.atom_xyz, s.lattice
    atoms = []  # (home atom, image)
    for a in range(s.n_atoms):
        atoms.append((a, (0, 0, 0)))
    for n in np.ndindex(5, 5, 5):
        nn = tuple(int(v) - 2 for v in n)
        if nn == (0, 0, 0):
            continue
        for a in range(s.n_atoms):
            p = xyz[a] + np.array(nn) @ lat
            if np.min(np.linalg.norm(xyz - p, axis=1)) <= 2 * rc + 1e-9:
                atoms.append((a, nn))
    cxyz = np.array([xyz[a] + np.array(n) @ lat for a, n in atoms])
    # same shells on each atom image
    per_atom = {}
    for I in range(s.n_shells):
        per_atom.setdefault(int(s.shell_atom[I]), []).append(I)
    po = s.shell_prim_offset()
    sh_atom, sh_l, sh_np, pe, pc, origin = [], [], [], [], [], []
    for ia, (a, n) in enumerate(atoms):
        for I in per_atom[a]:
            sh_atom.append(ia)
            sh_l.append(int(s.shell_l[I]))
            sh_np.append(int(s.shell_nprim[I]))
            pe.append(s.prim_exp[po[I]:po[I] + s.shell_nprim[I]])
            pc.append(s.prim_coef[po[I]:po[I] + s.shell_nprim[I]])
            origin.append((I, n))
    cl = systems.System(name="cluster", seed=s.seed, atom_xyz=cxyz,
                        shell_atom=np.array(sh_atom, dtype=np.int32),
                        shell_l=np.array(sh_l, dtype=np.int32),
                        shell_nprim=np.array(sh_np, dtype=np.int32),
                        prim_exp=np.concatenate(pe), prim_coef=np.concatenate(pc),
                        lattice=None, pair_cutoff=rc, op=s.op, omega=s.omega, tau=s.tau,
                        spherical_d=s.spherical_d, d_decay=s.d_decay)
    oc = oracle.Oracle(cl)
    # cluster D = periodic D of the translated block
    mapped = np.array([[origin[I][0], origin[J][0]] + list(np.subtract(origin[J][1], origin[I][1]))
                       for (I, J) in oc.blocks[:, :2]], dtype=np.int64)
    vals = systems.density_blocks(s, mapped)
    oc.set_density(np.concatenate([v.ravel() for v in vals]))
    n_home = s.n_shells
    req = np.nonzero(oc.blocks[:, 0] < n_home)[0]
    Kc, _ = oc.build_K(blocks=req, screened=False)
    keys = _block_map(o)
    checked = 0
    for i in req:
        I, J = int(oc.blocks[i, 0]), int(oc.blocks[i, 1])
        hj, nj = origin[J]
        kp = keys[(I, hj) + tuple(nj)]
        assert np.allclose(_blk(oc, Kc, i), _blk(o, Ku, kp), rtol=0, atol=1e-12)
        checked += 1
    assert checked == len(o.blocks)


def test_K_from_orbits_equals_plain_loop():
    """The oracle's K from a given quartet set, fed every member of every
    kept orbit, reproduces the plain screened loop (pins K_from_quartets for
    the sampled full-size parity test)."""
    from tests.helpers import canonical_keys, oracle_quartet_instances, orbit_members
    for s in (systems.molecule8(seed=321),
              systems.diamond_cell(seed=322, n=(1, 1, 1), nprim=1, shells=(0, 1), r_cut=4.0)):
        o = oracle.Oracle(s)
        o.schwarz()
        o.set_density(o.density_from_system())
        Kref, _ = o.build_K()
        rows, _ = o.quartets(gR=2)
        keys = canonical_keys(oracle_quartet_instances(rows))
        _, first = np.unique(keys, axis=0, return_index=True)
        members = orbit_members(rows[np.sort(first)])
        assert len(members) == len(rows), "orbits of the kept quartets are exactly the kept quartets"
        K, used = o.K_from_quartets(members)
        assert np.max(np.abs(K - Kref)) <= 1e-12 * max(1.0, np.max(np.abs(Kref)))
