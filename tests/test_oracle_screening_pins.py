"""Pins of the oracle's screening inputs: the Schwarz factors of Eq. schwarz
and the Cartesian density with its block maxima of Eq. dmscreening.

* Q_IJ = sqrt(max_{i in I, j in J} |(ij|ij)|) of every pattern block is
  recomputed without the oracle's integral code: contracted s-s pairs from
  the closed form of (ss|ss) at coincident centres of charge, p and d pairs
  from brute-force u-quadrature of each diagonal component, summed over the
  primitives.
* D_cart = T^T D T: the density function sum_mn D_mn phi_m(x) phi_n(y) of a
  block, with the spherical d functions built from scipy's spherical
  harmonics (real solid harmonics r^2 Y_2m scaled to the norm of the x^2
  component), equals sum_ac D_cart,ac x^a y^c at random points.
* P_max of a block is the largest |D_cart| of it, shared with its transpose
  block; a density with one nonzero element (and its mirror) gives exactly
  that magnitude on those two blocks and zero elsewhere.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import systems
from tests.quadrature import cart_powers, overlap_1d, uquad_eri, uquad_eri_fast

OMEGA = 0.11


def _tiny_system(periodic: bool, op: str, spherical_d: bool = True, nprim: int = 2, seed: int = 5):
    """Two atoms with shells s, p, d (nprim primitives each); periodic: a
    small cubic cell whose pair cutoff reaches a few images."""
    rng = np.random.default_rng(seed)
    xyz = np.array([[0.3, -0.2, 0.1], [1.4, 0.9, -0.6]])
    shell_atom = np.array([0, 0, 0, 1, 1, 1], dtype=np.int32)
    shell_l = np.array([0, 1, 2, 0, 1, 2], dtype=np.int32)
    shell_nprim = np.full(6, nprim, dtype=np.int32)
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), size=6 * nprim))
    co = rng.uniform(0.1, 1.0, size=6 * nprim)
    kw = dict(name="tiny_spd", seed=seed, atom_xyz=xyz, shell_atom=shell_atom, shell_l=shell_l,
              shell_nprim=shell_nprim, prim_exp=ex, prim_coef=co, op=op, omega=OMEGA if op == "erfc" else 0.0,
              spherical_d=spherical_d)
    if periodic:
        kw.update(lattice=np.diag([4.2, 4.6, 5.0]), pair_cutoff=5.0)
    return systems.System(**kw)


def _shell_data(s, I, img):
    off = int(np.sum(s.shell_nprim[:I]))
    n = int(s.shell_nprim[I])
    ex = s.prim_exp[off:off + n]
    cn = oracle.normalize(int(s.shell_l[I]), ex, s.prim_coef[off:off + n])
    R = np.array(s.atom_xyz[s.shell_atom[I]], dtype=float)
    if s.lattice is not None:
        R = R + np.asarray(img, dtype=float) @ np.asarray(s.lattice, dtype=float)
    return R, int(s.shell_l[I]), ex, cn


def _ss_pair(a, b, c, d, A, B, op):
    """(ss|ss) of unit-coefficient primitives a at A, b at B | c at A, d at B
    in closed form: pi^3 (pq)^-3/2 K_AB K_CD erf(sqrt(g) R)/R with g = rho
    (Coulomb), minus the same with g = rho s, s = omega^2/(omega^2 + rho)
    (erfc); R = |P - Q|, and 2 sqrt(g/pi) at R = 0."""
    p, q = a + b, c + d
    rho = p * q / (p + q)
    AB2 = float(np.sum((A - B) ** 2))
    P = (a * A + b * B) / p
    Q = (c * A + d * B) / q
    R = float(np.linalg.norm(P - Q))
    pref = math.pi ** 3 * (p * q) ** -1.5 * math.exp(-a * b / p * AB2) * math.exp(-c * d / q * AB2)

    def pot(gam):
        return 2.0 * math.sqrt(gam / math.pi) if R == 0.0 else math.erf(math.sqrt(gam) * R) / R

    g = pot(rho)
    if op == "erfc":
        g -= pot(rho * OMEGA * OMEGA / (OMEGA * OMEGA + rho))
    return pref * g


def _q_independent(s, I, J, img):
    """sqrt(max over diagonal components of (ij|ij)), by closed form (s-s) or
    u-quadrature (anything else), summed over primitives."""
    A, la, exa, ca = _shell_data(s, I, (0, 0, 0))
    B, lb, exb, cb = _shell_data(s, J, img)
    if la == 0 and lb == 0:
        v = 0.0
        for (i, j, k, l) in itertools.product(range(len(exa)), range(len(exb)), range(len(exa)), range(len(exb))):
            v += ca[i] * cb[j] * ca[k] * cb[l] * _ss_pair(exa[i], exb[j], exa[k], exb[l], A, B, s.op)
        return math.sqrt(abs(v))
    best = 0.0
    u0 = OMEGA if s.op == "erfc" else 0.0
    for pa in cart_powers(la):
        for pb in cart_powers(lb):
            v = 0.0
            for (i, j, k, l) in itertools.product(range(len(exa)), range(len(exb)), range(len(exa)),
                                                  range(len(exb))):
                v += ca[i] * cb[j] * ca[k] * cb[l] * uquad_eri_fast(A, B, A, B, exa[i], exb[j], exa[k], exb[l],
                                                                    pa, pb, pa, pb, u0=u0)
            best = max(best, abs(v))
    return math.sqrt(best)


def test_fast_quadrature_equals_reference_quadrature():
    rng = np.random.default_rng(4)
    for ls in [(0, 0, 0, 0), (1, 2, 1, 0), (2, 2, 2, 2)]:
        cen = rng.uniform(-1.5, 1.5, size=(4, 3))
        ex = np.exp(rng.uniform(np.log(0.1), np.log(5), size=4))
        pw = [cart_powers(l)[-1] for l in ls]
        for u0 in (0.0, OMEGA):
            ref = uquad_eri(*cen, *ex, *pw, u0=u0)
            assert uquad_eri_fast(*cen, *ex, *pw, u0=u0) == pytest.approx(ref, rel=1e-12, abs=1e-300)


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("op", ["coulomb", "erfc"])
def test_schwarz_factors_against_independent_integrals(periodic, op):
    s = _tiny_system(periodic, op)
    o = oracle.Oracle(s)
    Q = o.schwarz()
    blocks = o.blocks.astype(np.int64)
    key = {tuple(b): i for i, b in enumerate(blocks)}
    canon = [i for i, b in enumerate(blocks)
             if b[0] < b[1] or (b[0] == b[1] and tuple(b[2:5]) >= (0, 0, 0))]
    if periodic:
        # every canonical block would take minutes of quadrature: all s-s
        # blocks, and every other block class once per image distance shell
        seen = set()
        pick = []
        for i in canon:
            I, J = int(blocks[i, 0]), int(blocks[i, 1])
            cls = (int(s.shell_l[I]), int(s.shell_l[J]), int(np.sum(np.abs(blocks[i, 2:5]))))
            if (s.shell_l[I] == 0 and s.shell_l[J] == 0) or cls not in seen:
                seen.add(cls)
                pick.append(i)
        canon = pick
    assert len(canon) >= 10
    for i in canon:
        I, J = int(blocks[i, 0]), int(blocks[i, 1])
        img = tuple(int(x) for x in blocks[i, 2:5])
        ref = _q_independent(s, I, J, img)
        assert Q[i] == pytest.approx(ref, rel=1e-11, abs=1e-300), (I, J, img)
        # a pair and its transpose share the factor
        j = key[(J, I, -img[0], -img[1], -img[2])]
        assert Q[j] == Q[i]


def test_schwarz_contracted_ss_pairs_of_the_molecule_workload():
    # every s-s block of the 8-atom workload (3 primitives per shell)
    s = systems.molecule8()
    o = oracle.Oracle(s)
    Q = o.schwarz()
    ls = s.shell_l
    n = 0
    for i, b in enumerate(o.blocks):
        I, J = int(b[0]), int(b[1])
        if ls[I] == 0 and ls[J] == 0 and I <= J:
            assert Q[i] == pytest.approx(_q_independent(s, I, J, (0, 0, 0)), rel=1e-12)
            n += 1
    assert n == 16 * 17 // 2


# -------------------------------------------------------------- density
def _real_solid_harmonic_d(x):
    """The five real solid harmonics of degree 2, m = -2..2, at points x
    (n, 3), from scipy's complex spherical harmonics, each scaled to the norm
    of the x^2 component (same radial factor)."""
    r = np.linalg.norm(x, axis=1)
    pol = np.arccos(np.clip(x[:, 2] / r, -1.0, 1.0))
    azi = np.arctan2(x[:, 1], x[:, 0])
    out = np.zeros((len(x), 5))
    for k, m in enumerate(range(-2, 3)):
        if m < 0:
            y = math.sqrt(2.0) * (-1) ** m * sp.sph_harm_y(2, -m, pol, azi).imag
        elif m == 0:
            y = sp.sph_harm_y(2, 0, pol, azi).real
        else:
            y = math.sqrt(2.0) * (-1) ** m * sp.sph_harm_y(2, m, pol, azi).real
        out[:, k] = r * r * y
    # norm with radial factor exp(-beta r^2): int r^6 e^{-beta r^2} dr (unit Y)
    # against int x^4 e^{-beta r^2} d^3r; beta cancels in the ratio (beta = 1)
    n_sph = sp.gamma(3.5) / 2.0
    n_cart = overlap_1d(4, 1.0) * overlap_1d(0, 1.0) ** 2
    return out * math.sqrt(n_cart / n_sph)


def _boundary_functions(l, spherical, x):
    if l == 2 and spherical:
        return _real_solid_harmonic_d(x)
    return _cart_monomials(l, x)


def _cart_monomials(l, x):
    return np.stack([x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for (a, b, c) in cart_powers(l)], axis=1)


def _sym_density(o, rng):
    """A random density on the oracle's pattern with D^n_ij = D^-n_ji."""
    blocks = o.blocks.astype(np.int64)
    key = {tuple(b): i for i, b in enumerate(blocks)}
    nf = [o.offsets[i + 1] - o.offsets[i] for i in range(len(blocks))]
    d = np.zeros(o.nnz)
    for i, b in enumerate(blocks):
        j = key[(b[1], b[0], -b[2], -b[3], -b[4])]
        if j < i:
            continue
        ni = len(_boundary_functions(int(o.system.shell_l[b[0]]), o.system.spherical_d, np.ones((1, 3)))[0])
        nj = nf[i] // ni
        v = rng.uniform(-1, 1, size=(ni, nj))
        if j == i:  # (I, I, 0): symmetric itself
            v = 0.5 * (v + v.T)
        d[o.offsets[i]:o.offsets[i + 1]] = v.ravel()
        d[o.offsets[j]:o.offsets[j + 1]] = v.T.ravel()
    return d


@pytest.mark.parametrize("spherical", [True, False])
def test_density_cart_reproduces_the_density_function(spherical):
    s = _tiny_system(True, "erfc", spherical_d=spherical)
    o = oracle.Oracle(s)
    rng = np.random.default_rng(21)
    d = _sym_density(o, rng)
    pmax = o.set_density(d)
    coff, dc = o.density_cart()
    x = rng.normal(size=(7, 3))
    y = rng.normal(size=(7, 3))
    for i, b in enumerate(o.blocks):
        li, lj = int(s.shell_l[b[0]]), int(s.shell_l[b[1]])
        fi, fj = _boundary_functions(li, spherical, x), _boundary_functions(lj, spherical, y)
        D = d[o.offsets[i]:o.offsets[i + 1]].reshape(fi.shape[1], fj.shape[1])
        ci, cj = _cart_monomials(li, x), _cart_monomials(lj, y)
        Dc = dc[coff[i]:coff[i + 1]].reshape(ci.shape[1], cj.shape[1])
        lhs = np.einsum("pm,mn,pn->p", fi, D, fj)
        rhs = np.einsum("pa,ac,pc->p", ci, Dc, cj)
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-13 * np.max(np.abs(lhs)))
        assert pmax[i] == np.max(np.abs(Dc))


def test_density_cart_of_one_spherical_d_element():
    # D has one unit element between the m = 0 function z^2 - (x^2 + y^2)/2
    # of a d shell and an s shell: its Cartesian block is that function's
    # expansion in xx, xy, xz, yy, yz, zz
    s = _tiny_system(False, "coulomb", spherical_d=True)
    o = oracle.Oracle(s)
    blocks = o.blocks.astype(np.int64)
    key = {tuple(b): i for i, b in enumerate(blocks)}
    i = key[(2, 3, 0, 0, 0)]  # (d on atom 0, s on atom 1)
    j = key[(3, 2, 0, 0, 0)]
    d = np.zeros(o.nnz)
    d[o.offsets[i] + 2] = 1.0  # row m = 0 of a 5 x 1 block
    d[o.offsets[j] + 2] = 1.0
    pmax = o.set_density(d)
    coff, dc = o.density_cart()
    assert np.allclose(dc[coff[i]:coff[i + 1]], [-0.5, 0, 0, -0.5, 0, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(dc[coff[j]:coff[j + 1]], [-0.5, 0, 0, -0.5, 0, 1.0], rtol=0, atol=1e-15)
    assert pmax[i] == 1.0 and pmax[j] == 1.0
    assert np.count_nonzero(pmax) == 2


@pytest.mark.parametrize("periodic", [False, True])
def test_pmax_of_one_element_is_its_magnitude_on_its_two_blocks(periodic):
    # Cartesian d (no transform): one element and its mirror
    s = _tiny_system(periodic, "erfc", spherical_d=False)
    o = oracle.Oracle(s)
    blocks = o.blocks.astype(np.int64)
    key = {tuple(b): i for i, b in enumerate(blocks)}
    rng = np.random.default_rng(8)
    for trial in range(6):
        i = int(rng.integers(len(blocks)))
        b = blocks[i]
        j = key[(b[1], b[0], -b[2], -b[3], -b[4])]
        ni = len(cart_powers(int(s.shell_l[b[0]])))
        nj = len(cart_powers(int(s.shell_l[b[1]])))
        r, c = int(rng.integers(ni)), int(rng.integers(nj))
        v = -float(rng.uniform(0.2, 3.0))
        d = np.zeros(o.nnz)
        d[o.offsets[i] + r * nj + c] = v
        d[o.offsets[j] + c * ni + r] = v
        pmax = o.set_density(d)
        expect = np.zeros(len(blocks))
        expect[i] = expect[j] = abs(v)
        assert np.array_equal(pmax, expect), (trial, i, j)


def test_schwarz_of_chosen_rows_equals_the_full_table():
    # the row-restricted Schwarz step (for K blocks of chosen rows) agrees
    # with the pinned full table on those rows' blocks
    s = _tiny_system(True, "erfc")
    full = oracle.Oracle(s)
    Q = full.schwarz()
    part = oracle.Oracle(s)
    rows = [1, 4]
    q = part.schwarz_rows(rows)
    for i, b in enumerate(part.blocks):
        if int(b[0]) in rows:
            assert q[i] == pytest.approx(Q[i], rel=1e-13)
        else:
            assert q[i] == 0.0
