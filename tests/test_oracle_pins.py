"""Pins of the CPU oracle against mathematics it does not use itself.

Each test fixes something the paper's definitions (Background section:
full-range ERI, Eq. ERI-SR, the 8-fold permutation relations, Eq. schwarz,
Eq. H-HFX) or plain mathematics determine, computed by an independent route:
scipy special functions, closed forms, finite differences, brute-force
quadrature of the six-dimensional integral, exact index permutations.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
import systems
from tests.quadrature import cart_powers, overlap_1d, uquad_eri

RNG = np.random.default_rng(20240917)


# ----------------------------------------------------------------- Boys
@pytest.mark.parametrize("m", range(0, 9))
def test_boys_at_zero(m):
    assert oracle.boys(m, 0.0)[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)


@pytest.mark.parametrize("T", [1e-3, 0.05, 0.7, 3.3, 12.0, 29.5, 44.99, 45.01, 60.0, 250.0, 1e4])
def test_boys_vs_incomplete_gamma(T):
    F = oracle.boys(8, T)
    for m in range(9):
        ref = sp.gamma(m + 0.5) * sp.gammainc(m + 0.5, T) / (2.0 * T ** (m + 0.5))
        assert F[m] == pytest.approx(ref, rel=2e-14, abs=0)


@pytest.mark.parametrize("T", [1e-10, 1e-6, 0.01, 0.4, 2.0, 8.0])
def test_boys_vs_confluent_hypergeometric(T):
    F = oracle.boys(8, T)
    for m in range(9):
        ref = sp.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
        assert F[m] == pytest.approx(ref, rel=2e-14)


@pytest.mark.parametrize("T", [0.2, 1.0, 7.5, 40.0, 44.9, 45.1, 300.0])
def test_boys_f0_erf_closed_form(T):
    ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
    assert oracle.boys(0, T)[0] == pytest.approx(ref, rel=1e-15)


@pytest.mark.parametrize("T", [0.3, 4.0, 20.0, 50.0])
def test_boys_derivative_ladder(T):
    # dF_m/dT = -F_{m+1}, central difference with Richardson extrapolation
    h = 1e-3
    d1 = (oracle.boys(8, T + h) - oracle.boys(8, T - h)) / (2 * h)
    d2 = (oracle.boys(8, T + h / 2) - oracle.boys(8, T - h / 2)) / h
    d = (4 * d2 - d1) / 3
    F = oracle.boys(9, T)
    assert np.allclose(d, -F[1:10], rtol=1e-9, atol=0)


@pytest.mark.parametrize("T", [0.01, 1.0, 10.0, 44.0, 46.0, 100.0])
def test_boys_recursion_identities(T):
    F = oracle.boys(8, T)
    e = math.exp(-T)
    for m in range(8):
        assert F[m] == pytest.approx((2 * T * F[m + 1] + e) / (2 * m + 1), rel=1e-14)


# --------------------------------------------------------- normalisation
@pytest.mark.parametrize("l", [0, 1, 2])
def test_contracted_self_overlap_is_one(l):
    ex = np.exp(RNG.uniform(np.log(0.05), np.log(20), size=5))
    c = RNG.uniform(0.1, 1.0, size=5)
    cn = oracle.normalize(l, ex, c)
    S = 0.0
    for i, j in itertools.product(range(5), range(5)):
        p = ex[i] + ex[j]
        S += cn[i] * cn[j] * overlap_1d(2 * l, p) * overlap_1d(0, p) ** 2
    assert S == pytest.approx(1.0, rel=1e-13)


def test_spherical_d_orthonormal():
    # same-centre overlap of the x^l-normalised Cartesian d components
    pw = cart_powers(2)
    ex = np.array([0.8, 2.5])
    cn = oracle.normalize(2, ex, np.array([0.6, 0.4]))
    S = np.zeros((6, 6))
    for a, b in itertools.product(range(6), range(6)):
        for i, j in itertools.product(range(2), range(2)):
            p = ex[i] + ex[j]
            v = cn[i] * cn[j]
            for k in range(3):
                v *= overlap_1d(pw[a][k] + pw[b][k], p)
            S[a, b] += v
    T = oracle.sph_matrix(2, True)
    assert T.shape == (5, 6)
    assert np.allclose(T @ S @ T.T, np.eye(5), atol=1e-13)
    assert S[0, 0] == pytest.approx(1.0, rel=1e-13)  # xx normalised
    assert S[1, 1] == pytest.approx(1.0 / 3.0, rel=1e-13)  # xy at x^2 normalisation


# ----------------------------------------------------------- closed forms
def _prim(xyz, l, a):
    return (np.asarray(xyz, dtype=float), l, [a], [1.0])


def _ss_closed(A, B, C, D, a, b, c, d, op="coulomb", omega=0.0):
    p, q = a + b, c + d
    P = (a * A + b * B) / p
    Q = (c * C + d * D) / q
    rho = p * q / (p + q)
    R = np.linalg.norm(P - Q)
    kab = math.exp(-a * b / p * np.sum((A - B) ** 2))
    kcd = math.exp(-c * d / q * np.sum((C - D) ** 2))
    pref = math.pi ** 3 * (p * q) ** -1.5 * kab * kcd

    def pot(r, g):  # erf(sqrt(g) r) / r with its r -> 0 limit
        return 2 * math.sqrt(g / math.pi) if r == 0 else math.erf(math.sqrt(g) * r) / r

    if op == "coulomb":
        return pref * pot(R, rho)
    s = omega * omega / (omega * omega + rho)
    if op == "erf":
        return pref * pot(R, rho * s)
    return pref * (pot(R, rho) - pot(R, rho * s))


@pytest.mark.parametrize("op", ["coulomb", "erfc", "erf"])
@pytest.mark.parametrize("trial", range(4))
def test_ssss_closed_form(op, trial):
    A, B, C, D = RNG.uniform(-3, 3, size=(4, 3))
    if trial == 3:
        C, D = A.copy(), B.copy()  # P == Q: R -> 0 limit
    a, b, c, d = np.exp(RNG.uniform(np.log(0.05), np.log(20), size=4))
    if trial == 3:
        c, d = a, b
    v = oracle.eri([_prim(A, 0, a), _prim(B, 0, b), _prim(C, 0, c), _prim(D, 0, d)], op, 0.11)
    assert v[0, 0, 0, 0] == pytest.approx(_ss_closed(A, B, C, D, a, b, c, d, op, 0.11), rel=1e-13)


def _richardson_d1(f, x, h):
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + h / 2) - f(x - h / 2)) / h
    return (4 * d2 - d1) / 3


def _richardson_d2(f, x, h):
    def c(hh):
        return (f(x + hh) - 2 * f(x) + f(x - hh)) / (hh * hh)
    return (4 * c(h / 2) - c(h)) / 3


def test_p_and_d_from_ssss_by_differentiation():
    # x_A exp(-a r_A^2) = (1/2a) d/dA_x exp(-a r_A^2); d_xx adds the 1/2a term
    A, B, C, D = RNG.uniform(-2, 2, size=(4, 3))
    a, b, c, d = 0.9, 0.35, 1.7, 0.6

    def ss(Ax=None, Ay=None):
        AA = A.copy()
        if Ax is not None:
            AA[0] = Ax
        if Ay is not None:
            AA[1] = Ay
        return _ss_closed(AA, B, C, D, a, b, c, d)

    p = oracle.eri([_prim(A, 1, a), _prim(B, 0, b), _prim(C, 0, c), _prim(D, 0, d)])[:, 0, 0, 0]
    fx = _richardson_d1(lambda x: ss(Ax=x), A[0], 1e-3) / (2 * a)
    assert p[0] == pytest.approx(fx, rel=1e-9)
    dd = oracle.eri([_prim(A, 2, a), _prim(B, 0, b), _prim(C, 0, c), _prim(D, 0, d)])[:, 0, 0, 0]
    fxx = _richardson_d2(lambda x: ss(Ax=x), A[0], 2e-3) / (2 * a) ** 2 + ss() / (2 * a)
    assert dd[0] == pytest.approx(fxx, rel=1e-7)
    # mixed derivative for d_xy
    h = 1e-3

    def mixed(hh):
        return (ss(A[0] + hh, A[1] + hh) - ss(A[0] + hh, A[1] - hh) - ss(A[0] - hh, A[1] + hh)
                + ss(A[0] - hh, A[1] - hh)) / (4 * hh * hh)
    fxy = (4 * mixed(h / 2) - mixed(h)) / 3 / (2 * a) ** 2
    assert dd[1] == pytest.approx(fxy, rel=1e-7)


# ---------------------------------------------------- brute-force quadrature
_UQ_CASES = [((1, 0, 2, 1), "coulomb"), ((2, 2, 0, 0), "coulomb"), ((1, 1, 1, 1), "erfc"),
             ((2, 1, 2, 0), "erfc"), ((2, 2, 2, 2), "coulomb"), ((0, 2, 1, 2), "erfc")]


@pytest.mark.parametrize("ls,op", _UQ_CASES)
def test_quartet_vs_u_quadrature(ls, op):
    rng = np.random.default_rng(hash(ls) % 1000 + len(op))
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(np.log(0.1), np.log(5), size=4))
    v = oracle.eri([_prim(cen[k], ls[k], ex[k]) for k in range(4)], op, 0.11)
    pws = [cart_powers(l) for l in ls]
    # a few components (each is a full six-dimensional quadrature)
    comps = [tuple(rng.integers(0, len(p)) for p in pws) for _ in range(3)]
    for (i, j, k, l) in comps:
        ref = uquad_eri(cen[0], cen[1], cen[2], cen[3], *ex, pws[0][i], pws[1][j], pws[2][k],
                        pws[3][l], u0=0.11 if op == "erfc" else 0.0)
        assert v[i, j, k, l] == pytest.approx(ref, rel=1e-11, abs=1e-15)


# ------------------------------------------------------------ invariances
def _rand_shell(rng, l, K=3):
    return (rng.uniform(-2, 2, size=3), l, np.exp(rng.uniform(np.log(0.1), np.log(10), size=K)),
            rng.uniform(0.1, 1, size=K))


@pytest.mark.parametrize("ls", [(0, 1, 2, 1), (2, 2, 1, 0), (1, 1, 2, 2)])
@pytest.mark.parametrize("op", ["coulomb", "erfc"])
def test_eightfold_permutation_symmetry(ls, op):
    rng = np.random.default_rng(sum(ls) * 7 + len(op))
    sh = [_rand_shell(rng, l) for l in ls]
    v = oracle.eri(sh, op, 0.11)
    a, b, c, d = sh
    assert np.allclose(oracle.eri([b, a, c, d], op, 0.11), v.transpose(1, 0, 2, 3), rtol=1e-12, atol=1e-16)
    assert np.allclose(oracle.eri([a, b, d, c], op, 0.11), v.transpose(0, 1, 3, 2), rtol=1e-12, atol=1e-16)
    assert np.allclose(oracle.eri([c, d, a, b], op, 0.11), v.transpose(2, 3, 0, 1), rtol=1e-12, atol=1e-16)
    assert np.allclose(oracle.eri([d, c, b, a], op, 0.11), v.transpose(3, 2, 1, 0), rtol=1e-12, atol=1e-16)


def test_translation_invariance():
    rng = np.random.default_rng(5)
    sh = [_rand_shell(rng, l) for l in (2, 1, 1, 2)]
    shift = np.array([3.1, -7.2, 0.4])
    moved = [(s[0] + shift,) + s[1:] for s in sh]
    for op in ("coulomb", "erfc"):
        assert np.allclose(oracle.eri(sh, op, 0.11), oracle.eri(moved, op, 0.11), rtol=1e-11, atol=1e-15)


def test_translational_sum_rule():
    # sum over centres of d/dX (ss|ss) = 0  =>  sum_X 2 alpha_X (p_X ...) = 0
    rng = np.random.default_rng(11)
    cen = rng.uniform(-2, 2, size=(4, 3))
    ex = [0.7, 1.9, 0.3, 4.0]
    tot = np.zeros(3)
    for k in range(4):
        ls = [0, 0, 0, 0]
        ls[k] = 1
        v = oracle.eri([_prim(cen[i], ls[i], ex[i]) for i in range(4)]).reshape(-1)
        tot += 2 * ex[k] * v
    ref = oracle.eri([_prim(cen[i], 0, ex[i]) for i in range(4)]).reshape(-1)[0]
    assert np.all(np.abs(tot) <= 1e-13 * max(abs(ref), 1e-30) * 100)


def test_operator_decomposition_and_limits():
    rng = np.random.default_rng(3)
    sh = [_rand_shell(rng, l) for l in (1, 2, 0, 1)]
    c = oracle.eri(sh, "coulomb")
    assert np.allclose(oracle.eri(sh, "erf", 0.11) + oracle.eri(sh, "erfc", 0.11), c, rtol=1e-12, atol=1e-16)
    # the erf part is O(omega): 2 omega / sqrt(pi) times the two overlaps
    assert np.allclose(oracle.eri(sh, "erfc", 1e-10), c, rtol=1e-8, atol=1e-14)
    assert np.max(np.abs(oracle.eri(sh, "erfc", 1e4))) < 1e-6 * np.max(np.abs(c))


@pytest.mark.parametrize("op", ["coulomb", "erfc"])
def test_schwarz_inequality(op):
    rng = np.random.default_rng(17 + len(op))
    for _ in range(3):
        ls = rng.integers(0, 3, size=4)
        sh = [_rand_shell(rng, int(l)) for l in ls]
        v = oracle.eri(sh, op, 0.11)
        ab = oracle.eri([sh[0], sh[1], sh[0], sh[1]], op, 0.11)
        cd = oracle.eri([sh[2], sh[3], sh[2], sh[3]], op, 0.11)
        na, nb, nc, nd = v.shape
        dab = np.array([[ab[i, j, i, j] for j in range(nb)] for i in range(na)])
        dcd = np.array([[cd[k, l, k, l] for l in range(nd)] for k in range(nc)])
        bound = np.sqrt(np.einsum("ij,kl->ijkl", dab, dcd))
        assert np.all(np.abs(v) <= bound * (1 + 1e-12))
