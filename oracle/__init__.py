"""CPU oracle for the screened exchange build.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2009_03555_amd``)
never does, and this package never imports the product: the two share only
the seeded input generators in ``systems``.

The numerics live in ``hfx_oracle.c`` (plain FP64 C, long-double Boys
function, McMurchie-Davidson integrals, plain ordered-quartet loop); this
module is a ctypes wrapper.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hfx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OP = {"coulomb": 0, "erfc": 1, "erf": 2}


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.oracle_op_ladder.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_double, dp]
        L.oracle_normalize.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.oracle_eri_raw.argtypes = [dp, ip, ip, dp, dp, ctypes.c_int, ctypes.c_double, dp]
        L.oracle_sph_matrix.argtypes = [ctypes.c_int, ctypes.c_int, dp, ip]
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, ip, ip, dp, dp, dp,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_n_blocks.restype = ctypes.c_int64
        L.oracle_n_blocks.argtypes = [ctypes.c_void_p]
        L.oracle_nnz.restype = ctypes.c_int64
        L.oracle_nnz.argtypes = [ctypes.c_void_p]
        L.oracle_blocks.argtypes = [ctypes.c_void_p, i32p]
        L.oracle_block_offsets.argtypes = [ctypes.c_void_p, i64p]
        L.oracle_schwarz.argtypes = [ctypes.c_void_p, dp]
        L.oracle_set_density.argtypes = [ctypes.c_void_p, dp, dp]
        L.oracle_set_pmax.argtypes = [ctypes.c_void_p, dp]
        L.oracle_set_q.argtypes = [ctypes.c_void_p, dp]
        L.oracle_schwarz_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, i32p, dp]
        L.oracle_quartets_bra.restype = ctypes.c_int64
        L.oracle_quartets_bra.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, i64p, ctypes.c_int64,
                                          i32p, dp]
        L.oracle_density_cart.restype = ctypes.c_int64
        L.oracle_density_cart.argtypes = [ctypes.c_void_p, i64p, dp]
        L.oracle_build_K.restype = ctypes.c_int64
        L.oracle_build_K.argtypes = [ctypes.c_void_p, ctypes.c_int64, i64p, ctypes.c_int, dp]
        L.oracle_quartets.restype = ctypes.c_int64
        L.oracle_quartets.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, i32p, dp]
        L.oracle_eval_quartets.restype = ctypes.c_int64
        L.oracle_eval_quartets.argtypes = [ctypes.c_void_p, ctypes.c_int64, i32p, dp]
        L.oracle_K_from_quartets.restype = ctypes.c_int64
        L.oracle_K_from_quartets.argtypes = [ctypes.c_void_p, ctypes.c_int64, i32p, dp]
        _lib = L
    return _lib


def _p(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


# ---------------------------------------------------------------- pieces
def boys(mmax: int, T: float) -> np.ndarray:
    """F_m(T), m = 0..mmax (long-double evaluation, rounded to double)."""
    out = np.zeros(mmax + 1)
    lib().oracle_boys(mmax, float(T), _p(out))
    return out


def op_ladder(op: str, omega: float, mmax: int, rho: float, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().oracle_op_ladder(OP[op], float(omega), mmax, float(rho), float(T), _p(out))
    return out


def normalize(l: int, ex: Sequence[float], c_raw: Sequence[float]) -> np.ndarray:
    ex = np.ascontiguousarray(ex, dtype=np.float64)
    c_raw = np.ascontiguousarray(c_raw, dtype=np.float64)
    out = np.zeros_like(ex)
    lib().oracle_normalize(int(l), len(ex), _p(ex), _p(c_raw), _p(out))
    return out


def eri(shells, op: str = "coulomb", omega: float = 0.0) -> np.ndarray:
    """Contracted Cartesian quartet (ab|cd).

    ``shells`` is four tuples (xyz, l, exponents, coefficients); coefficients
    are used as given (normalise with :func:`normalize` first if wanted).
    Returns an array of shape (ncart(la), ncart(lb), ncart(lc), ncart(ld)).
    """
    xyz = np.ascontiguousarray(np.concatenate([np.asarray(s[0], dtype=np.float64) for s in shells]))
    ls = np.array([s[1] for s in shells], dtype=np.int32)
    nps = np.array([len(s[2]) for s in shells], dtype=np.int32)
    ex = np.ascontiguousarray(np.concatenate([np.asarray(s[2], dtype=np.float64) for s in shells]))
    co = np.ascontiguousarray(np.concatenate([np.asarray(s[3], dtype=np.float64) for s in shells]))
    nc = [(l + 1) * (l + 2) // 2 for l in ls]
    out = np.zeros(int(np.prod(nc)))
    lib().oracle_eri_raw(_p(xyz), _p(ls, ctypes.c_int), _p(nps, ctypes.c_int), _p(ex), _p(co),
                         OP[op], float(omega), _p(out))
    return out.reshape(nc)


def sph_matrix(l: int, spherical: bool = True) -> np.ndarray:
    T = np.zeros(36)
    n = ctypes.c_int(0)
    lib().oracle_sph_matrix(int(l), int(spherical), _p(T), ctypes.byref(n))
    nc = (l + 1) * (l + 2) // 2
    return T[: n.value * nc].reshape(n.value, nc).copy()


def nao2gto_fit(l, r, radial, n_gto):
    """GTO fit of a numerical radial function (NAO2GTO: the paper fits each
    numerical orbital with several GTOs; it gives no procedure, so this is
    the reading): minimise sum_i w_i (R_i - sum_k c_k r_i^l exp(-a_k r_i^2))^2,
    w_i = r_i^2 dr_i (trapezoid), with even-tempered exponents a_k = a_0 b^k,
    coefficients by weighted linear least squares (numpy lstsq) for given
    (a_0, b); (log a_0, log b) by brute force over a 64 x 48 grid of the box
    a_0 in [0.1 / r_max^2, 5], b in [1.5, 8], refined by scipy's bounded
    Nelder-Mead.  Returns (exponents ascending, coefficients, relative rms)."""
    from scipy.optimize import minimize
    r = np.asarray(r, dtype=float)
    R = np.asarray(radial, dtype=float)
    dr = np.zeros_like(r)
    dr[1:] += 0.5 * np.diff(r)
    dr[:-1] += 0.5 * np.diff(r)
    sw = np.sqrt(r * r * dr)
    lo = np.array([np.log(0.1 / r[-1] ** 2), np.log(1.5)])
    hi = np.array([np.log(5.0), np.log(8.0) if n_gto > 1 else np.log(1.5)])

    def fit(p):
        p = np.clip(p, lo, hi)
        a = np.exp(p[0] + np.arange(n_gto) * p[1])
        A = (r ** l)[:, None] * np.exp(-a[None, :] * (r * r)[:, None])
        c, *_ = np.linalg.lstsq(sw[:, None] * A, sw * R, rcond=None)
        return a, c, float(np.sum((sw * (R - A @ c)) ** 2))

    ga = np.linspace(lo[0], hi[0], 64)
    gb = np.linspace(lo[1], hi[1], 48) if n_gto > 1 else np.array([lo[1]])
    vals = np.array([[fit(np.array([x, y]))[2] for y in gb] for x in ga])
    i, j = np.unravel_index(np.argmin(vals), vals.shape)
    p0 = np.array([ga[i], gb[j]])
    if n_gto > 1:
        sol = minimize(lambda p: fit(p)[2], p0, method="Nelder-Mead", bounds=list(zip(lo, hi)),
                       options={"xatol": 1e-12, "fatol": 0.0, "maxiter": 20000, "maxfev": 40000})
        p0 = sol.x
    else:
        sol = minimize(lambda x: fit(np.array([x[0], lo[1]]))[2], p0[:1], method="Nelder-Mead",
                       bounds=[(lo[0], hi[0])], options={"xatol": 1e-12, "fatol": 0.0, "maxiter": 20000})
        p0 = np.array([sol.x[0], lo[1]])
    a, c, f = fit(p0)
    return a, c, float(np.sqrt(f / np.sum((sw * R) ** 2)))


def kspace(system, blocks, offsets, K, kpts, alpha):
    """Exchange part of the Hamiltonian at k-points from real-space K blocks
    (Background section: Bloch sum of the Hamiltonian applied to Eq. H-HFX
    with its -1/2, times the exact-exchange fraction alpha):
    H(k)_{mu nu} = -(alpha/2) sum_G K^G_{mu nu} exp(i k.(T_G + r_nu - r_mu)).
    Plain loop over the pattern blocks; returns complex (nk, nbf, nbf)."""
    from systems import nfunc
    ls = np.asarray(system.shell_l)
    nf = np.array([nfunc(int(l), system.spherical_d) for l in ls])
    fo = np.concatenate([[0], np.cumsum(nf)])
    nbf = int(fo[-1])
    r = np.asarray(system.atom_xyz, dtype=float)[np.asarray(system.shell_atom)]
    lat = np.zeros((3, 3)) if system.lattice is None else np.asarray(system.lattice, dtype=float)
    kp = np.asarray(kpts, dtype=float).reshape(-1, 3)
    H = np.zeros((len(kp), nbf, nbf), dtype=complex)
    for b, (I, J, n1, n2, n3) in enumerate(np.asarray(blocks)):
        d = n1 * lat[0] + n2 * lat[1] + n3 * lat[2] + r[J] - r[I]
        v = np.asarray(K[offsets[b]:offsets[b + 1]]).reshape(nf[I], nf[J])
        for k in range(len(kp)):
            H[k, fo[I]:fo[I + 1], fo[J]:fo[J + 1]] += -0.5 * alpha * v * np.exp(1j * float(kp[k] @ d))
    return H


# ---------------------------------------------------------------- system
class Oracle:
    """Oracle state for one system: its own pattern, Q, P_max and K."""

    def __init__(self, system):
        s = system
        self.system = s
        self._keep = []
        xyz = self._k(np.ascontiguousarray(s.atom_xyz, dtype=np.float64))
        sa = self._k(np.ascontiguousarray(s.shell_atom, dtype=np.int32))
        sl = self._k(np.ascontiguousarray(s.shell_l, dtype=np.int32))
        sn = self._k(np.ascontiguousarray(s.shell_nprim, dtype=np.int32))
        ex = self._k(np.ascontiguousarray(s.prim_exp, dtype=np.float64))
        co = self._k(np.ascontiguousarray(s.prim_coef, dtype=np.float64))
        lat = None
        if s.lattice is not None:
            lat = self._k(np.ascontiguousarray(s.lattice, dtype=np.float64).reshape(9))
        self.h = lib().oracle_create(
            s.n_atoms, _p(xyz), s.n_shells, _p(sa, ctypes.c_int), _p(sl, ctypes.c_int),
            _p(sn, ctypes.c_int), _p(ex), _p(co), _p(lat) if lat is not None else None,
            float(s.pair_cutoff), OP[s.op], float(s.omega), float(s.tau), int(bool(s.spherical_d)))
        nb = lib().oracle_n_blocks(self.h)
        self.blocks = np.zeros((nb, 5), dtype=np.int32)
        if nb:
            lib().oracle_blocks(self.h, _p(self.blocks, ctypes.c_int32))
        self.offsets = np.zeros(nb + 1, dtype=np.int64)
        lib().oracle_block_offsets(self.h, _p(self.offsets, ctypes.c_int64))
        self.nnz = int(self.offsets[-1])
        self.Q = None
        self.Pmax = None

    def _k(self, a):
        self._keep.append(a)
        return a

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().oracle_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def schwarz(self) -> np.ndarray:
        self.Q = np.zeros(len(self.blocks))
        lib().oracle_schwarz(self.h, _p(self.Q))
        return self.Q

    def set_density(self, d_values: np.ndarray) -> np.ndarray:
        d = np.ascontiguousarray(d_values, dtype=np.float64)
        assert d.shape == (self.nnz,)
        self._d = d
        self.Pmax = np.zeros(len(self.blocks))
        lib().oracle_set_density(self.h, _p(d), _p(self.Pmax))
        return self.Pmax

    def schwarz_rows(self, rows) -> np.ndarray:
        """Schwarz factors of the blocks of the given shell rows only (what
        K blocks of those rows need); other blocks are zero until computed."""
        if self.Q is None:
            self.Q = np.zeros(len(self.blocks))
            lib().oracle_set_q(self.h, _p(self.Q))
        r = np.ascontiguousarray(sorted(set(int(x) for x in rows)), dtype=np.int32)
        lib().oracle_schwarz_rows(self.h, len(r), _p(r, ctypes.c_int32), _p(self.Q))
        return self.Q

    def set_q(self, q: np.ndarray) -> None:
        """Replace the Schwarz factors (one per block) used by the screening."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (len(self.blocks),)
        self.Q = q.copy()
        lib().oracle_set_q(self.h, _p(q))

    def quartets_of_bra_blocks(self, bra_blocks, gR: int = 3):
        """Kept ordered quartets whose bra block is one of ``bra_blocks``
        (every ket block, G in the cube |G_i| <= gR): (rows[n,13], bounds[n])."""
        if self.Q is None:
            self.schwarz()
        bb = np.ascontiguousarray(bra_blocks, dtype=np.int64)
        n = lib().oracle_quartets_bra(self.h, gR, len(bb), _p(bb, ctypes.c_int64), 0, None, None)
        rows = np.zeros((max(n, 1), 13), dtype=np.int32)
        bnd = np.zeros(max(n, 1))
        lib().oracle_quartets_bra(self.h, gR, len(bb), _p(bb, ctypes.c_int64), n, _p(rows, ctypes.c_int32), _p(bnd))
        return rows[:n], bnd[:n]

    def set_pmax(self, pmax: np.ndarray) -> None:
        """Replace the block maxima used by the screening predicate."""
        p = np.ascontiguousarray(pmax, dtype=np.float64)
        assert p.shape == (len(self.blocks),)
        self.Pmax = p.copy()
        lib().oracle_set_pmax(self.h, _p(p))

    def build_K_spin(self, d_alpha: np.ndarray, d_beta: np.ndarray):
        """Collinear spin: K of each spin density (Eq. H-HFX per spin), both
        screened with one predicate whose block maxima are the larger of the
        two spins' (so that one quartet list serves both).  Returns
        (K_alpha, K_beta)."""
        if self.Q is None:
            self.schwarz()
        pb = self.set_density(d_beta)
        pa = self.set_density(d_alpha)
        pm = np.maximum(pa, pb)
        self.set_pmax(pm)
        ka, _ = self.build_K()
        self.set_density(d_beta)
        self.set_pmax(pm)
        kb, _ = self.build_K()
        return ka, kb

    def density_cart(self):
        """Cartesian density blocks of the last set_density: (block offsets
        [n_blocks + 1], values [nnz_cart]); block b is ncart(I) x ncart(J)
        row-major at offsets[b]."""
        n = lib().oracle_density_cart(self.h, None, None)
        coff = np.zeros(len(self.blocks) + 1, dtype=np.int64)
        dc = np.zeros(max(n, 1))
        lib().oracle_density_cart(self.h, _p(coff, ctypes.c_int64), _p(dc))
        return coff, dc[:n]

    def density_from_system(self, iteration: int = 0) -> np.ndarray:
        from systems import density_blocks
        vals = density_blocks(self.system, self.blocks.astype(np.int64), iteration=iteration)
        return np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0)

    def build_K(self, blocks: Optional[np.ndarray] = None, screened: bool = True):
        """K values (pattern layout).  ``blocks``: indices to compute (default all).
        Returns (K, number of ordered quartets evaluated)."""
        if self.Q is None:
            self.schwarz()
        if blocks is None:
            blocks = np.arange(len(self.blocks), dtype=np.int64)
        req = np.ascontiguousarray(blocks, dtype=np.int64)
        K = np.zeros(self.nnz)
        n = lib().oracle_build_K(self.h, len(req), _p(req, ctypes.c_int64), int(screened), _p(K))
        return K, int(n)

    def quartets(self, gR: int = 2, cap: int = 50_000_000):
        """Kept ordered quartets (tiny systems only): (rows[n,13], bounds[n])."""
        if self.Q is None:
            self.schwarz()
        n = lib().oracle_quartets(self.h, gR, 0, None, None)
        rows = np.zeros((max(n, 1), 13), dtype=np.int32)
        bnd = np.zeros(max(n, 1))
        lib().oracle_quartets(self.h, gR, n, _p(rows, ctypes.c_int32), _p(bnd))
        return rows[:n], bnd[:n]

    def eval_quartets(self, rows: np.ndarray):
        """Evaluate ordered quartets (rows of 13 ints) without screening;
        returns (count, checksum).  For timing samples of a workload."""
        rows = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 13)
        cs = ctypes.c_double(0.0)
        n = lib().oracle_eval_quartets(self.h, len(rows), _p(rows, ctypes.c_int32), ctypes.byref(cs))
        return int(n), float(cs.value)

    def K_from_quartets(self, rows: np.ndarray):
        """K (pattern layout) from the given ordered quartets only, each
        adding its plain term of Eq. H-HFX (no screening); returns (K, number
        of rows whose K and D blocks exist).  Needs set_density first."""
        rows = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1, 13)
        K = np.zeros(self.nnz)
        n = lib().oracle_K_from_quartets(self.h, len(rows), _p(rows, ctypes.c_int32), _p(K))
        return K, int(n)

    def sample_quartets(self, n: int, seed: int = 0) -> np.ndarray:
        """n ordered quartets (I^0 J^N | K^G L^H) drawn uniformly from the
        plain loop of Eq. H-HFX: a K block (I, K, G), a bra pair of row I, a
        ket pair of row K, kept when the density block (J, L, H-N) exists."""
        rng = np.random.default_rng(seed)
        b = self.blocks.astype(np.int64)
        rows_of = {}
        for i, r in enumerate(b[:, 0]):
            rows_of.setdefault(int(r), []).append(i)
        keys = self.block_key_index()
        out = []
        while len(out) < n:
            kb = b[rng.integers(len(b))]
            I, K, G = int(kb[0]), int(kb[1]), kb[2:5]
            pb = b[rows_of[I][rng.integers(len(rows_of[I]))]]
            qb = b[rows_of[K][rng.integers(len(rows_of[K]))]]
            J, N = int(pb[1]), pb[2:5]
            L, M = int(qb[1]), qb[2:5]
            H = G + M
            if (J, L) + tuple(int(v) for v in (H - N)) not in keys:
                continue
            out.append([I, J, *N, K, L, *M, *G])
        return np.array(out, dtype=np.int32)

    def block_key_index(self):
        return {tuple(int(v) for v in b): i for i, b in enumerate(self.blocks)}
