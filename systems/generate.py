"""Synthetic systems shaped like the paper's molecules and solids.

Recipes (all lengths in bohr, exponents in bohr^-2):

* ``molecule8``: 8 atoms uniform in a 10-bohr cube (min separation 2),
  one element with shells s,s,p, 3 primitives per shell, exponents
  log-uniform in [0.1, 10], raw coefficients uniform in [0.1, 1]; bare
  Coulomb; tau = 1e-10; density D_ij = u_ij exp(-0.3 r_ij).
* ``diamond_cell``: conventional diamond cell a = 10.26 repeated 2x2x2
  (64 atoms, cubic cell edge 20.52), one element with shells s,s,p,p,d
  (13 spherical functions), 6 primitives per shell, exponents log-uniform in
  [0.05, 20]; erfc-screened operator with omega = 0.11; shell pairs kept
  within 12 bohr; D_ij = u_ij exp(-0.5 r_ij).
* ``cluster_k4``: 256 atoms at density 0.1 atoms/bohr^3 (cube edge
  (N/0.1)^(1/3)), min separation 1.8, alternating heavy (s,s,p,p,d) and light
  (s,s,p) elements, 4 primitives per shell, exponents log-uniform in
  [0.1, 10]; bare Coulomb; FP32 cutoff 1e-6 on the product of Schwarz
  factors; D as in the molecule.
* ``cluster_batch``: 512 clusters with N uniform in {4..40}, each built with
  the cluster recipe and its own seed.
* ``request_stream``: a Poisson stream (rate 200/s) of requests, half
  clusters (N log-uniform in [10, 500], cluster recipe) and half periodic
  diamond cells of 8..128 atoms (cell recipe), each of 10 SCF
  iterations.

Draw order for a system with seed s: ``rng = Generator(PCG64(s))``; atom
positions first (rejection sampling, one candidate at a time), then for each
element in order, for each of its shells in order: the exponents, then the
raw coefficients.  Density values do not use ``rng``: each element of D is a
pure function of (seed, orbital i, orbital j, image n) through SplitMix64, so
that any consumer enumerating any subset of blocks in any order gets the same
numbers, and D^n_ij = D^-n_ji holds exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# counter-based hashing (SplitMix64, Steele, Lea & Flood, OOPSLA 2014)
# --------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 finaliser applied to ``x + golden gamma`` (uint64 array)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _mix(h, v):
    v = np.asarray(v).astype(np.int64).astype(np.uint64)
    return splitmix64(np.asarray(h, dtype=np.uint64) ^ v)


def hash_uniform(seed: int, *keys) -> np.ndarray:
    """Uniform doubles in [0, 1) from the 53 top bits of a chained hash."""
    h = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    for k in keys:
        h = _mix(h, k)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# system container
# --------------------------------------------------------------------------
def nfunc(l: int, spherical_d: bool) -> int:
    """Number of basis functions of a shell at the boundary."""
    if l == 2 and spherical_d:
        return 5
    return (l + 1) * (l + 2) // 2


@dataclasses.dataclass
class System:
    name: str
    seed: int
    atom_xyz: np.ndarray          # (n_atoms, 3) float64, bohr
    shell_atom: np.ndarray        # (n_shells,) int32
    shell_l: np.ndarray           # (n_shells,) int32
    shell_nprim: np.ndarray       # (n_shells,) int32
    prim_exp: np.ndarray          # (sum nprim,) float64
    prim_coef: np.ndarray         # (sum nprim,) float64, raw (not normalised)
    lattice: Optional[np.ndarray] = None   # (3, 3) rows a1, a2, a3, or None
    pair_cutoff: float = 0.0      # <= 0: all pairs
    op: str = "coulomb"           # "coulomb" | "erfc"
    omega: float = 0.0
    tau: float = 1e-10
    precision: str = "fp64"       # "fp64" | "mixed"
    fp32_cutoff: float = 0.0
    spherical_d: bool = True
    d_decay: float = 0.3          # D_ij = u exp(-d_decay r_ij)
    d_drop: float = 1e-8          # |D_ij| below this -> 0

    @property
    def n_atoms(self) -> int:
        return int(self.atom_xyz.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def periodic(self) -> bool:
        return self.lattice is not None

    def shell_nfunc(self) -> np.ndarray:
        return np.array([nfunc(int(l), self.spherical_d) for l in self.shell_l], dtype=np.int64)

    def shell_func_offset(self) -> np.ndarray:
        nf = self.shell_nfunc()
        return np.concatenate([[0], np.cumsum(nf)[:-1]]).astype(np.int64)

    def n_functions(self) -> int:
        return int(self.shell_nfunc().sum())

    def shell_prim_offset(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.shell_nprim)[:-1]]).astype(np.int64)

    def with_(self, **kw) -> "System":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def _rejection_positions(rng, n_atoms: int, edge: float, min_sep: float,
                         max_tries: int = 2_000_000) -> np.ndarray:
    pos = np.empty((n_atoms, 3))
    k = 0
    tries = 0
    while k < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling did not place all atoms")
        c = rng.uniform(0.0, edge, size=3)
        if k:
            d2 = np.sum((pos[:k] - c) ** 2, axis=1)
            if np.min(d2) < min_sep * min_sep:
                continue
        pos[k] = c
        k += 1
    return pos


def diamond_supercell(a: float, n1: int, n2: int, n3: int) -> Tuple[np.ndarray, np.ndarray]:
    """Atoms of n1 x n2 x n3 conventional cubic diamond cells of edge ``a``."""
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])
    pts = []
    for i in range(n1):
        for j in range(n2):
            for k in range(n3):
                pts.append((basis + np.array([i, j, k])) * a)
    xyz = np.concatenate(pts)
    lat = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return xyz, lat


# --------------------------------------------------------------------------
# basis
# --------------------------------------------------------------------------
def _draw_element(rng, shells: Sequence[int], nprim: int, lo: float, hi: float):
    out = []
    for l in shells:
        ex = np.exp(rng.uniform(math.log(lo), math.log(hi), size=nprim))
        co = rng.uniform(0.1, 1.0, size=nprim)
        out.append((int(l), ex, co))
    return out


def _assemble(name, seed, xyz, elem_of_atom, elements, **kw) -> System:
    sh_atom, sh_l, sh_np, pe, pc = [], [], [], [], []
    for ia, e in enumerate(elem_of_atom):
        for (l, ex, co) in elements[e]:
            sh_atom.append(ia)
            sh_l.append(l)
            sh_np.append(len(ex))
            pe.append(ex)
            pc.append(co)
    return System(
        name=name, seed=seed, atom_xyz=np.ascontiguousarray(xyz, dtype=np.float64),
        shell_atom=np.array(sh_atom, dtype=np.int32), shell_l=np.array(sh_l, dtype=np.int32),
        shell_nprim=np.array(sh_np, dtype=np.int32),
        prim_exp=np.concatenate(pe).astype(np.float64),
        prim_coef=np.concatenate(pc).astype(np.float64), **kw)


def random_cluster(n_atoms: int, seed: int, *, edge: Optional[float] = None,
                   density: float = 0.1, min_sep: float = 1.8,
                   heavy=(0, 0, 1, 1, 2), light=(0, 0, 1), nprim: int = 4,
                   exp_range=(0.1, 10.0), alternate: bool = True,
                   name: Optional[str] = None, **kw) -> System:
    """Random molecular cluster (the cluster recipe by default)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if edge is None:
        edge = (n_atoms / density) ** (1.0 / 3.0)
    xyz = _rejection_positions(rng, n_atoms, edge, min_sep)
    elements = [_draw_element(rng, heavy, nprim, *exp_range)]
    if alternate:
        elements.append(_draw_element(rng, light, nprim, *exp_range))
        elem_of_atom = [i % 2 for i in range(n_atoms)]
    else:
        elem_of_atom = [0] * n_atoms
    kw.setdefault("d_decay", 0.3)
    return _assemble(name or f"cluster{n_atoms}", seed, xyz, elem_of_atom, elements, **kw)


def molecule8(seed: int = 1000) -> System:
    """8-atom s,s,p molecule in a 10-bohr cube, bare Coulomb, FP64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = _rejection_positions(rng, 8, 10.0, 2.0)
    elements = [_draw_element(rng, (0, 0, 1), 3, 0.1, 10.0)]
    return _assemble("molecule8_ssp_K3", seed, xyz, [0] * 8, elements,
                     op="coulomb", tau=1e-10, d_decay=0.3)


def diamond_cell(seed: int = 1001, n=(2, 2, 2), a: float = 10.26, nprim: int = 6,
                 exp_range=(0.05, 20.0), shells=(0, 0, 1, 1, 2), r_cut: float = 12.0,
                 omega: float = 0.11, precision: str = "fp64", name: Optional[str] = None,
                 **kw) -> System:
    """Periodic diamond cell, erfc operator, shell pairs within ``r_cut``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz, lat = diamond_supercell(a, *n)
    elements = [_draw_element(rng, shells, nprim, *exp_range)]
    kw.setdefault("tau", 1e-10)
    kw.setdefault("d_decay", 0.5)
    nm = name or f"diamond{xyz.shape[0]}_ssppd_K{nprim}_erfc"
    return _assemble(nm, seed, xyz, [0] * xyz.shape[0], elements, lattice=lat,
                     pair_cutoff=r_cut, op="erfc", omega=omega, precision=precision,
                     fp32_cutoff=1e-6 if precision == "mixed" else 0.0, **kw)


def cluster_k4(seed: int = 1002, n_atoms: int = 256, precision: str = "mixed") -> System:
    return random_cluster(n_atoms, seed, name=f"cluster{n_atoms}_K4",
                          op="coulomb", tau=1e-10, precision=precision,
                          fp32_cutoff=1e-6 if precision == "mixed" else 0.0)


def cluster_batch(seed: int = 1003, n_clusters: int = 512, n_range=(4, 40),
                  precision: str = "mixed") -> List[System]:
    """Independent clusters for the fused batched launch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(n_range[0], n_range[1] + 1, size=n_clusters)
    return [random_cluster(int(n), seed * 100000 + i + 1, name=f"batch{i}_n{int(n)}",
                           op="coulomb", tau=1e-10, precision=precision,
                           fp32_cutoff=1e-6 if precision == "mixed" else 0.0)
            for i, n in enumerate(sizes)]


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    system: System
    n_iter: int = 10


def request_stream(seed: int = 1004, n_requests: int = 200, rate_per_s: float = 200.0,
                   cluster_range=(10, 500), cell_atoms=(8, 16, 32, 64, 128),
                   n_iter: int = 10, precision: str = "mixed",
                   cluster_nprim: int = 4, cell_nprim: int = 6) -> List[Request]:
    """The first n_requests of the seeded Poisson request stream (50%
    clusters, 50% cells).  Draw order, request by request: the gap to the
    previous arrival, the kind, the cluster size, the cell size; so the
    first k requests are the same for every n_requests >= k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = cluster_range
    gaps, kinds, sizes, cells = [], [], [], []
    for _ in range(n_requests):
        gaps.append(rng.exponential(1.0 / rate_per_s))
        kinds.append(int(rng.integers(0, 2)))
        sizes.append(float(np.exp(rng.uniform(math.log(lo), math.log(hi)))))
        cells.append(int(rng.integers(0, len(cell_atoms))))
    t = np.cumsum(gaps)
    shapes = {8: (1, 1, 1), 16: (2, 1, 1), 32: (2, 2, 1), 64: (2, 2, 2), 128: (4, 2, 2)}
    out = []
    for i in range(n_requests):
        s = seed * 1000003 + i + 1
        if kinds[i] == 0:
            sysm = random_cluster(int(round(sizes[i])), s, nprim=cluster_nprim,
                                  name=f"req{i}_cluster{int(round(sizes[i]))}",
                                  op="coulomb", tau=1e-10, precision=precision,
                                  fp32_cutoff=1e-6 if precision == "mixed" else 0.0)
        else:
            na = cell_atoms[int(cells[i])]
            sysm = diamond_cell(seed=s, n=shapes[na], nprim=cell_nprim, precision=precision,
                                   name=f"req{i}_diamond{na}")
        out.append(Request(rid=i, arrival_s=float(t[i]), system=sysm, n_iter=n_iter))
    return out


# --------------------------------------------------------------------------
# density matrix
# --------------------------------------------------------------------------
def _canonical_keys(i, j, n):
    """Orient (i, j, n) so that (i, j, n) and (j, i, -n) share one key."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64).reshape(-1, 3)
    n_pos = (n[:, 0] > 0) | ((n[:, 0] == 0) & ((n[:, 1] > 0) | ((n[:, 1] == 0) & (n[:, 2] >= 0))))
    keep = (i < j) | ((i == j) & n_pos)
    ci = np.where(keep, i, j)
    cj = np.where(keep, j, i)
    cn = np.where(keep[:, None], n, -n)
    return ci, cj, cn


def _image_vectors(system: System, n: np.ndarray) -> np.ndarray:
    if system.lattice is None:
        return np.zeros((n.shape[0], 3))
    return n.astype(np.float64) @ system.lattice


def density_blocks(system: System, blocks: np.ndarray, iteration: int = 0,
                   noise: float = 1e-3) -> List[np.ndarray]:
    """Density values for the given blocks.

    ``blocks`` is an (nb, 5) integer array of (I, J, n1, n2, n3): the block
    couples home-cell shell I with shell J translated by lattice vector n.
    Returns one (nfunc(I), nfunc(J)) array per block in the boundary basis
    (spherical d when ``system.spherical_d``).  D_ij = u_ij exp(-decay r_ij)
    with u uniform in [-1, 1] and r the distance between the two atom
    centres; |D_ij| < d_drop is set to 0.  For ``iteration`` k > 0 the values
    are D_0 * prod_{t=1..k} (1 + noise * xi_t) with xi_t standard normal,
    symmetric in (i, j, n) <-> (j, i, -n).
    """
    return density_series(system, blocks, iteration + 1, noise, first=iteration)[0]


def density_series(system: System, blocks: np.ndarray, n_iter: int, noise: float = 1e-3,
                   first: int = 0) -> List[List[np.ndarray]]:
    """density_blocks for iterations first .. n_iter-1 in one pass (each
    iteration's factor drawn once, the running product kept), the same
    values bit for bit."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 5)
    nf = system.shell_nfunc()
    off = system.shell_func_offset()
    xyz = system.atom_xyz
    sizes = nf[blocks[:, 0]] * nf[blocks[:, 1]]
    tot = int(sizes.sum())
    if tot == 0:
        return [[np.zeros((nf[b[0]], nf[b[1]])) for b in blocks] for _ in range(first, n_iter)]
    bi = np.repeat(np.arange(blocks.shape[0]), sizes)
    start = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    local = np.arange(tot) - start[bi]
    ncol = nf[blocks[bi, 1]]
    a = local // ncol
    b = local % ncol
    I = blocks[bi, 0]
    J = blocks[bi, 1]
    img = blocks[bi, 2:5]
    gi = off[I] + a
    gj = off[J] + b
    ci, cj, cn = _canonical_keys(gi, gj, img)
    u = 2.0 * hash_uniform(system.seed, ci, cj, cn[:, 0], cn[:, 1], cn[:, 2]) - 1.0
    rvec = xyz[system.shell_atom[I]] - (xyz[system.shell_atom[J]] + _image_vectors(system, img))
    r = np.sqrt(np.sum(rvec * rvec, axis=1))
    val = u * np.exp(-system.d_decay * r)
    series = []
    for k in range(0, n_iter):
        if k >= 1:
            u1 = hash_uniform(system.seed ^ 0x5A5A5A5A, k, ci, cj, cn[:, 0], cn[:, 1], cn[:, 2])
            u2 = hash_uniform(system.seed ^ 0x3C3C3C3C, k, ci, cj, cn[:, 0], cn[:, 1], cn[:, 2])
            xi = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
            val = val * (1.0 + noise * xi)
        if k < first:
            continue
        kept = np.where(np.abs(val) < system.d_drop, 0.0, val)
        out = []
        for q in range(blocks.shape[0]):
            s0 = int(start[q])
            out.append(kept[s0:s0 + int(sizes[q])].reshape(int(nf[blocks[q, 0]]), int(nf[blocks[q, 1]])))
        series.append(out)
    return series


def perturb_density(system: System, blocks: np.ndarray, iteration: int) -> List[np.ndarray]:
    """Density of SCF iteration ``iteration`` (0 = initial) of a request."""
    return density_blocks(system, blocks, iteration=iteration)


# --------------------------------------------------------------------------
# synthetic numerical atomic orbitals (radial tables with a strict cutoff)
# --------------------------------------------------------------------------
def nao_radial(l: int, zeta: float, r_cut: float, n_r: int = 400) -> Tuple[np.ndarray, np.ndarray]:
    """A radial table shaped like a confined numerical atomic orbital:
    R(r) = r^l exp(-zeta r) (1 - (r / r_cut)^2)^2 for r < r_cut and 0 beyond,
    on n_r uniform points of [0, r_cut] (the real NAO and pseudopotential
    files of the paper's systems are not available)."""
    r = np.linspace(0.0, r_cut, n_r)
    R = r ** l * np.exp(-zeta * r) * (1.0 - (r / r_cut) ** 2) ** 2
    return r, R


def nao_basis(seed: int, shells=(0, 0, 1, 1, 2)) -> List[Tuple[int, float, float]]:
    """Seeded (l, zeta, r_cut) of an element's numerical orbitals: zeta
    log-uniform in [0.6, 2.5] bohr^-1, r_cut uniform in [5, 8] bohr."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for l in shells:
        zeta = float(np.exp(rng.uniform(np.log(0.6), np.log(2.5))))
        rc = float(rng.uniform(5.0, 8.0))
        out.append((int(l), zeta, rc))
    return out
