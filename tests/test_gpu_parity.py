"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: K element by element within 1e-10 (FP64); Schwarz factors within
1e-12 relative; P_max bit-identical; the quartet list equal as a set of
canonical orbits, except quartets whose bound lies within 1e-12 relative of
tau (there either decision is correct, both are FP64).
"""
import numpy as np
import pytest

import oracle
import systems
from tests.helpers import canonical_keys, gpu_quartet_instances, key_set, oracle_quartet_instances

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL_FP64 = 1e-10


def _density(system, blocks, iteration=0):
    vals = systems.density_blocks(system, np.asarray(blocks, dtype=np.int64), iteration=iteration)
    return np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0)


class Case:
    def __init__(self, system):
        self.s = system
        self.plan = hfx.Plan(system)
        self.D = _density(system, self.plan.blocks)
        self.Dd = torch.from_numpy(self.D).to(DEV)
        self.Kd = torch.full_like(self.Dd, np.nan)
        self.info = self.plan.build_K(self.Dd, self.Kd, flags=hfx.HFX_SYNC, info=True)
        self.K = self.Kd.cpu().numpy()
        self.o = oracle.Oracle(system)
        self.o.schwarz()
        self.o.set_density(self.D)


def _tiny_cell(**kw):
    kw.setdefault("seed", 77)
    return systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, **kw)


@pytest.fixture(scope="module")
def c1():
    return Case(systems.molecule8())


@pytest.fixture(scope="module")
def cell():
    return Case(_tiny_cell())


def test_pattern_matches_oracle(c1, cell):
    for c in (c1, cell):
        assert np.array_equal(c.plan.blocks, c.o.blocks)
        assert np.array_equal(c.plan.offsets, c.o.offsets)


def test_schwarz_factors(c1, cell):
    for c in (c1, cell):
        q = c.plan.schwarz()
        assert np.allclose(q, c.o.Q, rtol=1e-12, atol=0)


def test_pmax_bit_identical_sp(c1):
    pm = c1.plan.export(0)
    assert np.array_equal(pm, c1.o.Pmax)


def test_pmax_close_spd(cell):
    pm = cell.plan.export(0)
    assert np.allclose(pm, cell.o.Pmax, rtol=1e-15, atol=0)


def test_K_molecule_full(c1):
    Kref, _ = c1.o.build_K()
    err = np.max(np.abs(c1.K - Kref))
    print(f"molecule: {c1.info['n_quartets']} quartets, max|dK| = {err:.3e}")
    assert err <= TOL_FP64


def test_K_periodic_erfc_spd(cell):
    Kref, _ = cell.o.build_K()
    err = np.max(np.abs(cell.K - Kref))
    print(f"tiny diamond cell: {cell.info['n_quartets']} quartets, max|dK| = {err:.3e}")
    assert err <= TOL_FP64


def _bounds_of(o, inst):
    """Oracle bound (Q_IJ Q_KL) P_scr of each quartet instance (n,4,4)."""
    keys = o.block_key_index()
    out = np.zeros(len(inst))
    for i, q in enumerate(inst):
        (I, *_), (J, *nJ), (K, *nK), (L, *nL) = [tuple(int(v) for v in r) for r in q]
        nJ, nK, nL = np.array(nJ), np.array(nK), np.array(nL)

        def blk(X, Y, n):
            return keys.get((X, Y) + tuple(int(v) for v in n), -1)

        def pm(X, Y, n):
            b = blk(X, Y, n)
            return 0.0 if b < 0 else o.Pmax[b]
        qij = o.Q[blk(I, J, nJ)]
        qkl = o.Q[blk(K, L, nL - nK)]
        ps = max(pm(I, K, nK), pm(I, L, nL), pm(J, K, nK - nJ), pm(J, L, nL - nJ))
        out[i] = (qij * qkl) * ps
    return out


@pytest.mark.parametrize("which", ["c1", "cell"])
def test_quartet_list_matches_oracle(which, c1, cell):
    c = c1 if which == "c1" else cell
    gl = hfx.unpack_quartets(c.plan.export(1))
    pairs = c.plan.export(2)
    gk = canonical_keys(gpu_quartet_instances(gl, pairs))
    # unique: no orbit listed twice
    assert len(key_set(gk)) == len(gk)
    rows, bnd = c.o.quartets(gR=3)
    ok = canonical_keys(oracle_quartet_instances(rows))
    gs, os_ = key_set(gk), key_set(ok)
    only_gpu = gs - os_
    only_orc = os_ - gs
    tau = c.s.tau
    # every disagreement must sit at the threshold
    if only_orc:
        idx = [i for i, k in enumerate(map(tuple, ok.tolist())) if k in only_orc]
        assert np.all(np.abs(bnd[idx] - tau) <= 1e-12 * tau), "oracle keeps quartets the GPU dropped"
    if only_gpu:
        inst = gpu_quartet_instances(gl, pairs)
        idx = [i for i, k in enumerate(map(tuple, gk.tolist())) if k in only_gpu]
        b = _bounds_of(c.o, inst[idx])
        assert np.all(np.abs(b - tau) <= 1e-12 * tau), "GPU keeps quartets the oracle dropped"
    print(f"{which}: {len(gs)} unique quartets, {len(only_gpu)}+{len(only_orc)} at the threshold")
    assert c.info["n_quartets"] == len(gl)


def test_cartesian_d_periodic():
    c = Case(_tiny_cell(seed=78, spherical_d=False))
    Kref, _ = c.o.build_K()
    assert np.max(np.abs(c.K - Kref)) <= TOL_FP64


def test_coulomb_molecule_with_d():
    s = systems.random_cluster(6, 4242, edge=7.0, min_sep=1.8, nprim=2)
    c = Case(s)
    Kref, _ = c.o.build_K()
    assert np.max(np.abs(c.K - Kref)) <= TOL_FP64


def test_repeat_builds_agree(c1):
    K2 = torch.zeros_like(c1.Dd)
    c1.plan.build_K(c1.Dd, K2, flags=hfx.HFX_SYNC)
    assert np.max(np.abs(K2.cpu().numpy() - c1.K)) <= 1e-13


def test_zero_density_gives_zero():
    s = systems.molecule8(seed=1234)
    plan = hfx.Plan(s)
    D = torch.zeros(plan.nnz, dtype=torch.float64, device=DEV)
    K = torch.full_like(D, 7.0)
    info = plan.build_K(D, K, flags=hfx.HFX_SYNC, info=True)
    assert info["n_quartets"] == 0
    assert torch.count_nonzero(K).item() == 0


def test_huge_tau_screens_everything():
    s = systems.molecule8().with_(tau=1e30)
    plan = hfx.Plan(s)
    D = torch.from_numpy(_density(s, plan.blocks)).to(DEV)
    K = torch.full_like(D, 3.0)
    info = plan.build_K(D, K, flags=hfx.HFX_SYNC, info=True)
    assert info["n_quartets"] == 0
    assert torch.count_nonzero(K).item() == 0


def test_single_shell_atom():
    s = systems.System(name="one_s", seed=5, atom_xyz=np.zeros((1, 3)),
                       shell_atom=np.array([0], np.int32), shell_l=np.array([0], np.int32),
                       shell_nprim=np.array([2], np.int32), prim_exp=np.array([0.5, 3.0]),
                       prim_coef=np.array([0.4, 0.6]))
    c = Case(s)
    Kref, _ = c.o.build_K()
    assert c.info["n_quartets"] == 1
    assert np.max(np.abs(c.K - Kref)) <= TOL_FP64


def test_destroyed_plan_is_rejected():
    s = systems.molecule8()
    plan = hfx.Plan(s)
    h = plan.handle.value
    plan.destroy()
    D = torch.zeros(plan.nnz, dtype=torch.float64, device=DEV)
    st = hfx.lib().hfx_build_K(hfx.ctypes.c_void_p(h), hfx.ctypes.c_void_p(D.data_ptr()),
                               hfx.ctypes.c_void_p(D.data_ptr()), 0, None)
    assert st == hfx.HFX_ERR_STATE


# ------------------------------------------------------------ mixed precision
TOL_MIXED = 1e-7


def _build(system, D=None):
    plan = hfx.Plan(system)
    if D is None:
        D = _density(system, plan.blocks)
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.zeros_like(Dd)
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    return plan, D, Kd.cpu().numpy(), info


@pytest.mark.parametrize("cutoff", [1e-6, 1e-2])
def test_mixed_precision_periodic_erfc(cutoff):
    s64 = _tiny_cell(seed=91)
    smx = s64.with_(precision="mixed", fp32_cutoff=cutoff)
    p64, D, K64, i64 = _build(s64)
    pmx, _, Kmx, imx = _build(smx, D)
    assert imx["n_quartets"] == i64["n_quartets"]
    assert imx["n_fp32_quartets"] > 0
    o = oracle.Oracle(s64)
    o.set_density(D)
    Kref, _ = o.build_K()
    err_o = np.max(np.abs(Kmx - Kref))
    err_g = np.max(np.abs(Kmx - K64))
    print(f"mixed cutoff {cutoff}: {imx['n_fp32_quartets']}/{imx['n_quartets']} FP32, "
          f"max|dK| vs oracle {err_o:.2e}, vs FP64 GPU {err_g:.2e}")
    assert err_o <= TOL_MIXED
    assert err_g <= TOL_MIXED
    # the two lists together are the FP64 list
    both = np.concatenate([pmx.export(1), pmx.export(5)])
    assert np.array_equal(np.sort(both), np.sort(p64.export(1)))
    # classes whose FP32 kernel is no faster keep every quartet on the FP64 list
    cls = pmx.export(2)[:, 5]
    q32 = pmx.export(5)
    bra_c = cls[(q32 & 0xFFFFFF).astype(np.int64)]
    ket_c = cls[((q32 >> 24) & 0xFFFFFF).astype(np.int64)]
    fp64_only = {(0, 0), (1, 0), (1, 1), (2, 1), (3, 0), (5, 0), (5, 5)}
    assert not any((max(int(b), int(k)), min(int(b), int(k))) in fp64_only for b, k in zip(bra_c, ket_c))
    assert len(q32) == imx["n_fp32_quartets"]


@pytest.mark.parametrize("cutoff", [1e-6, 1e-3])
def test_mixed_precision_cluster_recipe(cutoff):
    # small enough for the oracle: 5 atoms (3 heavy, 2 light), 3 primitives.
    # At the recipe's 1e-6 this cluster's quartets below the cutoff all fall
    # in classes that stay FP64; 1e-3 puts d-shell classes on the FP32 list.
    s = systems.random_cluster(5, 2024, nprim=3, op="coulomb", tau=1e-10, precision="mixed",
                               fp32_cutoff=cutoff)
    plan, D, K, info = _build(s)
    o = oracle.Oracle(s)
    o.set_density(D)
    Kref, _ = o.build_K()
    err = np.max(np.abs(K - Kref))
    print(f"cluster5 mixed {cutoff}: {info['n_fp32_quartets']}/{info['n_quartets']} FP32, max|dK| {err:.2e}")
    if cutoff > 1e-6:
        assert info["n_fp32_quartets"] > 0
    assert err <= TOL_MIXED


# ------------------------------------------------------ kernel variants
# every ERI kernel variant of the d-shell classes against the oracle
_VARIANTS = {
    "lane": ",".join(f"{cb}{ck}=lane" for cb in range(2, 6) for ck in range(cb + 1)),
    "coop": "42=coop,43=coop,44=coop,51=coop,52=coop,53=coop,54=coop,55=coop",
    "reg": "41=reg,42=reg,43=reg,51=reg",
}


@pytest.mark.parametrize("variant", sorted(_VARIANTS))
def test_kernel_variants_match_oracle(variant, cell, monkeypatch):
    monkeypatch.setenv("HFX_KERNELS", _VARIANTS[variant])
    plan = hfx.Plan(cell.s)
    Kd = torch.full_like(cell.Dd, np.nan)
    info = plan.build_K(cell.Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    Kref, _ = cell.o.build_K()
    err = np.max(np.abs(Kd.cpu().numpy() - Kref))
    print(f"{variant}: max|dK| = {err:.3e}")
    assert info["n_quartets"] == cell.info["n_quartets"]
    # every kernel applies the same primitive-quartet test (B_ket < thr / B_bra)
    assert info["n_prim_quartets"] == cell.info["n_prim_quartets"]
    assert err <= TOL_FP64


@pytest.mark.parametrize("variant", ["lane", "coop"])
def test_kernel_variants_mixed(variant, monkeypatch):
    monkeypatch.setenv("HFX_KERNELS", _VARIANTS[variant])
    s64 = _tiny_cell(seed=91)
    smx = s64.with_(precision="mixed", fp32_cutoff=1e-4)
    _, D, K64, _ = _build(s64)
    _, _, Kmx, imx = _build(smx, D)
    o = oracle.Oracle(s64)
    o.set_density(D)
    Kref, _ = o.build_K()
    err = np.max(np.abs(Kmx - Kref))
    print(f"{variant} mixed: {imx['n_fp32_quartets']}/{imx['n_quartets']} FP32, max|dK| {err:.2e}")
    assert err <= TOL_MIXED
    assert np.max(np.abs(K64 - Kref)) <= TOL_FP64


def test_kernel_override_rejects_unavailable(monkeypatch):
    monkeypatch.setenv("HFX_KERNELS", "55=reg")
    with pytest.raises(hfx.HfxError):
        hfx.Plan(_tiny_cell())


# ------------------------------------------------ quartet subsets, full size
def test_subset_of_whole_list_equals_build(cell):
    q = cell.plan.export(1)
    K = torch.full_like(cell.Dd, np.nan)
    cell.plan.build_K_subset(cell.Dd, K, q)
    assert np.max(np.abs(K.cpu().numpy() - cell.K)) <= 1e-13 * max(1.0, np.max(np.abs(cell.K)))
    # any order, and the empty subset gives zero
    K2 = torch.full_like(cell.Dd, np.nan)
    cell.plan.build_K_subset(cell.Dd, K2, q[::-1].copy())
    assert np.max(np.abs(K2.cpu().numpy() - cell.K)) <= 1e-13 * max(1.0, np.max(np.abs(cell.K)))
    cell.plan.build_K_subset(cell.Dd, K2, q[:0])
    assert torch.count_nonzero(K2).item() == 0


def test_subset_rejects_bad_quartets(cell):
    K = torch.zeros_like(cell.Dd)
    with pytest.raises(hfx.HfxError):
        cell.plan.build_K_subset(cell.Dd, K, np.array([np.uint64(1) << np.uint64(23)], dtype=np.uint64))


@pytest.mark.parametrize("which", ["c1", "cell"])
def test_quartet_list_exact_with_the_gpus_screening_inputs(which, c1, cell):
    """The oracle's predicate fed the GPU's exported Schwarz factors and
    P_max selects exactly the GPU's list (as a set of canonical orbits): the
    quartet selection is bit-identical, with no threshold window."""
    c = c1 if which == "c1" else cell
    o = oracle.Oracle(c.s)
    o.set_density(c.D)
    o.set_q(c.plan.schwarz())
    o.set_pmax(c.plan.export(0))
    gl = hfx.unpack_quartets(c.plan.export(1))
    gk = key_set(canonical_keys(gpu_quartet_instances(gl, c.plan.export(2))))
    rows, _ = o.quartets(gR=3)
    ok = key_set(canonical_keys(oracle_quartet_instances(rows)))
    assert gk == ok, (len(gk - ok), len(ok - gk))
    assert len(gk) == len(gl)


def _region(ls, I, J, K, L):
    def pc(a, b):
        a, b = max(a, b), min(a, b)
        return 0 if a == 0 else (1 + b if a == 1 else 3 + b)
    p, q = pc(ls[I], ls[J]), pc(ls[K], ls[L])
    cb, ck = max(p, q), min(p, q)
    return cb * (cb + 1) // 2 + ck


def test_full_size_list_on_sampled_bra_pairs():
    """The 64-atom periodic diamond workload at full size: for a seeded
    sample of shell pairs (three of each pair class), the orbits of the
    GPU's list containing the pair equal the oracle's kept orbits with that
    bra pair (the oracle screening with the GPU's Q and P_max: exact)."""
    s = systems.diamond_cell()
    plan = hfx.Plan(s)
    D = _density(s, plan.blocks)
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.zeros_like(Dd)
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    qb = plan.schwarz()
    pm = plan.export(0)
    pairs = plan.export(2)
    rng = np.random.default_rng(2024)
    pick = np.concatenate([rng.choice(np.flatnonzero(pairs[:, 5] == c), size=3, replace=False) for c in range(6)])
    lst = plan.export(1)
    assert len(lst) == info["n_quartets"]
    sel = np.zeros(len(pairs), dtype=bool)
    sel[pick] = True
    keep = []
    step = 1 << 26
    for a in range(0, len(lst), step):
        q = lst[a:a + step]
        bra = (q & np.uint64(0xFFFFFF)).astype(np.int64)
        ket = ((q >> np.uint64(24)) & np.uint64(0xFFFFFF)).astype(np.int64)
        keep.append(q[sel[bra] | sel[ket]])
    del lst
    gsel = np.concatenate(keep)
    gk = key_set(canonical_keys(gpu_quartet_instances(hfx.unpack_quartets(gsel), pairs)))
    o = oracle.Oracle(s)
    o.set_density(D)
    o.set_q(qb)
    o.set_pmax(pm)
    bkey = {tuple(int(v) for v in b): i for i, b in enumerate(plan.blocks)}
    bra_blocks = [bkey[tuple(int(v) for v in pairs[p, :5])] for p in pick]
    rows, _ = o.quartets_of_bra_blocks(bra_blocks, gR=3)
    ok = key_set(canonical_keys(oracle_quartet_instances(rows)))
    print(f"full-size list: {len(pick)} pairs, {len(gsel)} GPU quartets, {len(ok)} oracle orbits")
    assert len(gk) == len(gsel)
    assert gk == ok, (len(gk - ok), len(ok - gk))


@pytest.mark.parametrize("precision,cutoff", [("fp64", 0.0), ("mixed", 1e-4), ("mixed", 1e-6)])
def test_full_size_sampled_parity(precision, cutoff):
    """The 64-atom periodic diamond workload of the benchmark at full size:
    K from a seeded, class-stratified sample of quartets (eight orbits of
    each of the 21 classes drawn from the plain loop, one member of each
    orbit in device orientation) on the GPU against the oracle's plain terms
    of every member of the same orbits; FP64 (1e-10) and the mixed form at
    the benchmark's cutoff 1e-4 and at 1e-6 (1e-7), the quartets below the
    cutoff taking the FP32 kernels."""
    from tests.helpers import canonical_keys, gpu_rows, oracle_quartet_instances, orbit_members, to_gpu_quartets
    s = systems.diamond_cell(precision=precision)
    if precision == "mixed":
        s = s.with_(fp32_cutoff=cutoff)
    plan = hfx.Plan(s)
    o = oracle.Oracle(s)
    D = _density(s, plan.blocks)
    o.set_density(D)
    # at least 8 distinct orbits of every one of the 21 classes, drawn
    # uniformly from the plain loop (the rarest class, (dd|dd), is 0.2% of it)
    ls = s.shell_l
    chosen, seen = [], set()
    per = np.zeros(21, dtype=int)
    for seed in range(11, 31):
        pool = o.sample_quartets(20000, seed=seed)
        keys = canonical_keys(oracle_quartet_instances(pool))
        for row, k in zip(pool, map(tuple, keys.tolist())):
            r = _region(ls, row[0], row[1], row[5], row[6])
            if per[r] < 8 and k not in seen:
                seen.add(k)
                per[r] += 1
                chosen.append(row)
        if per.min() >= 8:
            break
    assert per.min() >= 8, per
    rows = np.array(chosen, dtype=np.int32)
    pairs = plan.export(2)
    q = to_gpu_quartets(rows, pairs, pairs[:, 5])
    # the device representatives are members of the same orbits
    rep = gpu_rows(hfx.unpack_quartets(q), pairs)
    assert np.array_equal(canonical_keys(oracle_quartet_instances(rep)), canonical_keys(oracle_quartet_instances(rows)))
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.full_like(Dd, np.nan)
    plan.build_K_subset(Dd, Kd, q)
    Kref, used = o.K_from_quartets(orbit_members(rows))
    err = np.max(np.abs(Kd.cpu().numpy() - Kref))
    print(f"full-size sample ({precision} {cutoff}): {len(rows)} orbits, {used} ordered terms, "
          f"max|dK| = {err:.3e}, max|K| = {np.max(np.abs(Kref)):.3e}")
    assert used > len(rows)
    assert err <= (TOL_FP64 if precision == "fp64" else 1e-7)


def test_max_primitives_and_angular_momentum():
    """HFX_MAX_PRIM primitives on s, p and d shells (64 primitive pairs per
    shell pair, the largest ragged primitive sets), Coulomb and erfc."""
    for op in ("coulomb", "erfc"):
        s = systems.random_cluster(2, 777, edge=4.0, min_sep=1.5, heavy=(0, 1, 2), light=(0, 1, 2), nprim=8,
                                   op=op, omega=0.3)
        c = Case(s)
        Kref, _ = c.o.build_K()
        err = np.max(np.abs(c.K - Kref))
        print(f"8 primitives {op}: {c.info['n_quartets']} quartets, max|dK| = {err:.3e}")
        assert err <= TOL_FP64


@pytest.mark.parametrize("rep", [(2, 1, 1), (2, 2, 2)])
def test_supercell_tiles_the_cell(rep):
    """A supercell of the periodic cell computed as a cell, with the cell's
    density tiled, gives the cell's K tiled (same pattern, same Q and P_max
    per corresponding block, so the same screened terms)."""
    kw = dict(seed=79, nprim=2, shells=(0, 1, 2), r_cut=4.6)
    small = systems.diamond_cell(n=(1, 1, 1), **kw)
    big = systems.diamond_cell(n=rep, **kw)
    assert np.array_equal(small.prim_exp, big.prim_exp[: len(small.prim_exp)])
    ps, pb = hfx.Plan(small), hfx.Plan(big)
    nsh = 3                                      # shells per atom
    Ds = _density(small, ps.blocks)
    skey = {tuple(int(v) for v in b): i for i, b in enumerate(ps.blocks)}
    reps = np.array(rep)

    def cellvec(shell):
        c = (shell // nsh) // 8                  # conventional cell of the atom
        return np.array([c // (rep[1] * rep[2]), (c // rep[2]) % rep[1], c % rep[2]])

    def small_shell(shell):
        return ((shell // nsh) % 8) * nsh + shell % nsh

    mapped = []
    for (I, J, n1, n2, n3) in pb.blocks:
        m = cellvec(J) - cellvec(I) + np.array([n1, n2, n3]) * reps
        mapped.append(skey[(small_shell(I), small_shell(J), *map(int, m))])
    Db = np.concatenate([Ds[ps.offsets[b]:ps.offsets[b + 1]] for b in mapped])
    Ks = torch.zeros(ps.nnz, dtype=torch.float64, device=DEV)
    Kb = torch.zeros(pb.nnz, dtype=torch.float64, device=DEV)
    ps.build_K(torch.from_numpy(Ds).to(DEV), Ks, flags=hfx.HFX_SYNC)
    pb.build_K(torch.from_numpy(Db).to(DEV), Kb, flags=hfx.HFX_SYNC)
    Ks, Kb = Ks.cpu().numpy(), Kb.cpu().numpy()
    Kt = np.concatenate([Ks[ps.offsets[b]:ps.offsets[b + 1]] for b in mapped])
    err = np.max(np.abs(Kb - Kt))
    print(f"supercell {rep}: {len(pb.blocks)} blocks, max|dK| = {err:.3e}")
    assert err <= 1e-12 * max(1.0, np.max(np.abs(Ks)))
