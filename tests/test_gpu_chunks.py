"""Chunked quartet lists (screening and compaction in chunks of bra-pair
ranges, the batched evaluation of Algorithm 4): a build whose list limit is
far below its screened size equals the unchunked build and the oracle.

Bars: 1e-10 against the oracle (FP64), 1e-7 (mixed precision); chunked
against unchunked builds of the same plan 1e-12 (only the order of the FP64
atomic additions differs).
"""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _density(system, blocks):
    vals = systems.density_blocks(system, np.asarray(blocks, dtype=np.int64))
    return np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0)


def _tiny_cell(**kw):
    kw.setdefault("seed", 77)
    return systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, **kw)


def _oracle_K(system, D):
    o = oracle.Oracle(system)
    o.schwarz()
    o.set_density(D)
    return o.build_K()[0]


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _run(system, limit, flags=hfx.HFX_SYNC):
    plan = hfx.Plan(system)
    D = _density(system, plan.blocks)
    Dd = torch.from_numpy(D).to(DEV)
    K0 = torch.full_like(Dd, np.nan)
    i0 = plan.build_K(Dd, K0, flags=hfx.HFX_SYNC, info=True)
    plan.set_list_limit(limit)
    K1 = torch.full_like(Dd, np.nan)
    i1 = plan.build_K(Dd, K1, flags=flags, info=True)
    return plan, D, Dd, K0.cpu().numpy(), K1.cpu().numpy(), i0, i1


@pytest.mark.parametrize("which", ["molecule8", "cell", "cell_mixed", "cluster_mixed"])
def test_chunked_equals_whole_and_oracle(which, oracle_cache):
    if which == "molecule8":
        s = systems.molecule8()
    elif which == "cell":
        s = _tiny_cell()
    elif which == "cell_mixed":
        s = _tiny_cell(precision="mixed").with_(fp32_cutoff=1e-2)
    else:
        s = systems.random_cluster(6, seed=31, nprim=2, precision="mixed").with_(fp32_cutoff=1e-4)
    plan, D, Dd, Kw, Kc, iw, ic = _run(s, 4096)
    assert iw["n_chunks"] == 0
    assert ic["n_chunks"] >= 3, ic["n_chunks"]
    assert ic["n_quartets"] == iw["n_quartets"]
    assert ic["n_quartets_class"] == iw["n_quartets_class"]
    assert ic["n_prim_quartets"] == iw["n_prim_quartets"]
    assert ic["n_fp32_quartets"] == iw["n_fp32_quartets"]
    if s.precision == "mixed":
        assert iw["n_fp32_quartets"] > 0
    scale = max(1.0, float(np.max(np.abs(Kw))))
    assert np.max(np.abs(Kc - Kw)) <= 1e-12 * scale
    key = which
    if key not in oracle_cache:
        oracle_cache[key] = _oracle_K(s, D)
    tol = 1e-10 if s.precision == "fp64" else 1e-7
    assert np.max(np.abs(Kc - oracle_cache[key])) <= tol
    plan.destroy()


def test_chunk_limit_below_one_work_item_is_an_error():
    s = systems.molecule8()
    plan = hfx.Plan(s)
    D = _density(s, plan.blocks)
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.zeros_like(Dd)
    plan.set_list_limit(1)
    with pytest.raises(hfx.HfxError) as e:
        plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC)
    assert e.value.status == hfx.HFX_ERR_OOM
    # the default limit works again
    plan.set_list_limit(0)
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    assert info["n_chunks"] == 0
    plan.destroy()


def test_chunked_build_keeps_no_list_and_graph_builds_run_eagerly():
    s = _tiny_cell()
    plan, D, Dd, Kw, Kc, iw, ic = _run(s, 2048)
    with pytest.raises(hfx.HfxError) as e:
        plan.export(1)
    assert e.value.status == hfx.HFX_ERR_STATE
    Kg = torch.full_like(Dd, np.nan)
    for _ in range(3):
        info = plan.build_K(Dd, Kg, flags=hfx.HFX_GRAPH, info=True)
        assert info["n_chunks"] > 0
        assert np.max(np.abs(Kg.cpu().numpy() - Kw)) <= 1e-12 * max(1.0, float(np.max(np.abs(Kw))))
    # back to one list: exported list has the full count, graphs replay
    plan.set_list_limit(0)
    plan.build_K(Dd, Kg, flags=hfx.HFX_SYNC)
    assert len(plan.export(1)) == iw["n_quartets"]
    for _ in range(2):
        plan.build_K(Dd, Kg, flags=hfx.HFX_GRAPH)
        assert np.max(np.abs(Kg.cpu().numpy() - Kw)) <= 1e-12 * max(1.0, float(np.max(np.abs(Kw))))
    plan.destroy()


def test_fused_multi_plan_build_in_chunks():
    ss = [systems.molecule8(), systems.random_cluster(5, seed=41, nprim=2)]
    plans = [hfx.Plan(s) for s in ss]
    Ds = [torch.from_numpy(_density(s, p.blocks)).to(DEV) for s, p in zip(ss, plans)]
    Kw = [torch.zeros_like(d) for d in Ds]
    hfx.build_K_multi(plans, Ds, Kw, flags=hfx.HFX_SYNC)
    plans[1].set_list_limit(3000)
    Kc = [torch.full_like(d, np.nan) for d in Ds]
    info = hfx.build_K_multi(plans, Ds, Kc, flags=hfx.HFX_SYNC, info=True)
    assert info["n_chunks"] >= 2
    for s, p, d, a, b in zip(ss, plans, Ds, Kw, Kc):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, float(np.max(np.abs(a))))
        assert np.max(np.abs(b - _oracle_K(s, d.cpu().numpy()))) <= 1e-10
    for p in plans:
        p.destroy()


def test_progress_reports_every_chunk():
    s = _tiny_cell(precision="mixed").with_(fp32_cutoff=1e-2)
    plan = hfx.Plan(s)
    D = torch.from_numpy(_density(s, plan.blocks)).to(DEV)
    K = torch.zeros_like(D)
    seen = []
    plan.set_progress(lambda lst, chunk, done, total: seen.append((lst, chunk, done, total)))
    plan.set_list_limit(3000)
    info = plan.build_K(D, K, flags=hfx.HFX_SYNC, info=True)
    assert len(seen) == info["n_chunks"] >= 4
    assert [c for _, c, _, _ in seen] == list(range(1, len(seen) + 1))
    for lst in (0, 1):
        rep = [(d, t) for l_, _, d, t in seen if l_ == lst]
        assert rep, lst
        assert all(b[0] > a[0] for a, b in zip(rep, rep[1:]))
        assert rep[-1][0] == rep[-1][1]
    assert seen[-1][3] + [t for l_, _, d, t in seen if l_ == 0][-1] == info["n_quartets"]
    plan.set_progress(None)
    plan.build_K(D, K, flags=hfx.HFX_SYNC)
    assert len(seen) == info["n_chunks"]
    plan.destroy()
