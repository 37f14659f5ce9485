"""GPU: the batched forms of the build against one-at-a-time builds.

* hfx_build_K_multi over several plans (mixed operators, precisions and
  sizes) equals separate hfx_build_K calls, and the oracle;
* HFX_GRAPH replays of a captured build equal eager builds, with eager work
  and synchronisations between the replays, across density updates written
  into the same buffers, and when the screened list outgrows the capacity
  fixed at capture time (detected on the device, redone eagerly).
"""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _density(system, blocks, iteration=0):
    vals = systems.density_blocks(system, np.asarray(blocks, dtype=np.int64), iteration=iteration)
    return np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0)


def _tiny_cell(**kw):
    kw.setdefault("seed", 77)
    return systems.diamond_cell(n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, **kw)


def _systems():
    return [
        systems.molecule8(),
        _tiny_cell(seed=301),
        systems.random_cluster(5, 2025, nprim=2, op="coulomb"),
        _tiny_cell(seed=302).with_(precision="mixed", fp32_cutoff=1e-4),
        systems.molecule8(seed=1003).with_(op="erfc", omega=0.2),
    ]


def _eager(plan, D):
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.zeros_like(Dd)
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    return Kd.cpu().numpy(), info


def test_multi_equals_separate_and_oracle():
    ss = _systems()
    plans = [hfx.Plan(s) for s in ss]
    Ds = [_density(s, p.blocks, iteration=1) for s, p in zip(ss, plans)]
    sep = [_eager(p, D) for p, D in zip(plans, Ds)]
    Dd = [torch.from_numpy(D).to(DEV) for D in Ds]
    Kd = [torch.full_like(d, np.nan) for d in Dd]
    info = hfx.build_K_multi(plans, Dd, Kd, flags=hfx.HFX_SYNC, info=True)
    assert info["n_quartets"] == sum(i["n_quartets"] for _, i in sep)
    for k, (s, (Ks, _)) in enumerate(zip(ss, sep)):
        Km = Kd[k].cpu().numpy()
        scale = max(1.0, np.max(np.abs(Ks)))
        err = np.max(np.abs(Km - Ks)) if Km.size else 0.0
        print(f"{s.name}: multi vs separate max|dK| {err:.2e}")
        assert err <= 1e-13 * scale
    # the oracle for the small FP64 members
    for k in (0, 2):
        o = oracle.Oracle(ss[k])
        o.set_density(Ds[k])
        Kref, _ = o.build_K()
        assert np.max(np.abs(Kd[k].cpu().numpy() - Kref)) <= 1e-10


def test_multi_repeat_and_subset_cache():
    ss = _systems()[:3]
    plans = [hfx.Plan(s) for s in ss]
    Ds = [torch.from_numpy(_density(s, p.blocks)).to(DEV) for s, p in zip(ss, plans)]
    K1 = [torch.zeros_like(d) for d in Ds]
    K2 = [torch.zeros_like(d) for d in Ds]
    hfx.build_K_multi(plans, Ds, K1, flags=hfx.HFX_SYNC)
    hfx.build_K_multi(plans[1:], Ds[1:], K2[1:], flags=hfx.HFX_SYNC)
    hfx.build_K_multi(plans, Ds, K2, flags=hfx.HFX_SYNC)
    for a, b in zip(K1, K2):
        assert torch.max(torch.abs(a - b)).item() <= 1e-13 * max(1.0, torch.max(torch.abs(a)).item())


def test_multi_rejects_duplicates_and_destroyed():
    s = systems.molecule8()
    p = hfx.Plan(s)
    D = torch.zeros(p.nnz, dtype=torch.float64, device=DEV)
    with pytest.raises(hfx.HfxError):
        hfx.build_K_multi([p, p], [D, D], [D, D])
    q = hfx.Plan(s)
    hfx.build_K_multi([p, q], [D, D], [torch.zeros_like(D), torch.zeros_like(D)], flags=hfx.HFX_SYNC)
    q.destroy()
    # a cached batch holding q is dropped with it; p alone still works
    hfx.build_K_multi([p], [D], [torch.zeros_like(D)], flags=hfx.HFX_SYNC)


@pytest.mark.parametrize("which", [1, 3])
def test_graph_replays_match_eager(which):
    s = _systems()[which]
    plan = hfx.Plan(s)
    iters = [_density(s, plan.blocks, iteration=i) for i in range(4)]
    ref = [_eager(hfx.Plan(s), D)[0] for D in iters]
    Dd = torch.from_numpy(iters[0]).to(DEV)
    Kd = torch.zeros_like(Dd)
    plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC)          # eager: sizes the lists
    for rep in range(3):
        for i, D in enumerate(iters):
            Dd.copy_(torch.from_numpy(D).to(DEV))
            Kd.fill_(np.nan)
            info = plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH, info=True)
            # eager work of the program between replays
            _ = (Dd * 2.0).sum().item()
            err = np.max(np.abs(Kd.cpu().numpy() - ref[i]))
            assert err <= 1e-13 * max(1.0, np.max(np.abs(ref[i]))), (rep, i, err)
            assert info["n_quartets"] > 0


def test_graph_new_buffers_recapture():
    s = _systems()[1]
    plan = hfx.Plan(s)
    D = _density(s, plan.blocks)
    ref, _ = _eager(hfx.Plan(s), D)
    for _ in range(2):
        Dd = torch.from_numpy(D).to(DEV)
        Kd = torch.zeros_like(Dd)
        plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH)
        plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH)
        assert np.max(np.abs(Kd.cpu().numpy() - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_graph_list_overflow_falls_back():
    s = _tiny_cell(seed=303)
    plan = hfx.Plan(s)
    D = _density(s, plan.blocks)
    _, full = _eager(hfx.Plan(s), D)
    # a density with only the on-site blocks (I == J, n = 0) screens most
    # quartets away
    small = np.zeros_like(D)
    for b, (I, J, n1, n2, n3) in enumerate(plan.blocks):
        if I == J and n1 == n2 == n3 == 0:
            small[plan.offsets[b]:plan.offsets[b + 1]] = D[plan.offsets[b]:plan.offsets[b + 1]]
    _, sm = _eager(hfx.Plan(s), small)
    assert full["n_quartets"] > 1.3 * sm["n_quartets"] + 4096, "the two densities must differ in list size"
    ref, _ = _eager(hfx.Plan(s), D)
    Dd = torch.from_numpy(small).to(DEV)
    Kd = torch.zeros_like(Dd)
    plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC)      # sizes the lists for the small density
    plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH)     # captures with that capacity
    Dd.copy_(torch.from_numpy(D).to(DEV))
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH, info=True)   # overflows -> eager
    assert info["n_quartets"] == full["n_quartets"]
    assert np.max(np.abs(Kd.cpu().numpy() - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    info = plan.build_K(Dd, Kd, flags=hfx.HFX_GRAPH, info=True)   # recaptured, replay
    assert info["n_quartets"] == full["n_quartets"]
    assert np.max(np.abs(Kd.cpu().numpy() - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_multi_graph():
    ss = _systems()[:4]
    plans = [hfx.Plan(s) for s in ss]
    Ds = [_density(s, p.blocks) for s, p in zip(ss, plans)]
    sep = [_eager(hfx.Plan(s), D)[0] for s, D in zip(ss, Ds)]
    Dd = [torch.from_numpy(D).to(DEV) for D in Ds]
    Kd = [torch.zeros_like(d) for d in Dd]
    hfx.build_K_multi(plans, Dd, Kd, flags=hfx.HFX_SYNC)
    for _ in range(3):
        for k in Kd:
            k.fill_(np.nan)
        hfx.build_K_multi(plans, Dd, Kd, flags=hfx.HFX_GRAPH)
        for k, r in zip(Kd, sep):
            assert np.max(np.abs(k.cpu().numpy() - r)) <= 1e-13 * max(1.0, np.max(np.abs(r)))


# ------------------------------------------------------------ autotuner
def test_autotune_keeps_results_and_reports_choices():
    s = _tiny_cell(seed=304).with_(precision="mixed", fp32_cutoff=1e-6)
    plan = hfx.Plan(s)
    D = _density(s, plan.blocks)
    ref, _ = _eager(hfx.Plan(s), D)
    Dd = torch.from_numpy(D).to(DEV)
    Kd = torch.full_like(Dd, np.nan)
    rep = plan.autotune(Dd, Kd, max_quartets=5000)
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(Kd.cpu().numpy() - ref)) <= 1e-9 * scale
    timed = [r for r in rep if r["candidates"]]
    assert timed, "no class was timed"
    for r in timed:
        assert 0 <= r["chosen"] < len(r["candidates"]) or r["chosen32"] >= 0
        best = min(ms for (_, f32, _, ms) in r["candidates"] if not f32) if r["chosen"] >= 0 else None
        if best is not None:
            assert r["candidates"][r["chosen"]][3] == best
    # later builds (eager and graph) use the tuned kernels and agree
    K2 = torch.zeros_like(Dd)
    plan.build_K(Dd, K2, flags=hfx.HFX_SYNC)
    plan.build_K(Dd, K2, flags=hfx.HFX_GRAPH)
    assert np.max(np.abs(K2.cpu().numpy() - ref)) <= 1e-9 * scale
    o = oracle.Oracle(s.with_(precision="fp64"))
    o.set_density(D)
    Kref, _ = o.build_K()
    assert np.max(np.abs(K2.cpu().numpy() - Kref)) <= 1e-7
