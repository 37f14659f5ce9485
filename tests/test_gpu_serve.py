"""GPU: the continuous-batching server.  A request's K is the same alone and
in a mix of requests that arrive while it runs (within 1e-12 relative: only
the order of the floating-point atomic additions differs), equals a direct
build with its last density, and equals the oracle's K of that density
(1e-10 in FP64, 1e-7 for the mixed-precision request)."""
import numpy as np
import pytest

import oracle
import systems

torch = pytest.importorskip("torch")
hfx = pytest.importorskip("paper_2009_03555_amd.hfx")
from paper_2009_03555_amd.serve import HipExecutor, Server, ServeRequest  # noqa: E402

pytestmark = pytest.mark.gpu


def _tiny_cell(seed, **kw):
    return systems.diamond_cell(seed=seed, n=(1, 1, 1), nprim=2, shells=(0, 1, 2), r_cut=4.6, **kw)


def _requests():
    return [
        # a build here takes milliseconds: the first request runs 8
        # iterations, the others arrive within its first one or two
        ServeRequest(0, _tiny_cell(501), n_iter=8, arrival_s=0.0),
        ServeRequest(1, systems.molecule8(seed=502), n_iter=3, arrival_s=0.0005),
        ServeRequest(2, _tiny_cell(503).with_(precision="mixed", fp32_cutoff=1e-6), n_iter=3, arrival_s=0.001),
        ServeRequest(3, systems.random_cluster(5, 504, nprim=2, op="coulomb"), n_iter=2, arrival_s=0.0015),
        ServeRequest(4, systems.molecule8(seed=505).with_(op="erfc", omega=0.2), n_iter=2, arrival_s=0.002),
    ]


def test_alone_equals_in_mix_and_direct_build():
    reqs = _requests()
    solo = Server(HipExecutor(), 1 << 40).run([reqs[0]])
    mix = Server(HipExecutor(), 1 << 40).run(reqs)
    assert len(mix.results) == len(reqs)
    assert mix.max_concurrent >= 2, "later arrivals must join the running request"
    K_solo = solo.results[0].result
    K_mix = mix.results[0].result
    scale = max(1.0, np.max(np.abs(K_solo)))
    assert np.max(np.abs(K_mix - K_solo)) <= 1e-12 * scale
    # every result equals a direct build with the request's last density
    for r, res in zip(reqs, mix.results):
        plan = hfx.Plan(r.system)
        vals = systems.perturb_density(r.system, plan.blocks.astype(np.int64), r.n_iter - 1)
        Dh = np.concatenate([v.ravel() for v in vals])
        D = torch.from_numpy(Dh).cuda()
        K = torch.zeros_like(D)
        plan.build_K(D, K, flags=hfx.HFX_SYNC)
        ref = K.cpu().numpy()
        assert np.max(np.abs(res.result - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), r.rid
        o = oracle.Oracle(r.system)
        o.set_density(Dh)
        Ko, _ = o.build_K()
        tol = 1e-10 if r.system.precision == "fp64" else 1e-7
        err = np.max(np.abs(res.result - Ko))
        print(f"request {r.rid} ({r.system.name}, {r.system.precision}): max|dK| vs oracle {err:.3e}")
        assert err <= tol, r.rid
    s = mix.summary()
    assert s["builds"] == sum(r.n_iter for r in reqs)
    assert 0 < s["latency_ms_p50"] <= s["latency_ms_p99"]


def test_admission_under_a_tight_limit():
    reqs = _requests()[:3]
    ex = HipExecutor()
    need = [ex.footprint(r) for r in reqs]
    limit = max(need) + min(need) - 1          # never all three at once
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = ex.device_bytes_in_use()
    st = Server(ex, limit).run(reqs)
    assert st.peak_reserved_bytes <= limit
    assert len(st.results) == 3
    # the device agrees with the accounting: the memory the admitted
    # requests really hold (plans, batches, lists, densities and K) stays
    # within the limit, up to the allocators' page rounding of each of a
    # plan's few dozen allocations
    used = ex.peak_device_bytes - base
    print(f"admission: limit {limit} B, accounted peak {st.peak_reserved_bytes} B, device peak {used} B")
    assert used <= limit + 2 * (4 << 20)
