"""Scheduler of the continuous-batching server on the host (no device):
a host executor with known footprints and a virtual clock."""
import numpy as np
import pytest

from paper_2009_03555_amd.serve import Server, ServeRequest


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class HostExecutor:
    """K_it = A @ D_it for a per-request matrix; a step costs a fixed time
    plus a time per request (a fused launch)."""

    def __init__(self, clock, fp, step_s=1.0, per_req_s=0.1, work_s=0.0):
        self.clock, self.fp, self.step_s, self.per_req_s, self.work_s = clock, fp, step_s, per_req_s, work_s
        self.live = {}
        self.batches = []
        self.peak_live_bytes = 0

    def static_footprint(self, r):
        return self.fp[r.rid]

    def footprint(self, r):
        return self.fp[r.rid]

    def admit(self, r):
        st = {"r": r, "it": 0, "K": np.zeros(3)}
        self.live[r.rid] = st
        self.peak_live_bytes = max(self.peak_live_bytes, sum(self.fp[k] for k in self.live))
        return st

    def step(self, states):
        self.batches.append(sorted(s["r"].rid for s in states))
        for s in states:
            rng = np.random.Generator(np.random.PCG64(1000 * s["r"].rid + s["it"]))
            s["K"] = s["K"] + rng.standard_normal(3)
            s["it"] += 1
        self.clock.t += self.step_s + self.per_req_s * len(states) + self.work_s * sum(self.cost(x) for x in states)

    def retire(self, st):
        del self.live[st["r"].rid]
        return st["K"].copy()

    def cost(self, st):
        return 1.0 + st["r"].rid % 3


def _reqs(n, gap, iters=3, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(gap, size=n))
    return [ServeRequest(rid=i, system=None, n_iter=iters, arrival_s=float(t[i])) for i in range(n)]


def _run(reqs, fp, limit, max_batch=64, budget=0.0, **cost):
    clk = VClock()
    ex = HostExecutor(clk, fp, **cost)
    st = Server(ex, limit, max_batch=max_batch, step_budget=budget, clock=clk, sleep=clk.sleep).run(reqs)
    return st, ex


def test_every_request_gets_its_iterations():
    reqs = _reqs(20, 0.5, iters=4)
    st, ex = _run(reqs, {r.rid: 10 for r in reqs}, 1000)
    assert len(st.results) == 20
    assert all(r.n_iter == 4 and len(r.steps) == 4 for r in st.results)
    assert st.builds == 80 == sum(len(b) for b in ex.batches)
    # consecutive steps: a request is never skipped while admitted
    assert all(r.steps == list(range(r.steps[0], r.steps[0] + 4)) for r in st.results)


def test_memory_limit_is_respected_and_fifo():
    reqs = _reqs(15, 0.1, iters=3)
    fp = {r.rid: 30 + 10 * (r.rid % 3) for r in reqs}
    st, ex = _run(reqs, fp, 100)
    assert ex.peak_live_bytes <= 100
    assert st.peak_reserved_bytes <= 100
    adm = [r.admitted_s for r in sorted(st.results, key=lambda r: r.rid)]
    assert adm == sorted(adm), "admission is first come, first served"


def test_arrivals_join_running_batches():
    # a long request starts alone; later ones join its steps (continuous batching)
    reqs = [ServeRequest(0, None, n_iter=10, arrival_s=0.0)] + \
           [ServeRequest(i, None, n_iter=2, arrival_s=2.0 + i) for i in range(1, 4)]
    st, ex = _run(reqs, {r.rid: 1 for r in reqs}, 100)
    assert ex.batches[0] == [0]
    assert any(len(b) > 1 and 0 in b for b in ex.batches)
    r0 = st.results[0]
    assert r0.latency_s < 10 * (1.0 + 0.1 * 4) + 1e-9


def test_result_independent_of_mix():
    # a request's results depend on its own iterations only
    solo, _ = _run([ServeRequest(7, None, n_iter=5, arrival_s=0.0)], {7: 1}, 10)
    others = [ServeRequest(100 + r.rid, None, r.n_iter, r.arrival_s) for r in _reqs(10, 0.3, iters=5)]
    st, _ = _run(others + [ServeRequest(7, None, n_iter=5, arrival_s=1.0)], {r: 1 for r in list(range(100, 110)) + [7]}, 10)
    got = [r for r in st.results if r.rid == 7][0]
    assert np.array_equal(got.result, solo.results[0].result)


def test_oversized_request_rejected():
    with pytest.raises(ValueError):
        _run([ServeRequest(0, None, 1, 0.0)], {0: 11}, 10)


def test_latency_percentiles():
    reqs = _reqs(30, 0.2, iters=2, seed=3)
    st, _ = _run(reqs, {r.rid: 1 for r in reqs}, 10, max_batch=4)
    s = st.summary()
    assert 0 < s["latency_ms_p50"] <= s["latency_ms_p99"]
    assert s["max_concurrent"] <= 4
    assert s["builds"] == 60


def test_step_budget_bounds_each_step_and_keeps_fifo():
    # compute-bound steps: a step takes time in proportion to its work
    work = dict(step_s=0.05, per_req_s=0.0, work_s=1.0)
    reqs = _reqs(12, 0.05, iters=3, seed=5)
    st, ex = _run(reqs, {r.rid: 1 for r in reqs}, 100, budget=4.0, **work)
    assert len(st.results) == 12 and st.builds == 36
    for b in ex.batches:
        cost = sum(1.0 + rid % 3 for rid in b)
        assert len(b) == 1 or cost <= 4.0
    # requests admitted earlier finish no later than those admitted after them
    fin = [r.finished_s for r in sorted(st.results, key=lambda r: (r.admitted_s, r.rid))]
    assert all(a <= b + 1e-12 for a, b in zip(fin, fin[1:]))
    # and the budgeted schedule has a lower median latency than running everyone every step
    st_all, _ = _run(reqs, {r.rid: 1 for r in reqs}, 100, **work)
    assert st.latency_percentile(50) <= st_all.latency_percentile(50)


def test_least_attained_service_lets_short_requests_past_a_long_one():
    # request 0 costs far more than the step budget; the others are short
    clock = VClock()

    class Ex(HostExecutor):
        def cost(self, st):
            return 50.0 if st["r"].rid == 0 else 1.0

    reqs = [ServeRequest(i, None, n_iter=4 if i == 0 else 2, arrival_s=0.001 * i) for i in range(6)]
    fifo = Server(Ex(clock, {i: 1 for i in range(6)}, work_s=0.1), 100, step_budget=10.0, clock=clock,
                  sleep=clock.sleep, policy="fifo").run(reqs)
    clock.t = 0.0
    las = Server(Ex(clock, {i: 1 for i in range(6)}, work_s=0.1), 100, step_budget=10.0, clock=clock,
                 sleep=clock.sleep, policy="las").run(reqs)
    lat = lambda st: {r.rid: r.latency_s for r in st.results}
    lf, ll = lat(fifo), lat(las)
    assert len(fifo.results) == len(las.results) == 6
    # under FIFO every short request waits for the long one; under LAS none does
    assert all(lf[i] > lf[0] * 0.9 for i in range(1, 6))
    assert all(ll[i] < ll[0] for i in range(1, 6))
    # the same work is done, and results do not depend on the policy
    assert fifo.builds == las.builds
    for a, b in zip(fifo.results, las.results):
        assert np.array_equal(a.result, b.result)


def test_stop_after_reports_unfinished_requests():
    clock = VClock()
    reqs = [ServeRequest(i, None, n_iter=5, arrival_s=0.5 * i) for i in range(8)]
    ex = HostExecutor(clock, {i: 1 for i in range(8)})
    st = Server(ex, 3, clock=clock, sleep=clock.sleep, stop_after_s=6.0).run(reqs)
    assert st.unfinished and len(st.results) + len(st.unfinished) == 8
    assert not ex.live  # cut-off requests were released
    assert all(r.finished_s <= 6.0 + 10.0 for r in st.results)


def test_shortest_remaining_work_first():
    clock = VClock()

    class Ex(HostExecutor):
        def cost(self, st):
            return 40.0 if st["r"].rid in (0, 2) else 1.0

    reqs = [ServeRequest(i, None, n_iter=3, arrival_s=0.001 * i) for i in range(6)]
    st = Server(Ex(clock, {i: 1 for i in range(6)}, work_s=0.1), 100, step_budget=5.0, clock=clock,
                sleep=clock.sleep, policy="srpt").run(reqs)
    lat = {r.rid: r.latency_s for r in st.results}
    assert len(st.results) == 6
    assert max(lat[i] for i in (1, 3, 4, 5)) < min(lat[0], lat[2])


def test_stop_time_keeps_out_requests_that_would_overrun_it():
    # a long request (cost 100) behind short ones: with a stop time, SRPT
    # runs the short ones, then leaves out the long one once the rate of the
    # finished steps says it would end after the stop time
    clock = VClock()

    class Ex(HostExecutor):
        def cost(self, st):
            return 100.0 if st["r"].rid == 0 else 1.0

    # the long request arrives just after the short ones: the first step
    # (short ones only) gives the rate
    reqs = [ServeRequest(i, None, n_iter=2, arrival_s=0.003 if i == 0 else 0.0) for i in range(4)]
    ex = Ex(clock, {i: 1 for i in range(4)}, step_s=0.0, per_req_s=0.0, work_s=0.1)
    st = Server(ex, 100, step_budget=5.0, clock=clock, sleep=clock.sleep, policy="srpt",
                stop_after_s=3.0).run(reqs)
    assert sorted(r.rid for r in st.results) == [1, 2, 3]
    assert st.unfinished == [0]
    assert st.wall_s <= 3.0 and not ex.live
    # without a stop time the long request runs to the end
    clock2 = VClock()
    st2 = Server(Ex(clock2, {i: 1 for i in range(4)}, step_s=0.0, per_req_s=0.0, work_s=0.1), 100,
                 step_budget=5.0, clock=clock2, sleep=clock2.sleep, policy="srpt").run(reqs)
    assert len(st2.results) == 4


def test_srpt_admission_passes_over_large_requests():
    # request 0 arrives first and would take most of the memory: FIFO
    # admission lets it hold the memory; shortest-work admission admits the
    # small requests first and request 0 once there is room
    clock = VClock()

    class Ex(HostExecutor):
        def cost(self, st):
            return 50.0 if st["r"].rid == 0 else 1.0

        def request_work(self, r):
            return (50.0 if r.rid == 0 else 1.0) * r.n_iter

    fp = {0: 8, **{i: 2 for i in range(1, 6)}}
    reqs = [ServeRequest(i, None, n_iter=3, arrival_s=0.0 if i == 0 else 0.001) for i in range(6)]
    st = Server(Ex(clock, fp, step_s=0.0, per_req_s=0.0, work_s=0.1), 10, step_budget=5.0, clock=clock,
                sleep=clock.sleep, policy="srpt").run(reqs)
    lat = {r.rid: r.latency_s for r in st.results}
    assert len(st.results) == 6
    assert max(lat[i] for i in range(1, 6)) < lat[0]
    assert st.peak_reserved_bytes <= 10
    # FIFO admission: request 0 is admitted first and the others queue behind it
    clock2 = VClock()
    st2 = Server(Ex(clock2, fp, step_s=0.0, per_req_s=0.0, work_s=0.1), 10, step_budget=5.0, clock=clock2,
                 sleep=clock2.sleep, policy="fifo").run(reqs)
    lat2 = {r.rid: r.latency_s for r in st2.results}
    assert min(lat2[i] for i in range(1, 6)) > min(lat[i] for i in range(1, 6))


def test_request_larger_than_the_limit_after_probing_is_an_error():
    clock = VClock()

    class Ex(HostExecutor):
        def static_footprint(self, r):
            return 1

        def footprint(self, r):
            return 100

    with pytest.raises(ValueError):
        Server(Ex(clock, {0: 1}), 10, clock=clock, sleep=clock.sleep).run([ServeRequest(0, None, 2, 0.0)])
