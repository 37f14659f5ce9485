"""Continuous-batching server of exchange builds.

Requests (a system, a number of SCF iterations, an arrival time) enter a
FIFO queue.  The scheduler works in steps at the granularity of one SCF
iteration (iteration-level batching): before each step it admits queued
requests that have arrived, in arrival order, as long as their device
footprint fits under the HBM limit; the step then runs one exchange build for
every admitted request together (one fused ``hfx_build_K_multi`` launch
sequence); requests that have done all their iterations retire and free their
memory, so requests that arrived meanwhile join the next step.  Each admitted
request keeps its plan (pairs, primitive pairs, Schwarz table), its densities
and its K on the device for its whole lifetime.

The paper's own scheme for this is the two-level master/worker distribution
of quartet batches over MPI ranks (its Sec. on parallelisation); here one GPU
serves many systems at once instead.

The scheduler is independent of the device: an executor object provides
``static_footprint(request) -> bytes`` (a host-only lower bound, used to
reject requests that can never fit), ``footprint(request) -> bytes`` (the
admission size, asked for the head of the queue only), ``admit(request) ->
state``,
``step(states)`` (one build for each state, at its current iteration),
``retire(state) -> result`` and, for a step budget, ``cost(state)``.  ``HipExecutor`` is the device executor; tests
drive the scheduler with a host-only executor and a virtual clock.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Any, Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    system: Any
    n_iter: int = 10
    arrival_s: float = 0.0


@dataclasses.dataclass
class ServeResult:
    rid: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    n_iter: int
    steps: List[int]            # scheduler steps this request took part in
    result: Any = None          # executor's result (e.g. the final K)

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


@dataclasses.dataclass
class ServeStats:
    results: List[ServeResult]
    wall_s: float
    n_steps: int
    builds: int
    max_concurrent: int
    peak_reserved_bytes: int
    unfinished: List[int] = dataclasses.field(default_factory=list)  # requests cut off by stop_after_s

    def latency_percentile(self, q: float) -> float:
        return float(np.percentile([r.latency_s for r in self.results], q)) if self.results else 0.0

    @property
    def builds_per_s(self) -> float:
        return self.builds / self.wall_s if self.wall_s > 0 else 0.0

    def summary(self) -> dict:
        return {"requests": len(self.results), "builds": self.builds, "steps": self.n_steps,
                "wall_s": self.wall_s, "builds_per_s": self.builds_per_s,
                "latency_ms_p50": self.latency_percentile(50) * 1e3,
                "latency_ms_p99": self.latency_percentile(99) * 1e3,
                "max_concurrent": self.max_concurrent, "peak_reserved_bytes": self.peak_reserved_bytes,
                "unfinished_requests": len(self.unfinished)}


class Server:
    """Iteration-level continuous batching under an HBM budget."""

    def __init__(self, executor, hbm_limit_bytes: int, max_batch: int = 64, step_budget: float = 0.0,
                 clock: Optional[Callable[[], float]] = None, sleep: Optional[Callable[[float], None]] = None,
                 policy: str = "fifo", stop_after_s: float = 0.0):
        """step_budget > 0: a step runs admitted requests only while their
        summed ``executor.cost`` stays within the budget (at least one); the
        others keep their device state and wait for the next step.  0: every
        admitted request runs every step.  policy: the order in which a
        budgeted step takes requests - "fifo" (admission order), "las"
        (least attained service: the request that has had the least work so
        far first) or "srpt" (shortest remaining work first: cost of one
        build times the iterations left); the first in that order always
        runs, the rest if they fit, so that under "las" and "srpt" short
        requests are not held behind a long one.  stop_after_s > 0: no step
        starts after this time, and (with a step budget) a request is left
        out of a step when its cost at the rate the finished steps have
        shown (summed cost over summed step time) would take it past that
        time; a step that would hold no request is not started.  Unfinished
        requests are reported, not retired results."""
        if policy not in ("fifo", "las", "srpt"):
            raise ValueError("policy must be 'fifo', 'las' or 'srpt'")
        self.ex = executor
        self.limit = int(hbm_limit_bytes)
        self.max_batch = int(max_batch)
        self.budget = float(step_budget)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.policy = policy
        self.stop_after = float(stop_after_s)

    def run(self, requests: Sequence[ServeRequest]) -> ServeStats:
        queue = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        for r in queue:
            if self.ex.static_footprint(r) > self.limit:
                raise ValueError(f"request {r.rid} needs more device memory than the limit")
        t0 = self.clock()
        active = []          # [request, state, reserved bytes, iterations done, admitted time, steps, work done]
        results: List[ServeResult] = []
        reserved = 0
        peak = 0
        n_steps = 0
        builds = 0
        max_conc = 0
        qi = 0
        waiting: List[ServeRequest] = []   # arrived, not admitted
        stopped = False
        cost_done, step_time = 0.0, 0.0  # for the rate of the deadline test
        by_work = self.policy != "fifo" and hasattr(self.ex, "request_work")
        while qi < len(queue) or waiting or active:
            now = self.clock() - t0
            if self.stop_after > 0 and now >= self.stop_after:
                stopped = True
                break
            while qi < len(queue) and queue[qi].arrival_s <= now:
                waiting.append(queue[qi])
                qi += 1
            # admission while they fit: FIFO stops at the first request that
            # does not fit; "las" and "srpt" (with an executor that tells a
            # request's work) take the arrived requests with the least work
            # first and pass over those that do not fit, so that large
            # requests do not hold the memory that small ones could run in
            order = sorted(waiting, key=lambda r: (self.ex.request_work(r), r.arrival_s, r.rid)) if by_work \
                else list(waiting)
            for r in order:
                if len(active) >= self.max_batch:
                    break
                need = self.ex.footprint(r)
                if reserved + need > self.limit:
                    if by_work:
                        continue
                    break
                st = self.ex.admit(r)
                reserved += need
                peak = max(peak, reserved)
                active.append([r, st, need, 0, now, [], 0.0])
                waiting.remove(r)
            if not active:
                if waiting:
                    raise ValueError(f"request {waiting[0].rid} needs more device memory than the limit")
                # idle until the next arrival
                self.sleep(max(0.0, queue[qi].arrival_s - (self.clock() - t0)))
                continue
            run = active
            if self.budget > 0:
                if self.policy == "fifo":
                    order = active
                elif self.policy == "las":
                    order = sorted(active, key=lambda a: a[6])
                else:
                    order = sorted(active, key=lambda a: self.ex.cost(a[1]) * (a[0].n_iter - a[3]))
                rate = cost_done / step_time if step_time > 0 else 0.0
                left = self.stop_after - now if self.stop_after > 0 else float("inf")
                run, used = [], 0.0
                for a in order:
                    c = self.ex.cost(a[1])
                    late = rate > 0 and (used + c) / rate > left
                    if (run and used + c > self.budget) or late:
                        if self.policy == "fifo":
                            break
                        continue
                    run.append(a)
                    used += c
                if not run:
                    stopped = True
                    break
            max_conc = max(max_conc, len(run))
            t_step = self.clock()
            self.ex.step([a[1] for a in run])
            if self.budget > 0:
                cost_done += sum(self.ex.cost(a[1]) for a in run)
                step_time += self.clock() - t_step
            n_steps += 1
            builds += len(run)
            now = self.clock() - t0
            ran = {id(a) for a in run}
            still = []
            for a in active:
                if id(a) not in ran:
                    still.append(a)
                    continue
                a[3] += 1
                a[5].append(n_steps - 1)
                a[6] += self.ex.cost(a[1]) if self.budget > 0 else 1.0
                if a[3] >= a[0].n_iter:
                    res = self.ex.retire(a[1])
                    reserved -= a[2]
                    results.append(ServeResult(a[0].rid, a[0].arrival_s, a[4], now, a[3], a[5], res))
                else:
                    still.append(a)
            active = still
        wall = self.clock() - t0
        results.sort(key=lambda r: r.rid)
        unfinished = sorted([a[0].rid for a in active] + [r.rid for r in waiting] + [r.rid for r in queue[qi:]]) \
            if stopped else []
        for a in active:
            self.ex.retire(a[1])
        return ServeStats(results, wall, n_steps, builds, max_conc, peak, unfinished)


class HipExecutor:
    """Device executor: one ``hfx`` plan per request, densities of all its SCF
    iterations and its K resident on the device, one fused build per step.

    Footprint = the plan's device memory (``hfx_footprint``: its tables, its
    own one-plan batch and its share of a fused batch) + the densities and K
    (one allocation, rounded up to the 2 MiB segments of torch's caching
    allocator) + the quartet lists, sized from the screened count of the
    first density (``hfx_screen_count``) with 25% headroom, at most the list
    limit per list (longer lists run in chunks).  Footprints and counts are
    kept per request id, so one executor can serve a stream more than once.  Sizing a
    request makes a probe plan and uploads its first density; both are
    released before the request can be admitted, so that nothing of a
    waiting request stays on the device.  Requests whose static part alone
    exceeds the limit are rejected by the server.  ``peak_device_bytes``: the
    largest device memory in use (hipMemGetInfo, through torch) seen after a
    step, for checking the accounting against the device."""

    SEGMENT = 2 << 20

    def __init__(self, keep_results: bool = True, flags: Optional[int] = None, list_headroom: float = 1.25,
                 list_limit: int = 1 << 33, progress: Optional[Callable] = None, cache_host: bool = False):
        """list_limit: quartets a request's list holds at once (its plans are
        set to it; a longer list runs in chunks, so the list memory charged
        is at most this many quartets per list).  progress: called as
        progress(rid, list, chunk, done, total) after every finished chunk of
        a chunked build (fused builds report under their first request).
        cache_host: keep each request's host densities once made (host
        memory: n_iter x nnz doubles per request)."""
        from paper_2009_03555_amd import hfx
        import torch
        self.hfx = hfx
        self.torch = torch
        self.keep = keep_results
        self.flags = hfx.HFX_SYNC if flags is None else flags
        self.headroom = list_headroom
        self.list_limit = int(list_limit)
        self.progress = progress
        self._fp = {}
        self._nq = {}
        self._host = {}
        self.cache_host = cache_host
        self.peak_device_bytes = 0
        self.quartets_done = 0  # screened quartets (of each request's first density) of the builds run

    def _densities(self, req: ServeRequest, blocks, first_only: bool = False):
        """host densities of every SCF iteration of the request (one pass of
        the seeded generator), kept per request id with cache_host;
        first_only (without a cache): the first iteration's alone"""
        if req.rid in self._host:
            return self._host[req.rid]
        import systems
        n = 1 if (first_only and not self.cache_host) else req.n_iter
        ser = systems.density_series(req.system, np.asarray(blocks, dtype=np.int64), n)
        out = np.stack([np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0) for vals in ser])
        if self.cache_host:
            self._host[req.rid] = out
        return out

    def prepare(self, req: ServeRequest) -> None:
        """size the request and make its host densities ahead of its arrival
        (with cache_host; the densities stand for what an SCF code hands
        over, so a benchmark makes them before its timed window)"""
        self.footprint(req)

    def device_bytes_in_use(self) -> int:
        free, total = self.torch.cuda.mem_get_info()
        return int(total - free)

    def static_footprint(self, req: ServeRequest) -> int:
        dev, _ = self.hfx.hfx_footprint(req.system)
        return dev

    def footprint(self, req: ServeRequest) -> int:
        if req.rid in self._fp:
            return self._fp[req.rid]
        dev, per_q = self.hfx.hfx_footprint(req.system)
        # the list part is known only after screening: a probe plan counts
        # the quartets of the first density, then goes away
        plan = self.hfx.Plan(req.system)
        D0 = self.torch.from_numpy(self._densities(req, plan.blocks, first_only=True)[0]).cuda()
        n64, n32 = plan.screen_count(D0)
        nnz = plan.nnz
        plan.destroy()
        del D0
        dk = -(-8 * nnz * (req.n_iter + 1) // self.SEGMENT) * self.SEGMENT
        lists = sum(min(int(self.headroom * n) + 4096, self.list_limit) for n in (n64, n32) if n)
        need = dev + dk + per_q * lists
        self._fp[req.rid] = need
        self._nq[req.rid] = n64 + n32
        return need

    def admit(self, req: ServeRequest):
        self.footprint(req)
        plan = self.hfx.Plan(req.system)
        plan.set_list_limit(self.list_limit)
        if self.progress is not None:
            plan.set_progress(lambda lst, chunk, done, total, rid=req.rid: self.progress(rid, lst, chunk, done, total))
        D = self._densities(req, plan.blocks)
        # densities of every iteration and K in one device allocation
        buf = self.torch.zeros((req.n_iter + 1, plan.nnz), dtype=self.torch.float64, device="cuda")
        buf[: req.n_iter] = self.torch.from_numpy(D).cuda()
        return {"req": req, "plan": plan, "buf": buf, "it": 0, "quartets": self._nq[req.rid]}

    def cost(self, state) -> float:
        """work of one build of the request: its screened quartet count"""
        return float(state["quartets"])

    def request_work(self, req: ServeRequest) -> float:
        """work of a whole request before admission: the screened quartet
        count of its first density (from its probe) times its iterations"""
        self.footprint(req)
        return float(self._nq[req.rid]) * req.n_iter

    def step(self, states) -> None:
        plans = [s["plan"] for s in states]
        Ds = [s["buf"][s["it"]] for s in states]
        Ks = [s["buf"][-1] for s in states]
        self.hfx.build_K_multi(plans, Ds, Ks, flags=self.flags)
        self.torch.cuda.synchronize()
        self.peak_device_bytes = max(self.peak_device_bytes, self.device_bytes_in_use())
        for s in states:
            s["it"] += 1
            self.quartets_done += s["quartets"]

    def retire(self, state):
        out = state["buf"][-1].cpu().numpy() if self.keep else None
        state["plan"].destroy()
        state["buf"] = None
        return out
