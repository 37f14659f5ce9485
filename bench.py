#!/usr/bin/env python3
"""Benchmark of the screened exchange build on one MI355X.

One step = one full exchange build (density transform + P_max, screening and
compaction, ERI + digest over every class, K finalisation) of the periodic
64-atom diamond workload (s,s,p,p,d shells, 6 primitives each, erfc operator
omega = 0.11, shell pairs within 12 bohr), with D and K resident in HBM.

Prints a JSON line after every timed build, each complete for the builds
timed so far; the last line is the result: quartets/s (unique screened
quartets per second), HFX builds/s with p50/p99 build latency, the roofline
of the dominant ERI kernel (algorithmic FP64 FLOPs per launch over its
HIP-event duration on the plan's stream), the mixed-precision form, and the
CPU oracle timed on a bounded sample of the same workload.  Warmups and
timed builds beyond one each run only inside a wall-clock budget from
process start (--budget-s), so that a run asked for many steps of a
half-minute build still ends in minutes; "steps" and "warmup" report what
actually ran.
"""
import argparse
import json
import os
import sys
import time

T_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_FP64_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


def class_labels():
    pc = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    out = []
    for cb in range(6):
        for ck in range(cb + 1):
            a, b = pc[cb]
            c, d = pc[ck]
            out.append(f"({'spd'[a]}{'spd'[b]}|{'spd'[c]}{'spd'[d]})")
    return out


def workload(name: str, precision: str):
    import systems
    if name == "diamond64":
        return systems.diamond_cell(precision=precision)
    if name == "diamond8":
        return systems.diamond_cell(n=(1, 1, 1), precision=precision)
    if name == "molecule8":
        return systems.molecule8()
    if name == "cluster256":
        return systems.cluster_k4(precision=precision)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(system, seconds: float):
    """The oracle, as it stands, on a bounded random sample of the workload's
    ordered quartets (plain loop of Eq. H-HFX), timed on this host's cores:
    samples of growing size are evaluated until the evaluation time adds up
    to about ``seconds``."""
    import oracle
    o = oracle.Oracle(system)
    D = o.density_from_system()
    o.set_density(D)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    o.eval_quartets(o.sample_quartets(32, seed=7))  # thread pool start-up, untimed
    cnt_tot, dt_tot, n, chunk = 0, 0.0, 64, 0
    while dt_tot < seconds:
        rows = o.sample_quartets(n, seed=100 + chunk)
        t = time.perf_counter()
        cnt, _ = o.eval_quartets(rows)
        dt = time.perf_counter() - t
        cnt_tot += cnt
        dt_tot += dt
        chunk += 1
        rate = cnt_tot / max(dt_tot, 1e-9)
        # next sample: the rest of the time at the rate so far, at most 4x
        n = int(max(64, min(4 * n, rate * (seconds - dt_tot) + 1)))
    ordered_rate = cnt_tot / dt_tot
    return {
        "value": ordered_rate / 8.0,
        "unit": "quartets/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{cnt_tot} ordered quartets drawn uniformly from the plain loop of the same workload "
                   f"({chunk} samples), evaluated (contracted integrals + D contraction) in {dt_tot:.1f} s; "
                   f"value = ordered rate {ordered_rate:.1f}/s divided by 8 (unique-equivalent)"),
        "cpu_model": _cpu_model(),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _build_series(plan, Dd, Kd, steps, warmup, label, deadline, reserve, on_step=None, est=0.0):
    """Warmup and timed builds of one plan inside a wall-clock budget.

    One timed build always runs, and one warmup unless a build of this plan
    already ran (est > 0: its duration).  A further timed build starts only
    if, at the duration of the last build, it ends ``reserve`` seconds before
    ``deadline`` (time.perf_counter()); a further warmup only if it also
    leaves room for min(steps, 10) timed builds (the first build loads the
    code and sizes the lists; later warmups are worth less than timed
    builds).  Returns (latencies s, infos, total timed s, warmups run)."""
    import torch
    from paper_2009_03555_amd import hfx
    w_done = 0
    for w in range(max(0 if est > 0 else 1, warmup)):
        if est > 0 and time.perf_counter() + est * (1 + min(steps, 10)) > deadline - reserve:
            break
        t = time.perf_counter()
        plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC)
        est = time.perf_counter() - t
        w_done += 1
        print(f"# {label} warmup {w}: {est:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for k in range(max(1, steps)):
        if k >= 1 and time.perf_counter() + est > deadline - reserve:
            print(f"# {label}: wall-clock budget reached after {k} timed builds", file=sys.stderr, flush=True)
            break
        t = time.perf_counter()
        info = plan.build_K(Dd, Kd, flags=hfx.HFX_TIMING, info=True)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t)
        est = lat[-1]
        infos.append(info)
        print(f"# {label} step {k}: {lat[-1]:.3f} s, {info['n_quartets']} quartets", file=sys.stderr, flush=True)
        if on_step is not None:
            on_step(lat, infos, time.perf_counter() - t0, w_done)
    torch.cuda.synchronize()
    return lat, infos, time.perf_counter() - t0, w_done


def _dens(system, plan):
    import systems
    vals = systems.density_blocks(system, plan.blocks.astype(np.int64))
    return np.concatenate([v.ravel() for v in vals]) if vals else np.zeros(0)


def bench_batch(args):
    """The batched form on the batch recipe (default: 512 independent
    clusters of 4-40 atoms, cluster recipe, each with its own seed and D):
    every cluster's plain FP64 build one after the other (per-build latency
    p50/p99), then one fused FP64 build of all of them, one fused mixed
    build (FP32 below Q_IJ Q_KL = 1e-6), and, when the fused lists fit the
    list limit whole, replays of the mixed build from a captured graph."""
    import torch
    import systems
    from paper_2009_03555_amd import hfx
    out = {}
    ss64 = systems.cluster_batch(n_clusters=args.n_clusters, n_range=tuple(args.cluster_atoms), precision="fp64")
    ssmx = [x.with_(precision="mixed", fp32_cutoff=1e-6) for x in ss64]
    p64 = [hfx.Plan(x) for x in ss64]
    pmx = [hfx.Plan(x) for x in ssmx]
    # the fused lists of all clusters (about 75 GB for the 512-cluster
    # recipe) fit the device whole: no chunks, so the graph form can run
    for p in p64 + pmx:
        p.set_list_limit(args.batch_list_limit)
    Ds = [torch.from_numpy(_dens(x, p)).cuda() for x, p in zip(ss64, p64)]
    K_sep = [torch.zeros_like(d) for d in Ds]
    atoms = [x.n_atoms for x in ss64]
    print(f"# batch: {len(ss64)} clusters, {sum(atoms)} atoms, {sum(x.n_shells for x in ss64)} shells",
          file=sys.stderr, flush=True)
    # plain: one synchronised FP64 build per cluster (the first build of
    # each plan sizes its lists; warm every plan once first)
    for p, d, k in zip(p64, Ds, K_sep):
        p.build_K(d, k, flags=hfx.HFX_SYNC)
    torch.cuda.synchronize()
    lat, nq = [], 0
    t0 = time.perf_counter()
    for p, d, k in zip(p64, Ds, K_sep):
        t = time.perf_counter()
        info = p.build_K(d, k, flags=hfx.HFX_SYNC, info=True)
        lat.append(time.perf_counter() - t)
        nq += info["n_quartets"]
    sep = time.perf_counter() - t0
    out["separate_fp64"] = {"wall_s": sep, "builds_per_s": len(p64) / sep, "quartets": nq, "quartets_per_s": nq / sep,
                            "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
                            "latency_ms_p99": float(np.percentile(lat, 99) * 1e3)}
    print(f"# separate FP64: {sep:.2f} s, {nq} quartets", file=sys.stderr, flush=True)
    K_f = [torch.zeros_like(d) for d in Ds]
    for name, plans, Ks in (("fused_fp64", p64, K_f), ("fused_mixed", pmx, [torch.zeros_like(d) for d in Ds])):
        t = time.perf_counter()
        hfx.build_K_multi(plans, Ds, Ks, flags=hfx.HFX_SYNC)  # sizes the fused lists
        torch.cuda.synchronize()
        print(f"# {name}: first (sizing) build {time.perf_counter() - t:.2f} s", file=sys.stderr, flush=True)
        t = time.perf_counter()
        info = hfx.build_K_multi(plans, Ds, Ks, flags=hfx.HFX_SYNC, info=True)
        dt = time.perf_counter() - t
        out[name] = {"wall_s": dt, "builds_per_s": len(plans) / dt, "quartets": info["n_quartets"],
                     "quartets_per_s": info["n_quartets"] / dt, "fp32_quartets": info["n_fp32_quartets"],
                     "chunks": info["n_chunks"], "speedup_vs_separate_fp64": sep / dt}
        if name == "fused_mixed":
            K_mx = Ks
            if info["n_chunks"] == 0:
                print(f"# {name}: {dt:.2f} s; capturing the graph", file=sys.stderr, flush=True)
                hfx.build_K_multi(plans, Ds, Ks, flags=hfx.HFX_GRAPH)  # capture
                torch.cuda.synchronize()
                print("# graph captured and replayed once", file=sys.stderr, flush=True)
                t = time.perf_counter()
                hfx.build_K_multi(plans, Ds, Ks, flags=hfx.HFX_GRAPH)
                dg = time.perf_counter() - t
                out["graph_mixed"] = {"wall_s": dg, "builds_per_s": len(plans) / dg, "speedup_vs_separate_fp64": sep / dg}
            else:
                out["graph_mixed"] = {"skipped": "the fused lists ran in chunks (longer than the list limit): "
                                                 "chunked builds are not graph-replayed"}
        print(f"# {name}: {dt:.2f} s, {info['n_chunks']} chunks", file=sys.stderr, flush=True)
    err_f = max(float(torch.max(torch.abs(a - b)).item()) for a, b in zip(K_f, K_sep))
    err_m = max(float(torch.max(torch.abs(a - b)).item()) for a, b in zip(K_mx, K_sep))
    out["max_abs_dK_fused_vs_separate_fp64"] = err_f
    out["max_abs_dK_mixed_vs_separate_fp64"] = err_m
    best = max(v.get("builds_per_s", 0.0) for v in out.values() if isinstance(v, dict))
    for p in p64 + pmx:
        p.destroy()
    print(json.dumps({"metric": "HFX builds/s, batched independent clusters", "unit": "builds/s",
                      "value": best, "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"{len(ss64)} clusters of {args.cluster_atoms[0]}-{args.cluster_atoms[1]} "
                                             f"atoms (heavy s,s,p,p,d / light s,s,p, 4 primitives, Coulomb), "
                                             f"{sum(atoms)} atoms in all"},
                      "forms": out}), flush=True)


def bench_spin(args):
    """Collinear spin on the 64-atom diamond workload: one spin build (both
    densities, one ERI evaluation) against two plain FP64 builds, one per
    spin density (the beta density: the alpha recipe with another seed,
    scaled by 0.4)."""
    import torch
    import systems
    from paper_2009_03555_amd import hfx
    s = workload("diamond64", "fp64")
    plan = hfx.Plan(s)
    Da = torch.from_numpy(_dens(s, plan)).cuda()
    Db = 0.4 * torch.from_numpy(_dens(s.with_(seed=s.seed + 17), plan)).cuda()
    Ka, Kb, Ks_a, Ks_b = (torch.zeros_like(Da) for _ in range(4))
    plan.build_K(Da, Ka, flags=hfx.HFX_SYNC)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ia = plan.build_K(Da, Ka, flags=hfx.HFX_SYNC, info=True)
    ib = plan.build_K(Db, Kb, flags=hfx.HFX_SYNC, info=True)
    two = time.perf_counter() - t
    print(f"# two plain builds: {two:.2f} s", file=sys.stderr, flush=True)
    plan.build_K_spin(Da, Db, Ks_a, Ks_b, flags=hfx.HFX_SYNC)
    torch.cuda.synchronize()
    t = time.perf_counter()
    isp = plan.build_K_spin(Da, Db, Ks_a, Ks_b, flags=hfx.HFX_SYNC, info=True)
    one = time.perf_counter() - t
    print(f"# one spin build: {one:.2f} s", file=sys.stderr, flush=True)
    out = {"two_plain_builds_s": two, "spin_build_s": one, "speedup": two / one,
           "quartets_plain_alpha": ia["n_quartets"], "quartets_plain_beta": ib["n_quartets"],
           "quartets_spin": isp["n_quartets"],
           "max_abs_dK_spin_vs_plain": max(float(torch.max(torch.abs(Ks_a - Ka)).item()),
                                           float(torch.max(torch.abs(Ks_b - Kb)).item()))}
    plan.destroy()
    print(json.dumps({"metric": "collinear-spin exchange build time", "unit": "s", "value": one,
                      "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": s.name + " with two spin densities"}, "forms": out}), flush=True)


def bench_kspace(args):
    """k-space assembly of the HSE06 exchange Hamiltonian of the 64-atom
    diamond workload from a K in the pattern layout, at --nk k-points."""
    import torch
    import systems
    from paper_2009_03555_amd import hfx
    s = workload("diamond64", "fp64")
    plan = hfx.Plan(s)
    K = torch.from_numpy(_dens(s, plan)).cuda()
    nbf = s.n_functions()
    rec = 2 * np.pi * np.linalg.inv(np.asarray(s.lattice)).T
    kp = np.random.default_rng(5).uniform(-0.5, 0.5, size=(args.nk, 3)) @ rec
    H = torch.empty((args.nk, nbf, nbf, 2), dtype=torch.float64, device="cuda")
    plan.kspace(K, kp, 0.25, H)
    torch.cuda.synchronize()
    reps = 5
    t = time.perf_counter()
    for _ in range(reps):
        plan.kspace(K, kp, 0.25, H)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    # algorithmic bytes: H written once (16 B per complex element), K read
    # once per k-point (8 B per value)
    byt = args.nk * (16 * nbf * nbf + 8 * plan.nnz)
    out = {"nk": args.nk, "nbf": nbf, "ms": dt * 1e3, "gb_per_s": byt / dt / 1e9, "bytes": byt}
    plan.destroy()
    print(json.dumps({"metric": "H^HFX(k) assembly time", "unit": "ms", "value": dt * 1e3,
                      "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"{s.name}, {args.nk} k-points"}, "forms": out}), flush=True)


def bench_serve(args):
    """The serving form on the request stream's recipe: Poisson arrivals at
    --rate (200/s) of clusters of 10-500 atoms (cluster recipe) and periodic
    diamond cells of 8-128 atoms (cell recipe), half and half, 10 SCF
    iterations each, HBM admission limit --hbm-gb (200 GB); the first
    --n-requests arrivals.  That stream offers orders of magnitude more work
    than one GPU does (a 300-atom cluster build alone takes minutes), so each
    form gets the same wall-clock window (--serve-seconds) from the first
    arrival and reports what it finished in it:
    offered work (screened quartets of each request's first density, times
    its iterations, from probe plans made with the requests' host densities
    before any window); plain FP64 (requests one at a time in arrival order,
    one synchronised build per iteration); served (continuous batching:
    fused builds of the admitted requests, each step within a
    --step-quartets budget in shortest-remaining-work order), FP64 and mixed
    precision.  No form starts a build that, at the rate it has shown so
    far, would end after its window.  Latency is from arrival to the last
    iteration's K."""
    import torch
    import systems
    from paper_2009_03555_amd import hfx
    from paper_2009_03555_amd.serve import HipExecutor, Server, ServeRequest

    def stream(prec):
        rq = systems.request_stream(n_requests=args.n_requests, rate_per_s=args.rate, precision=prec)
        return [ServeRequest(r.rid, r.system, r.n_iter, r.arrival_s) for r in rq]

    win = args.serve_seconds
    limit = int(args.hbm_gb * 1e9)
    out = {"window_s": win, "requests_offered": args.n_requests}

    def progress(rid, lst, chunk, done, total):
        print(f"# request {rid} list {lst}: chunk {chunk}, {done}/{total} quartets", file=sys.stderr, flush=True)

    # offered work, from the probes of the executor every form uses; the
    # requests' host densities are made here too, before the timed windows
    # (they stand for what an SCF code hands over with each request)
    exm = HipExecutor(keep_results=False, progress=progress, cache_host=True)
    reqs_m = stream("mixed")
    t = time.perf_counter()
    offered = []
    for r in reqs_m:
        exm.prepare(r)
        offered.append(exm._nq[r.rid] * r.n_iter)
        print(f"# probe {r.rid} ({r.system.name}): {exm._nq[r.rid]} quartets per build", file=sys.stderr,
              flush=True)
    out["offered_quartets"] = int(sum(offered))
    out["offered_arrival_span_s"] = reqs_m[-1].arrival_s
    out["probe_s"] = time.perf_counter() - t
    print(f"# offered: {sum(offered):.3e} quartets over {reqs_m[-1].arrival_s:.3f} s of arrivals "
          f"(probes {out['probe_s']:.1f} s)", file=sys.stderr, flush=True)
    # plain: one request at a time, arrival order, inside the window; a
    # build is not started when, at the rate of the plain builds so far, it
    # would end after the window (the queue's head then blocks the rest)
    # the FP64 stream has the mixed one's requests: the executor's probe
    # counts (per request id) serve every form
    reqs = stream("fp64")
    ex = exm
    t0 = time.perf_counter()
    lat, builds, done, q = [], 0, 0, 0
    bq, bt = 0, 0.0  # quartets and seconds of the plain builds (rate)
    blocked = None
    for r in reqs:
        now = time.perf_counter() - t0
        if now >= win:
            break
        if bt > 0 and now + exm._nq[r.rid] * bt / bq > win:
            blocked = r.rid
            break
        if now < r.arrival_s:
            time.sleep(r.arrival_s - now)
        st = ex.admit(r)
        print(f"# plain: request {r.rid} ({r.system.name}) admitted at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        finished = True
        for it in range(r.n_iter):
            now = time.perf_counter() - t0
            if now >= win or (bt > 0 and now + st["quartets"] * bt / bq > win):
                finished = False
                blocked = r.rid
                break
            tb = time.perf_counter()
            st["plan"].build_K(st["buf"][it], st["buf"][-1], flags=hfx.HFX_SYNC)
            bt += time.perf_counter() - tb
            bq += st["quartets"]
            builds += 1
            q += st["quartets"]
        ex.retire(st)
        if finished:
            done += 1
            lat.append(time.perf_counter() - t0 - r.arrival_s)
        if blocked is not None:
            break
    wall = time.perf_counter() - t0
    # every form is charged the whole window (a form that stops early,
    # blocked or out of work that fits, has used it)
    span = max(wall, win)
    out["plain_fp64"] = {"builds": builds, "builds_per_s": builds / span, "quartets_per_s_est": q / span,
                         "requests_done": done, "wall_s": wall, "blocked_by_request": blocked,
                         "latency_ms_p50": float(np.percentile(lat, 50) * 1e3) if lat else None,
                         "latency_ms_p99": float(np.percentile(lat, 99) * 1e3) if lat else None}
    print(f"# plain fp64: {builds} builds, {done} requests done in {wall:.1f} s", file=sys.stderr, flush=True)
    for prec in ("mixed", "fp64"):
        exm.quartets_done = 0
        st = Server(exm, limit, step_budget=args.step_quartets, policy="srpt",
                    stop_after_s=win).run(reqs_m if prec == "mixed" else stream("fp64"))
        d = st.summary()
        span = max(st.wall_s, win)
        d["builds_per_s"] = st.builds / span
        d["quartets_per_s_est"] = exm.quartets_done / span
        out[f"served_{prec}"] = d
        print(f"# served {prec}: {st.builds} builds, {len(st.results)} requests done in {st.wall_s:.1f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(json.dumps({"metric": "HFX builds/s (p50/p99 latency), served SCF request stream", "unit": "builds/s",
                      "value": out["served_mixed"]["builds_per_s"], "higher_is_better": True, "n_gpus": 1,
                      "data": "synthetic",
                      "config": {"workload": f"first {args.n_requests} requests of the Poisson stream at "
                                             f"{args.rate}/s (clusters 10-500 atoms, diamond cells 8-128 atoms, "
                                             f"10 SCF iterations each, HBM limit {args.hbm_gb} GB), "
                                             f"{win:.0f} s window (overloaded)"},
                      "forms": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diamond64")
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"],
                    help="fp64: the plain form only; both: also the mixed-precision form, its "
                         "throughput and max|dK| against the FP64 build")
    ap.add_argument("--fp32-cutoff", type=float, default=1e-4,
                    help="mixed form: quartets with Q_IJ*Q_KL below this take the FP32 recursion")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget from process start: warmups and timed builds beyond the "
                         "requested minimum (one each) start only if they end inside it; the JSON line "
                         "reports the steps actually timed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-clusters", type=int, default=512, help="batch workload: number of clusters")
    ap.add_argument("--cluster-atoms", type=int, nargs=2, default=(4, 40),
                    help="batch workload: atom counts drawn uniformly from this range")
    ap.add_argument("--n-requests", type=int, default=40, help="serve workload: first arrivals of the stream")
    ap.add_argument("--serve-seconds", type=float, default=120.0, help="serve workload: window per form")
    ap.add_argument("--rate", type=float, default=200.0, help="serve workload arrivals per second")
    ap.add_argument("--hbm-gb", type=float, default=200.0, help="serve workload admission limit")
    ap.add_argument("--step-quartets", type=float, default=3e8,
                    help="serve workload: screened quartets one scheduler step may take on")
    ap.add_argument("--nk", type=int, default=8, help="kspace workload: k-points")
    ap.add_argument("--batch-list-limit", type=int, default=1 << 34,
                    help="batch workload: quartets a fused list may hold (more run in chunks)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="first run one plain device-to-device copy of this many GiB (a reference "
                         "dispatch of known traffic for hardware-counter runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the exchange build shards by quartet ranges with one sparse-K all-reduce; "
              "that design is documented but not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_03555_amd import hfx

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    import systems
    if args.copy_gib > 0:
        n = int(args.copy_gib * (1 << 30)) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# reference copy: {n * 8} bytes read, {n * 8} bytes written", file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "spin":
        return bench_spin(args)
    if args.workload == "kspace":
        return bench_kspace(args)

    prec = "fp64" if args.precision in ("fp64", "both") else "mixed"
    s = workload(args.workload, prec)
    if prec == "mixed":
        s = s.with_(fp32_cutoff=args.fp32_cutoff, name=s.name)
    plan = hfx.Plan(s)
    D = np.concatenate([v.ravel() for v in systems.density_blocks(s, plan.blocks.astype(np.int64))])
    Dd = torch.from_numpy(D).cuda()
    Kd = torch.zeros_like(Dd)
    plan.schwarz()
    torch.cuda.synchronize()
    print(f"# {s.name}: {s.n_atoms} atoms, {s.n_shells} shells, {plan.n_blocks} blocks, nnz {plan.nnz}",
          file=sys.stderr, flush=True)
    deadline = T_START + args.budget_s
    # what has to fit after the plain series: the CPU baseline and, with
    # --precision both, one warmup and one timed mixed build (about the
    # plain build's duration each; the first plain warmup tells)
    cpu_reserve = 0.0 if args.no_cpu_baseline else args.cpu_seconds + 10.0
    labels = class_labels()
    state = {}

    def record(lat, infos, total, w_done):
        # w_done + 1: the first build (below) is a warmup too
        state["out"] = _line(args, s, plan, prec, lat, infos, total, w_done + 1, labels)
        if state.get("mixed") is not None:
            state["out"]["mixed"] = state["mixed"]
        if state.get("cpu") is not None:
            state["out"]["cpu_baseline"] = state["cpu"]
        # provisional line of the steps so far (stderr: stdout gets one line)
        print("# provisional: " + json.dumps(state["out"]), file=sys.stderr, flush=True)

    first = {}

    def reserve_plain():
        # the mixed form needs two builds at roughly the plain build's time
        est = first.get("est", 0.0)
        return cpu_reserve + (2.2 * est if args.precision == "both" else 0.0)

    # a first warmup sizes the reserve of the mixed block
    t = time.perf_counter()
    plan.build_K(Dd, Kd, flags=hfx.HFX_SYNC)
    first["est"] = time.perf_counter() - t
    print(f"# {prec} first build: {first['est']:.2f} s", file=sys.stderr, flush=True)
    lat, infos, total, w_done = _build_series(plan, Dd, Kd, args.steps, args.warmup - 1, prec, deadline,
                                              reserve_plain(), on_step=record, est=first["est"])
    w_done += 1
    out = state["out"]
    if args.precision == "both":
        K64 = Kd.clone()
        if time.perf_counter() + 2.0 * first["est"] <= deadline - cpu_reserve:
            smx = s.with_(precision="mixed", fp32_cutoff=args.fp32_cutoff, name=s.name)
            pmx = hfx.Plan(smx)
            Kmx = torch.zeros_like(Dd)
            pmx.schwarz()
            lat_m, inf_m, tot_m, wm = _build_series(pmx, Dd, Kmx, args.steps, 1, "mixed", deadline, cpu_reserve)
            err = float(torch.max(torch.abs(Kmx - K64)).item())
            state["mixed"] = {
                "fp32_cutoff": smx.fp32_cutoff,
                "steps": len(lat_m),
                "warmup": wm,
                "quartets_per_s": inf_m[-1]["n_quartets"] * len(lat_m) / tot_m,
                "builds_per_s": len(lat_m) / tot_m,
                "latency_ms_p50": float(np.percentile(lat_m, 50) * 1e3),
                "latency_ms_p99": float(np.percentile(lat_m, 99) * 1e3),
                "fp32_quartets": inf_m[-1]["n_fp32_quartets"],
                "quartets_per_build": inf_m[-1]["n_quartets"],
                "max_abs_dK_vs_fp64": err,
                "speedup_vs_fp64": (len(lat_m) / tot_m) / (len(lat) / total),
                "phase_ms": {k: float(np.mean([i[k] for i in inf_m])) for k in
                             ("ms_density", "ms_screen", "ms_eri", "ms_finalize", "ms_total")},
            }
            pmx.destroy()
        else:
            state["mixed"] = {"skipped": "wall-clock budget"}
        out["mixed"] = state["mixed"]
    if not args.no_cpu_baseline:
        cpu_s = max(2.0, min(args.cpu_seconds, deadline - time.perf_counter() - 5.0))
        state["cpu"] = cpu_baseline(s, cpu_s)
        # extrapolated, not measured: one whole build at the sampled rate
        state["cpu"]["full_build_s_extrapolated"] = infos[-1]["n_quartets"] / state["cpu"]["value"]
        out["cpu_baseline"] = state["cpu"]
    print(json.dumps(out), flush=True)


def _line(args, s, plan, prec, lat, infos, total, w_done, labels):
    """The bench JSON object of the timed builds so far."""
    steps = len(lat)
    nq = infos[-1]["n_quartets"]
    value = nq * steps / total
    ms_class = np.mean([i["ms_class"] for i in infos], axis=0)
    fl_class = np.mean([i["flops_class"] for i in infos], axis=0)
    dom = int(np.argmax(ms_class))
    achieved = fl_class[dom] / (ms_class[dom] * 1e-3) / 1e12
    eri_tflops = np.mean([i["flops"] / (i["ms_eri"] * 1e-3) / 1e12 for i in infos])
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tj = json.load(open(tpath))
            ent = tj.get(args.workload, {}).get(labels[dom])
            if ent and ent.get("kernel_hash") == kernel_hash():
                traffic = ent["bytes_per_launch"]
        except (OSError, ValueError):
            traffic = None
    return {
        "metric": "screened ERI quartets/s + HFX builds/s (p50/p99 latency) at max|ΔK|≤1e-7",
        "value": value,
        "unit": "quartets/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": w_done,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "budget_s": args.budget_s,
        "ms_per_step": total / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": s.name, "n_atoms": s.n_atoms, "n_shells": s.n_shells,
                   "n_basis": s.n_functions(), "periodic": s.periodic, "op": s.op, "omega": s.omega,
                   "pair_cutoff": s.pair_cutoff, "tau": s.tau, "precision": prec,
                   **({"fp32_cutoff": s.fp32_cutoff} if prec == "mixed" else {}),
                   "n_blocks": plan.n_blocks, "nnz": plan.nnz},
        "builds_per_s": steps / total,
        "latency_ms_p50": float(np.percentile(lat, 50) * 1e3),
        "latency_ms_p99": float(np.percentile(lat, 99) * 1e3),
        "quartets_per_build": nq,
        "prim_quartets_per_build": infos[-1]["n_prim_quartets"],
        "phase_ms": {k: float(np.mean([i[k] for i in infos])) for k in
                     ("ms_density", "ms_screen", "ms_eri", "ms_finalize", "ms_total")},
        "eri_phase_tflops": float(eri_tflops),
        "roofline": {"bound": "alu", "kernel": f"ERI+digest {labels[dom]}", "achieved": float(achieved),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": float(achieved / PEAK_FP64_TFLOPS),
                     "traffic": traffic},
        "classes": {labels[r]: {"quartets": int(infos[-1]["n_quartets_class"][r]), "ms": float(ms_class[r]),
                                "tflops": float(fl_class[r] / max(ms_class[r], 1e-9) / 1e9)}
                    for r in range(21) if infos[-1]["n_quartets_class"][r]},
        "mixed": None,
        "cpu_baseline": None,
    }


def kernel_hash():
    """Hash of the sources the ERI class kernels are compiled from (their
    translation units eri_*.hip and every header); traffic counters are
    valid only for it.  The auxiliary kernels (k_aux.hip) are not part of it."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2009_03555_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith(".hpp") or (f.startswith("eri_") and f.endswith(".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
