"""Full-size run of the mixed-precision cluster workload (256 atoms at 0.1
atoms/bohr^3, heavy s,s,p,p,d and light s,s,p atoms, 4 primitives, bare
Coulomb, FP32 allowed below Q_IJ Q_KL = 1e-6) on the GPU, with the mixed
build's error against the FP64 oracle reported per K block.

Not collected by pytest (minutes of GPU time, tens of minutes of host time
for the oracle's blocks, whose rows keep nearly every candidate quartet on
this diffuse basis).  Run as
``python tests/fullsize_cluster256.py --gpu-out P --forms fp64`` and
``... --gpu-out P --forms mixed`` on the GPU (counts, the timed build with a
progress line per list chunk, K saved to P_fp64.npz / P_mixed.npz and a
JSON line), then ``python tests/fullsize_cluster256.py --check P`` on any host
(mixed against FP64 on every element when both were saved, the oracle on
the seeded blocks, per-block errors of each saved form, a JSON line);
without --gpu-out or --check everything runs in one process.
Steps: screened counts (FP64 and FP32 lists); one FP64 and one mixed build,
timed, with the lists evaluated in chunks of at most the list limit; the
oracle's K on a seeded sample of K blocks (half uniform over the pattern,
half among blocks of shells within 5 bohr, where K is large), with the
Schwarz factors of only the rows those blocks need; per sampled block the
largest |dK| of the mixed and of the FP64 build against the oracle; the
mixed build against the FP64 build on every element.  Prints one JSON
object (and writes it to --out)."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--blocks", type=int, default=32)
    ap.add_argument("--list-limit", type=int, default=0, help="quartets per list chunk (0: the library default)")
    ap.add_argument("--atoms", type=int, default=256)
    ap.add_argument("--out", default="")
    ap.add_argument("--gpu-out", default="", help="GPU part only: save the sampled blocks' K here (.npz)")
    ap.add_argument("--check", default="", help="host part only: oracle against the K saved by --gpu-out")
    ap.add_argument("--forms", nargs="+", default=["fp64", "mixed"], choices=["fp64", "mixed"],
                    help="GPU part: which builds to run (both are needed for the check)")
    ap.add_argument("--oracle-cache", default="", help="host part: .npz holding (or to hold) the oracle's blocks")
    ap.add_argument("--oracle-only", action="store_true", help="host part: only compute (and cache) the oracle")
    ap.add_argument("--stride", type=int, default=1,
                    help="host part: check every stride-th saved block only (the oracle needs minutes per block)")
    args = ap.parse_args()

    def log(msg):
        print(f"# {msg}", file=sys.stderr, flush=True)

    import systems
    smx = systems.cluster_k4(n_atoms=args.atoms)
    s64 = smx.with_(precision="fp64")
    if args.check:
        return check(args, s64, log)
    import torch
    from paper_2009_03555_amd import hfx
    out = {"workload": smx.name, "n_atoms": smx.n_atoms, "n_shells": smx.n_shells,
           "n_basis": smx.n_functions(), "fp32_cutoff": smx.fp32_cutoff, "tau": smx.tau}
    forms = {"fp64": s64, "mixed": smx}
    K = {}
    for name in args.forms:
        plan = hfx.Plan(forms[name])
        if args.list_limit:
            plan.set_list_limit(args.list_limit)
        if "n_blocks" not in out:
            log(f"{smx.name}: {smx.n_shells} shells, {plan.n_blocks} blocks, nnz {plan.nnz}")
            D = np.concatenate([v.ravel() for v in systems.density_blocks(s64, plan.blocks.astype(np.int64))])
            Dd = torch.from_numpy(D).cuda()
            out.update(n_blocks=plan.n_blocks, nnz=plan.nnz)
        n64, n32 = plan.screen_count(Dd)
        log(f"{name}: screened {n64} + {n32} quartets (FP64 + FP32 lists)")
        plan.set_progress(lambda lst, chunk, done, total, name=name:
                          log(f"{name} list {lst}: chunk {chunk} done, {done}/{total} quartets"))
        Kd = torch.zeros_like(Dd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = plan.build_K(Dd, Kd, flags=hfx.HFX_TIMING, info=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = {"build_s": dt, "quartets": info["n_quartets"], "quartets_per_s": info["n_quartets"] / dt,
                     "fp32_quartets": info["n_fp32_quartets"], "fp32_fraction": info["n_fp32_quartets"] / max(
                         1, info["n_quartets"]), "prim_quartets": info["n_prim_quartets"],
                     "chunks": info["n_chunks"], "flops_algorithmic": info["flops"],
                     "eri_tflops_algorithmic": info["flops"] / dt / 1e12}
        log(f"{name} build: {dt:.1f} s, {info['n_quartets']} quartets, {info['n_chunks']} chunks, "
            f"{info['n_fp32_quartets']} FP32")
        K[name] = Kd.cpu().numpy()
        plan.destroy()
    if args.gpu_out:
        for name, k in K.items():
            np.savez(f"{args.gpu_out}_{name}.npz", k=k, summary=json.dumps(out))
        print(json.dumps(out), flush=True)
        return 0
    for name, k in K.items():
        np.savez(f"/tmp/_cluster256_{name}.npz", k=k, summary=json.dumps(out))
    args.check = "/tmp/_cluster256"
    return check(args, s64, log)


def sample_blocks(system, blocks, n):
    """Seeded K blocks: half uniform over the pattern, half among blocks of
    shells within 5 bohr (where K is large)."""
    blocks = np.asarray(blocks, dtype=np.int64)
    rng = np.random.default_rng(3003)
    xyz = np.asarray(system.atom_xyz)[np.asarray(system.shell_atom)]
    dist = np.linalg.norm(xyz[blocks[:, 0]] - xyz[blocks[:, 1]], axis=1)
    near = np.flatnonzero(dist < 5.0)
    half = n // 2
    return np.unique(np.concatenate([rng.choice(len(blocks), n - half, replace=False),
                                     rng.choice(near, half, replace=False)]))


def oracle_blocks(args, s64, log):
    """The oracle's K on the seeded sample of blocks (every stride-th), with
    the Schwarz factors of only the rows they need; cached in
    --oracle-cache if given (the oracle needs minutes per block here)."""
    import oracle
    o = oracle.Oracle(s64)
    blocks = o.blocks.astype(np.int64)
    sel = sample_blocks(s64, blocks, args.blocks)[::max(1, args.stride)]
    if args.oracle_cache and os.path.exists(args.oracle_cache):
        z = np.load(args.oracle_cache)
        if np.array_equal(z["sel"], sel):
            log(f"oracle: {len(sel)} K blocks from {args.oracle_cache}")
            return o, blocks, sel, z["K"], int(z["nterms"]), float(z["seconds"])
    t = time.perf_counter()
    o.schwarz_rows(np.concatenate([blocks[sel, 0], blocks[sel, 1]]))
    o.set_density(o.density_from_system())
    Kref, nterms = o.build_K(blocks=sel)
    dt = time.perf_counter() - t
    log(f"oracle: {len(sel)} K blocks, {nterms} ordered quartets, {dt:.1f} s")
    if args.oracle_cache:
        np.savez(args.oracle_cache, sel=sel, K=Kref, nterms=nterms, seconds=dt)
    return o, blocks, sel, Kref, nterms, dt


def check(args, s64, log):
    o, blocks, sel, Kref, nterms, dt = oracle_blocks(args, s64, log)
    if args.oracle_only:
        return 0
    # the forms whose K the GPU part saved (both, or one of them)
    zs = {name: np.load(f"{args.check}_{name}.npz") for name in ("fp64", "mixed")
          if os.path.exists(f"{args.check}_{name}.npz")}
    if not zs:
        raise SystemExit(f"no {args.check}_fp64.npz or {args.check}_mixed.npz")
    out = {}
    for name, z in zs.items():
        out.update(json.loads(str(z["summary"])))
    ks = {name: z["k"] for name, z in zs.items()}
    out["max_abs_K"] = float(max(np.max(np.abs(k)) for k in ks.values()))
    if len(ks) == 2:
        out["max_abs_dK_mixed_vs_fp64_all"] = float(np.max(np.abs(ks["mixed"] - ks["fp64"])))
        out["speedup_mixed_vs_fp64"] = out["fp64"]["build_s"] / out["mixed"]["build_s"]
        log(f"mixed vs FP64 on every element: {out['max_abs_dK_mixed_vs_fp64_all']:.3e}")
    per = []
    for b in sel:
        a, e = o.offsets[b], o.offsets[b + 1]
        ref = Kref[a:e]
        row = {"block": [int(v) for v in blocks[b]], "max_abs_K": float(np.max(np.abs(ref)))}
        for name, k in ks.items():
            row[f"max_abs_dK_{name}"] = float(np.max(np.abs(k[a:e] - ref)))
        per.append(row)
    out["oracle_blocks"] = per
    out["oracle_K_blocks"] = len(sel)
    out["oracle_ordered_quartets"] = int(nterms)
    out["oracle_s"] = dt
    bars = {"fp64": 1e-10, "mixed": 1e-7}
    ok = True
    for name in ks:
        out[f"max_abs_dK_{name}_vs_oracle"] = max(p[f"max_abs_dK_{name}"] for p in per)
        log(f"per-block max|dK| vs oracle, {name}: {out[f'max_abs_dK_{name}_vs_oracle']:.3e}")
        ok = ok and out[f"max_abs_dK_{name}_vs_oracle"] <= bars[name]
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
