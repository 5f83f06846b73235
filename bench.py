"""Benchmark of the BPMF sampling hot path on one MI355X.

Workload (default): the production-size single-ligand system -- a 48-atom
ligand, three float32 receptor grids of 128^3 nodes at 0.25 A from 2000
point atoms, 64 replicas on a coupled temperature/lambda ladder (600 K,
lambda 0 -> 300 K, lambda 1).  One step is one pass of the whole hot path:
5000 sweeps of (one 20-step velocity-Verlet HMC move per replica + one
neighbour replica-exchange sweep), a recorded sample per state every 10
sweeps, the 64 x 32000 float64 reduced-energy matrix u_kn recomputed from the
recorded configurations, and MBAR on it (BPMF_syn = f_{K-1} - f_0).
Replicas carry over from step to step (a production run in cycles).

value = atom-grid energy+force evaluations of the HMC moves per second of
whole-step time; one evaluation = one atom's trilinear interpolation of the
three grids with gradient (96 algorithmic grid bytes) plus its share of the
bonded terms and restraint.

A second leg ("batched") runs the batched workload -- 256 ligands of 10-80
atoms with 32 replicas each on one shared 160^3 grid, 2000 sweeps of 10
steps, per-ligand u_kn and MBAR -- with the launch shape picked by the
autotuner; --config 3 makes it the main workload instead.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
GRID_BYTES_PER_EVAL = 96  # 8 corners x 3 channels x 4 B


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", type=int, default=2)
    p.add_argument("--sweeps", type=int, default=None,
                   help="override sweeps per step (default: the workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-batched", dest="batched", action="store_false",
                   help="skip the batched 256-ligand leg")
    return p.parse_args()


def cpu_baseline(system, target_s):
    """The FP64 oracle running the same sweeps on the host cores, on a
    bounded number of sweeps."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    lig = system.ligands[0]
    og, ol = oracle.OGrid(system.grid), oracle.OLigand(lig)
    s = oracle.Sampler(og, ol, seed=system.seed, x0=lig.x0)
    L = system.n_leapfrog
    t0 = time.perf_counter()
    s.sweep(nleap=L, exchange_every=1)
    one = time.perf_counter() - t0
    n = max(2, int(target_s / max(one, 1e-4)))
    t0 = time.perf_counter()
    for _ in range(n):
        s.sweep(nleap=L, exchange_every=1)
    el = time.perf_counter() - t0
    evals = n * ol.K * lig.n_atoms * (L + 1)
    return dict(value=evals / el, unit="atom-evals/s",
                cores=int(oracle.num_threads()), kind="oracle",
                sample=f"{n} sweeps of the {system.name} workload "
                       f"({ol.K} replicas x {lig.n_atoms} atoms x {L + 1} "
                       f"energy+force evaluations per sweep, plus exchange), "
                       f"{el:.1f} s")


def run_workload(pkg, torch, system, steps, warmup, sweeps=None,
                 tune=False):
    """Set up every ligand of `system`, run `warmup` + `steps` timed steps
    of the hot path and return the measurements."""
    import numpy as np
    g = system.grid
    ligs = system.ligands
    L = system.n_leapfrog
    sweeps = sweeps or system.n_sweeps
    every = system.sample_every
    records = sweeps // every
    t_setup = time.perf_counter()
    ctx = pkg.Context(seed=system.seed, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    ids = [ctx.ligand_setup(l, sample_capacity=records) for l in ligs]
    ukn = [torch.empty((l.n_states, records * l.n_states),
                       dtype=torch.float64, device="cuda:0") for l in ligs]
    Nk = [np.full(l.n_states, records, np.int64) for l in ligs]
    tuned = None
    if tune:
        sig = (f"{system.name}|L{L}|" +
               ",".join(f"{l.n_atoms}x{l.n_states}" for l in ligs))
        cache = os.environ.get("BPMF_TUNE_CACHE", os.path.join(
            os.path.expanduser("~"), ".cache", "bpmf_autotune.json"))
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        chosen, table = ctx.autotune(n_sweeps=64, n_leapfrog=L,
                                     cache_path=cache, signature=sig)
        tuned = {"chosen_waves": chosen or "auto", "sweep_ms": table}
    setup_s = time.perf_counter() - t_setup
    results = []
    # MBAR of each cycle starts from the previous cycle's free energies
    f_prev = [None] * len(ids)

    def step():
        for i in ids:
            ctx.reset_samples(i)
        ctx.hmc_sweep(sweeps, L, exchange_every=1, exchange_scheme=0,
                      sample_every=every)
        out = []
        for q, (i, u, nk) in enumerate(zip(ids, ukn, Nk)):
            ctx.energy_matrix(i, None, n_samples=u.shape[1], out=u)
            r = ctx.mbar(u, nk, tol=1e-10, max_iter=100, f_init=f_prev[q])
            f_prev[q] = r[0] if np.all(np.isfinite(r[0])) else None
            out.append(r)
        return out

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True, every=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        results = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hmc_ms, hmc_n = ctx.get_timing(ctx.TIMER_HMC)
    cmp_ms, cmp_n = ctx.get_timing(ctx.TIMER_COMPONENTS)
    ctx.set_timing(False)
    stats = [ctx.get_stats(i) for i in ids]
    waves = sorted({ctx.get_waves(i) for i in ids})
    ctx.close()

    ms_per_step = el / steps * 1e3
    evals_per_sweep = sum(l.n_states * l.n_atoms for l in ligs) * (L + 1)
    value = sweeps * evals_per_sweep / (ms_per_step * 1e-3)
    achieved = evals_per_sweep * GRID_BYTES_PER_EVAL / (hmc_ms * 1e-3) / 1e9
    f, var, it = results[0]
    acc = sum(st["hmc_acc"].sum() for st in stats) / max(
        sum(st["hmc_try"].sum() for st in stats), 1)
    exa = sum(st["ex_acc"].sum() for st in stats) / max(
        sum(st["ex_try"].sum() for st in stats), 1)
    bpmf = np.array([r[0][-1] - r[0][0] for r in results])
    return dict(value=value, ms_per_step=ms_per_step, sweeps=sweeps,
                records=records, hmc_ms=hmc_ms, hmc_n=hmc_n, cmp_ms=cmp_ms,
                achieved=achieved, evals_per_sweep=evals_per_sweep,
                setup_s=setup_s, waves=waves, tuned=tuned,
                result={"bpmf_syn_kT": float(f[-1] - f[0]) if len(results)
                        == 1 else None,
                        "sigma_kT": float(np.sqrt(max(var[-1], 0.0))),
                        "mbar_iterations": int(it),
                        "bpmf_syn_kT_mean": float(bpmf.mean()),
                        "bpmf_syn_kT_range": [float(bpmf.min()),
                                              float(bpmf.max())],
                        "hmc_acceptance": float(acc),
                        "exchange_acceptance": float(exa)})


def describe(system, r):
    ligs = system.ligands
    g = system.grid
    L = system.n_leapfrog
    R = sum(l.n_states for l in ligs)
    if len(ligs) == 1:
        l = ligs[0]
        what = (f"{system.name}: {l.n_atoms}-atom ligand, {g.n[0]}^3 x 3 "
                f"float32 grids at {g.spacing} A, {R} replicas, "
                f"{r['sweeps']} sweeps x {L} leapfrog steps + neighbour "
                f"exchange, u_kn {l.n_states}x{r['records'] * l.n_states} "
                f"float64, MBAR")
    else:
        counts = [l.n_atoms for l in ligs]
        what = (f"{system.name}: {len(ligs)} ligands of {min(counts)}-"
                f"{max(counts)} atoms x {ligs[0].n_states} replicas ({R} "
                f"replicas), shared {g.n[0]}^3 x 3 float32 grids at "
                f"{g.spacing} A, {r['sweeps']} sweeps x {L} leapfrog steps "
                f"+ neighbour exchange, per-ligand u_kn and MBAR")
    return {"workload": what, "ligands": len(ligs), "replicas": R,
            "atoms": [l.n_atoms for l in ligs] if len(ligs) <= 4 else
            f"{sum(l.n_atoms for l in ligs)} total",
            "sweeps_per_step": r["sweeps"], "leapfrog": L,
            "samples_per_state": r["records"]}


def roofline(r):
    return {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS,
            "traffic": None, "kernel": "k_hmc_sweep",
            "mean_launch_ms": r["hmc_ms"], "launches_timed": r["hmc_n"],
            "algorithmic_bytes_per_launch": r["evals_per_sweep"] *
            GRID_BYTES_PER_EVAL}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the "
              "path shards by ligand/replica range without collectives, see "
              "the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    import paper_1507_03703_amd as pkg

    system = synth.make_system(args.config, grid_device="cuda:0")
    r = run_workload(pkg, torch, system, args.steps, args.warmup,
                     sweeps=args.sweeps, tune=len(system.ligands) > 1)
    out = {
        "metric": "atom-grid energy+force evals/s & HBM fraction; effective "
                  "samples/s vs plain HMC",
        "value": r["value"],
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": describe(system, r),
        "roofline": roofline(r),
        "kernels_ms": {"hmc_sweep": r["hmc_ms"], "components": r["cmp_ms"]},
        "result": r["result"],
        "setup_s": r["setup_s"],
    }
    if r["tuned"]:
        out["autotune"] = r["tuned"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_seconds)
    if args.batched and args.config != 3:
        bs = synth.make_system(3, grid_device="cuda:0")
        rb = run_workload(pkg, torch, bs, 1, 1, tune=True)
        out["batched"] = {"value": rb["value"], "unit": "atom-evals/s",
                          "ms_per_step": rb["ms_per_step"], "steps": 1,
                          "warmup": 1, "config": describe(bs, rb),
                          "roofline": roofline(rb),
                          "autotune": rb["tuned"], "waves": rb["waves"],
                          "result": rb["result"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
