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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the "
              "path shards by ligand/replica range without collectives, see "
              "the design notes.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_1507_03703_amd as pkg

    t_setup = time.perf_counter()
    system = synth.make_system(args.config)
    lig = system.ligands[0]
    g = system.grid
    K, n = lig.n_states, lig.n_atoms
    L = system.n_leapfrog
    sweeps = args.sweeps or system.n_sweeps
    every = system.sample_every
    records = sweeps // every
    ctx = pkg.Context(seed=system.seed, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    lid = ctx.ligand_setup(lig, sample_capacity=records)
    N = records * K
    ukn = torch.empty((K, N), dtype=torch.float64, device="cuda:0")
    Nk = np.full(K, records, np.int64)
    setup_s = time.perf_counter() - t_setup

    def step():
        ctx.reset_samples(lid)
        ctx.hmc_sweep(sweeps, L, exchange_every=1, exchange_scheme=0,
                      sample_every=every)
        ctx.energy_matrix(lid, None, n_samples=N, out=ukn)
        return ctx.mbar(ukn, Nk, tol=1e-10, max_iter=100)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(True, every=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, var, it = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hmc_ms, hmc_n = ctx.get_timing(ctx.TIMER_HMC)
    cmp_ms, cmp_n = ctx.get_timing(ctx.TIMER_COMPONENTS)
    tail_ms, tail_n = ctx.get_timing(ctx.TIMER_TAIL)
    ctx.set_timing(False)
    stats = ctx.get_stats(lid)

    ms_per_step = el / args.steps * 1e3
    evals_per_step = sweeps * K * n * (L + 1)
    value = evals_per_step / (ms_per_step * 1e-3)
    # dominant kernel: the HMC sweep (one launch = one sweep of all replicas)
    evals_per_launch = K * n * (L + 1)
    achieved = evals_per_launch * GRID_BYTES_PER_EVAL / (hmc_ms * 1e-3) / 1e9
    out = {
        "metric": "atom-grid energy+force evals/s & HBM fraction; effective "
                  "samples/s vs plain HMC",
        "value": value,
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{system.name}: {n}-atom ligand, {g.n[0]}^3 x 3 "
                        f"float32 grids at {g.spacing} A, {K} replicas, "
                        f"{sweeps} sweeps x {L} leapfrog steps + neighbour "
                        f"exchange, u_kn {K}x{N} float64, MBAR",
            "replicas": K, "atoms": n, "sweeps_per_step": sweeps,
            "leapfrog": L, "samples": N},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_hmc_sweep", "mean_launch_ms": hmc_ms,
            "launches_timed": hmc_n,
            "algorithmic_bytes_per_launch": evals_per_launch *
            GRID_BYTES_PER_EVAL},
        "kernels_ms": {"hmc_sweep": hmc_ms, "sweep_tail": tail_ms,
                       "components": cmp_ms},
        "result": {"bpmf_syn_kT": float(f[-1] - f[0]),
                   "sigma_kT": float(np.sqrt(max(var[-1], 0.0))),
                   "mbar_iterations": int(it),
                   "hmc_acceptance": float(stats["hmc_acc"].sum() /
                                           max(stats["hmc_try"].sum(), 1)),
                   "exchange_acceptance": float(stats["ex_acc"].sum() /
                                                max(stats["ex_try"].sum(),
                                                    1))},
        "setup_s": setup_s,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
