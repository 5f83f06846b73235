"""Benchmark of the BPMF sampling hot path on one MI355X.

Workload (default): the large batched workload with learned pose proposals
-- 32 ligands of 40-100 atoms, each with a 32-state ladder (1024 replicas;
600 K, lambda 0 -> 300 K, lambda 1), sharing three float32 receptor grids of
256^3 nodes at 0.25 A from 8000 point atoms, and one pose-proposal network
per ligand, trained before the timed steps on 200k poses that plain HMC
samples at the ligand's coupled state.  One step is one pass of the whole
hot path: 10000 sweeps of (one 10-step velocity-Verlet HMC move per replica
+ one neighbour replica-exchange sweep), a learned independence pose move
of every replica every 5 sweeps, a recorded sample per state every 50
sweeps, each ligand's 32 x 6400 float64 reduced-energy matrix u_kn
recomputed from its recorded configurations (one batched call), and MBAR on
all 32 (one batched call).  Replicas carry over from step to step (a
production run in cycles).

value = atom-grid energy+force evaluations of the HMC moves per second of
whole-step time (L per atom per sweep: the force at the start of a
trajectory is the previous sweep's last one); one evaluation = one atom's
trilinear interpolation of the three grids with gradient (96 algorithmic
grid bytes) plus its share of the bonded terms and restraint.  The
roofline's kernel time is the sweep kernel's mean launch time, measured
with HIP events on the library's stream over plain sweeps of the same
ligands after the timed steps.

Further legs in the same JSON line: "production_single_ligand" (a 48-atom
ligand, 64 replicas, 128^3 grids, 5000 sweeps of 20 steps, u_kn, MBAR),
"batched" (256 ligands of 10-80 atoms x 32 replicas on 160^3 grids, 2000
sweeps; the launch shape picked by the autotuner), each with the oracle
timed on a bounded sample of it as well, "bulk_interpolation"
(u_kn and the interpolation harness on the sample sets of the batched
workloads), "learned_proposal" (plain HMC, the paper's external moves and
learned pose moves on the 24-atom, 64-state soft-grid system, each over
independent ladders: BPMF error against a reference of 16 plain ladders and
effective samples per second),
"initialization" (the paper's ladder initialisation and production
protocol) and "pair_terms" (the ligand's intramolecular nonbonded and OBC
GB/SA energies and forces, and their cost inside the sampler: the Full
pathway's sweep against the plain one).  --config picks another main workload.
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

# HBM traffic measured with rocprofv3 counters (FETCH_SIZE and WRITE_SIZE in
# KiB per dispatch, scaled by what they read for a 1 GiB device copy), per
# kernel and workload: one sweep launch (at the given wavefronts per
# replica), one harness launch, one energy-matrix call (its launches
# summed); valid only while the kernel sources hash to TRAFFIC_SOURCES
TRAFFIC_SOURCES = "5bbe1275acda510c"
TRAFFIC_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC = {
    ("k_hmc_sweep", "c5_large_batched"):
        {"waves": 4, "fetch_kib": 9087.386, "write_kib": 4431.231},
    ("k_hmc_sweep", "c2_plain_production"):
        {"waves": None, "fetch_kib": 761.004, "write_kib": 198.215},
    ("k_hmc_sweep", "c3_batched_uneven"):
        {"waves": 2, "fetch_kib": 37105.157, "write_kib": 23616.926},
    ("k_grid_eval", "c3_batched_uneven"):
        {"waves": None, "fetch_kib": 3379937.406, "write_kib": 3383700.0},
    ("k_energy_matrix", "c3_batched_uneven"):
        {"waves": None, "fetch_kib": 1178483.14, "write_kib": 535488.633},
}
KERNEL_SOURCES = ("device.h", "kernels.hip", "internal.h")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1507_03703_amd", "csrc", f),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, waves=None):
    """Measured HBM bytes per launch (or call), or None when the workload,
    its launch shape or the kernel sources differ from those the counters
    were taken on."""
    t = TRAFFIC.get((kernel, workload))
    if t is None or kernel_sources_hash() != TRAFFIC_SOURCES:
        return None
    if t.get("waves") is not None and list(waves or []) != [t["waves"]]:
        return None
    return 1024.0 * (t["fetch_kib"] * TRAFFIC_SCALE["fetch"] +
                     t["write_kib"] * TRAFFIC_SCALE["write"])


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", type=int, default=5)
    p.add_argument("--sweeps", type=int, default=None,
                   help="override sweeps per step (default: the workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=16.0)
    p.add_argument("--metrics", default=None, metavar="PATH",
                   help="append the main workload's per-ligand counters and "
                        "throughput to this JSON-lines file")
    p.add_argument("--no-batched", dest="batched", action="store_false",
                   help="skip the batched 256-ligand leg")
    p.add_argument("--no-production", dest="production",
                   action="store_false",
                   help="skip the single-ligand production (config 2) leg")
    p.add_argument("--no-proposals", dest="proposals", action="store_false",
                   help="config 5 without its learned pose proposals")
    p.add_argument("--proposal-train-steps", type=int, default=1500)
    p.add_argument("--no-bulk", dest="bulk", action="store_false",
                   help="skip the bulk interpolation leg")
    p.add_argument("--bulk-configs", default="3,5",
                   help="batched workloads whose sample sets the bulk leg "
                        "uses")
    p.add_argument("--bulk-only", action="store_true")
    p.add_argument("--no-learned", dest="learned", action="store_false",
                   help="skip the learned-proposal leg")
    p.add_argument("--learned-only", action="store_true",
                   help="only the learned-proposal leg (with --long-sweeps, "
                        "--prod-sweeps, --train-steps)")
    p.add_argument("--no-init", dest="init", action="store_false",
                   help="skip the ladder-initialisation leg")
    p.add_argument("--init-only", action="store_true")
    p.add_argument("--no-pairs", dest="pairs", action="store_false",
                   help="skip the intramolecular pair-term leg")
    p.add_argument("--pairs-only", action="store_true")
    p.add_argument("--long-sweeps", type=int, default=500000,
                   help="learned leg: sweeps of each reference ladder")
    p.add_argument("--prod-sweeps", type=int, default=200000,
                   help="learned leg: sweeps of each sampler's ladders")
    p.add_argument("--burn-sweeps", type=int, default=200000)
    p.add_argument("--train-steps", type=int, default=4000)
    p.add_argument("--waves", type=int, default=None,
                   help="wavefronts per replica for every ligand instead of "
                        "the autotuner's choice (0 = per-ligand minimum)")
    p.add_argument("--task-order", type=int, default=None, choices=(0, 1, 2),
                   help="workgroup order of the sweep (0 ligand by ligand, 1 "
                        "heaviest ligands first) instead of the autotuner's")
    p.add_argument("--grid-device", default="cuda:0",
                   help="torch device that sums the synthetic receptor grids "
                        "(input generation, outside the timed region)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                   help="only run a plain device-to-device copy of BYTES "
                        "bytes five times (reference for memory counters)")
    return p.parse_args()


def cpu_model():
    """The host CPU's model name (as lscpu reports it, from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, target_s, n_ligands=2):
    """The FP64 oracle's sampler (HMC moves + neighbour exchange, the same
    sweeps as the library's) on a bounded sample of the workload: its first
    `n_ligands` ligands, each for as many sweeps as fit about target_s / 2
    seconds split over the ligands, once on one host thread and once on all
    of them (OpenMP across replicas).  The oracle evaluates every atom L + 1
    times per sweep (it recomputes the force at the start of a trajectory),
    and its rate counts them all."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    L = system.n_leapfrog
    ligs = system.ligands[:n_ligands]
    og = oracle.OGrid(system.grid)
    all_threads = int(oracle.num_threads())
    runs = {}
    for threads in (1, all_threads):
        oracle.set_num_threads(threads)
        evals = sweeps_done = 0
        el = 0.0
        for q, lig in enumerate(ligs):
            ol = oracle.OLigand(lig)
            s = oracle.Sampler(og, ol, seed=system.seed, lig_id=q, x0=lig.x0)
            t0 = time.perf_counter()
            s.sweep(nleap=L, exchange_every=1)
            one = time.perf_counter() - t0
            n = max(2, int(target_s / 2 / len(ligs) / max(one, 1e-4)))
            t0 = time.perf_counter()
            for _ in range(n):
                s.sweep(nleap=L, exchange_every=1)
            el += time.perf_counter() - t0
            evals += n * ol.K * lig.n_atoms * (L + 1)
            sweeps_done += n
        runs[threads] = (evals / el, sweeps_done, el)
    oracle.set_num_threads(all_threads)
    counts = [l.n_atoms for l in ligs]
    v1, n1, e1 = runs[1]
    va, na, ea = runs[all_threads]
    return dict(value=va, unit="atom-evals/s", cores=all_threads,
                kind="oracle", single_core_value=v1,
                cpu_model=cpu_model(),
                sample=f"{system.name}: ligands 0-{len(ligs) - 1} "
                       f"({', '.join(map(str, counts))} atoms, "
                       f"{ligs[0].n_states} replicas each), oracle sweeps of "
                       f"{L} leapfrog steps + neighbour exchange, "
                       f"{ligs[0].n_states} x n_atoms x {L + 1} energy+force "
                       f"evaluations per ligand sweep; {n1} sweeps in "
                       f"{e1:.1f} s on 1 thread, {na} sweeps in {ea:.1f} s "
                       f"on {all_threads} threads")


def train_proposals(pkg, torch, system, sweeps=31250, burn=400, every=5,
                    steps=1500, batch=512, lr=2e-3):
    """One pose proposal per ligand, trained as the learned workloads state
    it: poses sampled by plain HMC at the coupled state (lambda = 1, 300 K;
    K independent chains per ligand, every ligand in one context, a record
    every `every` sweeps after `burn` sweeps: K x sweeps / every poses, 200k
    at the defaults), then each ligand's network trained on its own poses
    by the library's kernels (Adam, minibatches drawn with replacement).
    Returns the parameters per ligand and what the training cost."""
    import dataclasses
    import numpy as np
    g, ligs, L = system.grid, system.ligands, system.n_leapfrog
    coupled = [dataclasses.replace(
        l, T=np.full(l.n_states, l.T[-1]),
        w=np.repeat(l.w[-1:], l.n_states, axis=0),
        dt=np.full(l.n_states, float(l.dt[-1]))) for l in ligs]
    records = sweeps // every
    ctx = pkg.Context(seed=system.seed + 17, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    ids = [ctx.ligand_setup(l, sample_capacity=records) for l in coupled]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.hmc_sweep(burn, L, exchange_every=0)
    ctx.hmc_sweep(sweeps, L, exchange_every=0, sample_every=every)
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t0
    rng = np.random.default_rng(system.seed)
    params, first, last = [], [], []
    train_s = 0.0
    for lid, l in zip(ids, coupled):
        xs, _ = ctx.get_samples(lid)
        xd = torch.from_numpy(xs.reshape(-1, l.n_atoms, 3)).to("cuda:0")
        del xs
        ctx.proposal_setup(lid, l.frame_atoms, l.tors[l.cond_tors],
                           init_params(rng))
        feats, poses = ctx.pose_features(lid, xd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = ctx.proposal_train(lid, feats, poses, batch=batch,
                                    steps=steps, lr=lr, losses=True)
        torch.cuda.synchronize()
        train_s += time.perf_counter() - t0
        params.append(ctx.proposal_params(lid))
        first.append(float(np.mean(losses[:20])))
        last.append(float(np.mean(losses[-20:])))
        del xd, feats, poses
    ctx.close()
    return params, {"poses_per_ligand": records * ligs[0].n_states,
                    "sampling_sweeps": burn + sweeps, "sampling_s": sample_s,
                    "adam_steps": steps, "batch": batch, "lr": lr,
                    "train_s": train_s,
                    "loss_first_mean": float(np.mean(first)),
                    "loss_last_mean": float(np.mean(last))}


def run_workload(pkg, torch, system, steps, warmup, sweeps=None,
                 tune=False, waves=None, task_order=None, proposals=None,
                 pose_every=5,
                 kernel_sweeps=512, metrics_path=None):
    """Set up every ligand of `system`, run `warmup` + `steps` timed steps
    of the hot path and return the measurements.  proposals: per-ligand
    network parameters; the sweeps then carry a learned pose move of every
    replica every `pose_every` sweeps.  After the timed steps,
    `kernel_sweeps` plain sweeps (graph replays of 64 sweeps, each replay
    bracketed by HIP events on the library's stream) give the sweep
    kernel's own mean launch time for the roofline.  metrics_path: append
    each ligand's counters (acceptances, round trips, non-finite moves) and
    the run's throughput to this JSON-lines file."""
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
    if proposals is not None:
        for i, l, p in zip(ids, ligs, proposals):
            ctx.proposal_setup(i, l.frame_atoms, l.tors[l.cond_tors], p)
    moves = dict(pose_move_every=pose_every if proposals is not None else 0)
    ukn = [torch.empty((l.n_states, records * l.n_states),
                       dtype=torch.float64, device="cuda:0") for l in ligs]
    Nk = [np.full(l.n_states, records, np.int64) for l in ligs]
    tuned = None
    if waves is not None:
        ctx.set_waves(waves)
        tuned = {"chosen_waves": waves or "auto", "fixed": True}
    elif tune:
        sig = (f"{system.name}|L{L}|" +
               ",".join(f"{l.n_atoms}x{l.n_states}" for l in ligs))
        cache = os.environ.get("BPMF_TUNE_CACHE", os.path.join(
            os.path.expanduser("~"), ".cache", "bpmf_autotune.json"))
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        chosen, table = ctx.autotune(n_sweeps=64, n_leapfrog=L,
                                     cache_path=cache, signature=sig)
        tuned = {"chosen_waves": chosen or "auto", "sweep_ms": table}
    if task_order is not None:
        ctx.set_task_order(task_order)
    setup_s = time.perf_counter() - t_setup
    results = []
    # MBAR of each cycle starts from the previous cycle's free energies
    f_prev = [None] * len(ids)

    def step():
        for i in ids:
            ctx.reset_samples(i)
        ctx.hmc_sweep(sweeps, L, exchange_every=1, exchange_scheme=0,
                      sample_every=every, **moves)
        # every ligand's u_kn, then every ligand's MBAR, in batched calls
        ctx.energy_matrix_batch(ids, n_samples=[u.shape[1] for u in ukn],
                                outs=ukn)
        out = ctx.mbar_batch(ukn, Nk, tol=1e-10, max_iter=100,
                             f_init=f_prev)
        for q, r in enumerate(out):
            f_prev[q] = r[0] if np.all(np.isfinite(r[0])) else None
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
    unit_ms, unit_n = ctx.get_timing(ctx.TIMER_HMC)
    cmp_ms, cmp_n = ctx.get_timing(ctx.TIMER_COMPONENTS)
    ctx.set_timing(False)
    stats = [ctx.get_stats(i) for i in ids]
    pose = None
    if proposals is not None:
        ps = [ctx.get_pose_stats(i) for i in ids]
        pose = {"pose_moves": int(sum(p["tries"].sum() for p in ps)),
                "pose_acceptance": float(sum(p["acc"].sum() for p in ps) /
                                         max(sum(p["tries"].sum()
                                                 for p in ps), 1)),
                "pose_acceptance_coupled_states": float(
                    sum(p["acc"][-1] for p in ps) /
                    max(sum(p["tries"][-1] for p in ps), 1))}
    # the sweep kernel alone: plain sweeps replayed from captured graphs of
    # 64 (as the library runs them), each replay timed and counted as 64
    # sweep launches
    ctx.set_graph(64)
    ctx.hmc_sweep(64, L, exchange_every=1)
    torch.cuda.synchronize()
    ctx.set_timing(True, every=1)
    ctx.hmc_sweep(kernel_sweeps, L, exchange_every=1)
    hmc_ms, hmc_n = ctx.get_timing(ctx.TIMER_HMC)
    ctx.set_timing(False)
    waves = sorted({ctx.get_waves(i) for i in ids})
    lig_metrics = None
    if metrics_path:
        from paper_1507_03703_amd import metrics as M
        lig_metrics = [M.ligand_metrics(ctx, i) for i in ids]
    ctx.close()

    ms_per_step = el / steps * 1e3
    # the kernel evaluates every atom L times per sweep (the force at the
    # start of a trajectory comes from the previous sweep's last step)
    evals_per_sweep = sum(l.n_states * l.n_atoms for l in ligs) * L
    value = sweeps * evals_per_sweep / (ms_per_step * 1e-3)
    achieved = evals_per_sweep * GRID_BYTES_PER_EVAL / (hmc_ms * 1e-3) / 1e9
    f, var, it = results[0]
    acc = sum(st["hmc_acc"].sum() for st in stats) / max(
        sum(st["hmc_try"].sum() for st in stats), 1)
    exa = sum(st["ex_acc"].sum() for st in stats) / max(
        sum(st["ex_try"].sum() for st in stats), 1)
    bpmf = np.array([r[0][-1] - r[0][0] for r in results])
    res = {"bpmf_syn_kT": float(f[-1] - f[0]) if len(results) == 1 else None,
           "sigma_kT": float(np.sqrt(max(var[-1], 0.0))),
           "mbar_iterations": int(it),
           "mbar_iterations_max": int(max(r[2] for r in results)),
           "bpmf_syn_kT_mean": float(bpmf.mean()),
           "bpmf_syn_kT_range": [float(bpmf.min()), float(bpmf.max())],
           "hmc_acceptance": float(acc),
           "exchange_acceptance": float(exa)}
    if pose:
        res.update(pose)
    if lig_metrics is not None:
        M.MetricsLog(metrics_path).write(
            lig_metrics, workload=system.name, atom_evals_per_s=value,
            ms_per_step=ms_per_step, sweep_kernel_ms=hmc_ms,
            effective_gbs=achieved)
    return dict(value=value, ms_per_step=ms_per_step, sweeps=sweeps,
                records=records, hmc_ms=hmc_ms, hmc_n=hmc_n,
                unit_ms=unit_ms, unit_n=unit_n, cmp_ms=cmp_ms,
                achieved=achieved, evals_per_sweep=evals_per_sweep,
                setup_s=setup_s, waves=waves, tuned=tuned,
                pose_every=moves["pose_move_every"], result=res)


def bulk_leg(pkg, torch, system, reps=3, harness_min=10 ** 8):
    """Throughput of the bulk interpolation kernels on the sample set of a
    batched workload: every ligand's ladder is sampled for the workload's
    sweeps (a record per state every `sample_every`), then (1) u_kn is
    recomputed from every recorded configuration (the component kernel,
    energy only) and (2) the interpolation harness (bpmf_grid_eval: energy
    and force of all channels) runs at every atom position of those
    configurations, tiled to at least `harness_min` points.  Both are timed
    with HIP events around every launch on the context's stream."""
    import numpy as np
    g, ligs = system.grid, system.ligands
    L = system.n_leapfrog
    every = system.sample_every
    records = system.n_sweeps // every
    ctx = pkg.Context(seed=system.seed, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    ids = [ctx.ligand_setup(l, sample_capacity=records) for l in ligs]
    t0 = time.perf_counter()
    ctx.hmc_sweep(system.n_sweeps, L, exchange_every=1, sample_every=every)
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t0
    ukn = [torch.empty((l.n_states, records * l.n_states),
                       dtype=torch.float64, device="cuda:0") for l in ligs]

    def all_ukn():
        ctx.energy_matrix_batch(ids, n_samples=[u.shape[1] for u in ukn],
                                outs=ukn)

    all_ukn()
    torch.cuda.synchronize()
    ctx.set_timing(True, every=1)
    for _ in range(reps):
        all_ukn()
    cmp_ms, cmp_n = ctx.get_timing(ctx.TIMER_COMPONENTS)
    ctx.set_timing(False)
    evals_ukn = sum(records * l.n_states * l.n_atoms for l in ligs)
    ukn_s = cmp_ms * cmp_n * 1e-3 / reps
    # harness points: every atom of every recorded configuration, with the
    # atom's per-channel scale
    pos, scl = [], []
    for i, l in zip(ids, ligs):
        xs, _ = ctx.get_samples(i)
        pos.append(xs.reshape(-1, 3))
        scl.append(np.tile(l.scale.astype(np.float32), (xs.shape[0] *
                                                         xs.shape[1], 1)))
    # tiled on the host and uploaded by plain copies (no torch kernels, so
    # that the leg also runs under hardware counter collection)
    pos, scl = np.concatenate(pos), np.concatenate(scl)
    tile = -(-harness_min // pos.shape[0])
    pos = torch.from_numpy(np.tile(pos, (tile, 1))).to("cuda:0")
    scl = torch.from_numpy(np.tile(scl, (tile, 1))).to("cuda:0")
    npts = pos.shape[0]
    w = np.ones(g.nodes.shape[-1])
    energy, force = ctx.grid_eval(pos, scl, w)
    torch.cuda.synchronize()
    ctx.set_timing(True, every=1)
    for _ in range(reps):
        ctx.grid_eval(pos, scl, w, energy=energy, force=force)
    ge_ms, ge_n = ctx.get_timing(ctx.TIMER_GRID_EVAL)
    ctx.set_timing(False)
    head = 1 << 20
    finite = all(bool(np.isfinite(a[sl].cpu().numpy()).all())
                 for a in (energy, force)
                 for sl in (slice(0, head), slice(npts - head, npts)))
    ctx.close()
    io = 4 * (3 + 2 * g.nodes.shape[-1] + 3)   # pos, scale, energy, force

    def line(evals, sec, io_bytes, kernel):
        gbs = evals * GRID_BYTES_PER_EVAL / sec / 1e9
        return {"value": evals / sec, "unit": "atom-evals/s",
                "roofline": {"bound": "hbm", "achieved": gbs,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS,
                             "traffic": measured_traffic(kernel,
                                                         system.name),
                             "algorithmic_bytes_per_eval":
                                 GRID_BYTES_PER_EVAL,
                             "streamed_bytes_per_eval": io_bytes}}
    counts = [l.n_atoms for l in ligs]
    return {
        "workload": f"{system.name} sample set: {len(ligs)} ligands of "
                    f"{min(counts)}-{max(counts)} atoms x "
                    f"{ligs[0].n_states} states x {records} records, "
                    f"{g.n[0]}^3 x {g.nodes.shape[-1]} float32 grids",
        "sampling_s": sample_s,
        "energy_matrix": dict(line(evals_ukn, ukn_s, 12, "k_energy_matrix"),
                              atom_evals=evals_ukn, kernel="k_energy_matrix",
                              timed_intervals_per_call=cmp_n // reps,
                              kernel_ms_total=ukn_s * 1e3),
        "harness": dict(line(npts, ge_ms * 1e-3, io, "k_grid_eval"),
                        points=npts,
                        kernel="k_grid_eval", launch_ms=ge_ms,
                        outputs_finite=finite),
    }


def describe(system, r):
    ligs = system.ligands
    g = system.grid
    L = system.n_leapfrog
    R = sum(l.n_states for l in ligs)
    moves = (f" + a learned independence pose move per replica every "
             f"{r['pose_every']} sweeps (one trained network per ligand)"
             if r.get("pose_every") else "")
    if len(ligs) == 1:
        l = ligs[0]
        what = (f"{system.name}: {l.n_atoms}-atom ligand, {g.n[0]}^3 x 3 "
                f"float32 grids at {g.spacing} A, {R} replicas, "
                f"{r['sweeps']} sweeps x {L} leapfrog steps + neighbour "
                f"exchange{moves}, u_kn "
                f"{l.n_states}x{r['records'] * l.n_states} float64, MBAR")
    else:
        counts = [l.n_atoms for l in ligs]
        what = (f"{system.name}: {len(ligs)} ligands of {min(counts)}-"
                f"{max(counts)} atoms x {ligs[0].n_states} replicas ({R} "
                f"replicas), shared {g.n[0]}^3 x 3 float32 grids at "
                f"{g.spacing} A, {r['sweeps']} sweeps x {L} leapfrog steps "
                f"+ neighbour exchange{moves}, per-ligand u_kn "
                f"({ligs[0].n_states} x {r['records'] * ligs[0].n_states}) "
                f"and batched MBAR")
    return {"workload": what, "ligands": len(ligs), "replicas": R,
            "atoms": [l.n_atoms for l in ligs] if len(ligs) <= 4 else
            f"{sum(l.n_atoms for l in ligs)} total",
            "sweeps_per_step": r["sweeps"], "leapfrog": L,
            "samples_per_state": r["records"],
            "pose_move_every": r.get("pose_every") or None}


def roofline(r, workload):
    return {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": r["achieved"] / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_hmc_sweep", workload, r["waves"]),
            "kernel": "k_hmc_sweep",
            "mean_launch_ms": r["hmc_ms"], "launches_timed": r["hmc_n"],
            "evals_per_launch": r["evals_per_sweep"],
            "algorithmic_bytes_per_launch": r["evals_per_sweep"] *
            GRID_BYTES_PER_EVAL}


def stat_inefficiency(a):
    """g = 1 + 2 sum_t (1 - t/N) rho(t), summed while the normalised
    autocorrelation rho stays positive (ESS = N / g); the lagged sums come
    from one FFT."""
    import numpy as np
    a = np.asarray(a, np.float64)
    N = len(a)
    d = a - a.mean()
    var = float(d @ d) / N
    if N < 3 or var <= 0.0:
        return 1.0
    m = 1 << int(np.ceil(np.log2(2 * N)))
    f = np.fft.rfft(d, m)
    lag = np.fft.irfft(f * np.conj(f), m)[:N - 1]   # sum_i d_i d_{i+t}
    t = np.arange(1, N - 1)
    rho = lag[1:] / (N - t) / var
    stop = np.nonzero(rho <= 0.0)[0]
    k = int(stop[0]) if len(stop) else len(rho)
    g = 1.0 + 2.0 * float(np.sum(rho[:k] * (1.0 - t[:k] / N)))
    return max(g, 1.0)


def batch_means_inefficiency(a, n_batches=30):
    """g = b var(batch means) / var(a) over n_batches consecutive batches of
    b samples: for slow observables, whose autocorrelation estimate turns
    negative from noise long before it has decayed."""
    import numpy as np
    a = np.asarray(a, np.float64)
    b = len(a) // n_batches
    var = float(a.var())
    if b < 2 or var <= 0.0:
        return 1.0
    means = a[:b * n_batches].reshape(n_batches, b).mean(axis=1)
    return max(b * float(means.var(ddof=1)) / var, 1.0)


def init_params(rng):
    """Random fan-in-scaled weights of the 16-256-256-104 proposal network in
    the library's flat layout (W1 b1 W2 b2 W3 b3, weights [in][out])."""
    import numpy as np
    parts = []
    for i, o, gain in ((16, 256, 1.0), (256, 256, 1.0), (256, 104, 0.1)):
        parts.append(rng.normal(size=(i, o)) * gain / np.sqrt(i))
        parts.append(np.zeros(o))
    return np.concatenate([q.reshape(-1) for q in parts]).astype(np.float32)


def learned_leg(pkg, torch, pose_every=5, train_steps=4000,
                long_sweeps=500000, prod_sweeps=200000, burn=200000,
                n_ref=16, n_seeds=8):
    """Plain HMC, the paper's external moves and learned independence pose
    moves on the 24-atom, 64-state system with the paper's soft-grid
    switching protocol, each estimate over independent ladders.

    The reference: `n_ref` independent copies of the ladder in one context
    (one launch per sweep covers all of them), `burn` sweeps of
    equilibration, then `long_sweeps` sweeps with a record every
    `sample_every`; each ladder's BPMF by MBAR over its records, the
    reference the mean over ladders with its standard error (their spread
    / sqrt(n_ref)).  The coupled state's records of every ladder are the
    poses the network is trained on.  Each sampler then runs `n_seeds`
    independent ladders in one context for `prod_sweeps` sweeps, started
    from the final states of the first `n_seeds` reference ladders: plain
    HMC, HMC with the paper's external moves (20 per sweep in the states
    with alpha < 0.01) and HMC with a learned pose move every `pose_every`
    sweeps.  Reported per sampler: the mean BPMF over its ladders, its error
    against the reference with the standard error of that difference, the
    spread of the per-ladder estimates, and effective samples per second of
    two observables of the coupled state, summed over the ladders: its
    reduced potential (fast) and the distance of its centre of mass from
    the site (the pose, which the pose moves act on)."""
    import numpy as np
    import synth
    system = synth.make_system(4, grid_device="cuda:0")
    g, (lig,) = synth.add_soft_grids(system.grid, system.ligands)
    K, L, n = lig.n_states, system.n_leapfrog, lig.n_atoms
    every = system.sample_every
    mass = lig.mass / lig.mass.sum()

    def fresh(copies, capacity):
        ctx = pkg.Context(seed=system.seed, device=0)
        ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
        ids = [ctx.ligand_setup(lig, sample_capacity=capacity)
               for _ in range(copies)]
        return ctx, ids

    def estimate(ctx, lid, n_rec):
        """One ladder: BPMF over all its records and the coupled state's
        observables."""
        u = ctx.energy_matrix(lid, None, n_samples=n_rec * K)
        f, var, _ = ctx.mbar(u, np.full(K, n_rec), tol=1e-10, max_iter=200)
        # the coupled state's reduced potential on its own samples
        # (round-major) and its pose: centre-of-mass distance from the site
        pot = u[K - 1, K - 1::K].cpu().numpy()
        del u
        xs, _ = ctx.get_samples(lid)
        com = (xs[:, K - 1].astype(np.float64) * mass[None, :, None]).sum(1)
        dist = np.linalg.norm(com - lig.site_center[None, :], axis=1)
        return dict(bpmf=float(f[-1] - f[0]),
                    sigma_mbar=float(np.sqrt(max(var[-1], 0.0))),
                    g_pot=stat_inefficiency(pot),
                    g_pose=batch_means_inefficiency(dist)), xs

    # reference ladders: BPMF and training poses
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    long_rec = long_sweeps // every
    ctx, ids = fresh(n_ref, long_rec)
    ctx.hmc_sweep(burn, L, exchange_every=1)
    ctx.hmc_sweep(long_sweeps, L, exchange_every=1, sample_every=every)
    torch.cuda.synchronize()
    long_s = time.perf_counter() - t0
    finals = [ctx.get_replicas(i) for i in ids]
    ref_b, ref_gpose, pose_x = [], [], []
    for i in ids:
        e, xs = estimate(ctx, i, long_rec)
        ref_b.append(e["bpmf"])
        ref_gpose.append(e["g_pose"])
        pose_x.append(np.ascontiguousarray(xs[:, K - 1]))
        del xs
    ref_b = np.array(ref_b)
    ref_mean = float(ref_b.mean())
    ref_se = float(ref_b.std(ddof=1) / np.sqrt(n_ref))
    poses_x = torch.as_tensor(np.concatenate(pose_x), device="cuda:0")
    del pose_x
    lid0 = ids[0]
    ctx.proposal_setup(lid0, lig.frame_atoms, lig.tors[lig.cond_tors],
                       init_params(np.random.default_rng(system.seed)))
    feats, poses = ctx.pose_features(lid0, poses_x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = ctx.proposal_train(lid0, feats, poses, batch=512,
                                steps=train_steps, lr=2e-3, losses=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    params = ctx.proposal_params(lid0)
    n_poses = int(feats.shape[0])
    ctx.close()
    del poses_x, feats, poses

    # the paper's external moves: 20 per sweep in the states whose grid
    # coupling alpha is below 0.01
    alpha = np.linspace(0.0, 1.0, K)
    k_ext = int(np.sum(alpha < 0.01))

    def production(mode):
        records = prod_sweeps // every
        ctx, ids = fresh(n_seeds, records)
        learned = mode == "learned"
        for q, i in enumerate(ids):
            fq = finals[q]
            ctx.set_replicas(i, fq["x"], fq["state_of_replica"], fq["comps"],
                             int(fq["counter"]))
            if learned:
                ctx.proposal_setup(i, lig.frame_atoms,
                                   lig.tors[lig.cond_tors], params)
        moves = dict(pose_move_every=pose_every if learned else 0)
        if mode == "external":
            moves.update(external_moves=20, external_k_max=k_ext,
                         external_sigma=0.6)
        ctx.hmc_sweep(2 * pose_every, L, exchange_every=1, **moves)
        for i in ids:
            ctx.reset_samples(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.hmc_sweep(prod_sweeps, L, exchange_every=1, sample_every=every,
                      **moves)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        es = [estimate(ctx, i, records)[0] for i in ids]
        b = np.array([e["bpmf"] for e in es])
        mean = float(b.mean())
        sd = float(b.std(ddof=1))
        err = mean - ref_mean
        err_se = float(np.sqrt(sd ** 2 / n_seeds + ref_se ** 2))
        ess_pot = sum(records / e["g_pot"] for e in es)
        ess_pose = sum(records / e["g_pose"] for e in es)
        out = dict(seconds=el, ladders=n_seeds, bpmf_kT=mean,
                   ladder_bpmf_kT=[float(v) for v in b],
                   ladder_sd_kT=sd,
                   sigma_mbar_kT=float(np.mean([e["sigma_mbar"]
                                                for e in es])),
                   error_vs_reference_kT=float(err),
                   error_standard_error_kT=err_se,
                   within_1kT=bool(abs(err) <= 1.0),
                   stat_inefficiency_potential=float(np.mean(
                       [e["g_pot"] for e in es])),
                   stat_inefficiency_pose=float(np.mean(
                       [e["g_pose"] for e in es])),
                   ess_potential=ess_pot, ess_pose=ess_pose,
                   ess_per_s=ess_pot / el, ess_pose_per_s=ess_pose / el)
        if learned:
            ps = [ctx.get_pose_stats(i) for i in ids]
            out["pose_acceptance"] = float(
                sum(p["acc"].sum() for p in ps) /
                max(sum(p["tries"].sum() for p in ps), 1))
            out["pose_acceptance_coupled_state"] = float(
                sum(p["acc"][-1] for p in ps) /
                max(sum(p["tries"][-1] for p in ps), 1))
        if mode == "external":
            xs_ = [ctx.get_external_stats(i) for i in ids]
            out["external_states"] = k_ext
            out["external_acceptance"] = float(
                sum(x["acc"].sum() for x in xs_) /
                max(sum(x["tries"].sum() for x in xs_), 1))
        ctx.close()
        return out

    progress("learned leg: reference ladders and training")
    plain = production("plain")
    progress("learned leg: plain sampler")
    external = production("external")
    progress("learned leg: external-move sampler")
    learned = production("learned")
    progress("learned leg: learned sampler")
    return {
        "workload": f"{system.name} with the soft-grid switching protocol "
                    f"(5 channels): {n}-atom ligand, {g.n[0]}^3 grids, {K} "
                    f"replicas per ladder; reference: {n_ref} independent "
                    f"ladders, {burn} sweeps of burn-in and {long_sweeps} "
                    f"sweeps each; samplers: {n_seeds} ladders each, "
                    f"{prod_sweeps} sweeps x {L} leapfrog steps from "
                    f"reference ladders' final states, a sample per state "
                    f"every {every}; learned: one independence pose move "
                    f"per replica every {pose_every} sweeps (captured with "
                    f"the sweeps); external: 20 of the paper's external "
                    f"moves per sweep in the states with alpha < 0.01",
        "ess_observables": "coupled state: reduced potential on its own "
                           "samples (initial positive autocorrelation sum); "
                           "centre-of-mass distance from the site (batch "
                           "means over 30 batches); summed over ladders",
        "reference": {"ladders": n_ref, "burn_in_sweeps": burn,
                      "sweeps": long_sweeps, "seconds": long_s,
                      "bpmf_kT": ref_mean,
                      "ladder_bpmf_kT": [float(v) for v in ref_b],
                      "ladder_sd_kT": float(ref_b.std(ddof=1)),
                      "standard_error_kT": ref_se,
                      "stat_inefficiency_pose": float(np.mean(ref_gpose))},
        "plain": plain, "external": external, "learned": learned,
        "ess_per_s_ratio": learned["ess_per_s"] / plain["ess_per_s"],
        "ess_pose_per_s_ratio": learned["ess_pose_per_s"] /
                                plain["ess_pose_per_s"],
        "external_ess_per_s_ratio": external["ess_per_s"] /
                                    plain["ess_per_s"],
        "external_ess_pose_per_s_ratio": external["ess_pose_per_s"] /
                                         plain["ess_pose_per_s"],
        "training": {"poses": n_poses, "steps": train_steps, "batch": 512,
                     "train_s": train_s,
                     "loss_first": float(np.mean(losses[:20])),
                     "loss_last": float(np.mean(losses[-20:]))},
    }


def init_leg(pkg, torch, n_seeds=50, n_trials=200, n_com=453, n_orient=100,
             prod_sweeps=2000):
    """The paper's ladder initialisation on the 24-atom soft-grid system:
    wall time of bpmf_initialize_ladder, the ladder it builds, and the
    neighbour exchange acceptance of a production run on it next to the
    fixed 64-state ladder (alpha_k = k/63) of the learned-proposal leg."""
    import dataclasses
    import numpy as np
    import synth
    system = synth.make_system(4, grid_device="cuda:0")
    g, (lig,) = synth.add_soft_grids(system.grid, system.ligands)
    L = system.n_leapfrog
    init = dataclasses.replace(
        lig, T=np.full(n_seeds, 600.0), w=np.zeros((n_seeds, 5)),
        dt=np.full(n_seeds, float(lig.dt[0])),
        x0=np.repeat(lig.x0[:1], n_seeds, axis=0).astype(np.float32))
    ctx = pkg.Context(seed=system.seed + 7, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    lid = ctx.ligand_setup(init, sample_capacity=n_trials)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.initialize_ladder(lid, pkg.SCHEDULE_SOFT, 600.0, 300.0,
                                speed=0.2, n_trials=n_trials, n_leapfrog=L,
                                dt_start=float(lig.dt[0]), dt_min=0.25,
                                max_dt_rounds=8, max_selections=6,
                                n_conf=n_seeds, n_com=n_com,
                                n_orient=n_orient, max_states=1024)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ctx.close()
    K = res["n_states"]

    def exchange_rates(T, w, dt, x0, alpha=None):
        """Neighbour exchange (even/odd) sweeps, or the paper's iteration:
        an HMC move, 20 external moves in the states with alpha < 0.01,
        then 25 exchange sweeps over separations 1..5."""
        lg = dataclasses.replace(lig, T=np.asarray(T), w=np.asarray(w),
                                 dt=np.asarray(dt),
                                 x0=np.ascontiguousarray(x0, np.float32))
        c = pkg.Context(seed=system.seed + 11, device=0)
        c.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
        i = c.ligand_setup(lg)
        kw = dict(exchange_every=1)
        if alpha is not None:
            kw.update(exchange_scheme=1, max_sep=5, exchange_sweeps=25,
                      external_moves=20,
                      external_k_max=int((np.asarray(alpha) < 0.01).sum()))
        c.hmc_sweep(prod_sweeps // 4, L, **kw)   # equilibration
        s0 = c.get_stats(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.hmc_sweep(prod_sweeps, L, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / prod_sweeps * 1e3
        s1 = c.get_stats(i)
        c.close()
        acc = (s1["ex_acc"] - s0["ex_acc"]) / np.maximum(
            s1["ex_try"] - s0["ex_try"], 1)
        hmc = (s1["hmc_acc"] - s0["hmc_acc"]) / np.maximum(
            s1["hmc_try"] - s0["hmc_try"], 1)
        return {"states": int(len(T)), "ms_per_iteration": ms,
                "exchange_min": float(acc.min()),
                "exchange_mean": float(acc.mean()),
                "pairs_below_0.4": int((acc < 0.4).sum()),
                "hmc_acceptance_min": float(hmc.min())}

    protocol = paper_production(pkg, torch, g, lig, res, L, system.seed)
    built = exchange_rates(res["T"], res["w"], res["dt"], res["x"][:, 0])
    fixed = exchange_rates(lig.T, lig.w, lig.dt, lig.x0)
    built_paper = exchange_rates(res["T"], res["w"], res["dt"],
                                 res["x"][:, 0], alpha=res["alpha"])
    fixed_paper = exchange_rates(lig.T, lig.w, lig.dt, lig.x0,
                                 alpha=np.linspace(0.0, 1.0, lig.n_states))
    pv = res["pacc"][1:]
    return {
        "workload": "c4_soft_grid_ladder_initialisation",
        "seconds": sec, "states": K, "selections": res["n_selections"],
        "runs": res["n_runs"], "removed": res["n_removed"],
        "reached_target": res["reached_target"],
        "seeds_per_state": n_seeds, "trials_per_run": n_trials,
        "leapfrog": L, "placements": n_seeds * n_com * n_orient,
        "verified_pacc_min": float(pv.min()) if len(pv) else None,
        "verified_pacc_median": float(np.median(pv)) if len(pv) else None,
        "dt_fs_range": [float(res["dt"].min()), float(res["dt"].max())],
        "hmc_acceptance_range": [float(res["acc"].min()),
                                 float(res["acc"].max())],
        "production_sweeps": prod_sweeps,
        "built_ladder": built, "fixed_ladder": fixed,
        "built_ladder_paper_iteration": built_paper,
        "fixed_ladder_paper_iteration": fixed_paper,
        "paper_protocol": protocol,
    }


def pair_leg(pkg, torch, n_conf=32000, reps=5):
    """Intramolecular LJ + Coulomb + OBC GB/SA energies and forces of
    n_conf configurations per call (bpmf_pair_evaluate), timed with HIP
    events on the library's stream: the 48-atom production ligand and a
    100-atom ligand (the largest of the large batched workload)."""
    import numpy as np
    import synth
    g = synth.make_system(1).grid
    lig48 = synth.make_system(2, with_grid=False).ligands[0]
    lig100 = synth.make_ligand(np.random.default_rng([105, 7]), 100, 2)
    out = []
    for name, lig in (("c2_ligand_48_atoms", lig48),
                      ("ligand_100_atoms", lig100)):
        ctx = pkg.Context(seed=1, device=0)
        ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
        lid = ctx.ligand_setup(dataclasses_replace_states(lig, 1))
        ctx.pair_setup(lid, synth.pair_params(lig))
        rng = np.random.default_rng(3)
        xs = torch.as_tensor(
            (lig.x0[0][None] + rng.normal(scale=0.1, size=(n_conf,
                                                           lig.n_atoms, 3))
             ).astype(np.float32), device="cuda:0").contiguous()
        res = {}
        for forces in (True, False):
            ctx.pair_evaluate(lid, xs, forces=forces)       # warm-up
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                terms, _f = ctx.pair_evaluate(lid, xs, forces=forces)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            assert np.isfinite(terms.cpu().numpy()).all()
            n = lig.n_atoms
            res["forces" if forces else "energies_only"] = {
                "ms_per_call": ms, "configs_per_s": n_conf / ms * 1e3,
                "ordered_pairs_per_s": n_conf * n * (n - 1) / ms * 1e3}
        ctx.close()
        out.append({"workload": name, "atoms": lig.n_atoms,
                    "configurations": n_conf, **res})
    return {"kernel": out, "in_sampler": full_pathway_cost(pkg, torch)}


def full_pathway_cost(pkg, torch, sweeps=512):
    """What the pair terms cost inside the sampler (the paper's Full
    pathway): a 48-atom ligand grown without nonbonded clashes, 64 replicas
    of the production ladder (L = 20) on 128^3 grids of 2000 receptor atoms
    kept 3 A from it, the mean sweep time over graph replays of 64 sweeps
    (HIP events on the library's stream) and the HMC acceptance, with the
    ligand's pair terms out of and in its energy."""
    import dataclasses
    import numpy as np
    import synth
    c2 = synth.make_system(2, with_grid=False)
    base = c2.ligands[0]
    lig = synth.make_ligand(np.random.default_rng([102, 77]), base.n_atoms,
                            base.n_states, box=10.0, far_sep=3.0)
    nn, h = 128, 0.25
    edge = (nn - 1) * h
    pts, q, sig, eps = synth.make_receptor(
        np.random.default_rng([102, 78]), 2000, edge, 0.3 * edge,
        avoid_xyz=lig.x0[0])
    nodes = synth.grids_from_points(pts, q, sig, eps, nn, h,
                                    device="cuda:0")
    g = synth.Grid((nn,) * 3, (-(nn - 1) * h / 2,) * 3, h, (4, 0, 0), nodes)
    L = c2.n_leapfrog
    res = {"atoms": lig.n_atoms, "replicas": lig.n_states, "leapfrog": L,
           "sweeps_timed": sweeps}
    for on in (False, True):
        # each from the start geometry: configurations sampled without the
        # pair terms are not relaxed with respect to them
        ctx = pkg.Context(seed=c2.seed, device=0)
        ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
        lid = ctx.ligand_setup(lig)
        ctx.pair_setup(lid, synth.pair_params(lig, seed=2))
        ctx.pair_sample(lid, on)
        ctx.hmc_sweep(128, L, exchange_every=1)
        torch.cuda.synchronize()
        before = ctx.get_stats(lid)
        ctx.set_timing(True, every=1)
        ctx.hmc_sweep(sweeps, L, exchange_every=1)
        ms, n = ctx.get_timing(ctx.TIMER_HMC)
        ctx.set_timing(False)
        after = ctx.get_stats(lid)
        acc = (after["hmc_acc"].sum() - before["hmc_acc"].sum()) / max(
            after["hmc_try"].sum() - before["hmc_try"].sum(), 1)
        res["with_pair_terms" if on else "without"] = {
            "sweep_us": ms * 1e3, "hmc_acceptance": float(acc)}
        ctx.close()
    res["cost_ratio"] = (res["with_pair_terms"]["sweep_us"] /
                         res["without"]["sweep_us"])
    return res


def dataclasses_replace_states(lig, K):
    """The ligand with a K-state ladder (the pair terms do not depend on
    the state)."""
    import dataclasses
    import numpy as np
    return dataclasses.replace(lig, T=np.full(K, 300.0),
                               w=np.ones((K, lig.scale.shape[1])),
                               dt=np.ones(K), x0=lig.x0[:K])


def paper_production(pkg, torch, g, lig, res, L, seed, n_cycles=15,
                     iters=1000, snaps=50):
    """Production on the initialised ladder as the paper runs it (Equilibration
    and production): cycles of `iters` iterations of an HMC move, 20
    external moves in the states with alpha < 0.01 and 25 exchange sweeps
    over separations 1..5, `snaps` snapshots per cycle; between cycles the
    state-insertion check (neighbour exchange acceptance below 0.4); the
    equilibrated start by equilibration detection on the sum over states of
    each state's reduced potential; BPMF by MBAR over every other state of the ladder
    (one solve holds at most 128 states), with its spread over cycles."""
    import dataclasses
    import numpy as np
    K = res["n_states"]
    alpha = np.asarray(res["alpha"])
    every = iters // snaps
    lg = dataclasses.replace(lig, T=res["T"], w=res["w"], dt=res["dt"],
                             x0=np.ascontiguousarray(res["x"][:, 0],
                                                     np.float32))
    ctx = pkg.Context(seed=seed + 13, device=0)
    ctx.grid_upload(g.nodes, g.origin, g.spacing, g.transform)
    lid = ctx.ligand_setup(lg, sample_capacity=n_cycles * snaps)
    kw = dict(exchange_every=1, exchange_scheme=1, max_sep=5,
              exchange_sweeps=25, external_moves=20,
              external_k_max=int((alpha < 0.01).sum()), sample_every=every)
    inserts = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prev = ctx.get_stats(lid)
    for _ in range(n_cycles):
        ctx.hmc_sweep(iters, L, **kw)
        st = ctx.get_stats(lid)
        acc = (st["ex_acc"] - prev["ex_acc"]) / np.maximum(
            st["ex_try"] - prev["ex_try"], 1)
        prev = st
        inserts.append(len(pkg.protocol_insert(alpha, acc, 0.4)) - K)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    n_rec = n_cycles * snaps
    u = ctx.energy_matrix(lid, None, n_samples=n_rec * K)
    # equilibration detected on the whole ladder: the sum over states of
    # each state's reduced potential on its own sample of that snapshot
    tot = torch.diagonal(u.view(K, n_rec, K), dim1=0, dim2=2).sum(dim=1)
    t_eq, g_eq, _ = pkg.detect_equilibration(tot.cpu().numpy(), 50)
    sub = np.arange(0, K, 2)
    if sub[-1] != K - 1:
        sub = np.append(sub, K - 1)
    rec = np.arange(t_eq, n_rec)
    cols = torch.as_tensor((rec[:, None] * K + sub[None, :]).reshape(-1),
                           device=u.device)
    rows = torch.as_tensor(sub, device=u.device)
    us = u.index_select(0, rows).index_select(1, cols).contiguous()
    f, var, _ = ctx.mbar(us, np.full(len(sub), len(rec)), tol=1e-10,
                         max_iter=200)
    per = snaps
    parts, ns = [], []
    for cyc in range(n_cycles):
        r = np.arange(max(cyc * per, t_eq), (cyc + 1) * per)
        if len(r) < per // 2:
            continue
        cc = torch.as_tensor((r[:, None] * K + sub[None, :]).reshape(-1),
                             device=u.device)
        parts.append(u.index_select(0, rows).index_select(1, cc).contiguous())
        ns.append(np.full(len(sub), len(r)))
    fb = ctx.mbar_batch(parts, ns, tol=1e-10, max_iter=200)
    blk = np.array([r[0][-1] - r[0][0] for r in fb])
    st = ctx.get_stats(lid)
    acc = st["ex_acc"] / np.maximum(st["ex_try"], 1)
    ctx.close()
    return {"states": int(K), "cycles": n_cycles, "iterations_per_cycle": iters,
            "snapshots_per_cycle": snaps, "seconds": sec,
            "ms_per_iteration": sec / (n_cycles * iters) * 1e3,
            "states_to_insert_per_cycle": inserts,
            "neighbour_exchange_min": float(acc.min()),
            "equilibrated_from_snapshot": int(t_eq),
            "equilibration_observable_inefficiency": float(g_eq),
            "mbar_states": int(len(sub)),
            "bpmf_kT": float(f[-1] - f[0]),
            "sigma_mbar_kT": float(np.sqrt(max(var[-1], 0.0))),
            "cycle_bpmf_kT": [float(b) for b in blk],
            "cycle_sd_kT": float(blk.std(ddof=1)) if len(blk) > 1 else None}


T_START = time.perf_counter()


def progress(what):
    """One line on stderr as each part of the run ends (the JSON result
    line goes to stdout at the end)."""
    print(f"bench: {what} ({time.perf_counter() - T_START:.1f} s)",
          file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the "
              "path shards by ligand/replica range without collectives, see "
              "the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "repeats": 5}))
        return

    import synth
    import paper_1507_03703_amd as pkg

    if args.pairs_only:
        print(json.dumps({"pair_terms": pair_leg(pkg, torch)}))
        return

    if args.init_only:
        print(json.dumps(init_leg(pkg, torch)))
        return

    if args.learned_only:
        print(json.dumps(learned_leg(pkg, torch, train_steps=args.train_steps,
                                     burn=args.burn_sweeps,
                                     long_sweeps=args.long_sweeps,
                                     prod_sweeps=args.prod_sweeps)))
        return

    def bulk():
        return [bulk_leg(pkg, torch, synth.make_system(
            int(c), grid_device=args.grid_device))
            for c in args.bulk_configs.split(",") if c]

    if args.bulk_only:
        print(json.dumps({"bulk_interpolation": bulk()}))
        return

    system = synth.make_system(args.config, grid_device=args.grid_device)
    proposals = training = None
    if args.config == 5 and args.proposals:
        proposals, training = train_proposals(
            pkg, torch, system, steps=args.proposal_train_steps)
        progress("proposals trained")
    r = run_workload(pkg, torch, system, args.steps, args.warmup,
                     sweeps=args.sweeps, tune=len(system.ligands) > 1,
                     waves=args.waves, task_order=args.task_order,
                     proposals=proposals, metrics_path=args.metrics)
    progress(f"{system.name}: {args.steps} timed steps")
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
        "roofline": roofline(r, system.name),
        "kernels_ms": {"hmc_sweep": r["hmc_ms"],
                       "sweep_unit_per_sweep": r["unit_ms"],
                       "energy_matrix": r["cmp_ms"]},
        "result": r["result"],
        "setup_s": r["setup_s"],
    }
    if training:
        out["proposal_training"] = training
    if r["tuned"]:
        out["autotune"] = r["tuned"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_seconds)
        progress("cpu baseline")
    del system

    def extra(config):
        es = synth.make_system(config, grid_device=args.grid_device)
        re = run_workload(pkg, torch, es, 1, 1, tune=len(es.ligands) > 1,
                          waves=args.waves, task_order=args.task_order)
        leg = {"value": re["value"], "unit": "atom-evals/s",
               "ms_per_step": re["ms_per_step"], "steps": 1, "warmup": 1,
               "config": describe(es, re),
               "roofline": roofline(re, es.name),
               "autotune": re["tuned"], "waves": re["waves"],
               "result": re["result"]}
        if not args.no_cpu_baseline:
            # the oracle on a bounded sample of this workload too (half the
            # headline's CPU time)
            leg["cpu_baseline"] = cpu_baseline(es, args.cpu_seconds / 2)
        return leg

    if args.production and args.config != 2:
        out["production_single_ligand"] = extra(2)
        progress("production single-ligand leg")
    if args.batched and args.config != 3:
        out["batched"] = extra(3)
        progress("batched leg")
    if args.bulk:
        out["bulk_interpolation"] = bulk()
        progress("bulk interpolation leg")
    if args.init:
        out["initialization"] = init_leg(pkg, torch)
        progress("initialisation leg")
    if args.pairs:
        out["pair_terms"] = pair_leg(pkg, torch)
        progress("pair-term leg")
    if args.learned:
        out["learned_proposal"] = learned_leg(
            pkg, torch, train_steps=args.train_steps, burn=args.burn_sweeps,
            long_sweeps=args.long_sweeps, prod_sweeps=args.prod_sweeps)
        if args.init:
            # both ladders end in the same two states: the same BPMF
            pp = out["initialization"]["paper_protocol"]
            ref = out["learned_proposal"]["reference"]
            pp["bpmf_minus_long_plain_run_kT"] = pp["bpmf_kT"] - ref["bpmf_kT"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
