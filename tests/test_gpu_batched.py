"""Batched sampling of many ligands of uneven size in one context: every
ligand's replicas go through the same per-sweep launches (grouped by the
number of wavefronts a replica uses), each ligand with its own ladder,
Philox stream, exchange and sample store.  Parity is lock-step against one
oracle sampler per checked ligand (tests/lockstep.py), at test size and on
sampled ligands of the full 256-ligand, 160^3-grid workload and of the
32-ligand, 256^3-grid workload; the autotuner must leave the sampler state
untouched.
"""
import json

import numpy as np
import pytest

import oracle
import synth
from gpu_util import make_context, print_case, require_gpu, torch
from lockstep import lockstep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _uneven_ligands():
    """The 24-atom, 8-state ligand plus batched-workload ligands (32 states
    each) spanning 10..80 atoms, so that one and two wavefront replicas
    share a sweep."""
    c1 = synth.make_system(1)
    c3 = synth.make_system(3, n_ligands=60, with_grid=False)
    counts = np.array([l.n_atoms for l in c3.ligands])
    pick = [int(np.argmin(counts)), int(np.argmax(counts)),
            int(np.argsort(counts)[len(counts) // 2]),
            int(np.nonzero(counts > 64)[0][0])]
    ligs = [c1.ligands[0]] + [c3.ligands[i] for i in dict.fromkeys(pick)]
    return c1.grid, ligs


@pytest.mark.parametrize("waves", [0, 4, "pins"])
def test_lockstep_uneven_batch(waves):
    """Automatic, uniform and per-ligand launch shapes; the shapes' launches
    of one sweep run side by side."""
    g, ligs = _uneven_ligands()
    print_case("batched lockstep", [l.n_atoms for l in ligs], "waves", waves)
    ctx, ids = make_context(g, ligs, seed=41)
    if waves == "pins":
        pins = [8, 1, 2, 4, 1, 2][:len(ids)]
        for i, w in zip(ids, pins):
            ctx.set_ligand_waves(i, w)
        used = [ctx.get_waves(i) for i in ids]
        assert used == [max(w, -(-l.n_atoms // 64))
                        for w, l in zip(pins, ligs)]
    else:
        ctx.set_waves(waves)
        used = [ctx.get_waves(i) for i in ids]
    for lig, w in zip(ligs, used):
        assert w >= -(-lig.n_atoms // 64)
    if waves != 4:
        assert len(set(used)) >= 2       # several launch shapes in one sweep
    n = lockstep(ctx, oracle.OGrid(g), list(zip(ids, ligs)), 41, 3, 10,
                 "uneven")
    assert sum(n.values()) >= len(ligs)
    ctx.close()


def _state(ctx, lid):
    st = ctx.get_replicas(lid)
    xs, cs = ctx.get_samples(lid)
    return st, ctx.get_stats(lid), xs, cs


def _same(a, b):
    (sa, ta, xa, ca), (sb, tb, xb, cb) = a, b
    for key in ("x", "state_of_replica", "comps", "counter"):
        if not np.array_equal(sa[key], sb[key]):
            return key
    for key in ("hmc_acc", "hmc_try", "ex_acc", "ex_try", "nonfinite"):
        if not np.array_equal(ta[key], tb[key]):
            return key
    if not (np.array_equal(xa, xb) and np.array_equal(ca, cb)):
        return "samples"
    return None


def test_task_order_does_not_change_results():
    """Heaviest ligands first (the default) and ligand by ligand give the
    same sampler state bit for bit: plain and graph sweeps, deferred
    exchange and records, round trips."""
    g, ligs = _uneven_ligands()
    print_case("task order", [l.n_atoms for l in ligs])
    runs = []
    for order in (1, 0):
        ctx, ids = make_context(g, ligs, seed=23, capacity=24)
        assert ctx.get_task_order() == 1
        ctx.set_task_order(order)
        assert ctx.get_task_order() == order
        ctx.set_graph(0)
        ctx.hmc_sweep(5, 10, exchange_every=1, sample_every=1)
        ctx.set_graph(8)
        ctx.hmc_sweep(17, 10, exchange_every=1, sample_every=1)
        runs.append(([_state(ctx, i) for i in ids],
                     [ctx.get_round_trips(i) for i in ids]))
        if order == 0:
            with pytest.raises(RuntimeError):
                ctx.set_task_order(2)
        ctx.close()
    (sa, ta), (sb, tb) = runs
    for i, (x, y) in enumerate(zip(sa, sb)):
        assert _same(x, y) is None, (i, _same(x, y))
    assert ta == tb


def test_autotune_leaves_state_unchanged(tmp_path):
    g, ligs = _uneven_ligands()
    print_case("autotune state")
    a, ids = make_context(g, ligs, seed=5, capacity=12)
    a.hmc_sweep(3, 10, exchange_every=1, sample_every=1)
    before = [_state(a, i) for i in ids]
    cache = tmp_path / "tune.json"
    chosen, table = a.autotune(n_sweeps=4, n_leapfrog=10,
                               cache_path=str(cache), signature="uneven")
    assert chosen in (0, 1, 2, 4, 8)
    assert np.isfinite(table[str(chosen) if chosen else "auto"])
    after = [_state(a, i) for i in ids]
    for i, (x, y) in enumerate(zip(before, after)):
        assert _same(x, y) is None, (i, _same(x, y))
    # the run continues as if tuned from the start of its second half
    a.hmc_sweep(5, 10, exchange_every=1, sample_every=1)
    b, ids_b = make_context(g, ligs, seed=5, capacity=12)
    b.hmc_sweep(3, 10, exchange_every=1, sample_every=1)
    b.set_waves(chosen)
    order = a.get_task_order()
    assert order in (0, 1)
    b.set_task_order(order)
    tuned = [a.get_waves(i) for i in ids]
    for j, w in zip(ids_b, tuned):
        b.set_ligand_waves(j, w)
    b.hmc_sweep(5, 10, exchange_every=1, sample_every=1)
    for i, j in zip(ids, ids_b):
        assert _same(_state(a, i), _state(b, j)) is None, i
    # the cached choice is reused without timing
    rec = json.loads(cache.read_text())
    assert len(rec) == 1 and list(rec.values())[0]["chosen"] == chosen
    assert list(rec.values())[0]["waves"] == tuned
    assert list(rec.values())[0]["task_order"] == order
    for j in ids_b:
        b.set_ligand_waves(j, 0)
    b.set_task_order(1 - order)
    again, table2 = b.autotune(cache_path=str(cache), signature="uneven")
    assert again == chosen and table2 == table
    assert [b.get_waves(j) for j in ids_b] == tuned
    assert b.get_task_order() == order
    with pytest.raises(RuntimeError):
        b.set_ligand_waves(ids_b[0], 3)
    a.close()
    b.close()


def test_full_batched_workload_sampled_ligands():
    """All 256 ligands (10..80 atoms, 32 states each) on the shared 160^3
    grid, tuned as the benchmark tunes them: two lock-step sweeps checked on
    sampled ligands, then a 64-sweep graph replay that must equal plain
    launches bit for bit on every ligand."""
    system = synth.make_system(3, grid_device="cuda:0")
    g, ligs = system.grid, system.ligands
    counts = np.array([l.n_atoms for l in ligs])
    print_case("c3 full", len(ligs), counts.min(), counts.max())
    ctx, ids = make_context(g, ligs, seed=system.seed)
    chosen, _ = ctx.autotune(n_sweeps=8, n_leapfrog=system.n_leapfrog)
    print_case("c3 waves", chosen)
    check = sorted({0, int(np.argmin(counts)), int(np.argmax(counts)),
                    len(ligs) // 2, len(ligs) - 1})
    lockstep(ctx, oracle.OGrid(g), [(ids[i], ligs[i]) for i in check],
             system.seed, 2, system.n_leapfrog, "c3")
    ref, ids_r = make_context(g, ligs, seed=system.seed)
    ref.set_waves(chosen)
    ref.set_graph(0)
    ref.hmc_sweep(2, system.n_leapfrog, exchange_every=1)
    ctx.hmc_sweep(64, system.n_leapfrog, exchange_every=1)
    ref.hmc_sweep(64, system.n_leapfrog, exchange_every=1)
    torch.cuda.synchronize()
    for i, j in zip(ids, ids_r):
        a, b = ctx.get_replicas(i), ref.get_replicas(j)
        for key in ("x", "state_of_replica", "comps", "counter"):
            assert np.array_equal(a[key], b[key]), (i, key)
    acc = np.concatenate([ctx.get_stats(i)["hmc_acc"] for i in ids])
    assert acc.sum() > 0.5 * 66 * 32 * len(ids)
    ctx.close()
    ref.close()


def test_large_grid_workload_sampled_ligands():
    """32 ligands of 40..100 atoms (one or two wavefronts of atoms) with 32
    states each on the shared 256^3 grid (201 MB, flat indices up to 5e7):
    lock-step sweeps on sampled ligands, including the widest, and the
    energy matrix of recorded samples against the oracle's brute force."""
    system = synth.make_system(5, grid_device="cuda:0")
    g, ligs = system.grid, system.ligands
    counts = np.array([l.n_atoms for l in ligs])
    print_case("c5 full", len(ligs), counts.min(), counts.max())
    ctx, ids = make_context(g, ligs, seed=system.seed, capacity=2)
    check = sorted({int(np.argmin(counts)), int(np.argmax(counts)),
                    len(ligs) // 2})
    og = oracle.OGrid(g)
    lockstep(ctx, og, [(ids[i], ligs[i]) for i in check], system.seed, 2,
             system.n_leapfrog, "c5")
    ctx.hmc_sweep(4, system.n_leapfrog, exchange_every=1, sample_every=2)
    i = check[-1]
    lig, lid = ligs[i], ids[i]
    K = lig.n_states
    u = ctx.energy_matrix(lid, None, n_samples=2 * K).cpu().numpy()
    xs, _ = ctx.get_samples(lid)
    X = xs.reshape(-1, lig.n_atoms, 3)
    ol = oracle.OLigand(lig)
    ref = oracle.ukn(og, ol, X)
    _, mags = oracle.components(og, ol, X)
    beta = 1.0 / (oracle.R_GAS * lig.T)
    assert np.all(np.abs(u - ref) <=
                  1e-5 * beta[:, None] * mags.sum(axis=1)[None, :] + 1e-12)
    ctx.close()


@pytest.mark.parametrize("large", ["most", "few"])
def test_energy_matrix_batch_equals_per_ligand_calls(large):
    """One batched u_kn call over ligands of one and two wavefronts (recorded
    samples for some, explicit device samples for others) writes exactly
    the matrices of per-ligand calls, and matches the oracle's brute force.
    "most": the ligands of over 64 atoms hold most of the work (one launch
    for all); "few": three samples each (the two launches side by side)."""
    g, ligs = _uneven_ligands()
    print_case("energy_matrix batch", [l.n_atoms for l in ligs], large)
    ctx, ids = make_context(g, ligs, seed=9, capacity=6)
    ctx.hmc_sweep(12, 10, exchange_every=1, sample_every=2)
    rng = np.random.default_rng(9)
    samples, ns = [], []
    for p, l in enumerate(ligs):
        if large == "few" and l.n_atoms > 64:
            x = l.x0[0][None] + rng.normal(scale=0.3, size=(3, l.n_atoms, 3))
            samples.append(torch.tensor(x, dtype=torch.float32,
                                        device="cuda:0"))
            ns.append(3)
        elif p % 2:
            x = l.x0[0][None] + rng.normal(scale=0.3, size=(37, l.n_atoms, 3))
            samples.append(torch.tensor(x, dtype=torch.float32,
                                        device="cuda:0"))
            ns.append(37)
        else:
            samples.append(None)
            ns.append(6 * l.n_states)
    batch = ctx.energy_matrix_batch(ids, samples=samples, n_samples=ns)
    og = oracle.OGrid(g)
    for p, (lid, l) in enumerate(zip(ids, ligs)):
        one = ctx.energy_matrix(lid, samples[p], n_samples=ns[p])
        assert torch.equal(batch[p], one), p
        if samples[p] is None:
            xs, _ = ctx.get_samples(lid)
            X = xs.reshape(-1, l.n_atoms, 3)
        else:
            X = samples[p].cpu().numpy()
        ol = oracle.OLigand(l)
        ref = oracle.ukn(og, ol, X)
        _, mags = oracle.components(og, ol, X)
        beta = 1.0 / (oracle.R_GAS * l.T)
        u = batch[p].cpu().numpy()
        assert np.all(np.abs(u - ref) <=
                      1e-5 * beta[:, None] * mags.sum(axis=1)[None, :] +
                      1e-12), p
    with pytest.raises(RuntimeError, match="entry 1"):
        ctx.energy_matrix_batch(ids[:2], samples=[None, None],
                                n_samples=[6 * ligs[0].n_states, 5])
    assert ctx.energy_matrix_batch([], samples=[]) == []
    ctx.close()
