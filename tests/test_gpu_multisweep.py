"""Multi-sweep sampler calls against the oracle and against single-sweep
calls (Sampling: HMC moves, replica exchange every sweep, samples recorded).

Inside a call of several neighbour-scheme sweeps the exchange and record
that end sweep s are taken at the start of sweep s + 1, by both replicas of
each pair, from double-buffered components; a call of one sweep instead
applies them in its closing kernel.  These tests tie the multi-sweep path
to the oracle and to the one-sweep path:

* one call of N sweeps gives the bits of N calls of one sweep (positions,
  labels, components, counters, statistics, recorded samples), with plain
  launches and with captured graphs, at one and two wavefronts of atoms;
* the oracle runs N sweeps on its own while the GPU runs one N-sweep call
  from the same state; where no decision on the oracle's path lies within
  its margin (|ln u + beta dH| > 1e-3 for every HMC move, |ln u + Delta| >
  1e-6 for every exchange attempt) the final labels, statistics and
  recorded states are identical and positions agree to 1e-3 A (float32
  trajectories run N sweeps without being reset to the oracle's; the
  one-sweep lock-step tolerance is 1e-4 A), components to 1e-5 of their
  magnitude sum.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import make_context, print_case, require_gpu
from lockstep import exchange_margins

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _system(which):
    system = synth.make_system(1)
    if which == "c1":
        return system.grid, system.ligands[0]
    lig = synth.make_ligand(np.random.default_rng(90), 90, 8, box=9.0)
    return system.grid, lig


def _snapshot(ctx, lid):
    st = ctx.get_replicas(lid)
    xs, cs = ctx.get_samples(lid)
    stats = ctx.get_stats(lid)
    return st, xs, cs, stats


@pytest.mark.parametrize("which,waves,chunk", [
    ("c1", 0, 0), ("c1", 0, 4), ("c1", 2, 0), ("wide90", 2, 0),
    ("wide90", 2, 4), ("wide90", 4, 0)])
def test_multi_sweep_call_equals_single_sweep_calls(which, waves, chunk):
    print_case("multi-sweep = single sweeps", which, waves, chunk)
    g, lig = _system(which)
    N, L, every = 13, 8, 3
    ctx_a, (la,) = make_context(g, [lig], seed=41, capacity=8)
    ctx_b, (lb,) = make_context(g, [lig], seed=41, capacity=8)
    for c in (ctx_a, ctx_b):
        c.set_waves(waves)
        c.set_graph(chunk)
    ctx_a.hmc_sweep(N, L, exchange_every=1, sample_every=every)
    for _ in range(N):
        ctx_b.hmc_sweep(1, L, exchange_every=1, sample_every=every)
    a, b = _snapshot(ctx_a, la), _snapshot(ctx_b, lb)
    for key in ("x", "state_of_replica", "comps", "counter"):
        assert np.array_equal(a[0][key], b[0][key]), key
    assert a[1].shape[0] == N // every
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    for key in a[3]:
        assert np.array_equal(a[3][key], b[3][key]), key
    assert a[3]["ex_try"].sum() > 0 and a[3]["ex_acc"].sum() > 0
    ctx_a.close()
    ctx_b.close()


def _oracle_run(ol, og, seed, lid, st, N, L, every):
    """N oracle sweeps from the GPU state `st`; returns the sampler and
    whether every decision on its path was clear of the margins."""
    s = oracle.Sampler(og, ol, seed=seed, lig_id=lid, x0=st["x"])
    s.x = np.ascontiguousarray(st["x"].astype(np.float64))
    s.state = np.ascontiguousarray(st["state_of_replica"].astype(np.int32))
    s.rep_of_state = np.ascontiguousarray(
        np.argsort(s.state).astype(np.int32))
    s.comps = np.ascontiguousarray(st["comps"].copy())
    s.sweep_count = int(st["counter"])
    clear = True
    for _ in range(N):
        before = s.state.copy()
        acc, dH, lnu = s.hmc(L)
        beta = 1.0 / (oracle.R_GAS * ol.T[before])
        clear &= bool(np.all(np.abs(lnu + beta * dH) > 1e-3))
        m = exchange_margins(ol, s.comps, s.rep_of_state, s.sweep_count,
                             seed, lid)
        clear &= bool(m.min() > 1e-6)
        s.exchange()
        if (s.sweep_count + 1) % every == 0:
            s.record()
        s.sweep_count += 1
    return s, clear


@pytest.mark.parametrize("which,waves,chunk", [
    ("c1", 0, 0), ("c1", 0, 2), ("wide90", 2, 0), ("wide90", 2, 2)])
def test_multi_sweep_call_lockstep_with_oracle(which, waves, chunk):
    print_case("multi-sweep oracle", which, waves, chunk)
    g, lig = _system(which)
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    N, L, every = 6, 8, 2
    seed = 57
    ctx, (lid,) = make_context(g, [lig], seed=seed, capacity=64)
    ctx.set_waves(waves)
    ctx.set_graph(chunk)
    ctx.hmc_sweep(3, L, exchange_every=1)     # leave the start geometry
    n_clear = 0
    for trial in range(5):
        st = ctx.get_replicas(lid)
        stats0 = ctx.get_stats(lid)
        rec0 = ctx.n_records(lid)
        s, clear = _oracle_run(ol, og, seed, lid, st, N, L, every)
        ctx.hmc_sweep(N, L, exchange_every=1, sample_every=every)
        st2 = ctx.get_replicas(lid)
        stats = ctx.get_stats(lid)
        assert int(st2["counter"]) == int(st["counter"]) + N
        if not clear:
            continue
        n_clear += 1
        assert np.array_equal(st2["state_of_replica"], s.state), trial
        err = np.abs(st2["x"].astype(np.float64) - s.x).max()
        assert err < 1e-3, (trial, err)
        t, m, _ = oracle.energy_batch(og, ol, s.x, np.zeros((ol.K, og.nc)))
        S = m.sum(axis=1)
        assert np.all(np.abs(st2["comps"] - s.comps) <=
                      1e-5 * S[:, None] + 1e-9), trial
        for key, ref in (("hmc_acc", s.hmc_acc), ("hmc_try", s.hmc_try),
                         ("ex_acc", s.ex_acc), ("ex_try", s.ex_try)):
            d = stats[key] - stats0[key]
            # the oracle sampler counts from zero at its start
            assert np.array_equal(d, ref), (trial, key, d, ref)
        xs, cs = ctx.get_samples(lid)
        n_new = N // every
        assert xs.shape[0] == rec0 + n_new
        rx = np.array(s.samples_x).reshape(n_new, ol.K, ol.n, 3)
        rc = np.array(s.samples_c).reshape(n_new, ol.K, -1)
        assert np.abs(xs[rec0:].astype(np.float64) - rx).max() < 1e-3
        _, mr, _ = oracle.energy_batch(og, ol, rx.reshape(-1, ol.n, 3),
                                       np.zeros((n_new * ol.K, og.nc)))
        Sr = mr.sum(axis=1).reshape(n_new, ol.K)
        assert np.all(np.abs(cs[rec0:] - rc) <= 1e-5 * Sr[..., None] + 1e-9)
    assert n_clear >= 3, n_clear
    ctx.close()
