"""GPU parity of the external-coordinate moves (Sampling: random rotation
about the centre of mass from a random unit quaternion, Gaussian
translation, Metropolis) against the oracle's moves on the same Philox
draws, their integration into sweep calls, and argument checks.

Tolerances: positions 2e-4 A after up to 8 moves (float rotation and
translation against double); components as for u_kn (1e-5 of the
magnitude sum); decisions compared where |ln u - ln alpha| > 5e-2 for every
move of the replica.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import make_context, print_case, require_gpu
from oracle import external as Ex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("which,sigma,n_moves", [
    ("c1", 0.6, 4), ("c1", 0.25, 8), ("wide90", 0.6, 4),
    ("wide100", 0.3, 6)])
def test_external_moves_match_oracle(which, sigma, n_moves):
    """The 24-atom ligand (one wavefront) and ligands of 90 and 100 atoms
    (two wavefronts: the move's two-wavefront centre of mass and
    evaluation)."""
    print_case("external moves", which, sigma, n_moves)
    system = synth.make_system(1)
    g = system.grid
    if which == "c1":
        lig = system.ligands[0]
    else:
        n = int(which[4:])
        lig = synth.make_ligand(np.random.default_rng(n + 1), n, 8, box=9.0)
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    ctx, (lid,) = make_context(g, [lig], seed=system.seed)
    K = lig.n_states
    checked = accepted = 0
    for rnd in range(3):
        ctx.hmc_sweep(2, 10, exchange_every=1)
        st = ctx.get_replicas(lid)
        before = ctx.get_external_stats(lid)
        ctx.external_move(lid, n_moves=n_moves, k_max=K, sigma=sigma)
        st2 = ctx.get_replicas(lid)
        after = ctx.get_external_stats(lid)
        d_acc = after["acc"] - before["acc"]
        assert np.array_equal(after["tries"] - before["tries"],
                              np.full(K, n_moves))
        for r in range(K):
            k = st["state_of_replica"][r]
            xo, n_acc, lns = Ex.external_moves(
                og, ol, st["x"][r], k, system.seed, lid, r, st["counter"],
                n_moves, sigma)
            if min(abs(lu - la) for la, lu in lns) < 5e-2:
                continue
            checked += 1
            accepted += n_acc
            assert d_acc[k] == n_acc, (rnd, r, d_acc[k], n_acc)
            assert np.max(np.abs(st2["x"][r] - xo)) < 2e-4, (rnd, r)
            if n_acc == 0:
                assert np.array_equal(st2["x"][r], st["x"][r])
                assert np.array_equal(st2["comps"][r], st["comps"][r])
            else:
                c, mags = oracle.components(og, ol, xo[None])
                assert np.all(np.abs(st2["comps"][r] - c[0]) <=
                              1e-5 * mags.sum() + 1e-9), (rnd, r)
    assert checked >= 12 and accepted >= 3, (checked, accepted)
    ctx.close()


@pytest.mark.parametrize("which", ["c1", "wide90"])
def test_long_move_chains_cross_random_number_batches(which):
    """70 moves per call: the rounds of candidate moves cross the 64-move
    batches of random numbers (a batch made anew mid-chain), one and two
    wavefronts, against the oracle's sequential chain."""
    print_case("external moves, 70 per call", which)
    system = synth.make_system(1)
    g = system.grid
    lig = system.ligands[0] if which == "c1" else synth.make_ligand(
        np.random.default_rng(91), 90, 8, box=9.0)
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    ctx, (lid,) = make_context(g, [lig], seed=system.seed)
    K, n_moves, sigma = lig.n_states, 70, 0.25
    checked = 0
    for rnd in range(2):
        ctx.hmc_sweep(2, 10, exchange_every=1)
        st = ctx.get_replicas(lid)
        before = ctx.get_external_stats(lid)
        ctx.external_move(lid, n_moves=n_moves, k_max=K, sigma=sigma)
        st2 = ctx.get_replicas(lid)
        after = ctx.get_external_stats(lid)
        assert np.array_equal(after["tries"] - before["tries"],
                              np.full(K, n_moves))
        d_acc = after["acc"] - before["acc"]
        for r in range(K):
            k = st["state_of_replica"][r]
            xo, n_acc, lns = Ex.external_moves(
                og, ol, st["x"][r], k, system.seed, lid, r, st["counter"],
                n_moves, sigma)
            # ln alpha of a move is good to ~1e-4 in float32 (grid energies
            # of some hundred kT): decisions within 2e-3 of ln u are left out
            if min(abs(lu - la) for la, lu in lns) < 2e-3:
                continue
            checked += 1
            assert d_acc[k] == n_acc, (rnd, r, d_acc[k], n_acc)
            assert np.max(np.abs(st2["x"][r] - xo)) < 5e-4, (rnd, r)
    assert checked >= 8, checked
    ctx.close()


def test_replicas_above_k_max_are_untouched():
    print_case("external k_max")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    ctx, (lid,) = make_context(g, [lig], seed=system.seed)
    ctx.hmc_sweep(3, 10, exchange_every=1)
    st = ctx.get_replicas(lid)
    ctx.external_move(lid, n_moves=5, k_max=2, sigma=0.3)
    st2 = ctx.get_replicas(lid)
    tries = ctx.get_external_stats(lid)["tries"]
    assert np.array_equal(tries, np.where(np.arange(lig.n_states) < 2, 5, 0))
    for r in range(lig.n_states):
        if st["state_of_replica"][r] >= 2:
            assert np.array_equal(st2["x"][r], st["x"][r])
            assert np.array_equal(st2["comps"][r], st["comps"][r])
    ctx.close()


def test_external_moves_inside_sweep_calls_match_host_loop():
    """Units of one sweep closed by external moves (three to a captured
    graph, replayed, and the rest launched plainly) equal sweep and move
    calls from the host, bit for bit, and
    the chain keeps sampling the same states' statistics."""
    print_case("external in sweeps")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    a, (la,) = make_context(g, [lig], seed=system.seed, capacity=8)
    b, (lb,) = make_context(g, [lig], seed=system.seed, capacity=8)
    a.set_graph(3)  # three one-sweep units per graph, two left over
    a.hmc_sweep(8, 10, exchange_every=1, sample_every=2, external_moves=3,
                external_k_max=4, external_sigma=0.4)
    for _ in range(8):
        b.hmc_sweep(1, 10, exchange_every=1, sample_every=2)
        b.external_move(lb, n_moves=3, k_max=4, sigma=0.4)
    sa, sb = a.get_replicas(la), b.get_replicas(lb)
    for key in ("x", "state_of_replica", "comps", "counter"):
        assert np.array_equal(sa[key], sb[key]), key
    xa, ca = a.get_samples(la)
    xb, cb = b.get_samples(lb)
    assert np.array_equal(xa, xb) and np.array_equal(ca, cb)
    ea, eb = a.get_external_stats(la), b.get_external_stats(lb)
    assert np.array_equal(ea["acc"], eb["acc"])
    assert np.array_equal(ea["tries"], eb["tries"])
    assert ea["tries"][:4].sum() == 8 * 3 * 4 and ea["tries"][4:].sum() == 0
    a.close()
    b.close()


def test_external_moves_of_several_ligands_in_one_launch():
    """Ligands of one and two wavefronts and different state counts moved
    by one sweep call (a launch per wavefront count, every ligand's states
    below k_max in it) equal each ligand moved by its own call, bit for
    bit; a ligand with fewer states than k_max has all of them moved."""
    print_case("external, several ligands")
    system = synth.make_system(1)
    g = system.grid
    ligs = [system.ligands[0],
            synth.make_ligand(np.random.default_rng(91), 90, 8, box=9.0),
            synth.make_ligand(np.random.default_rng(5), 30, 4)]
    k_max, nx, sweeps = 6, 3, 4
    a, ia = make_context(g, ligs, seed=system.seed)
    b, ib = make_context(g, ligs, seed=system.seed)
    a.set_graph(2)  # two one-sweep units per graph
    a.hmc_sweep(sweeps, 10, exchange_every=1, external_moves=nx,
                external_k_max=k_max, external_sigma=0.5)
    for _ in range(sweeps):
        b.hmc_sweep(1, 10, exchange_every=1)
        for lb in ib:
            b.external_move(lb, n_moves=nx, k_max=k_max, sigma=0.5)
    for lig, la, lb in zip(ligs, ia, ib):
        sa, sb = a.get_replicas(la), b.get_replicas(lb)
        for key in ("x", "state_of_replica", "comps", "counter"):
            assert np.array_equal(sa[key], sb[key]), (lig.n_atoms, key)
        ea, eb = a.get_external_stats(la), b.get_external_stats(lb)
        assert np.array_equal(ea["acc"], eb["acc"]), lig.n_atoms
        kk = min(k_max, lig.n_states)
        assert np.array_equal(ea["tries"], np.where(
            np.arange(lig.n_states) < kk, sweeps * nx, 0)), lig.n_atoms
    a.close()
    b.close()


def test_external_move_argument_errors():
    print_case("external errors")
    system = synth.make_system(1)
    ctx, (lid,) = make_context(system.grid, system.ligands,
                               seed=system.seed)
    for kw in (dict(n_moves=-1), dict(k_max=-1), dict(sigma=0.0),
               dict(sigma=math.inf)):
        args = dict(ligand_id=lid, n_moves=1, k_max=1, sigma=0.6)
        args.update(kw)
        with pytest.raises(RuntimeError):
            ctx.external_move(**args)
    with pytest.raises(RuntimeError):
        ctx.hmc_sweep(1, 10, external_moves=2, external_sigma=-1.0)
    ctx.external_move(lid, n_moves=0, k_max=3)     # nothing to do
    assert ctx.get_external_stats(lid)["tries"].sum() == 0
    ctx.close()
