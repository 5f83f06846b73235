"""Replica round trips (the walk of replicas between the two end states of
the ladder) counted by the library against the definition applied on the
host to the state maps observed after every sweep: a trip counts when a
replica that has visited state K-1 since it was last in state 0 returns to
state 0; at setup replica r holds state r.  Bit-equal runs (one
multi-sweep call against single-sweep calls, deferred against immediate
exchange bookkeeping) must count the same trips.
"""
import numpy as np
import pytest

import synth
from gpu_util import make_context, print_case, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def host_round_trips(history, K):
    """The definition on a list of state_of_replica arrays (the first is the
    initial map), one per observation."""
    end = [0 if k == 0 else -1 for k in history[0]]
    trips = 0
    for sor in history[1:]:
        for r, k in enumerate(sor):
            if k == 0:
                trips += end[r] == 1
                end[r] = 0
            elif k == K - 1 and end[r] == 0:
                end[r] = 1
    return trips


def test_host_definition_on_a_hand_made_walk():
    # replica 0: 0 -> 1 -> 2 (top) -> 1 -> 0: one trip; replica 2 starts at
    # the top and reaches 0 without having left 0 first: none
    hist = [[0, 1, 2], [1, 0, 2], [2, 0, 1], [1, 2, 0], [0, 2, 1]]
    assert host_round_trips(hist, 3) == 1


def equal_states(lig):
    """The ligand with every state a copy of its last one: every exchange is
    accepted, so replicas walk the ladder end to end and trips are many."""
    import copy
    l1 = copy.deepcopy(lig)
    K = lig.n_states
    l1.T = np.full(K, lig.T[-1])
    l1.w = np.repeat(lig.w[-1:], K, axis=0)
    l1.dt = np.full(K, lig.dt[-1])
    return l1


@pytest.mark.parametrize("scheme,ladder", [(0, "equal"), (1, "equal"),
                                           (0, "config")])
def test_round_trips_match_the_state_maps(scheme, ladder):
    print_case("round trips", scheme, ladder)
    system = synth.make_system(1)
    g = system.grid
    lig = system.ligands[0]
    if ladder == "equal":
        lig = equal_states(lig)
    K, n = lig.n_states, 300
    kw = dict(exchange_every=1, exchange_scheme=scheme,
              max_sep=3 if scheme else 1)
    a, (la,) = make_context(g, [lig], seed=system.seed)
    hist = [a.get_replicas(la)["state_of_replica"].copy()]
    for _ in range(n):
        a.hmc_sweep(1, 10, **kw)
        hist.append(a.get_replicas(la)["state_of_replica"].copy())
    trips = host_round_trips(hist, K)
    if ladder == "equal":
        assert trips >= 10, trips
    assert a.get_round_trips(la) == trips
    # one call of n sweeps: the same run, the same trips
    b, (lb,) = make_context(g, [lig], seed=system.seed)
    b.hmc_sweep(n, 10, **kw)
    assert np.array_equal(b.get_replicas(lb)["state_of_replica"], hist[-1])
    assert b.get_round_trips(lb) == trips
    a.close()
    b.close()


def test_round_trips_of_a_single_state_and_after_restore():
    print_case("round trips, edge cases")
    system = synth.make_system(1)
    lig, g = system.ligands[0], system.grid
    one = synth.make_ligand(np.random.default_rng(3), 12, 1)
    ctx, (l8, l1) = make_context(g, [lig, one], seed=system.seed)
    ctx.hmc_sweep(50, 10, exchange_every=1)
    assert ctx.get_round_trips(l1) == 0
    before = ctx.get_round_trips(l8)
    # restoring states restarts the tracking from them and keeps the count
    st = ctx.get_replicas(l8)
    ctx.set_replicas(l8, st["x"], st["state_of_replica"], st["comps"],
                     st["counter"])
    assert ctx.get_round_trips(l8) == before
    hist = [st["state_of_replica"].copy()]
    for _ in range(300):
        ctx.hmc_sweep(1, 10, exchange_every=1)
        hist.append(ctx.get_replicas(l8)["state_of_replica"].copy())
    assert ctx.get_round_trips(l8) == before + host_round_trips(
        hist, lig.n_states)
    ctx.close()
