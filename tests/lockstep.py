"""Lock-step parity harness shared by the GPU sampling tests (not collected
by pytest).

Before every sweep the oracle sampler of each checked ligand is set to the
GPU's state; both run one sweep with the same Philox streams and the results
must agree: positions to 1e-4 A, accept decisions exactly except where the
oracle's own margin |ln u + beta dH| < 1e-3 (there float32 rounding may
decide), cached components to 1e-5 of their magnitude sum, state maps exactly
unless an exchange exponent lies within 1e-6 of its uniform.
"""
import numpy as np

import oracle


def sync_oracle(s, st):
    s.x = np.ascontiguousarray(st["x"].astype(np.float64))
    s.state = np.ascontiguousarray(st["state_of_replica"].astype(np.int32))
    s.rep_of_state = np.ascontiguousarray(np.argsort(s.state).astype(np.int32))
    s.comps = np.ascontiguousarray(st["comps"].copy())
    s.sweep_count = int(st["counter"])


def exchange_margins(ol, comps, rep_of_state, sweep, seed, lig):
    """|ln u + delta| of every neighbour attempt the oracle makes this sweep
    (even/odd scheme)."""
    K = ol.K
    out = []
    beta = 1.0 / (oracle.R_GAS * ol.T)
    ros = rep_of_state.copy()
    for a in range(sweep & 1, K - 1, 2):
        ra, rb = ros[a], ros[a + 1]

        def E(k, r):
            return comps[r, 0] + ol.w[k] @ comps[r, 1:]
        delta = beta[a] * (E(a, rb) - E(a, ra)) + \
            beta[a + 1] * (E(a + 1, ra) - E(a + 1, rb))
        lnu = np.log(oracle.uniform(seed, a, lig, 0, sweep, 3 | (1 << 8)))
        out.append(abs(lnu + delta))
    return np.array(out) if out else np.array([np.inf])


def lockstep(ctx, og, checked, seed, n_sweeps, nleap, label, pairs=None):
    """Run n_sweeps single sweeps of every ligand in ctx (exchange every
    sweep) and check each (ligand_id, Ligand) pair of `checked` against its
    own oracle sampler (pairs: {ligand_id: pair parameters} of ligands whose
    pair terms are in the energy).  Returns, per checked ligand, the number
    of sweeps whose decisions were all clear of the rounding margin."""
    samplers = []
    for lid, lig in checked:
        ol = oracle.OLigand(lig, pairs=(pairs or {}).get(lid))
        samplers.append((lid, lig, ol, oracle.Sampler(
            og, ol, seed=seed, lig_id=lid, x0=lig.x0)))
    n_clear = {lid: 0 for lid, _ in checked}
    start = {lid: int(ctx.get_replicas(lid)["counter"]) for lid, _ in checked}
    for sweep in range(n_sweeps):
        pending = []
        for lid, lig, ol, s in samplers:
            sync_oracle(s, ctx.get_replicas(lid))
            state_before = s.state.copy()
            acc, dH, lnu = s.hmc(nleap)
            margin = exchange_margins(ol, s.comps, s.rep_of_state,
                                      s.sweep_count, seed, lid)
            s.exchange()
            s.sweep_count += 1
            beta = 1.0 / (oracle.R_GAS * lig.T[state_before])
            pending.append((np.abs(lnu + beta * dH) > 1e-3, margin))
        ctx.hmc_sweep(1, nleap, exchange_every=1)
        for (lid, lig, ol, s), (ok, margin) in zip(samplers, pending):
            st2 = ctx.get_replicas(lid)
            err = np.abs(st2["x"].astype(np.float64) - s.x).max(axis=(1, 2))
            assert np.all(err[ok] < 1e-4), (label, lid, sweep, err)
            if np.all(ok):
                n_clear[lid] += 1
                t, m, _ = oracle.energy_batch(og, ol, s.x,
                                              np.zeros((ol.K, og.nc)))
                S = m.sum(axis=1)
                assert np.all(np.abs(st2["comps"] - s.comps) <=
                              1e-5 * S[:, None] + 1e-9), (label, lid, sweep)
                if margin.min() > 1e-6:
                    assert np.array_equal(st2["state_of_replica"], s.state), \
                        (label, lid, sweep)
            assert int(st2["counter"]) == start[lid] + sweep + 1
    for lid, lig, ol, s in samplers:
        stats = ctx.get_stats(lid)
        assert stats["hmc_try"].sum() >= n_sweeps * ol.K
    return n_clear
