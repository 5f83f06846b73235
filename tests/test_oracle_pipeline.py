"""Whole-pipeline pin of the oracle: replica-exchange HMC + u_kn + MBAR on the
solvable toy must recover the exact reduced free energies f_k - f_0, and in
particular the synthetic BPMF f_CD' = f_{lambda=1, 300 K} - f_{lambda=0,
600 K} (Estimation section), within three standard errors."""
import math

import numpy as np

import oracle
import synth
from oracle import estimators, toy

TOY = dict(n_atoms=3, bond_K=50.0, q=0.3, field=(2.0, 1.0, -1.5), phi0=3.0,
           d0=2.0, k_rest=100.0, K=6, n_grid=32, h=0.5)


def toy_system():
    """Three-atom chain in a linear electrostatic field (see oracle.toy)."""
    t = TOY
    grid = synth.linear_field_grid(t["n_grid"], t["h"], t["field"], t["phi0"])
    x = np.array([[-1.5, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 1.5, 0.0]])
    T, w = synth.ladder(t["K"])
    lig = synth.toy_ligand(x, [[0, 1], [1, 2]], t["bond_K"], T, w[:, 0],
                           q=t["q"], mass=1.0, dt=2.0, d0=t["d0"],
                           k_restraint=t["k_rest"])
    exact = toy.exact_f(T, w[:, 2], [t["bond_K"]] * 2, lig.bond_par[:, 1],
                        t["q"], t["n_atoms"], np.array(t["field"]), t["phi0"],
                        t["k_rest"], t["d0"])
    return grid, lig, exact


def block_estimate(ukn, K, S, n_blocks=10):
    """MBAR on the whole run, with the standard error taken from the spread
    of MBAR estimates over contiguous time blocks.  Samples are recorded in
    rounds of K (one per state), so a block is a contiguous range of rounds.
    Block averaging covers the correlations that replica exchange creates
    between the sample series of different states."""
    f, _, _ = estimators.mbar(ukn, np.full(K, S))
    per = S // n_blocks
    fb = []
    for b in range(n_blocks):
        cols = slice(b * per * K, (b + 1) * per * K)
        fb.append(estimators.mbar(ukn[:, cols], np.full(K, per))[0])
    fb = np.array(fb)
    sd = fb.std(axis=0, ddof=1) / math.sqrt(n_blocks)
    return f, sd


def test_exact_toy_pipeline_oracle(oracle_lib):
    grid, lig, exact = toy_system()
    og, ol = oracle.OGrid(grid), oracle.OLigand(lig)
    s = oracle.Sampler(og, ol, seed=2024, x0=lig.x0)
    n_sweeps, every = 24000, 8
    for it in range(n_sweeps):
        s.sweep(nleap=10, exchange_every=1,
                sample_every=every if it >= 2000 else 0)
    xs = np.array(s.samples_x)
    K = ol.K
    S = len(xs) // K
    # the ligand must stay well inside the linear-field region
    lo = grid.origin[0] + grid.spacing
    assert np.all(np.abs(xs) < abs(lo))
    ukn = oracle.ukn(og, ol, xs)
    f, sd = block_estimate(ukn, K, S)
    err = f - (exact - exact[0])
    # within 4 block standard errors (the error bar itself is estimated
    # from 10 blocks)
    assert np.all(np.abs(err[1:]) < 4 * sd[1:] + 1e-3), (f, exact, sd)
    acc = s.ex_acc / np.maximum(s.ex_try, 1)
    assert np.all(acc > 0.05)
