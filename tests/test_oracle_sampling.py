"""Pins of the oracle's HMC (velocity-Verlet trial moves, Sampling section),
replica exchange (Eq. repXacc) and counter-based random numbers."""
import math

import numpy as np
import pytest
from scipy import stats, integrate

import oracle
import synth


def _zero_grid(n=4):
    nodes = np.zeros((n, n, n, 3), np.float32)
    return synth.Grid((n, n, n), (-1.0,) * 3, 0.5, (4, 0, 0), nodes)


# ---------------------------------------------------------------- Philox ---

def test_philox_known_answers(oracle_lib):
    # published known-answer vectors of Philox-4x32-10 (Random123)
    assert oracle.philox((0, 0, 0, 0), (0, 0)) == \
        (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)
    assert oracle.philox((0xffffffff,) * 4, (0xffffffff,) * 2) == \
        (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)
    assert oracle.philox((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344),
                         (0xa4093822, 0x299f31d0)) == \
        (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)


def test_momenta_are_maxwell_boltzmann(oracle_lib):
    lig = synth.toy_ligand(np.zeros((400, 3)), [[0, 1]], 0.0, [450.0], [0.0],
                           mass=3.0)
    ol = oracle.OLigand(lig)
    zs = []
    for sweep in range(10):
        v = oracle.momenta(ol, 450.0, 1234, 0, 0, sweep)
        zs.append(v.reshape(-1) / math.sqrt(oracle.R_GAS * 450.0 / 3.0 * 1e-4))
    z = np.concatenate(zs)
    assert stats.kstest(z, "norm").pvalue > 1e-3


# --------------------------------------------------------- velocity Verlet

@pytest.fixture(scope="module")
def smooth_system(oracle_lib):
    rng = np.random.default_rng(5)
    lig = synth.make_ligand(rng, 12, 2)
    return oracle.OGrid(_zero_grid()), oracle.OLigand(lig), lig


def test_verlet_reversibility(smooth_system):
    og, ol, lig = smooth_system
    x0 = lig.x0[0].astype(np.float64)
    v0 = oracle.momenta(ol, 600.0, 7, 0, 0, 0)
    x1, v1, H, _ = oracle.verlet(og, ol, np.zeros(3), 1.0, 50, x0, v0)
    x2, v2, H2, _ = oracle.verlet(og, ol, np.zeros(3), 1.0, 50, x1, -v1)
    assert np.max(np.abs(x2 - x0)) < 1e-10
    assert np.max(np.abs(v2 + v0)) < 1e-10
    # detailed balance of the HMC kernel: the reversed move has -dH, so
    # pi(x)phi(p) min(1, e^{-b dH}) == pi(x')phi(p') min(1, e^{b dH})
    beta = 1.0 / (oracle.R_GAS * 600.0)
    dH, dHr = H[1] - H[0], H2[1] - H2[0]
    assert abs(dH + dHr) < 1e-9
    lhs = math.exp(-beta * H[0]) * min(1.0, math.exp(-beta * dH))
    rhs = math.exp(-beta * H[1]) * min(1.0, math.exp(-beta * dHr))
    assert abs(lhs - rhs) <= 1e-12 * max(lhs, rhs)


def test_verlet_energy_error_scales_as_dt_squared(smooth_system):
    og, ol, lig = smooth_system
    rng = np.random.default_rng(3)
    x0 = lig.x0[0].astype(np.float64) + rng.normal(scale=0.05,
                                                   size=lig.x0[0].shape)
    v0 = oracle.momenta(ol, 600.0, 9, 0, 0, 0)
    errs = []
    for dt in (0.4, 0.2, 0.1):
        n = int(round(20.0 / dt))
        # max |H(t) - H(0)| over the trajectory, sampled every 1 fs
        x, v = x0.copy(), v0.copy()
        H0 = None
        m = 0.0
        per = int(round(1.0 / dt))
        for _ in range(n // per):
            x, v, H, _ = oracle.verlet(og, ol, np.zeros(3), dt, per, x, v)
            if H0 is None:
                H0 = H[0]
            m = max(m, abs(H[1] - H0))
        errs.append(m)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


# ----------------------------------------------------- HMC distributions

def test_two_atom_toy_exact_marginals(oracle_lib):
    """One bond, no grid coupling: the bond length has density
    r^2 exp(-beta K (r - r0)^2) and the COM distance from the site has
    density d^2 exp(-beta k (d - d0)_+^2 / 2)."""
    T, K, r0, d0, kr = 450.0, 30.0, 1.5, 1.0, 40.0
    x = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]])
    lig = synth.toy_ligand(x, [[0, 1]], K, [T], [0.0], mass=1.0, dt=2.0,
                           d0=d0, k_restraint=kr)
    og = oracle.OGrid(_zero_grid())
    ol = oracle.OLigand(lig)
    R = 1
    s = oracle.Sampler(og, ol, seed=77, x0=lig.x0)
    rs, ds = [], []
    for it in range(30000):
        s.sweep(nleap=10, exchange_every=0)
        if it >= 500 and it % 10 == 0:
            xx = s.x[0]
            rs.append(np.linalg.norm(xx[0] - xx[1]))
            ds.append(np.linalg.norm(xx.mean(0)))
    beta = 1.0 / (oracle.R_GAS * T)

    def cdf_factory(pdf, lo, hi):
        grid = np.linspace(lo, hi, 4001)
        p = np.array([pdf(v) for v in grid])
        c = integrate.cumulative_trapezoid(p, grid, initial=0.0)
        c /= c[-1]
        return lambda v: np.interp(v, grid, c)
    cdf_r = cdf_factory(lambda r: r * r * math.exp(-beta * K * (r - r0) ** 2),
                        0.0, 4.0)
    cdf_d = cdf_factory(lambda d: d * d * math.exp(
        -0.5 * beta * kr * max(d - d0, 0.0) ** 2), 0.0, 4.0)
    # thin further to reduce autocorrelation before the KS test
    assert stats.kstest(np.array(rs)[::3], cdf_r).pvalue > 1e-3
    assert stats.kstest(np.array(ds)[::3], cdf_d).pvalue > 1e-3
    assert s.hmc_acc[0] / s.hmc_try[0] > 0.5


def test_creutz_identity(smooth_system):
    """<exp(-beta dH)> = 1 for trial moves started from equilibrium."""
    og, ol, lig = smooth_system
    s = oracle.Sampler(og, ol, seed=5, x0=lig.x0)
    vals = []
    for it in range(3000):
        acc, dH, lnu = s.sweep(nleap=10, exchange_every=0)
        if it >= 300:
            for r in range(ol.K):
                beta = 1.0 / (oracle.R_GAS * ol.T[s.state[r]])
                vals.append(math.exp(-beta * dH[r]))
    vals = np.array(vals)
    g = 1.0
    err = vals.std() / math.sqrt(len(vals) / g)
    assert abs(vals.mean() - 1.0) < 4 * err + 1e-3


# ------------------------------------------------------ replica exchange

def _comps_for_delta(K, T, w, delta_target):
    """Components such that the neighbour attempt (0,1) has delta_target."""
    R = oracle.R_GAS
    comps = np.zeros((K, 4))
    # only psi_ele differs: delta = (b0*w0 - b1*w1) * (P1 - P0)
    b0, b1 = 1 / (R * T[0]), 1 / (R * T[1])
    coef = b0 * w[0, 2] - b1 * w[1, 2]
    comps[1, 3] = delta_target / coef
    return comps


def test_exchange_acceptance_frequency(oracle_lib):
    import ctypes as C
    K = 2
    T = np.array([600.0, 300.0])
    w = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    for target in (-0.5, 0.0, 0.7, 2.0):
        comps = _comps_for_delta(K, T, w, target)
        n, acc = 4000, 0
        for sweep in range(0, 2 * n, 2):  # even sweeps attempt pair (0,1)
            st = np.arange(K, dtype=np.int32)
            rp = np.arange(K, dtype=np.int32)
            a = np.zeros(1, np.int64)
            t = np.zeros(1, np.int64)
            oracle.lib().ora_exchange(
                K, 3, T.ctypes.data_as(C.POINTER(C.c_double)),
                w.ctypes.data_as(C.POINTER(C.c_double)), 99, 0, sweep, 0, 1,
                0, comps.ctypes.data_as(C.POINTER(C.c_double)),
                st.ctypes.data_as(C.POINTER(C.c_int)),
                rp.ctypes.data_as(C.POINTER(C.c_int)),
                a.ctypes.data_as(C.POINTER(C.c_int64)),
                t.ctypes.data_as(C.POINTER(C.c_int64)))
            acc += int(a[0])
            assert t[0] == 1
            assert sorted(st) == [0, 1] and np.all(rp[st] == np.arange(K))
        p = min(1.0, math.exp(-target))
        sd = math.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(acc / n - p) <= 4 * sd + 1e-9


def test_exchange_detailed_balance_and_permutation(oracle_lib):
    """pi_a(x) pi_b(y) p(x,y) == pi_a(y) pi_b(x) p(y,x) for the acceptance
    used by the oracle, and the state<->replica maps stay inverse."""
    rng = np.random.default_rng(4)
    K = 6
    T, w = synth.ladder(K)
    R = oracle.R_GAS
    comps = rng.normal(scale=20, size=(K, 4))
    beta = 1 / (R * T)

    def E(k, c):
        return c[0] + w[k] @ c[1:]
    for a in range(K - 1):
        b = a + 1
        x, y = comps[a], comps[b]
        d_xy = beta[a] * (E(a, y) - E(a, x)) + beta[b] * (E(b, x) - E(b, y))
        lhs = math.exp(-beta[a] * E(a, x) - beta[b] * E(b, y)) * \
            min(1, math.exp(-d_xy))
        rhs = math.exp(-beta[a] * E(a, y) - beta[b] * E(b, x)) * \
            min(1, math.exp(d_xy))
        assert abs(lhs - rhs) <= 1e-12 * max(lhs, rhs)
    lig = synth.toy_ligand(np.zeros((2, 3)), [[0, 1]], 1.0, T, w[:, 0])
    og, ol = oracle.OGrid(_zero_grid()), oracle.OLigand(lig)
    s = oracle.Sampler(og, ol, seed=3, x0=lig.x0)
    s.comps = np.ascontiguousarray(comps)
    for sweep in range(200):
        s.sweep_count = sweep
        s.exchange(scheme=1 if sweep % 3 == 0 else 0, max_sep=5)
        assert np.all(s.rep_of_state[s.state] == np.arange(K))
    assert s.ex_try.sum() > 0


def test_repeated_exchange_sweeps_two_state_chain(oracle_lib):
    """n exchange sweeps in a row at one counter are n steps of the two-state
    Markov chain: from the favoured labelling a swap is accepted with
    p = exp(-delta), the swap back always.  Independent uniforms per sweep
    give P(swapped after n) = (e0 M^n)[1] with M = [[1-p, p], [1, 0]];
    reusing one uniform for every sweep would give 0 for n = 2."""
    K = 2
    T = np.array([600.0, 300.0])
    w = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    lig = synth.toy_ligand(np.zeros((2, 3)), [[0, 1]], 1.0, T, w[:, 0])
    og, ol = oracle.OGrid(_zero_grid()), oracle.OLigand(lig)
    delta = math.log(2.0)
    comps = _comps_for_delta(K, T, w, delta)
    p = math.exp(-delta)
    M = np.array([[1 - p, p], [1.0, 0.0]])
    trials = 3000
    for n in (1, 2, 3, 4):
        s = oracle.Sampler(og, ol, seed=17, x0=lig.x0)
        swapped = 0
        for t in range(trials):
            s.comps = np.ascontiguousarray(comps)
            s.state = np.arange(K, dtype=np.int32)
            s.rep_of_state = np.arange(K, dtype=np.int32)
            s.sweep_count = t
            s.exchange(scheme=1, max_sep=1, n_sweeps=n)
            assert np.all(s.rep_of_state[s.state] == np.arange(K))
            swapped += int(s.state[0] == 1)
        q = np.linalg.matrix_power(M, n)[0, 1]
        sd = math.sqrt(q * (1 - q) / trials)
        assert abs(swapped / trials - q) < 5 * sd + 1e-9, (n, swapped, q)
        assert s.ex_try[0] == n * trials


def test_repeated_exchange_sweeps_stationary_law(oracle_lib):
    """Exchange is Gibbs sampling of the state labelling: with fixed
    configurations, repeated sweeps (scheme 1, all separations) leave the
    law P(labelling) ~ exp(-sum_k beta_k E_k(x_replica in k)) invariant, so
    the labellings seen after each call follow it."""
    import itertools
    K = 3
    T = np.array([600.0, 450.0, 300.0])
    w = np.array([[0.0] * 3, [0.5] * 3, [1.0] * 3])
    R = oracle.R_GAS
    beta = 1 / (R * T)
    rng = np.random.default_rng(8)
    comps = np.ascontiguousarray(rng.normal(scale=1.0, size=(K, 4)))
    lig = synth.toy_ligand(np.zeros((2, 3)), [[0, 1]], 1.0, T, w[:, 0])
    og, ol = oracle.OGrid(_zero_grid()), oracle.OLigand(lig)

    def E(k, c):
        return c[0] + w[k] @ c[1:]
    perms = list(itertools.permutations(range(K)))   # replica in state k
    logp = np.array([-sum(beta[k] * E(k, comps[pm[k]]) for k in range(K))
                     for pm in perms])
    pi = np.exp(logp - logp.max())
    pi /= pi.sum()
    assert pi.min() > 0.02    # a law with every labelling visible
    s = oracle.Sampler(og, ol, seed=23, x0=lig.x0)
    s.comps = comps
    calls = 6000
    seen = np.zeros(len(perms))
    for t in range(calls):
        s.sweep_count = t
        s.exchange(scheme=1, max_sep=2, n_sweeps=4)
        seen[perms.index(tuple(int(r) for r in s.rep_of_state))] += 1
    f = seen / calls
    sd = np.sqrt(pi * (1 - pi) / calls)
    assert np.all(np.abs(f - pi) < 6 * sd), (f, pi)


def test_identical_hamiltonians_always_exchange(oracle_lib):
    K = 5
    T = np.full(K, 300.0)
    lig = synth.toy_ligand(np.zeros((2, 3)), [[0, 1]], 1.0, T, np.zeros(K))
    og, ol = oracle.OGrid(_zero_grid()), oracle.OLigand(lig)
    s = oracle.Sampler(og, ol, seed=3, x0=lig.x0)
    s.comps = np.ascontiguousarray(np.random.default_rng(0).normal(
        size=(K, 4)))
    for sweep in range(100):
        s.sweep_count = sweep
        s.exchange()
    assert np.all(s.ex_acc == s.ex_try)
