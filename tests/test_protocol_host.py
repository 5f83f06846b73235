"""The library's ladder-initialisation steps (host code in libbpmf, no GPU
needed) against the oracle (oracle/protocol.py) on the same inputs:
schedule, per-state spreads, parameter selection on both paths, SIR indices
(bitwise), the time-step rule, mean exchange acceptance, state insertion and
equilibration detection."""
import numpy as np
import pytest

from oracle import protocol as P

pkg = pytest.importorskip("paper_1507_03703_amd")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        pkg.library()
    except ImportError as e:
        pytest.skip(str(e))


@pytest.mark.parametrize("kind,C", [(P.LINEAR, 3), (P.SOFT, 5)])
def test_state_matches_oracle(kind, C):
    for a in np.linspace(0, 1, 23):
        T, w = pkg.protocol_state(a, kind, C, 600.0, 300.0)
        To, wo = P.state_of(a, kind, C, 600.0, 300.0)
        assert T == To
        assert np.allclose(w, wo, rtol=1e-15, atol=0)


@pytest.mark.parametrize("kind,C", [(P.LINEAR, 3), (P.SOFT, 5)])
def test_sigmas_match_oracle(kind, C):
    rng = np.random.default_rng(1 + kind)
    comps = rng.normal(size=(5000, 1 + C)) * np.array([40.0] + [15.0] * C)
    for a in (0.0, 0.2, 0.5, 0.93):
        s = pkg.protocol_sigmas(comps, a, kind, 600.0, 300.0)
        so = P.state_sigmas(comps, a, kind, 600.0, 300.0)
        assert np.allclose(s, so, rtol=1e-12, atol=1e-300)


def test_next_alpha_and_temperature_match_oracle():
    rng = np.random.default_rng(5)
    for _ in range(300):
        kind = int(rng.integers(0, 2))
        a = float(rng.uniform(0, 1))
        sig = rng.uniform(0, 80, size=3) * (rng.uniform(size=3) > 0.15)
        s = float(rng.uniform(0.01, 0.5))
        TH, TT = float(rng.uniform(300, 700)), float(rng.uniform(250, 400))
        got = pkg.protocol_next_alpha(a, sig, kind, s, TH, TT)
        ref = P.next_alpha(a, sig[0], sig[1], sig[2], kind, s, TH, TT)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-15)
        T = float(rng.uniform(250, 700))
        sU, tgt = float(rng.uniform(0, 50)), float(rng.uniform(250, 700))
        assert pkg.protocol_next_temperature(T, sU, 20.0, tgt) == \
            pytest.approx(P.next_temperature(T, sU, 20.0, tgt), rel=1e-13)


def test_sir_indices_bitwise():
    rng = np.random.default_rng(8)
    for trial in range(6):
        n = int(rng.integers(1, 3000))
        logw = rng.normal(scale=[0.5, 3.0, 30.0][trial % 3], size=n)
        if trial % 2:
            logw[rng.uniform(size=n) < 0.2] = -np.inf
            logw[0] = 0.0
        idx = pkg.protocol_sir(logw, 257, 1234 + trial, trial, 3 + trial)
        ref = P.sir(logw, 257, 1234 + trial, trial, 3 + trial)
        assert np.array_equal(idx, ref), trial
        assert np.all(np.isfinite(logw[idx]))


def test_time_step_rule_matches_oracle():
    for dt in (0.125, 0.25, 0.5, 1.0, 1.75, 3.0):
        for acc in (0.0, 0.05, 0.0999, 0.1, 0.25, 0.3999, 0.4, 0.6, 0.8,
                    0.8001, 1.0):
            nd, done = pkg.protocol_adapt_dt(dt, acc, 0.125)
            ref = P.adapt_dt(dt, acc, 0.125)
            assert (nd, done) == ref, (dt, acc)


def test_mean_pacc_matches_oracle():
    rng = np.random.default_rng(4)
    v = [rng.normal(scale=3, size=4000) for _ in range(4)]
    v[0][:7] = np.inf
    got = pkg.protocol_mean_pacc(*v)
    ref = P.mean_pacc(*v)
    assert got == pytest.approx(ref, rel=1e-13)


def test_insert_matches_oracle():
    rng = np.random.default_rng(2)
    for _ in range(20):
        K = int(rng.integers(1, 12))
        al = np.sort(rng.uniform(size=K))
        pa = rng.uniform(size=max(K - 1, 0))
        got = pkg.protocol_insert(al, pa, 0.4)
        assert np.array_equal(got, np.array(P.insert_states(al, pa, 0.4)))


def test_equilibration_detection_matches_oracle():
    rng = np.random.default_rng(9)
    for phi, L in ((0.5, 0.0), (0.9, 40.0), (0.0, 10.0)):
        N = 3000
        e = rng.normal(size=N)
        z = np.zeros(N)
        for t in range(1, N):
            z[t] = phi * z[t - 1] + e[t]
        z += L * np.exp(-np.arange(N) / 80.0)
        t0, g, ne = pkg.detect_equilibration(z, 60)
        r0, rg, rn = P.detect_equilibration(z, 60)
        assert t0 == r0
        assert g == pytest.approx(rg, rel=1e-9)
        assert ne == pytest.approx(rn, rel=1e-9)
