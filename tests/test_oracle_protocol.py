"""Pins of the ladder-initialisation oracle (oracle/protocol.py) against
what the paper and the mathematics fix: derivative formulas against finite
differences, the schedule's end points, thermodynamic length in closed form
for a harmonic family (the number of states s-spaced steps take), the
geometric temperature ladder of a constant-heat-capacity system, agreement
of the grid path's temperature term with the temperature-only formula, the
resampled law of SIR, the paper's time-step rule, the exchange acceptance of
two Gaussian states by quadrature, the inefficiency of an AR(1) series and
equilibration detection on a series with a transient, and the placements'
rigidity and uniform law in the site sphere."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import protocol as P


@pytest.mark.parametrize("a", [0.0, 0.1, 0.3, 0.45, 0.55, 0.7, 0.9, 1.0])
def test_schedule_derivatives_match_finite_differences(a):
    h = 1e-6
    lo, hi = max(a - h, 0.0), min(a + h, 1.0)
    fd_sg = (P.alpha_sg(hi) - P.alpha_sg(lo)) / (hi - lo)
    fd_g = (P.alpha_g(hi) - P.alpha_g(lo)) / (hi - lo)
    assert abs(P.d_alpha_sg(a) - fd_sg) < 1e-5
    assert abs(P.d_alpha_g(a) - fd_g) < 1e-4 * max(1.0, abs(fd_g))


def test_schedule_end_points():
    T, w = P.state_of(0.0, P.SOFT, 5, 600.0, 300.0)
    assert T == 600.0 and np.all(np.abs(w) < 1e-200)
    T, w = P.state_of(1.0, P.SOFT, 5, 600.0, 300.0)
    assert T == 300.0 and np.allclose(w, [1, 1, 1, 0, 0], atol=1e-15)
    T, w = P.state_of(0.5, P.SOFT, 5, 600.0, 300.0)
    assert T == 450.0 and np.allclose(w, [0, 0, 0, 1, 1])
    T, w = P.state_of(0.25, P.LINEAR, 3, 600.0, 300.0)
    assert T == 525.0 and np.all(w == 0.25)


def test_thermodynamic_length_of_a_harmonic_family():
    """u_alpha(x) = (1 + c alpha) x^2 / 2 in units of kT: du/dalpha =
    c x^2 / 2 has sigma = c / (sqrt(2) lambda) with lambda = 1 + c alpha,
    so the length is ln(1 + c) / sqrt(2) and steps of speed s take about
    length / s of them."""
    c, s = 9.0, 0.01
    T = 1.0 / oracle.R_GAS              # k T = 1
    a, n = 0.0, 0
    while a < 1.0:
        lam = 1.0 + c * a
        sig_psi = c / (math.sqrt(2.0) * lam)     # sigma of Psi = c x^2 / 2
        a = P.next_alpha(a, sig_psi, 0.0, 123.0, P.LINEAR, s, T, T)
        n += 1
    L = math.log(1.0 + c) / math.sqrt(2.0)
    assert abs(n - L / s) <= 2, (n, L / s)


def test_temperature_ladder_is_geometric_for_constant_heat_capacity():
    """U = x^2 / 2 per degree of freedom: sigma[U] = k T / sqrt(2) per
    degree, so each step multiplies T by 1 + sqrt(2) s / sqrt(d) -- the
    geometric ladder -- and stops at the target."""
    d, s = 24, 0.05
    T, Ts = 300.0, []
    while T < 600.0:
        sig = oracle.R_GAS * T * math.sqrt(d / 2.0)
        T = P.next_temperature(T, sig, s, 600.0)
        Ts.append(T)
    ratio = 1.0 + math.sqrt(2.0 / d) * s
    assert Ts[-1] == 600.0
    assert np.allclose(np.array(Ts[1:-1]) / np.array(Ts[:-2]), ratio,
                       rtol=1e-12)
    assert P.next_temperature(400.0, 5.0, s, 300.0) < 400.0


def test_grid_path_temperature_term_matches_temperature_path():
    """With no grid coupling (sigma of Psi zero) the grid path's third term
    moves T(alpha) by exactly the temperature-only step s k T^2 / sigma[U]
    (sigma[u] = sigma[U] / (k T))."""
    T_H, T_T, s = 600.0, 300.0, 0.2
    for a, sig_U in ((0.0, 40.0), (0.3, 12.0), (0.8, 70.0)):
        T = P.temperature(a, T_H, T_T)
        sig_u = sig_U / (oracle.R_GAS * T)
        a2 = P.next_alpha(a, 0.0, 0.0, sig_u, P.SOFT, s, T_H, T_T)
        T2 = P.temperature(a2, T_H, T_T)
        T2_ref = P.next_temperature(T, sig_U, s, T_T)
        assert abs(T2 - T2_ref) < 1e-9 * T


def test_next_alpha_clips_and_handles_zero_spread():
    assert P.next_alpha(0.9, 0.0, 0.0, 0.0, P.SOFT, 0.2, 600, 300) == 1.0
    assert P.next_alpha(0.99, 1.0, 1.0, 1e-3, P.SOFT, 0.2, 600, 300) == 1.0
    a = P.next_alpha(0.0, 50.0, 50.0, 3.0, P.SOFT, 0.2, 600, 300)
    assert 0.0 < a < 0.01


def test_sir_resamples_the_target_law():
    """Samples of N(0, 1) resampled with weights exp[u_k - u_k+1] for
    u_k+1 = (x - 1)^2 / 2 follow N(1, 1)."""
    rng = np.random.default_rng(3)
    x = rng.normal(size=40000)
    logw = x * x / 2 - (x - 1.0) ** 2 / 2
    idx = P.sir(logw, 4000, seed=5, lig=0, state=1)
    y = x[idx]
    assert abs(y.mean() - 1.0) < 0.08
    assert abs(y.std() - 1.0) < 0.06


def test_sir_frequencies_and_zero_weights():
    logw = np.log(np.array([1.0, 0.0, 3.0, 2.0, 4.0]) + 1e-300)
    logw[1] = -np.inf
    idx = P.sir(logw, 20000, seed=9, lig=2, state=3)
    f = np.bincount(idx, minlength=5) / 20000
    p = np.array([1, 0, 3, 2, 4]) / 10
    assert f[1] == 0.0
    assert np.all(np.abs(f - p) < 5 * np.sqrt(p * (1 - p) / 20000) + 1e-12)


def test_time_step_rule():
    assert P.adapt_dt(1.0, 0.9, 0.125) == (1.125, False)
    assert P.adapt_dt(1.0, 0.6, 0.125) == (1.0, True)
    assert P.adapt_dt(1.0, 0.4, 0.125) == (1.0, True)
    assert P.adapt_dt(1.0, 0.8, 0.125) == (1.0, True)
    assert P.adapt_dt(1.0, 0.3, 0.125) == (0.75, False)
    assert P.adapt_dt(1.0, 0.05, 0.125) == (0.5, False)
    assert P.adapt_dt(0.25, 0.05, 0.125) == (0.125, False)
    assert P.adapt_dt(0.125, 0.05, 0.125) == (0.125, True)


def test_mean_exchange_acceptance_of_two_gaussian_states():
    """States u_a = a x^2 / 2 and u_b = b x^2 / 2: E[min(1, exp(-Delta))]
    over x ~ N(0, 1/a), y ~ N(0, 1/b) by quadrature equals the oracle's
    sample mean, and identical states always exchange."""
    a, b = 1.0, 2.5
    rng = np.random.default_rng(11)
    n = 200000
    x = rng.normal(scale=1 / math.sqrt(a), size=n)
    y = rng.normal(scale=1 / math.sqrt(b), size=n)
    m = P.mean_pacc(a * x * x / 2, b * x * x / 2, a * y * y / 2, b * y * y / 2)

    def f(yv, xv):
        d = (a - b) * (yv * yv - xv * xv) / 2
        px = math.sqrt(a / (2 * math.pi)) * math.exp(-a * xv * xv / 2)
        py = math.sqrt(b / (2 * math.pi)) * math.exp(-b * yv * yv / 2)
        return px * py * min(1.0, math.exp(-d))
    ref, _ = integrate.dblquad(f, -8, 8, -8, 8, epsabs=1e-7)
    assert abs(m - ref) < 0.005, (m, ref)
    assert P.mean_pacc(x, x, y, y) == 1.0


def test_inefficiency_and_equilibration_detection():
    rng = np.random.default_rng(7)
    phi, N = 0.8, 20000
    e = rng.normal(size=N)
    z = np.zeros(N)
    for t in range(1, N):
        z[t] = phi * z[t - 1] + e[t]
    g_ref = (1 + phi) / (1 - phi)
    t0, g, neff = P.detect_equilibration(z)
    assert t0 < N // 10
    assert abs(g - g_ref) < 0.2 * g_ref
    # a transient of about 5 * 100 samples in front of the stationary part
    zt = z[:4000] + 30.0 * np.exp(-np.arange(4000) / 100.0)
    t0, g, neff = P.detect_equilibration(zt)
    assert 200 <= t0 <= 1000, t0
    for cand in range(0, 4000, 40):
        from oracle.estimators import statistical_inefficiency
        assert (4000 - cand) / statistical_inefficiency(zt[cand:]) <= neff + 1e-9


def test_insert_states():
    out = P.insert_states([0.0, 0.2, 0.5, 1.0], [0.9, 0.3, 0.5])
    assert out == [0.0, 0.2, 0.35, 0.5, 1.0]
    assert P.insert_states([0.0, 1.0], [0.1]) == [0.0, 0.5, 1.0]


def test_placements_are_rigid_and_uniform_in_the_site():
    rng = np.random.default_rng(2)
    n = 7
    conf = rng.normal(scale=2.0, size=(2, n, 3))
    mass = rng.uniform(1, 16, size=n)
    center, radius = np.array([1.0, -2.0, 0.5]), 6.0
    poses = P.placements(conf, mass, center, radius, 300, 4, seed=13, lig=1)
    assert poses.shape == (2 * 300 * 4, n, 3)
    poses = poses.reshape(2, 300, 4, n, 3)
    com = (mass[None, None, None, :, None] * poses).sum(3) / mass.sum()
    r = np.linalg.norm(com - center, axis=-1)
    assert np.all(r <= radius * (1 + 1e-12))
    # uniform in the ball: P(r < R/2) = 1/8, mean r = 3R/4
    rr = r[0, :, 0]
    assert abs((rr < radius / 2).mean() - 0.125) < 5 * math.sqrt(
        0.125 * 0.875 / 300)
    assert abs(rr.mean() / radius - 0.75) < 0.05
    # same site position for every orientation and configuration
    assert np.allclose(com[0, :, 0], com[1, :, 3])
    for c in range(2):
        d0 = np.linalg.norm(conf[c][:, None] - conf[c][None], axis=-1)
        for i, o in ((0, 0), (17, 2), (299, 3)):
            d = np.linalg.norm(poses[c, i, o][:, None] - poses[c, i, o][None],
                               axis=-1)
            assert np.allclose(d, d0, atol=1e-10)
