"""Pins of the oracle's estimators: MBAR (used for f_BC,L and f_CD',
Estimation section), the reduced-energy matrix u_kn, the statistical
inefficiency / effective sample size, and the exact-toy quadrature."""
import math

import numpy as np
import pytest
from scipy import optimize, special

import oracle
import synth
from oracle import estimators, toy


def _bar_textbook(w_f, w_r):
    """Bennett's acceptance ratio: the root in df of
    sum_F 1/(1 + (N_F/N_R) exp(w_F - df)) - sum_R 1/(1 + (N_R/N_F)
    exp(w_R + df)) = 0, with w_F = u_1 - u_0 on samples of state 0 and
    w_R = u_0 - u_1 on samples of state 1."""
    nf, nr = len(w_f), len(w_r)
    M = math.log(nf / nr)

    def h(df):
        return np.sum(special.expit(-(M + w_f - df))) - \
            np.sum(special.expit(-(-M + w_r + df)))
    return optimize.brentq(h, -100, 100, xtol=1e-14)


def test_mbar_two_states_equals_bar():
    rng = np.random.default_rng(0)
    x0 = rng.normal(0.0, 1.0, 700)
    x1 = rng.normal(0.8, 1.3, 500)
    x = np.concatenate([x0, x1])
    u = np.stack([0.5 * x ** 2, 0.5 * ((x - 0.8) / 1.3) ** 2])
    f, var, _ = estimators.mbar(u, [700, 500])
    df_bar = _bar_textbook(u[1, :700] - u[0, :700], u[0, 700:] - u[1, 700:])
    assert abs(f[1] - df_bar) < 1e-8


def test_mbar_harmonic_oscillators_exact():
    """Reduced potentials u_k = k_k |x|^2 / 2 in d dimensions have
    f_k - f_0 = (d/2) ln(k_k / k_0)."""
    rng = np.random.default_rng(1)
    d = 3
    ks = np.array([1.0, 1.7, 3.0, 5.0])
    Nk = np.array([400, 300, 300, 500])
    xs = np.concatenate([rng.normal(0, 1 / math.sqrt(k), (n, d))
                         for k, n in zip(ks, Nk)])
    r2 = (xs ** 2).sum(1)
    u = 0.5 * ks[:, None] * r2[None, :]
    f, var, _ = estimators.mbar(u, Nk)
    exact = 0.5 * d * np.log(ks / ks[0])
    assert abs(f[-1] - exact[-1]) < 3 * math.sqrt(var)
    for i in range(1, len(ks)):
        v = estimators.mbar_var(u, Nk, f, i, 0)
        assert abs(f[i] - exact[i]) < 3.5 * math.sqrt(v)


def test_mbar_variance_is_calibrated():
    rng = np.random.default_rng(2)
    ks = np.array([1.0, 2.5, 6.0])
    Nk = np.array([200, 200, 200])
    est, pred = [], []
    for _ in range(150):
        xs = np.concatenate([rng.normal(0, 1 / math.sqrt(k), n)
                             for k, n in zip(ks, Nk)])
        u = 0.5 * ks[:, None] * xs[None, :] ** 2
        f, var, _ = estimators.mbar(u, Nk)
        est.append(f[-1])
        pred.append(math.sqrt(var))
    ratio = np.std(est) / np.mean(pred)
    assert 0.8 < ratio < 1.25
    assert abs(np.mean(est) - 0.5 * math.log(6.0)) < 4 * np.std(est) / \
        math.sqrt(150)


def test_statistical_inefficiency_ar1():
    rng = np.random.default_rng(3)
    for rho in (0.0, 0.5, 0.9):
        n = 200000
        e = rng.normal(size=n)
        a = np.empty(n)
        a[0] = e[0]
        for t in range(1, n):
            a[t] = rho * a[t - 1] + math.sqrt(1 - rho * rho) * e[t]
        g = estimators.statistical_inefficiency(a)
        assert abs(g / ((1 + rho) / (1 - rho)) - 1) < 0.1


def test_ukn_brute_force_equals_factorised(oracle_lib):
    rng = np.random.default_rng(4)
    g = synth.random_grid(rng, n=(20, 20, 20), spacing=0.5,
                          origin=(-4.75,) * 3)
    lig = synth.make_ligand(rng, 10, 5)
    og, ol = oracle.OGrid(g), oracle.OLigand(lig)
    xs = lig.x0[0][None].astype(np.float64) + rng.normal(
        scale=0.3, size=(40, 10, 3))
    u = oracle.ukn(og, ol, xs)
    comps, _ = oracle.components(og, ol, xs)
    beta = 1 / (oracle.R_GAS * lig.T)
    fact = beta[:, None] * (comps[None, :, 0] +
                            np.einsum("kc,nc->kn", lig.w, comps[:, 1:]))
    assert np.allclose(u, fact, rtol=1e-12, atol=1e-12)


def test_toy_quadrature_closed_forms():
    # bond integral: int_0^inf b^2 exp(-a (b - r0)^2) db in closed form
    beta, K, r0 = 0.3, 20.0, 1.2
    a = beta * K
    closed = (1 / (2 * a) + r0 ** 2) * math.sqrt(math.pi) / (2 * math.sqrt(a)) \
        * (1 + math.erf(math.sqrt(a) * r0)) + r0 * math.exp(-a * r0 ** 2) / \
        (2 * a)
    assert abs(toy._ln_zb(beta, K, r0) - math.log(4 * math.pi * closed)) < 1e-11
    # COM integral without field: d0^3/3 + Gaussian shell moments
    k, d0 = 40.0, 1.5
    gam = 0.5 * beta * k
    closed = d0 ** 3 / 3 + math.sqrt(math.pi) / (4 * gam ** 1.5) + d0 / gam + \
        d0 ** 2 * math.sqrt(math.pi) / (2 * math.sqrt(gam))
    assert abs(toy._ln_zc(beta, 0.0, 1.0, 1.0, 0.0, k, d0) -
               math.log(4 * math.pi * closed)) < 1e-11
    # COM integral with field and d0 = 0: a tilted 3-D Gaussian,
    # int exp(-gam |c|^2 - a c_z) d^3c = (pi/gam)^{3/2} exp(a^2 / (4 gam))
    lam, Q, E, phi0 = 0.7, 0.9, 2.5, 1.3
    aa = beta * lam * Q * E
    closed = 1.5 * math.log(math.pi / gam) + aa * aa / (4 * gam) - \
        beta * lam * Q * phi0
    assert abs(toy._ln_zc(beta, lam, Q, E, phi0, k, 0.0) - closed) < 1e-10
