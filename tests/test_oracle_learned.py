"""Pins of the oracle's learned pose proposal: rotation maps, pose
decomposition, MLP gradients, the mixture density folded onto SE(3), exact
sampling, and invariance of the target under the independence
Metropolis-Hastings move (Sampling: external-coordinate moves, here with a
learned proposal)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats
from scipy.spatial.transform import Rotation

from oracle import learned as Lr


def test_rodrigues_matches_scipy_and_log_inverts():
    rng = np.random.default_rng(0)
    for _ in range(200):
        w = rng.normal(size=3)
        w *= rng.uniform(0, math.pi) / np.linalg.norm(w)
        R = Lr.rodrigues(w)
        assert np.allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=1e-13)
        assert np.allclose(Lr.log_rotation(R), w, atol=1e-8)
    # near the identity and near pi
    for th in (1e-9, 1e-5, math.pi - 1e-3, math.pi - 3e-5, math.pi - 1e-6,
               math.pi):
        n = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
        R = Lr.rodrigues(th * n)
        w = Lr.log_rotation(R)
        assert np.allclose(Lr.rodrigues(w), R, atol=1e-9)


def test_pose_decomposition_rebuilds_configuration():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(9, 3)) * 2
    m = rng.uniform(1, 12, 9)
    c0 = np.array([0.5, -0.2, 0.1])
    t, R, y = Lr.pose(x, m, (0, 1, 2), c0)
    assert np.allclose(R.T @ R, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(R) - 1) < 1e-12
    assert np.allclose(Lr.rebuild(t, R, y, c0), x, atol=1e-12)
    # internal coordinates are invariant under rigid motion
    Q = Rotation.random(random_state=3).as_matrix()
    x2 = x @ Q.T + 1.7
    _, _, y2 = Lr.pose(x2, m, (0, 1, 2), c0)
    assert np.allclose(y, y2, atol=1e-12)


def _params(rng):
    p = Lr.init_weights(rng)
    for k in p:
        p[k] = p[k] + 0.05 * rng.normal(size=p[k].shape)
    return p


def test_nll_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = _params(rng)
    B = 6
    f = rng.normal(size=(B, Lr.N_FEAT))
    t = rng.normal(size=(B, 3))
    w = rng.normal(size=(B, 3))
    loss, g, _ = Lr.nll_grad(p, f, t, w)
    eta = 1e-5
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, 12, replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eta
            lp, _, _ = Lr.nll_grad(p, f, t, w)
            flat[i] = old - eta
            lm, _, _ = Lr.nll_grad(p, f, t, w)
            flat[i] = old
            fd = (lp - lm) / (2 * eta)
            an = g[name].reshape(-1)[i]
            # relative 1e-6, with a floor at the round-off of the
            # difference quotient (~1e-16 * |loss| / eta)
            assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-9, (name, i, fd, an)


def test_mixture_density_is_normalised_in_r6():
    rng = np.random.default_rng(3)
    p = _params(rng)
    out, _ = Lr.forward(p, rng.normal(size=(1, Lr.N_FEAT)))
    mp = Lr.mixture(out)
    # importance sampling from the mixture itself: E[1] trivially; instead
    # integrate p_mix over a box by Monte Carlo with uniform points
    n = 400000
    lo = np.minimum(mp["mu_t"][0] - 6 * mp["s_t"][0], -0.1).min()
    hi = np.maximum(mp["mu_t"][0] + 6 * mp["s_t"][0], 0.1).max()
    lw = np.minimum(mp["mu_w"][0] - 6 * mp["s_w"][0], 0).min()
    hw = np.maximum(mp["mu_w"][0] + 6 * mp["s_w"][0], 0).max()
    t = rng.uniform(lo, hi, (n, 3))
    w = rng.uniform(lw, hw, (n, 3))
    mp_n = {k: np.repeat(v, n, axis=0) for k, v in mp.items()}
    val = np.exp(Lr.log_pmix(mp_n, t, w))
    vol = (hi - lo) ** 3 * (hw - lw) ** 3
    est = val.mean() * vol
    err = val.std() * vol / math.sqrt(n)
    assert abs(est - 1) < 4 * err


def _fib_sphere(n):
    i = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * i / n)
    th = math.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi),
                     np.cos(phi)], 1)


def test_folded_density_gives_the_rotation_angle_law_of_samples():
    """Rotation angles of exp(omega) for omega drawn from the mixture follow
    the density 2 (1 - cos th) * int_{S^2} q_R(th n) dOmega obtained from the
    folded SE(3) density; KS test."""
    rng = np.random.default_rng(4)
    p = _params(rng)
    out, _ = Lr.forward(p, rng.normal(size=(1, Lr.N_FEAT)))
    mp = Lr.mixture(out)
    row = {k: v[0] for k, v in mp.items()}
    # samples
    th_s = []
    for _ in range(4000):
        _, t, w = Lr.sample(row, rng.uniform(), rng.normal(size=3),
                            rng.normal(size=3))
        th_s.append(np.linalg.norm(Lr.log_rotation(Lr.rodrigues(w))))
    # angle density from the folded density (t integrated out: evaluate at a
    # fixed t and divide by the translation marginal, which factorises per
    # component only, so integrate t numerically through ln q with t fixed at
    # each component mean would be wrong; use the rotation marginal mixture)
    rot = {"logit": row["logit"], "mu_t": np.zeros((8, 3)),
           "s_t": np.ones((8, 3)), "mu_w": row["mu_w"], "s_w": row["s_w"]}
    dirs = _fib_sphere(240)
    ths = np.linspace(1e-4, math.pi, 160)
    dens = []
    for th in ths:
        acc = 0.0
        for nvec in dirs:
            R = Lr.rodrigues(th * nvec)
            # q over (t, R) with a standard-normal t factor in every
            # component: divide it out at t = 0
            lq = Lr.log_q_se3(rot, np.zeros(3), R) + 1.5 * math.log(TWO_PI)
            acc += math.exp(lq)
        dens.append(2 * (1 - math.cos(th)) * acc * 4 * math.pi / len(dirs))
    dens = np.array(dens)
    cdf = integrate.cumulative_trapezoid(dens, ths, initial=0.0)
    assert abs(cdf[-1] - 1) < 5e-3
    cdf /= cdf[-1]
    pv = stats.kstest(th_s, lambda v: np.interp(v, ths, cdf)).pvalue
    assert pv > 1e-3


TWO_PI = 2 * math.pi


def test_independence_move_preserves_the_target():
    """With the grid switched off the target over the pose is the restraint
    on the centre of mass times Haar on the orientation; a chain of
    independence moves from an arbitrary (fixed) mixture must reproduce the
    Haar angle law (1 - cos th)/pi and the COM radial law."""
    rng = np.random.default_rng(5)
    x0 = np.array([[0.0, 0, 0], [1.5, 0, 0], [0.3, 1.4, 0.2], [-1.0, -0.8,
                                                                 0.9]])
    m = np.ones(4)
    c0 = np.zeros(3)
    d0, k, beta = 1.0, 40.0, 1.0 / (8.314462618e-3 * 300.0)

    def energy(x):
        d = np.linalg.norm((m[:, None] * x).sum(0) / m.sum() - c0)
        return 0.5 * k * max(d - d0, 0.0) ** 2
    row = {"logit": np.array([0.2, -0.3, 0.0, 0.5, -1.0, 0.1, 0.3, -0.2]),
           "mu_t": rng.normal(scale=0.3, size=(8, 3)),
           "s_t": rng.uniform(0.4, 0.9, (8, 3)),
           "mu_w": rng.normal(scale=1.0, size=(8, 3)),
           "s_w": rng.uniform(0.5, 1.4, (8, 3))}
    x = x0.copy()
    ths, ds = [], []
    nacc = 0
    for it in range(20000):
        x, a, _ = Lr.pose_move(x, m, (0, 1, 2), c0, row, energy, beta,
                               rng.uniform(), rng.normal(size=3),
                               rng.normal(size=3), rng.uniform())
        nacc += a
        if it >= 200 and it % 4 == 0:
            _, R, _ = Lr.pose(x, m, (0, 1, 2), c0)
            # orientation relative to the starting frame
            _, R0, _ = Lr.pose(x0, m, (0, 1, 2), c0)
            ths.append(np.linalg.norm(Lr.log_rotation(R @ R0.T)))
            ds.append(np.linalg.norm((m[:, None] * x).sum(0) / m.sum()))
    assert nacc > 1000
    haar = lambda v: (np.asarray(v) - np.sin(v)) / math.pi  # noqa: E731
    assert stats.kstest(ths, haar).pvalue > 1e-3
    g = np.linspace(0, 3, 3001)
    pdf = g ** 2 * np.exp(-0.5 * beta * k * np.maximum(g - d0, 0) ** 2)
    cdf = integrate.cumulative_trapezoid(pdf, g, initial=0)
    cdf /= cdf[-1]
    assert stats.kstest(ds, lambda v: np.interp(v, g, cdf)).pvalue > 1e-3
