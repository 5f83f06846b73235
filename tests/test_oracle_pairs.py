"""Pins of the intramolecular nonbonded / implicit-solvent oracle
(oracle/pairs.py): the descreening integral against a Monte Carlo volume
integral, the Born energy of a lone ion, Coulomb's law with the constant
from CODATA values, screening of two distant ions, the LJ minimum and 1-4
scaling, rigid-motion invariance, the Born-radius limits and the lone-atom
surface term, and the finite-difference forces against an analytic pair."""
import math

import numpy as np
import pytest
from scipy import constants

from oracle import pairs as O


def _params(n, q=None, rho=None, S=None, sigma=None, eps=None, excl=(),
            p14=(), gamma=0.0):
    ex, o4 = O.masks(n, excl, p14)
    return dict(charge=np.zeros(n) if q is None else np.asarray(q, float),
                sigma=np.full(n, 3.0) if sigma is None else np.asarray(sigma),
                eps=np.zeros(n) if eps is None else np.asarray(eps, float),
                rho=np.full(n, 1.5) if rho is None else np.asarray(rho, float),
                S=np.full(n, 0.8) if S is None else np.asarray(S, float),
                excluded=ex, one_four=o4, lj14=0.5, el14=1 / 1.2,
                eps_solute=1.0, eps_solvent=78.5, gamma=gamma, probe=1.4)


@pytest.mark.parametrize("r,a,s", [(3.0, 1.4, 1.2), (1.5, 1.4, 1.3),
                                   (0.5, 0.8, 2.0), (2.2, 1.0, 1.8),
                                   (1.0, 2.5, 1.0)])
def test_descreening_integral_matches_monte_carlo(r, a, s):
    rng = np.random.default_rng(1)
    m = 2_000_000
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pts = v * (s * rng.uniform(size=m) ** (1 / 3))[:, None]
    pts[:, 0] += r
    d = np.linalg.norm(pts, axis=1)
    f = np.where(d > a, d ** -4, 0.0)
    vol = 4 / 3 * math.pi * s ** 3
    mc = f.mean() * vol / (4 * math.pi)
    se = f.std() * vol / (4 * math.pi) / math.sqrt(m)
    h = O.hct_integral(r, a, s)
    assert abs(h - mc) < 5 * se + 1e-12, (h, mc, se)


def test_coulomb_constant_from_codata():
    k = constants.e ** 2 / (4 * math.pi * constants.epsilon_0) * \
        constants.N_A / 1000.0 * 1e10
    assert abs(k - O.K_COULOMB) < 1e-6 * k


def test_lone_ion_born_energy_and_surface_term():
    q, rho = 0.7, 1.7
    p = _params(1, q=[q], rho=[rho], gamma=0.0225936)
    e = O.energy_terms(np.zeros((1, 3)), p)
    rt = rho - O.DIELECTRIC_OFFSET
    tau = 1.0 - 1.0 / 78.5
    assert e[2] == pytest.approx(-0.5 * O.K_COULOMB * tau * q * q / rt,
                                 rel=1e-14)
    assert e[3] == pytest.approx(4 * math.pi * 0.0225936 * (rho + 1.4) ** 2 *
                                 (rho / rt) ** 6, rel=1e-14)
    assert e[0] == 0.0 and e[1] == 0.0


def test_coulomb_and_screening_of_distant_ions():
    r = 60.0
    x = np.array([[0.0, 0, 0], [r, 0, 0]])
    p = _params(2, q=[0.4, -0.3])
    e = O.energy_terms(x, p)
    assert e[1] == pytest.approx(O.K_COULOMB * 0.4 * -0.3 / r, rel=1e-14)
    R = O.born_radii(x, p["rho"], p["S"])
    tau = 1.0 - 1.0 / 78.5
    self_e = -0.5 * O.K_COULOMB * tau * (0.4 ** 2 / R[0] + 0.3 ** 2 / R[1])
    cross = -O.K_COULOMB * tau * 0.4 * -0.3 / r
    assert e[2] == pytest.approx(self_e + cross, rel=1e-6)
    # the distant partner barely descreens: R close to the offset radius
    assert np.all(np.abs(R - (p["rho"] - O.DIELECTRIC_OFFSET)) < 1e-3)


def test_lj_minimum_exclusions_and_one_four_scaling():
    sg, ep = [3.2, 3.6], [0.2, 0.05]
    s, e = 3.4, math.sqrt(0.01)
    x = np.array([[0.0, 0, 0], [2 ** (1 / 6) * s, 0, 0]])
    p = _params(2, sigma=sg, eps=ep)
    assert O.energy_terms(x, p)[0] == pytest.approx(-e, rel=1e-13)
    p14 = _params(2, sigma=sg, eps=ep, p14=[(0, 1)], q=[0.3, 0.3])
    full = _params(2, sigma=sg, eps=ep, q=[0.3, 0.3])
    a, b = O.energy_terms(x, p14), O.energy_terms(x, full)
    assert a[0] == pytest.approx(0.5 * b[0], rel=1e-14)
    assert a[1] == pytest.approx(b[1] / 1.2, rel=1e-14)
    ex = _params(2, sigma=sg, eps=ep, excl=[(0, 1)], p14=[(0, 1)],
                 q=[0.3, 0.3])
    c = O.energy_terms(x, ex)
    assert c[0] == 0.0 and c[1] == 0.0 and c[2] == b[2]


def test_born_radius_limits():
    rho, S = np.array([1.5, 1.6]), np.array([0.8, 0.8])
    rt = rho - O.DIELECTRIC_OFFSET
    prev = None
    for r in (8.0, 5.0, 4.0, 3.0, 2.5, 1.8, 1.2):
        R = O.born_radii(np.array([[0.0, 0, 0], [r, 0, 0]]), rho, S)
        assert np.all(R >= rt - 1e-12)
        assert np.all(R <= 1.0 / (1.0 / rt - 1.0 / rho) + 1e-9)
        # while the spheres do not overlap, a closer neighbour descreens
        # more (overlapping volume inside an atom's own sphere does not
        # count, so the trend can turn)
        if prev is not None and r >= 3.0:
            assert np.all(R >= prev - 1e-12)
        prev = R


def test_rigid_motion_invariance_and_fd_forces():
    rng = np.random.default_rng(6)
    n = 7
    x = rng.uniform(-3, 3, size=(n, 3))
    p = _params(n, q=rng.uniform(-0.5, 0.5, n), sigma=rng.uniform(3, 4, n),
                eps=rng.uniform(0.05, 0.3, n), rho=rng.uniform(1.3, 1.9, n),
                S=rng.uniform(0.72, 0.9, n), excl=[(0, 1), (1, 2), (0, 2)],
                p14=[(0, 3)], gamma=0.0225936)
    e = O.energy_terms(x, p)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0],
                   [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    e2 = O.energy_terms(x @ Rz.T + np.array([1.0, -2.0, 0.5]), p)
    assert np.allclose(e, e2, rtol=1e-11, atol=1e-11)
    F = O.forces(x, p)
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-6 * np.abs(F).max())


def test_fd_forces_of_a_coulomb_pair():
    r = 4.0
    x = np.array([[0.0, 0, 0], [r, 0, 0]])
    p = _params(2, q=[0.5, 0.5])
    p["eps_solvent"] = 1.0   # no GB: tau = 0
    F = O.forces(x, p)
    f = O.K_COULOMB * 0.25 / r ** 2
    assert F[1, 0] == pytest.approx(f, rel=1e-8)
    assert F[0, 0] == pytest.approx(-f, rel=1e-8)


# --------------------------------------------------------------------------
# the pair terms inside the sampled energy (oracle.c): the same definition
# as the pair oracle above, its forces, and the integrator with them
# --------------------------------------------------------------------------

def _pair_system(n=12, seed=5, K=2):
    import synth
    lig = synth.make_ligand(np.random.default_rng(seed), n, K, box=10.0,
                            far_sep=3.0)
    p = synth.pair_params(lig, seed=seed)
    return lig, p


def _oracle_params(p, n):
    ex, o4 = O.masks(n, p["exclusions"], p["pairs14"])
    q = dict(p)
    q.update(excluded=ex, one_four=o4)
    return q


def _zero_grid(n=4):
    import synth
    nodes = np.zeros((n, n, n, 3), np.float32)
    return synth.Grid((n, n, n), (-1.0,) * 3, 0.5, (4, 0, 0), nodes)


@pytest.mark.parametrize("n", [12, 30])
def test_c_pair_energy_is_the_pair_oracle(oracle_lib, n):
    import oracle
    lig, p = _pair_system(n, seed=n)
    og = oracle.OGrid(_zero_grid())
    on, off = oracle.OLigand(lig, pairs=p), oracle.OLigand(lig)
    q = _oracle_params(p, n)
    rng = np.random.default_rng(1)
    for _ in range(4):
        x = lig.x0[0] + rng.normal(scale=0.2, size=(n, 3))
        t1, m1, _ = oracle.energy(og, on, np.zeros(3), x, forces=False)
        t0, m0, _ = oracle.energy(og, off, np.zeros(3), x, forces=False)
        e = O.energy_terms(x, q)
        assert abs((t1[3] - t0[3]) - e.sum()) <= 1e-12 * np.abs(e).sum()
        assert np.all(t1[:3] == t0[:3]) and np.all(t1[4:] == t0[4:])
        assert m1[3] - m0[3] >= abs(e.sum()) * (1 - 1e-12)


def test_c_pair_forces_are_minus_the_gradient(oracle_lib):
    import oracle
    n = 10
    lig, p = _pair_system(n, seed=3)
    og = oracle.OGrid(_zero_grid())
    on, off = oracle.OLigand(lig, pairs=p), oracle.OLigand(lig)
    q = _oracle_params(p, n)
    x = lig.x0[0] + np.random.default_rng(2).normal(scale=0.2, size=(n, 3))
    _, _, F1 = oracle.energy(og, on, np.zeros(3), x)
    _, _, F0 = oracle.energy(og, off, np.zeros(3), x)
    Fp = F1 - F0
    ref = np.zeros_like(x)
    h = 1e-4
    for i in range(n):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            ref[i, a] = -(O.energy_terms(xp, q).sum() -
                          O.energy_terms(xm, q).sum()) / (2 * h)
    assert np.max(np.abs(Fp - ref)) <= 1e-6 * np.max(np.abs(ref)) + 1e-8
    # rigid-motion invariance of the pair energy: no net force or torque
    s = np.max(np.abs(Fp))
    assert np.max(np.abs(Fp.sum(0))) < 1e-6 * s
    assert np.max(np.abs(np.cross(x, Fp).sum(0))) < 1e-5 * s


def test_verlet_with_pair_terms_is_reversible_and_second_order(oracle_lib):
    import oracle
    lig, p = _pair_system(12, seed=7)
    og, ol = oracle.OGrid(_zero_grid()), oracle.OLigand(lig, pairs=p)
    x0 = lig.x0[0].astype(np.float64)
    v0 = oracle.momenta(ol, 600.0, 7, 0, 0, 0)
    x1, v1, H, _ = oracle.verlet(og, ol, np.zeros(3), 0.5, 40, x0, v0)
    x2, v2, _, _ = oracle.verlet(og, ol, np.zeros(3), 0.5, 40, x1, -v1)
    assert np.max(np.abs(x2 - x0)) < 1e-9 and np.max(np.abs(v2 + v0)) < 1e-9
    errs = []
    for dt in (0.4, 0.2, 0.1):
        n = int(round(8.0 / dt))
        _, _, H, _ = oracle.verlet(og, ol, np.zeros(3), dt, n, x0, v0)
        errs.append(abs(H[1] - H[0]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs
