"""Pins of the oracle's external-coordinate moves (Sampling: random rotation
about the centre of mass from a random unit quaternion, Gaussian
translation, Metropolis): the quaternion-to-matrix map against an
independent library, the uniform (Haar) law of the rotations it draws, the
rigidity of a move, and invariance of the target distribution."""
import math

import numpy as np
from scipy import integrate, stats
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import external as Ex


def test_quaternion_matrix_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(300):
        u = rng.uniform(0, 1, 3)
        q = Ex.unit_quaternion(*u)
        assert abs(np.linalg.norm(q) - 1) < 1e-14
        R = Ex.quaternion_matrix(q)
        # scipy orders quaternions (x, y, z, w)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(R, ref, atol=1e-13)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-13


def test_random_rotations_are_uniform():
    """Angles of the drawn rotations follow the Haar law (theta - sin
    theta) / pi, and their axes are isotropic."""
    rng = np.random.default_rng(1)
    th, ax = [], []
    for _ in range(20000):
        R = Ex.quaternion_matrix(Ex.unit_quaternion(*rng.uniform(0, 1, 3)))
        v = Rotation.from_matrix(R).as_rotvec()
        th.append(np.linalg.norm(v))
        ax.append(v / max(np.linalg.norm(v), 1e-300))
    haar = lambda t: (np.asarray(t) - np.sin(t)) / math.pi  # noqa: E731
    assert stats.kstest(th, haar).pvalue > 1e-3
    ax = np.array(ax)
    # cos of the polar angle of the axis is uniform on [-1, 1]
    assert stats.kstest(ax[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_move_is_rigid_about_the_centre_of_mass():
    """A move keeps every interatomic distance (so the bonded energy) and
    displaces the centre of mass by exactly sigma z."""
    system = synth.make_system(1)
    lig = system.ligands[0]
    og, ol = oracle.OGrid(system.grid), oracle.OLigand(lig)
    rng = np.random.default_rng(2)
    x = lig.x0[0].astype(np.float64)
    m = lig.mass
    for _ in range(20):
        u3, z3 = rng.uniform(0, 1, 3), rng.normal(size=3)
        xn = Ex.propose(x, m, u3, z3, sigma=0.6)
        d0 = np.linalg.norm(x[:, None] - x[None], axis=-1)
        d1 = np.linalg.norm(xn[:, None] - xn[None], axis=-1)
        assert np.max(np.abs(d0 - d1)) < 1e-12
        c0 = (m[:, None] * x).sum(0) / m.sum()
        c1 = (m[:, None] * xn).sum(0) / m.sum()
        assert np.allclose(c1 - c0, 0.6 * z3, atol=1e-12)
        t0, _, _ = oracle.energy(og, ol, ol.w[0], x, forces=False)
        t1, _, _ = oracle.energy(og, ol, ol.w[0], xn, forces=False)
        assert np.allclose(t0[:3], t1[:3], rtol=1e-9, atol=1e-9)


def test_moves_preserve_the_target():
    """With only the flat-bottom centre-of-mass restraint the target over
    the pose is the restraint on the centre of mass times Haar on the
    orientation; a chain of external moves must reproduce both laws."""
    rng = np.random.default_rng(3)
    x0 = np.array([[0.0, 0, 0], [1.5, 0, 0], [0.3, 1.4, 0.2],
                   [-1.0, -0.8, 0.9]])
    m = np.array([12.0, 14.0, 12.0, 16.0])
    d0, k, beta = 1.0, 40.0, 1.0 / (oracle.R_GAS * 300.0)

    def energy(x):
        c = (m[:, None] * x).sum(0) / m.sum()
        d = np.linalg.norm(c)
        return 0.5 * k * max(d - d0, 0.0) ** 2

    x, e = x0.copy(), energy(x0)
    ths, ds, nacc = [], [], 0
    R0 = None
    for it in range(40000):
        x, a, _, e = Ex.external_move(x, m, energy, beta, rng.uniform(0, 1, 3),
                                      rng.normal(size=3), rng.uniform(),
                                      e_cur=e, sigma=0.6)
        nacc += a
        if it >= 200 and it % 5 == 0:
            c = (m[:, None] * x).sum(0) / m.sum()
            # orientation: the rotation taking the first three atoms' frame
            # of x0 to that of x (rigid, so one Kabsch fit is exact)
            H = (x0 - (m[:, None] * x0).sum(0) / m.sum()).T @ (x - c)
            U, _, Vt = np.linalg.svd(H)
            D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
            R = Vt.T @ D @ U.T
            ths.append(np.linalg.norm(Rotation.from_matrix(R).as_rotvec()))
            ds.append(np.linalg.norm(c))
    assert nacc > 4000
    haar = lambda t: (np.asarray(t) - np.sin(t)) / math.pi  # noqa: E731
    assert stats.kstest(ths, haar).pvalue > 1e-3
    g = np.linspace(0, 3, 3001)
    pdf = g ** 2 * np.exp(-0.5 * beta * k * np.maximum(g - d0, 0) ** 2)
    cdf = integrate.cumulative_trapezoid(pdf, g, initial=0)
    cdf /= cdf[-1]
    assert stats.kstest(ds, lambda v: np.interp(v, g, cdf)).pvalue > 1e-3
