"""Pins of the oracle's intramolecular force field (GAFF functional forms:
harmonic bonds and angles, proper torsions; the U_s(r_L) term of the
alchemical protocol equation) and of the flat-bottom COM restraint
(Eq. binding_site)."""
import math

import numpy as np
import pytest

import oracle
import synth


def _zero_grid(n=4):
    nodes = np.zeros((n, n, n, 3), np.float32)
    return synth.Grid((n, n, n), (-1.0,) * 3, 0.5, (4, 0, 0), nodes)


@pytest.fixture(scope="module")
def system(oracle_lib):
    rng = np.random.default_rng(42)
    lig = synth.make_ligand(rng, 20, 4)
    return oracle.OGrid(_zero_grid()), oracle.OLigand(lig), lig


def test_generated_geometry_is_bonded_minimum(system):
    og, ol, lig = system
    terms, mags, F = oracle.energy(og, ol, np.zeros(3), lig.x0[0])
    assert np.all(np.abs(terms[:4]) < 1e-9)
    assert np.max(np.abs(F)) < 1e-6


def test_bonded_forces_match_central_differences(system):
    og, ol, lig = system
    rng = np.random.default_rng(1)
    x = lig.x0[0].astype(np.float64) + rng.normal(scale=0.15,
                                                  size=lig.x0[0].shape)
    w = np.zeros(3)
    _, _, F = oracle.energy(og, ol, w, x)
    eta = 1e-5
    fd = np.zeros_like(x)
    for i in range(len(x)):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += eta
            xm[i, a] -= eta
            tp, _, _ = oracle.energy(og, ol, w, xp, forces=False)
            tm, _, _ = oracle.energy(og, ol, w, xm, forces=False)
            fd[i, a] = -(tp[:4].sum() - tm[:4].sum()) / (2 * eta)
    rms = np.sqrt(np.mean(F ** 2))
    assert np.max(np.abs(fd - F)) <= 1e-7 * rms + 1e-9


def test_zero_net_force_and_torque(system):
    og, ol, lig = system
    rng = np.random.default_rng(2)
    x = lig.x0[0].astype(np.float64) + rng.normal(scale=0.2,
                                                  size=lig.x0[0].shape)
    _, _, F = oracle.energy(og, ol, np.zeros(3), x)
    scale = np.max(np.abs(F))
    assert np.max(np.abs(F.sum(0))) < 1e-10 * max(scale, 1)
    tau = np.cross(x, F).sum(0)
    assert np.max(np.abs(tau)) < 1e-10 * max(scale, 1) * 10


def _rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def test_rigid_motion_invariance(system):
    og, ol, lig = system
    rng = np.random.default_rng(3)
    x = lig.x0[0].astype(np.float64) + rng.normal(scale=0.2,
                                                  size=lig.x0[0].shape)
    t0, _, F0 = oracle.energy(og, ol, np.zeros(3), x)
    Rm = _rot(rng)
    y = x @ Rm.T + np.array([0.3, -0.2, 0.1])
    t1, _, F1 = oracle.energy(og, ol, np.zeros(3), y)
    assert np.allclose(t0[:3], t1[:3], rtol=1e-12, atol=1e-10)
    assert np.allclose(F0 @ Rm.T, F1, atol=1e-9)


def test_dihedral_closed_forms(oracle_lib):
    L = oracle.lib()
    import ctypes as C

    def dih(a, b, c, d):
        arr = [np.ascontiguousarray(v, np.float64) for v in (a, b, c, d)]
        return L.ora_dihedral(*[v.ctypes.data_as(C.POINTER(C.c_double))
                                for v in arr])
    j, k = np.zeros(3), np.array([0.0, 0.0, 1.0])
    i = np.array([1.0, 0.0, 0.0])
    # cis (eclipsed): 0; trans: pi
    assert abs(dih(i, j, k, np.array([1.0, 0.0, 1.0]))) < 1e-15
    assert abs(abs(dih(i, j, k, np.array([-1.0, 0.0, 1.0]))) - math.pi) < 1e-15
    # IUPAC sign: looking along j->k (+z), the front bond j->i lies on +x and
    # the back bond k->l at angle a measured from +x towards +y; that
    # rotation is clockwise for this viewer, so the torsion angle is +a
    for a in (0.3, 1.2, 2.5, -0.7, -2.9):
        l = np.array([math.cos(a), math.sin(a), 1.0])
        assert abs(dih(i, j, k, l) - a) < 1e-14


def test_angle_closed_form(oracle_lib):
    L = oracle.lib()
    import ctypes as C
    for th in (0.5, 1.0, 1.9, 2.8):
        i = np.array([1.0, 0.0, 0.0]) * 1.3
        j = np.zeros(3)
        k = np.array([math.cos(th), math.sin(th), 0.0]) * 0.7
        arr = [np.ascontiguousarray(v, np.float64) for v in (i, j, k)]
        got = L.ora_angle(*[v.ctypes.data_as(C.POINTER(C.c_double))
                            for v in arr])
        assert abs(got - th) < 1e-14


def test_torsion_energy_closed_form(oracle_lib):
    # 4-atom chain with one torsion, V/2 = 2, n = 3, gamma = 0.4 and no
    # bonds/angles in the energy: E = 2 (1 + cos(3 phi - 0.4))
    x = np.array([[1.0, 0.0, 0.0], [0, 0, 0], [0, 0, 1.0], [0, 0, 1.0]])
    lig = synth.toy_ligand(x[:2], [[0, 1]], 0.0, [300.0], [0.0])
    lig.n_atoms = 4
    lig.mass = np.ones(4)
    lig.scale = np.zeros((4, 3))
    lig.bonds = np.zeros((0, 2), np.int32)
    lig.bond_par = np.zeros((0, 2))
    lig.tors = np.array([[0, 1, 2, 3]], np.int32)
    lig.tors_par = np.array([[2.0, 3.0, 0.4]])
    lig.d0 = 100.0
    ol = oracle.OLigand(lig)
    og = oracle.OGrid(_zero_grid())
    for phi in (0.1, 1.0, -2.0, 3.0):
        xx = x.copy()
        xx[3] = [math.cos(phi), math.sin(phi), 1.0]
        t, _, _ = oracle.energy(og, ol, np.zeros(3), xx, forces=False)
        assert abs(t[2] - 2 * (1 + math.cos(3 * phi - 0.4))) < 1e-13


def test_restraint_closed_form_and_force_split(oracle_lib):
    rng = np.random.default_rng(9)
    x = rng.normal(size=(3, 3))
    lig = synth.toy_ligand(x, [[0, 1], [1, 2]], 0.0, [300.0], [0.0],
                           d0=1.0, k_restraint=100.0)
    lig.mass = np.array([1.0, 2.0, 5.0])
    ol = oracle.OLigand(lig)
    og = oracle.OGrid(_zero_grid())
    for shift in (np.zeros(3), np.array([0.5, 0.2, -0.1]),
                  np.array([2.0, -1.0, 0.7])):
        y = x + shift
        com = (lig.mass[:, None] * y).sum(0) / lig.mass.sum()
        d = np.linalg.norm(com)
        ref = 0.0 if d <= 1.0 else 0.5 * 100.0 * (d - 1.0) ** 2
        t, _, F = oracle.energy(og, ol, np.zeros(3), y)
        assert abs(t[3] - ref) < 1e-12 * max(ref, 1)
        if d > 1.0:
            # bond K = 0, so F is the restraint force; it is shared in
            # proportion to the masses and points back to the site
            Ftot = F.sum(0)
            assert np.allclose(F, lig.mass[:, None] / lig.mass.sum() * Ftot,
                               atol=1e-12)
            assert np.allclose(Ftot, -100.0 * (d - 1.0) * com / d, atol=1e-10)
        else:
            assert np.all(F == 0)


def test_angle_energy_closed_form(oracle_lib):
    """Harmonic angle term K_theta (theta - theta0)^2 on a 3-atom ligand
    with one angle and nothing else: the energy at a placed angle theta and
    the force on the end atoms from the planar geometry.  With i on the x
    axis at distance r1 from the vertex j and k at distance r2 in direction
    (cos theta, sin theta, 0), increasing theta moves k along (-sin theta,
    cos theta, 0) / r2 per radian and i along (0, -1, 0) / r1, so
    F_k = -dE/dtheta (-sin theta, cos theta, 0) / r2,
    F_i = -dE/dtheta (0, -1, 0) / r1 and F_j = -(F_i + F_k),
    with dE/dtheta = 2 K (theta - theta0).  theta0 is in radians: a
    degree/radian slip or a factor 1/2 in the energy fails here."""
    K, th0 = 250.0, 1.9
    x = np.zeros((3, 3))
    lig = synth.toy_ligand(x, np.zeros((0, 2)), 0.0, [300.0], [0.0],
                           d0=100.0)
    lig.scale = np.zeros((3, 3))
    lig.angles = np.array([[0, 1, 2]], np.int32)
    lig.angle_par = np.array([[K, th0]])
    ol = oracle.OLigand(lig)
    og = oracle.OGrid(_zero_grid())
    r1, r2 = 1.3, 0.7
    for th in (0.6, 1.5, 1.9, 2.4, 3.0):
        xx = np.array([[r1, 0.0, 0.0], [0.0, 0.0, 0.0],
                       [r2 * math.cos(th), r2 * math.sin(th), 0.0]])
        t, _, F = oracle.energy(og, ol, np.zeros(3), xx)
        E = K * (th - th0) ** 2
        assert abs(t[1] - E) <= 1e-12 * max(E, 1.0), (th, t[1], E)
        assert abs(t[0]) == 0.0 and abs(t[2]) == 0.0
        dE = 2.0 * K * (th - th0)
        Fk = -dE * np.array([-math.sin(th), math.cos(th), 0.0]) / r2
        Fi = -dE * np.array([0.0, -1.0, 0.0]) / r1
        ref = np.stack([Fi, -(Fi + Fk), Fk])
        assert np.allclose(F, ref, atol=1e-10 * max(abs(dE), 1.0)), (th, F,
                                                                    ref)
    # the bent-at-right-angle case written out: theta = pi/2, theta0 = 1.9
    xx = np.array([[r1, 0, 0], [0, 0, 0], [0, r2, 0]], np.float64)
    t, _, _ = oracle.energy(og, ol, np.zeros(3), xx, forces=False)
    assert abs(t[1] - 250.0 * (math.pi / 2 - 1.9) ** 2) < 1e-12
