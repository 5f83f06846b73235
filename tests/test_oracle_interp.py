"""Pins of the oracle's grid interpolation (trilinear interpolation of the
electrostatic and van der Waals grids with the power-4 inverse transform on
the repulsive channel; Methodology, "Thermodynamic Cycle").  Each check is
fixed by mathematics that is independent of the oracle's own formula."""
import numpy as np
import pytest

import oracle
import synth


def _grid(nodes, origin, h, transform):
    nz, ny, nx, _ = nodes.shape
    return synth.Grid((nx, ny, nz), tuple(origin), h, tuple(transform),
                      np.ascontiguousarray(nodes, np.float32))


def test_node_values_exact(oracle_lib):
    rng = np.random.default_rng(1)
    g = synth.random_grid(rng, n=(6, 5, 4), transform=(0, 0, 0))
    og = oracle.OGrid(g)
    nx, ny, nz = g.n
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                p = np.array(g.origin) + g.spacing * np.array([ix, iy, iz])
                v, _ = oracle.interp(og, p)
                assert np.array_equal(v, g.nodes[iz, iy, ix].astype(np.float64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_multilinear_field_reproduced(oracle_lib, seed):
    # a + bx + cy + dz + exy + fxz + gyz + hxyz with dyadic coefficients is
    # exactly representable at the nodes and is reproduced everywhere inside
    rng = np.random.default_rng(seed)
    coef = rng.integers(-8, 9, size=(3, 8)) / 4.0
    g = synth.multilinear_grid(coef)
    og = oracle.OGrid(g)
    nx, ny, nz = g.n
    lo = np.array(g.origin)
    hi = lo + g.spacing * (np.array([nx, ny, nz]) - 1)
    for _ in range(200):
        p = rng.uniform(lo, hi)
        x, y, z = p
        v, dv = oracle.interp(og, p)
        for c in range(3):
            a, b, cc, d, e, f, gg, h = coef[c]
            ref = a + b * x + cc * y + d * z + e * x * y + f * x * z + \
                gg * y * z + h * x * y * z
            grad = np.array([b + e * y + f * z + h * y * z,
                             cc + e * x + gg * z + h * x * z,
                             d + f * x + gg * y + h * x * y])
            assert abs(v[c] - ref) <= 1e-12 * (1 + abs(ref))
            assert np.allclose(dv[c], grad, rtol=0, atol=1e-11)


def test_single_cell_is_unique_multilinear_interpolant(oracle_lib):
    # On a 2x2x2 grid the interpolant is the unique function of the form
    # sum_{ijk in {0,1}} a_ijk x^i y^j z^k through the 8 node values; find
    # its coefficients by a linear solve and compare at random points.
    rng = np.random.default_rng(5)
    nodes = rng.normal(size=(2, 2, 2, 1))
    h, o = 0.75, np.array([0.3, -0.2, 0.1])
    g = _grid(nodes.astype(np.float32), o, h, (0,))
    vals = g.nodes.astype(np.float64)
    A, rhs = [], []
    for iz in range(2):
        for iy in range(2):
            for ix in range(2):
                x, y, z = o + h * np.array([ix, iy, iz])
                A.append([1, x, y, z, x * y, x * z, y * z, x * y * z])
                rhs.append(vals[iz, iy, ix, 0])
    coef = np.linalg.solve(np.array(A), np.array(rhs))
    og = oracle.OGrid(g)
    for _ in range(50):
        p = o + h * rng.uniform(0, 1, 3)
        x, y, z = p
        ref = coef @ np.array([1, x, y, z, x * y, x * z, y * z, x * y * z])
        v, _ = oracle.interp(og, p)
        assert abs(v[0] - ref) < 1e-12


def test_gradient_matches_central_differences_inside_cells(oracle_lib):
    rng = np.random.default_rng(7)
    g = synth.random_grid(rng, n=(7, 6, 5), transform=(4, 0, 0))
    og = oracle.OGrid(g)
    eta = 1e-5
    lo = np.array(g.origin)
    for _ in range(100):
        cell = rng.integers(0, [g.n[0] - 1, g.n[1] - 1, g.n[2] - 1])
        t = rng.uniform(0.05, 0.95, 3)   # stay away from faces
        p = lo + g.spacing * (cell + t)
        scale = np.array([1.3, -0.7, 0.4])
        e, de = oracle.atom_grid(og, p, scale)
        for a in range(3):
            dp = np.zeros(3)
            dp[a] = eta
            ep, _ = oracle.atom_grid(og, p + dp, scale)
            em, _ = oracle.atom_grid(og, p - dp, scale)
            fd = (ep - em) / (2 * eta)
            # linear channels: central differences are exact inside a cell
            assert np.allclose(fd[1:], de[1:, a], rtol=1e-9, atol=1e-9)
            # v^4 channel: O(eta^2) truncation
            assert abs(fd[0] - de[0, a]) <= 1e-7 * (1 + abs(de[0, a]))


def test_continuity_across_faces_and_grid_boundary(oracle_lib):
    rng = np.random.default_rng(11)
    g = synth.random_grid(rng, n=(5, 5, 5), transform=(4, 0, 0))
    og = oracle.OGrid(g)
    lo = np.array(g.origin)
    h = g.spacing
    eps = 1e-10
    for _ in range(60):
        p = lo + h * rng.uniform(0, 4, 3)
        ax = rng.integers(0, 3)
        k = rng.integers(0, 5)      # face index 0..4 (0 and 4 = boundary)
        p[ax] = lo[ax] + h * k
        a, b = p.copy(), p.copy()
        a[ax] -= eps
        b[ax] += eps
        va, _ = oracle.interp(og, a)
        vb, _ = oracle.interp(og, b)
        assert np.allclose(va, vb, atol=1e-8)


def test_outside_grid_clamps_to_edge(oracle_lib):
    rng = np.random.default_rng(13)
    g = synth.random_grid(rng, n=(5, 4, 6), transform=(4, 0, 0))
    og = oracle.OGrid(g)
    lo = np.array(g.origin)
    hi = lo + g.spacing * (np.array(g.n) - 1)
    for _ in range(100):
        p = rng.uniform(lo - 3, hi + 3)
        q = np.clip(p, lo, hi)
        v, dv = oracle.interp(og, p)
        vq, dvq = oracle.interp(og, q)
        assert np.allclose(v, vq, atol=1e-12)
        for a in range(3):
            if p[a] < lo[a] or p[a] > hi[a]:
                assert np.all(dv[:, a] == 0.0)
            else:
                assert np.allclose(dv[:, a], dvq[:, a], atol=1e-12)


def test_quartic_transform(oracle_lib):
    # if G^(1/4) is multilinear, G = v^4 is reproduced exactly; at nodes
    # the energy equals scale * G
    coef = np.array([[2.0, 0.25, -0.5, 0.75, 0.0, 0.0, 0.0, 0.0]])
    g = synth.multilinear_grid(coef, n=(4, 4, 4), origin=(0.0, 0.0, 0.0))
    nodes = np.abs(g.nodes)
    g = _grid(nodes, g.origin, g.spacing, (4,))
    og = oracle.OGrid(g)
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = rng.uniform(0, 1.5, 3)
        root = 2.0 + 0.25 * p[0] - 0.5 * p[1] + 0.75 * p[2]
        e, de = oracle.atom_grid(og, p, np.array([1.5]))
        assert abs(e[0] - 1.5 * root ** 4) <= 1e-12 * 1.5 * root ** 4
        grad = 1.5 * 4 * root ** 3 * np.array([0.25, -0.5, 0.75])
        assert np.allclose(de[0], grad, rtol=1e-12)


def test_grids_reduce_to_direct_pair_sum(oracle_lib):
    """With no softening and no cap, the three grids times the per-atom
    factors reproduce the direct Lennard-Jones (geometric-mean rule) plus
    Coulomb sum between receptor points and ligand atoms placed on nodes."""
    rng = np.random.default_rng(21)
    n, h = 12, 0.5
    pts, q, sig, eps = synth.make_receptor(rng, 6, 5.5, 0.0)
    # keep the points off the lattice (no singular node)
    pts = pts + 0.123
    nodes = synth.grids_from_points(pts, q, sig, eps, n, h, delta=0.0,
                                    cap=np.inf)
    origin = -(n - 1) * h / 2
    g = synth.Grid((n, n, n), (origin,) * 3, h, (4, 0, 0), nodes)
    og = oracle.OGrid(g)
    m = 5
    idx = rng.integers(0, n, size=(m, 3))
    xl = origin + h * idx
    ql = rng.uniform(-0.5, 0.5, m)
    sl = rng.uniform(3, 4, m)
    el = rng.uniform(0.05, 0.3, m)
    scale = np.stack([2 * np.sqrt(el) * sl ** 6, -2 * np.sqrt(el) * sl ** 3,
                      ql], axis=1)
    total = 0.0
    direct = 0.0
    mag = 0.0
    for i in range(m):
        e, _ = oracle.atom_grid(og, xl[i], scale[i])
        total += e.sum()
        mag += np.abs(e).sum()
        for j in range(len(pts)):
            r = np.linalg.norm(xl[i] - pts[j])
            eij = np.sqrt(el[i] * eps[j])
            sij = np.sqrt(sl[i] * sig[j])
            direct += 4 * eij * ((sij / r) ** 12 - (sij / r) ** 6) + \
                synth.COULOMB * ql[i] * q[j] / r
    # grid values are float32 (rep stored as a float32 quartic root)
    assert abs(total - direct) <= 2e-6 * mag
