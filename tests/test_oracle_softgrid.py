"""Pins of the oracle's soft grids and switching schedule (Thermodynamic
Cycle: soft repulsive and electrostatic grids v_max tanh(v / v_max) between
milestones C and D, the electrostatic cap bounded by the repulsive one, and
the alpha_sg / alpha_g protocol), and the check that the synthetic inputs
both sides of every parity test receive are the oracle's definition."""
import math

import numpy as np
import pytest

import synth
from oracle import protocol as P


def test_soft_grid_limits_and_closed_forms():
    vm = 7.5
    # slope 1 at the origin: the soft grid equals the original for small
    # values (central difference, and the cubic remainder of tanh)
    eta = 1e-6
    slope = (P.soft_grid(eta, vm) - P.soft_grid(-eta, vm)) / (2 * eta)
    assert abs(slope - 1.0) < 1e-9
    v = np.array([1e-3, -2e-3, 5e-3])
    assert np.all(np.abs(P.soft_grid(v, vm) - v) <= np.abs(v) ** 3 /
                  (3 * vm * vm) * 1.0001)
    # saturation at +-v_max, never beyond
    big = np.array([1e3, 1e6, -1e3, -1e6]) * vm
    assert np.allclose(P.soft_grid(big, vm), np.sign(big) * vm, rtol=0,
                       atol=1e-12)
    grid = np.linspace(-50 * vm, 50 * vm, 10001)
    s = P.soft_grid(grid, vm)
    assert np.all(np.abs(s) <= vm)
    # odd and strictly increasing
    assert np.allclose(P.soft_grid(-grid, vm), -s, atol=0)
    assert np.all(np.diff(s) >= 0) and np.all(np.diff(s[4000:6001]) > 0)
    # half the cap at v_max artanh(1/2) = v_max ln(3) / 2
    assert abs(P.soft_grid(vm * math.log(3.0) / 2, vm) - vm / 2) < 1e-13


def test_soft_caps_bound_electrostatics_by_repulsion():
    rng = np.random.default_rng(3)
    s_rep = rng.uniform(1e3, 5e4, 37)
    q = rng.uniform(-0.5, 0.5, 37)
    q[5] = 0.0
    v_rep, v_ele = P.soft_caps(s_rep, q, cap_energy=10.0)
    # the median atom's soft repulsion saturates at 10 kJ/mol
    assert abs(np.median(s_rep) * v_rep - 10.0) < 1e-12
    # every atom's largest soft electrostatic energy is at most its largest
    # soft repulsive energy, and the bound is tight for one charged atom
    e_ele = np.abs(q) * v_ele
    e_rep = s_rep * v_rep
    assert np.all(e_ele <= e_rep * (1 + 1e-12))
    tight = np.abs(e_ele - e_rep) <= 1e-12 * e_rep
    assert tight.sum() == 1 and q[np.argmax(tight)] != 0.0
    # brute force: the largest cap with the bound holding
    nz = q != 0
    cand = np.sort(s_rep[nz] * v_rep / np.abs(q[nz]))
    assert abs(v_ele - cand[0]) <= 1e-12 * cand[0]
    # no charged atom: the electrostatic cap equals the repulsive one
    assert P.soft_caps(s_rep, np.zeros(37)) == (v_rep, v_rep)


def test_schedule_end_points_and_midpoint():
    for C in (5,):
        T, w = P.state_of(0.0, P.SOFT, C, 600.0, 300.0)
        # alpha_g(0) = 1 / (1 + e^500): decoupled up to 1e-217
        assert T == 600.0 and np.all(w[3:] == 0.0)
        assert np.all(w[:3] == 1.0 / (1.0 + math.exp(500.0)))
        T, w = P.state_of(0.5, P.SOFT, C, 600.0, 300.0)
        assert T == 450.0 and np.allclose(w, [0, 0, 0, 1, 1], atol=0)
        T, w = P.state_of(1.0, P.SOFT, C, 600.0, 300.0)
        g = 1.0 / (1.0 + math.exp(-500.0))
        assert T == 300.0 and np.allclose(w, [g, g, g, 0, 0], atol=0)


def test_synthetic_schedule_is_the_oracles():
    for K in (2, 9, 32, 64, 163):
        T, w = synth.soft_schedule(K)
        for k in range(K):
            To, wo = P.state_of(k / (K - 1), P.SOFT, 5, 600.0, 300.0)
            # alpha from linspace may differ from k / (K - 1) by an ulp,
            # which the logistic's slope of 1000 amplifies to ~1e-13
            assert abs(T[k] - To) <= 1e-12 * To
            assert np.allclose(w[k], wo, rtol=1e-12, atol=1e-300), (K, k)


@pytest.mark.parametrize("extra", [(), (10, 40, 90, 100)])
def test_synthetic_soft_grids_are_the_oracles(extra):
    """The 24-atom system's grids, alone or shared by ligands of 10-100
    atoms (whose factors then set the caps together)."""
    system = synth.make_system(1)
    rng = np.random.default_rng(77)
    system.ligands += [synth.make_ligand(rng, n, 32) for n in extra]
    g, ligs = synth.add_soft_grids(system.grid, system.ligands)
    nodes = system.grid.nodes
    assert g.nodes.shape[-1] == 5 and tuple(g.transform) == (4, 0, 0, 0, 0)
    assert np.array_equal(g.nodes[..., :3], nodes)
    s_rep = np.concatenate([l.scale[:, 0] for l in system.ligands])
    q = np.concatenate([l.scale[:, 2] for l in system.ligands])
    v_rep, v_ele = P.soft_caps(s_rep, q)
    # the repulsive channel stores a quartic root: the cap acts on its
    # fourth power
    rep = P.soft_grid(nodes[..., 0].astype(np.float64) ** 4, v_rep)
    ele = P.soft_grid(nodes[..., 2].astype(np.float64), v_ele)
    assert np.array_equal(g.nodes[..., 3], rep.astype(np.float32))
    assert np.array_equal(g.nodes[..., 4], ele.astype(np.float32))
    # grids this strong saturate somewhere: both caps are reached
    assert g.nodes[..., 3].max() >= np.float32(v_rep) * 0.999
    assert np.abs(g.nodes[..., 4]).max() > 0.5 * v_ele
    for l0, l in zip(system.ligands, ligs):
        assert np.array_equal(l.scale[:, :3], l0.scale)
        assert np.array_equal(l.scale[:, 3], l0.scale[:, 0])
        assert np.array_equal(l.scale[:, 4], l0.scale[:, 2])
        K = l.n_states
        for k in range(K):
            To, wo = P.state_of(k / (K - 1), P.SOFT, 5, 600.0, 300.0)
            assert abs(l.T[k] - To) <= 1e-12 * To
            assert np.allclose(l.w[k], wo, rtol=1e-12, atol=1e-300)
