"""Initialisation and adaptation of the thermodynamic-state ladder -- oracle,
TEST INFRASTRUCTURE ONLY (imported by tests/, the package smoke check and the
benchmark's CPU baseline; never by the library).

Initialization section: states are added one at a time from alpha = 0
(decoupled, hot) towards alpha = 1 (coupled, cold).  For each new state:

* parameter selection -- the step in alpha is the thermodynamic speed s over
  the standard deviation of the derivative of the log probability, in the
  paper's three-term form for the grid path (soft grids, grids,
  temperature) and as s k T^2 / sigma[U] for a temperature-only path;
* seed selection -- sampling importance resampling of the previous state's
  samples with weights exp[u_k(x) - u_k+1(x)];
* sampling and adaptation -- runs from the seeds, with the time step raised
  by 0.125 fs above acceptance 0.8, lowered by 0.25 fs below 0.4 and by
  0.5 fs below 0.1, repeated until the acceptance lies in [0.4, 0.8];
* verification -- the mean exchange acceptance over pairs of initial samples
  at the same time index; below 0.4 the speed shrinks by 4/5 and the state
  is selected again, above 0.99 the previous state is dropped.

Between cycles a state is inserted between neighbours whose exchange
acceptance fell below 0.4 (Equilibration and production); the production
data start where the number of uncorrelated samples is largest (equilibration
detection, Chodera 2016).  The grid path's schedule is the Thermodynamic
Cycle's: T(alpha) linear between T_H and T_T, the soft grids weighted by
alpha_sg = 1 - (2 alpha - 1)^2, the original grids by
alpha_g = (2 alpha - 1)^2 / (1 + exp(-1000 (alpha - 1/2))).

Readings where the paper is silent: sigma is the population standard
deviation (ddof 0); a step never passes alpha = 1 (the target is used); the
time step has a floor dt_min below which it is not lowered (the adaptation
then ends); the end state alpha = 0 is never dropped; an inserted state
sits at the midpoint in alpha; SIR draws with replacement by inverting the
cumulative weights with Philox uniforms (purpose P_INIT, sub-purpose 0,
index = draw, sweep field = the new state's index); "the same time index"
pairs sample i of one state with sample i of the other for i below the
smaller count.

Random placements of a configuration in the binding site (the start of the
grid path when no bound pose is known): centre of mass uniform in the sphere
of radius d0 about the site (radius d0 u^(1/3), cos(theta) = 2u - 1,
phi = 2 pi u from the Philox uniforms of sub-purpose 1, index = position),
orientation from a uniform unit quaternion (sub-purpose 2, index =
orientation), applied about the configuration's centre of mass.
"""
from __future__ import annotations

import math

import numpy as np

from . import R_GAS, uniform, uniform4
from .estimators import statistical_inefficiency
from .external import quaternion_matrix, unit_quaternion

P_INIT = 7
SUB_SIR, SUB_COM, SUB_ORIENT = 0, 1, 2

# paper's constants (Initialization)
S_CD = 0.2
S_BC = 20.0
P_LOW, P_HIGH = 0.4, 0.99
SPEED_FACTOR = 0.8
ACC_LOW, ACC_HIGH, ACC_VERY_LOW = 0.4, 0.8, 0.1
DT_UP, DT_DOWN, DT_DOWN_MORE = 0.125, 0.25, 0.5

LINEAR, SOFT = 0, 1


# ---------------------------------------------------------------------------
# the schedule (Thermodynamic Cycle)
# ---------------------------------------------------------------------------
def alpha_sg(a):
    return 1.0 - (2.0 * a - 1.0) ** 2


def alpha_g(a):
    return (2.0 * a - 1.0) ** 2 / (1.0 + math.exp(-1000.0 * (a - 0.5)))


def d_alpha_sg(a):
    return -4.0 * (2.0 * a - 1.0)


def d_alpha_g(a):
    # with the logistic sig = 1 / (1 + exp(-1000 (a - 1/2))), whose
    # derivative is 1000 sig (1 - sig)
    sig = 1.0 / (1.0 + math.exp(-1000.0 * (a - 0.5)))
    return (4.0 * (2.0 * a - 1.0) * sig +
            (2.0 * a - 1.0) ** 2 * 1000.0 * sig * (1.0 - sig))


def temperature(a, T_H, T_T):
    return (T_T - T_H) * a + T_H


def state_of(a, kind, C, T_H, T_T):
    """(T, w[C]) of the state at alpha.  LINEAR: every channel weighted by
    alpha; SOFT (C = 5: rep, att, ele, soft rep, soft ele): the original
    grids by alpha_g, the soft grids by alpha_sg."""
    T = temperature(a, T_H, T_T)
    if kind == LINEAR:
        return T, np.full(C, float(a))
    assert C == 5
    g, sg = alpha_g(a), alpha_sg(a)
    return T, np.array([g, g, g, sg, sg])


def soft_caps(s_rep, q, cap_energy=10.0):
    """Caps (v_max,rep, v_max,ele) of the soft grids (Thermodynamic Cycle,
    soft grids between milestones C and D).

    The paper caps the soft repulsive grid at 10 in its own grid units and
    sets the electrostatic cap so that no atom's soft electrostatic energy
    exceeds its soft repulsive energy: the repulsive cap times the smallest
    ratio of repulsive to electrostatic scaling factor over the atoms.
    Reading for grids in this build's units (repulsive factor times grid
    value is an energy): the repulsive cap makes the soft repulsion of the
    median atom (median over the listed atoms' repulsive factors) equal to
    cap_energy kJ/mol; atoms without charge do not bound the electrostatic
    cap (and with no charged atom it equals the repulsive one)."""
    s_rep = np.asarray(s_rep, np.float64)
    q = np.abs(np.asarray(q, np.float64))
    v_rep = cap_energy / float(np.median(s_rep))
    charged = q > 0.0
    if not charged.any():
        return v_rep, v_rep
    return v_rep, v_rep * float(np.min(s_rep[charged] / q[charged]))


def soft_grid(values, v_max):
    """Soft grid value v_max tanh(v / v_max) of original grid values v
    (Thermodynamic Cycle: the hyperbolic-tangent cap of the soft repulsive
    and electrostatic grids), in double.  A repulsive grid stored as a
    quartic root is raised to the fourth power first by the caller: the cap
    acts on the grid's value, not on its stored root."""
    return v_max * np.tanh(np.asarray(values, np.float64) / v_max)


def channel_groups(kind, C):
    """Boolean masks (original grids, soft grids) over the C channels."""
    g = np.ones(C, bool)
    sg = np.zeros(C, bool)
    if kind == SOFT:
        g[3:] = False
        sg[3:] = True
    return g, sg


def reduced(comps, T, w):
    """u = (U0 + sum_c w_c Psi_c) / (R T) of samples whose cached
    components are comps (N, 1 + C)."""
    comps = np.asarray(comps, np.float64)
    return (comps[:, 0] + comps[:, 1:] @ np.asarray(w, np.float64)) / (R_GAS * T)


# ---------------------------------------------------------------------------
# parameter selection (Initialization, thermodynamic length)
# ---------------------------------------------------------------------------
def state_sigmas(comps, a, kind, T_H, T_T):
    """sigma[Psi_g], sigma[Psi_sg], sigma[u_alpha] over a state's samples."""
    comps = np.asarray(comps, np.float64)
    C = comps.shape[1] - 1
    g, sg = channel_groups(kind, C)
    T, w = state_of(a, kind, C, T_H, T_T)
    psi_g = comps[:, 1:][:, g].sum(axis=1)
    psi_sg = comps[:, 1:][:, sg].sum(axis=1) if sg.any() else np.zeros(len(comps))
    u = reduced(comps, T, w)
    return float(np.std(psi_g)), float(np.std(psi_sg)), float(np.std(u))


def next_alpha(a, sig_g, sig_sg, sig_u, kind, s, T_H, T_T):
    """alpha of the next state: a + s / [ |d alpha_sg/d alpha| sigma[Psi_sg]
    / (k T) + |d alpha_g/d alpha| sigma[Psi_g] / (k T) + |T_T - T_H|
    sigma[u] / T ], never past 1.  For LINEAR every channel's weight is
    alpha, so the grid term is sigma[Psi_g] / (k T) with no soft term."""
    T = temperature(a, T_H, T_T)
    kT = R_GAS * T
    if kind == LINEAR:
        dg, dsg = 1.0, 0.0
    else:
        dg, dsg = d_alpha_g(a), d_alpha_sg(a)
    denom = (abs(dsg) * sig_sg / kT + abs(dg) * sig_g / kT +
             abs(T_T - T_H) * sig_u / T)
    if denom <= 0.0:
        return 1.0
    return min(a + s / denom, 1.0)


def next_temperature(T, sig_U, s, T_target):
    """Temperature-only path: T moves towards T_target by s k T^2 /
    sigma[U], and stops there."""
    if sig_U <= 0.0:
        return float(T_target)
    step = s * R_GAS * T * T / sig_U
    if T_target >= T:
        return min(T + step, float(T_target))
    return max(T - step, float(T_target))


# ---------------------------------------------------------------------------
# seed selection (sampling importance resampling)
# ---------------------------------------------------------------------------
def sir(logw, n_draw, seed, lig, state):
    """Indices of n_draw samples drawn with replacement with probability
    proportional to exp(logw): draw j takes the first i whose cumulative
    weight (summed in index order after subtracting max logw) reaches
    u_j times the total."""
    logw = np.asarray(logw, np.float64)
    ok = np.isfinite(logw)
    if not ok.any():
        raise ValueError("no finite weight")
    m = logw[ok].max()
    w = np.where(ok, np.exp(np.where(ok, logw, m) - m), 0.0)
    cum = np.cumsum(w)
    total = cum[-1]
    out = np.zeros(n_draw, np.int64)
    for j in range(n_draw):
        u = uniform(seed, j, lig, 0, state, P_INIT | (SUB_SIR << 8))
        i = int(np.searchsorted(cum, u * total, side="left"))
        out[j] = min(i, len(cum) - 1)
    return out


# ---------------------------------------------------------------------------
# time-step adaptation and verification
# ---------------------------------------------------------------------------
def adapt_dt(dt, acc, dt_min):
    """(new dt, done): +0.125 fs above acceptance 0.8, -0.5 fs below 0.1,
    -0.25 fs below 0.4; done when the acceptance is in [0.4, 0.8] or dt
    cannot be lowered further (floor dt_min)."""
    if acc > ACC_HIGH:
        return dt + DT_UP, False
    if acc < ACC_LOW:
        if dt <= dt_min:
            return dt, True
        step = DT_DOWN_MORE if acc < ACC_VERY_LOW else DT_DOWN
        return max(dt - step, dt_min), False
    return dt, True


def mean_pacc(uk_x, uk1_x, uk_y, uk1_y):
    """Mean of min(1, exp(-[u_k(y) + u_k+1(x) - u_k(x) - u_k+1(y)])) over
    pairs (x_i from state k, y_i from state k+1) -- Eq. repXacc."""
    d = (np.asarray(uk_y) + np.asarray(uk1_x) - np.asarray(uk_x) -
         np.asarray(uk1_y))
    p = np.where(np.isfinite(d), np.exp(-np.maximum(d, 0.0)), 0.0)
    return float(p.mean())


def insert_states(alphas, pacc, threshold=P_LOW):
    """Ladder with a state at the midpoint between each neighbour pair whose
    exchange acceptance is below threshold."""
    out = [float(alphas[0])]
    for k in range(len(alphas) - 1):
        if pacc[k] < threshold:
            out.append(0.5 * (alphas[k] + alphas[k + 1]))
        out.append(float(alphas[k + 1]))
    return out


# ---------------------------------------------------------------------------
# equilibration detection (Chodera 2016)
# ---------------------------------------------------------------------------
def detect_equilibration(a, n_candidates=100):
    """(t0, g, N_eff): the start t0 among n_candidates evenly spaced
    candidates (t0 = floor(i N / n_candidates)) that maximises the number of
    uncorrelated samples (N - t0) / g(a[t0:]); ties go to the smaller t0."""
    a = np.asarray(a, np.float64)
    N = len(a)
    best = (0, 1.0, -1.0)
    for i in range(n_candidates):
        t0 = (i * N) // n_candidates
        if N - t0 < 2:
            break
        g = statistical_inefficiency(a[t0:])
        neff = (N - t0) / g
        if neff > best[2]:
            best = (t0, g, neff)
    return best


# ---------------------------------------------------------------------------
# random placements in the binding site
# ---------------------------------------------------------------------------
def site_position(seed, lig, i, center, radius):
    u = uniform4(seed, i, lig, 0, 0, P_INIT | (SUB_COM << 8))
    r = radius * u[0] ** (1.0 / 3.0)
    ct = 2.0 * u[1] - 1.0
    st = math.sqrt(max(0.0, 1.0 - ct * ct))
    ph = 2.0 * math.pi * u[2]
    return np.asarray(center, np.float64) + r * np.array(
        [st * math.cos(ph), st * math.sin(ph), ct])


def orientation(seed, lig, o):
    u = uniform4(seed, o, lig, 0, 0, P_INIT | (SUB_ORIENT << 8))
    return quaternion_matrix(unit_quaternion(u[0], u[1], u[2]))


def placements(confs, mass, center, radius, n_com, n_orient, seed, lig):
    """Poses (n_conf * n_com * n_orient, n, 3), pose (c, i, o) at flat index
    (c * n_com + i) * n_orient + o: configuration c rotated by orientation o
    about its centre of mass, which is moved to site position i."""
    confs = np.asarray(confs, np.float64)
    mass = np.asarray(mass, np.float64)
    n_conf, n = confs.shape[:2]
    pos = [site_position(seed, lig, i, center, radius) for i in range(n_com)]
    rot = [orientation(seed, lig, o) for o in range(n_orient)]
    out = np.zeros((n_conf, n_com, n_orient, n, 3))
    for c in range(n_conf):
        com = (mass[:, None] * confs[c]).sum(0) / mass.sum()
        rel = confs[c] - com
        for o in range(n_orient):
            rr = rel @ rot[o].T
            for i in range(n_com):
                out[c, i, o] = rr + pos[i]
    return out.reshape(n_conf * n_com * n_orient, n, 3)
