"""External-coordinate Monte Carlo moves of the ligand -- oracle, TEST
INFRASTRUCTURE ONLY (imported by tests/, the package smoke check and the
benchmark's CPU baseline; never by the library).

Sampling section (external coordinate Markov chain Monte Carlo): a move
rotates the ligand rigidly about its centre of mass by a rotation made from
a random unit quaternion, translates it by a Gaussian displacement of
standard deviation sigma (0.6 A in the paper) per axis, and is accepted by
the Metropolis criterion; the paper attempts such moves only in states whose
grid coupling alpha is below 0.01.  The proposal is symmetric: the rotation
is uniform (Haar), so a rotation and its inverse are equally likely, and so
are t and -t.

Random numbers come from the Philox draws every other move uses (ligand,
replica, sweep counter), purpose P_EXTERNAL; move m of a run of moves uses
draw index 3m (three uniforms for the quaternion), 3m + 1 (three normals for
the translation) and 3m + 2 (the acceptance uniform).
"""
from __future__ import annotations

import math

import numpy as np

from . import P_EXTERNAL, R_GAS, energy, normals3, uniform4

SIGMA_PAPER = 0.6  # A per axis


def unit_quaternion(u1, u2, u3):
    """Uniformly distributed unit quaternion (w, x, y, z) from three
    uniforms in (0, 1] (Shoemake, Graphics Gems III, 1992): with a =
    sqrt(1 - u1), b = sqrt(u1), (x, y) = a (sin, cos)(2 pi u2) and (z, w) =
    b (sin, cos)(2 pi u3)."""
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    return np.array([b * math.cos(2 * math.pi * u3),
                     a * math.sin(2 * math.pi * u2),
                     a * math.cos(2 * math.pi * u2),
                     b * math.sin(2 * math.pi * u3)])


def quaternion_matrix(q):
    """Rotation matrix of the unit quaternion q = (w, x, y, z)."""
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def propose(x, mass, u3, z3, sigma=SIGMA_PAPER):
    """The moved configuration: R (x - c) + c + sigma z, c the centre of
    mass, R the rotation of the quaternion made from u3."""
    c = (mass[:, None] * x).sum(0) / mass.sum()
    R = quaternion_matrix(unit_quaternion(*u3))
    return (x - c) @ R.T + c + sigma * np.asarray(z3)


def external_move(x, mass, energy_fn, beta, u3, z3, u_acc, e_cur=None,
                  sigma=SIGMA_PAPER):
    """One Metropolis move: returns (new x, accepted, ln alpha, energy of
    the returned configuration).  energy_fn(x) -> U_k(x) in kJ/mol."""
    e0 = energy_fn(x) if e_cur is None else e_cur
    xn = propose(x, mass, u3, z3, sigma)
    e1 = energy_fn(xn)
    ln_a = -beta * (e1 - e0)
    acc = bool(math.isfinite(ln_a) and math.log(u_acc) < ln_a)
    return (xn, True, ln_a, e1) if acc else (x, False, ln_a, e0)


def state_energy(og, ol, k, x):
    """U_k(x) = U_bonded + U_restraint + sum_c w_kc Psi_c(x)."""
    t, _, _ = energy(og, ol, ol.w[k], x, forces=False)
    return float(t[:4].sum() + ol.w[k] @ t[4:])


def external_moves(og, ol, x, k, seed, lig, rep, sweep, n_moves,
                   sigma=SIGMA_PAPER):
    """n_moves moves in a row of replica `rep` (in state k) at sweep counter
    `sweep`; returns (x, number accepted, [ln alpha of each move])."""
    beta = 1.0 / (R_GAS * ol.T[k])
    x = np.asarray(x, np.float64)
    e = state_energy(og, ol, k, x)
    n_acc, lns = 0, []
    for m in range(n_moves):
        u3 = uniform4(seed, 3 * m, lig, rep, sweep, P_EXTERNAL)[:3]
        z3 = normals3(seed, 3 * m + 1, lig, rep, sweep, P_EXTERNAL)
        ua = uniform4(seed, 3 * m + 2, lig, rep, sweep, P_EXTERNAL)[0]
        x, acc, ln_a, e = external_move(
            x, ol.mass, lambda y: state_energy(og, ol, k, y), beta, u3, z3,
            ua, e_cur=e, sigma=sigma)
        n_acc += acc
        lns.append((ln_a, math.log(ua)))
    return x, n_acc, lns
