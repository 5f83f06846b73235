"""Intramolecular nonbonded and implicit-solvent energy of the ligand --
oracle, TEST INFRASTRUCTURE ONLY (imported by tests/, the package smoke check
and the benchmark's CPU baseline; never by the library).

Force field (Thermodynamic Cycle: the ligand's force field with an OBC
generalised-Born/surface-area implicit solvent, the solvation model the
paper adapts):

* Lennard-Jones 12-6 over atom pairs more than two bonds apart, with the
  Lorentz-Berthelot rules sigma_ij = (sigma_i + sigma_j) / 2 and eps_ij =
  sqrt(eps_i eps_j); 1-4 pairs scaled by lj14.
* Coulomb k_e q_i q_j / r over the same pairs in a dielectric of 1
  (eps_solute), 1-4 pairs scaled by el14.
* Generalised Born (Onufriev, Bashford, Case 2004, "OBC II"):
  E_GB = -(k_e / 2) (1/eps_solute - 1/eps_solvent) sum_i sum_j q_i q_j /
  f_ij over all ordered pairs including i = j, f_ij = sqrt(r^2 + R_i R_j
  exp(-r^2 / (4 R_i R_j))), f_ii = R_i.  Born radii 1/R_i = 1/rt_i -
  tanh(a psi - b psi^2 + c psi^3) / rho_i with psi = I_i rt_i, (a, b, c) =
  (1, 0.8, 4.85), rt_i = rho_i - 0.09 A, and I_i the descreening integral of
  Hawkins, Cramer, Truhlar (1996): the integral of |x - x_i|^-4 / (4 pi)
  over each other atom's sphere of radius S_j rt_j, outside the sphere of
  radius rt_i about atom i.
* Surface area (ACE form): sum_i 4 pi gamma (rho_i + r_probe)^2 (rho_i /
  R_i)^6.

All terms are written as plain sums in float64.  Forces are -grad E by
central differences of the energy (no derivative formula of its own).
"""
from __future__ import annotations

import math

import numpy as np

# Coulomb constant e^2 / (4 pi eps0) in kJ/mol A e^-2
K_COULOMB = 1389.35457644382
OBC_ABG = (1.0, 0.8, 4.85)
DIELECTRIC_OFFSET = 0.09  # A
TERMS = ("lj", "coulomb", "gb", "sa")


def masks(n, exclusions, pairs14):
    """(excluded, one_four) boolean n x n matrices."""
    ex = np.zeros((n, n), bool)
    for i, j in np.asarray(exclusions, int).reshape(-1, 2):
        ex[i, j] = ex[j, i] = True
    o4 = np.zeros((n, n), bool)
    for i, j in np.asarray(pairs14, int).reshape(-1, 2):
        if not ex[i, j]:
            o4[i, j] = o4[j, i] = True
    return ex, o4


def hct_integral(r, a, s):
    """(1/4pi) * integral of |x|^-4 over the ball of radius s centred at
    distance r from the origin, outside the ball of radius a about the
    origin (r > 0)."""
    if a >= r + s:
        return 0.0
    L = max(a, abs(r - s))
    U = r + s
    l, u = 1.0 / L, 1.0 / U
    h = (0.5 * (l - u) + (s * s - r * r) * (l * l - u * u) / (8.0 * r) +
         math.log(u / l) / (4.0 * r))
    if a < s - r:   # the origin lies inside the ball: shells a..s-r whole
        h += 1.0 / a - 1.0 / (s - r)
    return h


def born_radii(x, rho, S):
    n = len(rho)
    rt = rho - DIELECTRIC_OFFSET
    a, b, c = OBC_ABG
    R = np.zeros(n)
    for i in range(n):
        I = 0.0
        for j in range(n):
            if j == i:
                continue
            r = float(np.linalg.norm(x[i] - x[j]))
            I += hct_integral(r, rt[i], S[j] * rt[j])
        psi = I * rt[i]
        R[i] = 1.0 / (1.0 / rt[i] - math.tanh(a * psi - b * psi ** 2 +
                                              c * psi ** 3) / rho[i])
    return R


def energy_terms(x, p, magnitudes=False):
    """(E_LJ, E_Coulomb, E_GB, E_SA) of one configuration x (n, 3); p is a
    dict with charge, sigma, eps, rho, S (n each), excluded and one_four
    (n x n), lj14, el14, eps_solute, eps_solvent, gamma, probe.  With
    magnitudes, also the sums of the absolute values of each energy's
    contributions (pair terms, GB pair terms, per-atom SA terms): the scale
    against which the rounding of a float32 evaluation is judged."""
    x = np.asarray(x, np.float64)
    n = len(x)
    q, sg, ep = p["charge"], p["sigma"], p["eps"]
    ex, o4 = p["excluded"], p["one_four"]
    e_lj = e_c = 0.0
    m_lj = m_c = m_gb = 0.0
    for i in range(n):
        for j in range(i + 1, n):
            if ex[i, j]:
                continue
            r = float(np.linalg.norm(x[i] - x[j]))
            s = 0.5 * (sg[i] + sg[j])
            e = math.sqrt(ep[i] * ep[j])
            sr6 = (s / r) ** 6
            lj = 4.0 * e * (sr6 * sr6 - sr6)
            cl = K_COULOMB * q[i] * q[j] / (p["eps_solute"] * r)
            if o4[i, j]:
                lj *= p["lj14"]
                cl *= p["el14"]
            e_lj += lj
            e_c += cl
            m_lj += abs(lj)
            m_c += abs(cl)
    R = born_radii(x, p["rho"], p["S"])
    tau = 1.0 / p["eps_solute"] - 1.0 / p["eps_solvent"]
    e_gb = 0.0
    for i in range(n):
        for j in range(n):
            if i == j:
                f = R[i]
            else:
                r2 = float(np.sum((x[i] - x[j]) ** 2))
                RR = R[i] * R[j]
                f = math.sqrt(r2 + RR * math.exp(-r2 / (4.0 * RR)))
            e_gb += q[i] * q[j] / f
            m_gb += abs(q[i] * q[j] / f)
    e_gb *= -0.5 * K_COULOMB * tau
    m_gb *= 0.5 * K_COULOMB * abs(tau)
    e_sa = 0.0
    for i in range(n):
        e_sa += (4.0 * math.pi * p["gamma"] * (p["rho"][i] + p["probe"]) ** 2 *
                 (p["rho"][i] / R[i]) ** 6)
    e = np.array([e_lj, e_c, e_gb, e_sa])
    if magnitudes:
        return e, np.array([m_lj, m_c, m_gb, e_sa])
    return e


def forces(x, p, h=1e-5):
    """-grad of the total by central differences (n, 3)."""
    x = np.asarray(x, np.float64)
    F = np.zeros_like(x)
    for i in range(len(x)):
        for d in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            F[i, d] = -(energy_terms(xp, p).sum() -
                        energy_terms(xm, p).sum()) / (2 * h)
    return F
