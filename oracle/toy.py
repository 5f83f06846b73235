"""Exact free energies of the solvable toy used to pin the whole pipeline --
TEST INFRASTRUCTURE ONLY.

Toy: a tree-shaped ligand with bonds only (no angles or torsions), equal
masses, equal charges q on n atoms (Q = n q), zero LJ factors, and an
electrostatic grid holding the linear potential G(x) = E.(x - c0) + phi0.
Under state k (inverse temperature beta_k, grid weight lambda_k) the reduced
potential is

    u_k = beta_k [ sum_b K_b (|b| - r0_b)^2 + U_I(c) + lambda_k Q (E.(c-c0) + phi0) ]

because with equal masses the centre of mass c is the mean position and the
electrostatic term only sees it.  Changing variables from atom positions to
(c, bond vectors) has a constant Jacobian, so the configurational integral
factorises into one radial integral per bond and one for the centre of mass
(angular part of exp(-a r cos theta) integrated in closed form):

    Z_b(beta)    = 4 pi int_0^inf b^2 exp(-beta K (b - r0)^2) db
    Z_c(beta, l) = exp(-beta l Q phi0) 4 pi int_0^inf r^2 sinh(a r)/(a r)
                   exp(-beta k (r - d0)_+^2 / 2) dr,   a = beta l Q |E|.

f_k - f_0 = -ln(Z_k / Z_0) is the quantity MBAR must reproduce
(restraint Eq. binding_site; alchemical protocol in "Thermodynamic Cycle").
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

R_GAS = 8.314462618e-3


def _ln_zb(beta, K, r0):
    s = 1.0 / math.sqrt(2.0 * beta * K)
    lo, hi = max(0.0, r0 - 40 * s), r0 + 40 * s
    # scale out the peak value to keep the integrand O(1)
    val, _ = integrate.quad(lambda b: (b / r0) ** 2 *
                            math.exp(-beta * K * (b - r0) ** 2), lo, hi,
                            epsabs=0, epsrel=1e-13, limit=400, points=[r0])
    return math.log(4 * math.pi) + 2 * math.log(r0) + math.log(val)


def _ln_zc(beta, lam, Q, Emag, phi0, k, d0):
    a = beta * lam * Q * Emag
    tail = d0 + 40.0 / math.sqrt(beta * k)

    def shape(r):
        # sinh(a r)/(a r) * exp(-a tail), arranged to avoid overflow
        if a * r > 1e-8:
            return (math.exp(a * r - a * tail) -
                    math.exp(-a * r - a * tail)) / (2 * a * r)
        return math.exp(-a * tail)

    def f(r):
        e = 0.0 if r <= d0 else 0.5 * beta * k * (r - d0) ** 2
        return r * r * shape(r) * math.exp(-e)

    val, _ = integrate.quad(f, 0.0, tail, epsabs=0, epsrel=1e-13, limit=400,
                            points=[d0])
    ln = math.log(4 * math.pi) + math.log(val)
    if a > 0:
        ln += a * tail
    return ln - beta * lam * Q * phi0


def exact_f(T, lam, bond_K, bond_r0, q, n_atoms, field, phi0, k_rest, d0):
    """Reduced free energies f_k - f_0 of the toy for each state."""
    T = np.asarray(T, np.float64)
    lam = np.asarray(lam, np.float64)
    Q = n_atoms * q
    Emag = float(np.linalg.norm(field))
    lnZ = np.zeros(len(T))
    for k in range(len(T)):
        beta = 1.0 / (R_GAS * T[k])
        s = 0.0
        for K, r0 in zip(bond_K, bond_r0):
            s += _ln_zb(beta, K, r0)
        s += _ln_zc(beta, lam[k], Q, Emag, phi0, k_rest, d0)
        lnZ[k] = s
    f = -lnZ
    return f - f[0]
