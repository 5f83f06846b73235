"""FP64 estimators for the oracle -- TEST INFRASTRUCTURE ONLY.

* MBAR (Shirts & Chodera 2008; the paper estimates f_BC,L and f_CD' with it,
  Methodology, "Estimation"): the reduced free energies f_i solve
      f_i = -ln sum_n exp(-u_in) / sum_k N_k exp(f_k - u_kn),
  equivalently they minimise the convex function
      F(f) = sum_n ln sum_k N_k exp(f_k - u_kn) - sum_i N_i f_i
  under the gauge f_0 = 0.  Solved here by Newton's method with a
  backtracking line search, falling back to the fixed-point equation while
  the Hessian is not numerically positive definite; float64, log-sum-exp.
  The asymptotic variance of f_i - f_j is (e_i - e_j)^T H^- (e_i - e_j)
  - 1/N_i - 1/N_j, with H the Hessian of F at the solution and H^- any
  generalised inverse (the gauge-fixed block inverse is used).
* statistical inefficiency g and effective sample size N/g of a time series
  (the paper separates equilibration and production by maximising the
  number of uncorrelated samples, after Chodera 2016):
      g = 1 + 2 sum_{t>=1} (1 - t/N) C_t / C_0, truncated at the first
      C_t <= 0.
"""
from __future__ import annotations

import numpy as np
from scipy.special import logsumexp


def _objective(f, u_kn, logN):
    a = (logN + f)[:, None] - u_kn
    return float(np.sum(logsumexp(a, axis=0)) - np.sum(np.exp(logN) * f))


def _self_consistent(f, u_kn, logN):
    """One step of the MBAR fixed-point equation, gauge f_0 = 0."""
    logD = logsumexp((logN + f)[:, None] - u_kn, axis=0)
    fn = -logsumexp(-u_kn - logD[None, :], axis=1)
    return fn - fn[0]


def mbar(u_kn, N_k, tol=1e-10, max_iter=10000):
    """Return (f, var_diff_last, n_iter).

    u_kn : (K, N) reduced energies of every sample n in every state k.
    N_k  : (K,) number of samples drawn from each state (all > 0).
    f[0] == 0 (gauge); var_diff_last is the asymptotic variance of
    f[K-1] - f[0].

    Each iteration takes a Newton step (with backtracking on F) when the
    gauge-fixed Hessian is numerically positive definite, otherwise one
    step of the fixed-point equation; far from the solution the weights of
    whole states can underflow and leave the Hessian singular.
    """
    u_kn = np.asarray(u_kn, np.float64)
    N_k = np.asarray(N_k, np.float64)
    K, N = u_kn.shape
    assert np.all(N_k > 0) and abs(N_k.sum() - N) < 0.5
    logN = np.log(N_k)
    f = np.zeros(K)
    it = 0
    for it in range(1, max_iter + 1):
        a = (logN + f)[:, None] - u_kn               # K x N
        logD = logsumexp(a, axis=0)                   # N
        W = np.exp(f[:, None] - u_kn - logD[None, :])  # K x N  (W_ni^T)
        colsum = W.sum(axis=1)                        # sum_n W_ni
        g = N_k * (colsum - 1.0)
        H = np.diag(N_k * colsum) - (N_k[:, None] * N_k[None, :]) * (W @ W.T)
        Hg = H[1:, 1:]
        try:
            Lc = np.linalg.cholesky(Hg)
            ok = np.min(np.diag(Lc)) ** 2 > 1e-13 * np.max(np.diag(Hg))
        except np.linalg.LinAlgError:
            ok = False
        if ok:
            step = np.zeros(K)
            step[1:] = -np.linalg.solve(Hg, g[1:])
            F0 = _objective(f, u_kn, logN)
            t = 1.0
            while True:
                fn = f + t * step
                if _objective(fn, u_kn, logN) <= F0 + 1e-4 * t * \
                        float(g @ step) + 1e-13 * abs(F0) or t < 1e-8:
                    break
                t *= 0.5
        else:
            fn = _self_consistent(f, u_kn, logN)
        change = np.max(np.abs(fn - f))
        f = fn
        if change < tol:
            break
    # asymptotic variance at the solution
    a = (logN + f)[:, None] - u_kn
    logD = logsumexp(a, axis=0)
    W = np.exp(f[:, None] - u_kn - logD[None, :])
    H = np.diag(N_k * W.sum(axis=1)) - (N_k[:, None] * N_k[None, :]) * (W @ W.T)
    G = np.zeros((K, K))
    G[1:, 1:] = np.linalg.inv(H[1:, 1:])
    e = np.zeros(K)
    e[-1], e[0] = 1.0, -1.0
    var = float(e @ G @ e - 1.0 / N_k[-1] - 1.0 / N_k[0])
    return f, var, it


def mbar_var(u_kn, N_k, f, i, j):
    """Asymptotic variance of f_i - f_j at a converged f."""
    u_kn = np.asarray(u_kn, np.float64)
    N_k = np.asarray(N_k, np.float64)
    K = len(N_k)
    logN = np.log(N_k)
    a = (logN + f)[:, None] - u_kn
    logD = logsumexp(a, axis=0)
    W = np.exp(f[:, None] - u_kn - logD[None, :])
    H = np.diag(N_k * W.sum(axis=1)) - (N_k[:, None] * N_k[None, :]) * (W @ W.T)
    G = np.zeros((K, K))
    G[1:, 1:] = np.linalg.inv(H[1:, 1:])
    e = np.zeros(K)
    e[i] += 1.0
    e[j] -= 1.0
    return float(e @ G @ e - (1.0 / N_k[i] + 1.0 / N_k[j] if i != j else 0.0))


def statistical_inefficiency(a):
    """g of a scalar time series (truncated autocorrelation sum)."""
    a = np.asarray(a, np.float64)
    N = len(a)
    d = a - a.mean()
    c0 = float(d @ d) / N
    if c0 <= 0:
        return 1.0
    g = 1.0
    for t in range(1, N - 1):
        ct = float(d[:-t] @ d[t:]) / (N - t)
        if ct <= 0:
            break
        g += 2.0 * (1.0 - t / N) * ct / c0
    return max(g, 1.0)


def ess(a):
    return len(a) / statistical_inefficiency(a)
