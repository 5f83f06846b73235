"""FP64 oracle of the learned rigid-body pose proposal -- TEST INFRASTRUCTURE
ONLY.

The paper accelerates pose transitions with external-coordinate Monte Carlo
moves: a random rotation about the centre of mass plus a Gaussian
translation, accepted by the Metropolis criterion (Sampling section).  The
learned variant replaces the random proposal by an independence
Metropolis-Hastings proposal drawn from a conditional density q(xi | tau)
over the ligand's rigid-body pose xi = (t, R): t = centre of mass minus the
site centre, R = orientation of a body frame, tau = sin/cos of internal
torsions (unchanged by the move).  Internal coordinates y_i = R^T (x_i - c)
are kept, so x'_i = c0 + t' + R' y_i.

Density.  q is an 8-component diagonal Gaussian mixture over the 6-vector
(t, omega) in R^3 x R^3, omega a rotation vector, produced by an MLP
16 -> 256 -> 256 -> 104 (SiLU).  Pushed forward to SE(3), its density with
respect to Lebesgue(t) x Haar(R) (Haar written as J(omega) d^3omega with
J = 2 (1 - cos|omega|) / |omega|^2) is

    q(t, R) = sum_{m} p_mix(t, (theta + 2 pi m) n) / J((theta + 2 pi m) n)

over the preimages of R = exp(theta n), theta in (0, pi], m in -M..M.  The
Cartesian measure splits into Lebesgue(c) x Haar(R) x (internal measure), so
the move is exact with

    ln alpha = -beta_k [E_k(x') - E_k(x)] + ln q(xi) - ln q(xi').

Output layout of the network (per component j = 0..7, 13 numbers):
    [logit, mu_t (3), raw_mu_w (3), raw_s_t (3), raw_s_w (3)]
    mu_w = pi tanh(raw),  s = s_min + (s_max - s_min) sigmoid(raw)
with s_t in [0.02, 3] A and s_w in [0.02, 1.5] rad.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import logsumexp

N_FEAT, N_HID, N_COMP = 16, 256, 8
N_OUT = N_COMP * 13
S_T = (0.02, 3.0)
S_W = (0.02, 1.5)
M_FOLD = 3
TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# rotations
# --------------------------------------------------------------------------

def rodrigues(w):
    """Rotation matrix exp([w]_x) of a rotation vector (float64)."""
    w = np.asarray(w, np.float64)
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-8:
        return np.eye(3) + K + 0.5 * K @ K
    return np.eye(3) + math.sin(th) / th * K + \
        (1 - math.cos(th)) / th ** 2 * K @ K


def log_rotation(R):
    """Rotation vector omega with |omega| in [0, pi] and exp(omega) = R.

    theta = atan2(|v|/2, (tr R - 1)/2) with v the axial vector of R - R^T
    (|v| = 2 sin theta), axis v/|v|: well conditioned up to theta -> pi,
    where the axis comes from the symmetric part (R + I)/2 = n n^T."""
    R = np.asarray(R, np.float64)
    c = (np.trace(R) - 1.0) / 2.0
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    s2 = np.linalg.norm(v)            # 2 sin theta
    th = math.atan2(0.5 * s2, c)
    if s2 < 1e-12:
        if c > 0:
            return 0.5 * v
    elif s2 > 1e-4 or c > 0:
        return th * v / s2
    # theta within ~5e-5 of pi: axis from the symmetric part
    B = (R + R.T) / 4.0 + np.eye(3) / 2.0
    k = int(np.argmax(np.diag(B)))
    n = B[:, k] / math.sqrt(max(B[k, k], 1e-300))
    n /= np.linalg.norm(n)
    if np.dot(n, v) < 0:
        n = -n
    return th * n


# --------------------------------------------------------------------------
# pose and features
# --------------------------------------------------------------------------

def body_frame(x, frame_atoms):
    a0, a1, a2 = frame_atoms
    e1 = x[a1] - x[a0]
    e1 = e1 / np.linalg.norm(e1)
    v = x[a2] - x[a0]
    e2 = v - np.dot(v, e1) * e1
    e2 = e2 / np.linalg.norm(e2)
    e3 = np.cross(e1, e2)
    return np.stack([e1, e2, e3], axis=1)   # columns


def pose(x, mass, frame_atoms, c0):
    """(t, R, y): t = COM - c0, R body frame, y_i = R^T (x_i - COM)."""
    x = np.asarray(x, np.float64)
    c = (mass[:, None] * x).sum(0) / mass.sum()
    R = body_frame(x, frame_atoms)
    y = (x - c) @ R
    return c - c0, R, y


def rebuild(t, R, y, c0):
    return c0 + t + y @ R.T


def dihedral(a, b, c, d):
    b1, b2, b3 = b - a, c - b, d - c
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    return math.atan2(np.linalg.norm(b2) * np.dot(b1, n2), np.dot(n1, n2))


def features(x, cond_tors):
    """sin/cos of up to 8 conditioning torsions, zero padded to 16."""
    f = np.zeros(N_FEAT)
    for q, (i, j, k, l) in enumerate(cond_tors[:8]):
        phi = dihedral(x[i], x[j], x[k], x[l])
        f[2 * q] = math.sin(phi)
        f[2 * q + 1] = math.cos(phi)
    return f


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------

def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_weights(rng):
    """Weights W1 (16,256), b1, W2 (256,256), b2, W3 (256,104), b3 with
    fan-in scaling; returned as float64 arrays."""
    def lin(i, o, g=1.0):
        return (rng.normal(size=(i, o)) * g / math.sqrt(i),
                np.zeros(o))
    W1, b1 = lin(N_FEAT, N_HID)
    W2, b2 = lin(N_HID, N_HID)
    W3, b3 = lin(N_HID, N_OUT, 0.1)
    return dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


def forward(p, f):
    """f (B,16) -> out (B,104) and the activations for backward."""
    z1 = f @ p["W1"] + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = silu(z2)
    out = h2 @ p["W3"] + p["b3"]
    return out, (f, z1, h1, z2, h2)


def backward(p, cache, dout):
    f, z1, h1, z2, h2 = cache
    g = {}
    g["W3"] = h2.T @ dout
    g["b3"] = dout.sum(0)
    dz2 = (dout @ p["W3"].T) * dsilu(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * dsilu(z1)
    g["W1"] = f.T @ dz1
    g["b1"] = dz1.sum(0)
    return g


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def mixture(out):
    """Split network outputs (B,104) into mixture parameters."""
    o = np.asarray(out, np.float64).reshape(-1, N_COMP, 13)
    logit = o[..., 0]
    mu_t = o[..., 1:4]
    mu_w = math.pi * np.tanh(o[..., 4:7])
    s_t = S_T[0] + (S_T[1] - S_T[0]) * _sig(o[..., 7:10])
    s_w = S_W[0] + (S_W[1] - S_W[0]) * _sig(o[..., 10:13])
    return dict(logit=logit, mu_t=mu_t, mu_w=mu_w, s_t=s_t, s_w=s_w)


def log_pmix(mp, t, w):
    """ln p_mix(t, w) per row; mp from mixture(); t, w (B,3)."""
    t = np.asarray(t, np.float64)[:, None, :]
    w = np.asarray(w, np.float64)[:, None, :]
    lw = mp["logit"] - logsumexp(mp["logit"], axis=1, keepdims=True)
    zt = (t - mp["mu_t"]) / mp["s_t"]
    zw = (w - mp["mu_w"]) / mp["s_w"]
    lg = -0.5 * (zt ** 2).sum(-1) - np.log(mp["s_t"]).sum(-1) \
        - 0.5 * (zw ** 2).sum(-1) - np.log(mp["s_w"]).sum(-1) \
        - 6 * 0.5 * math.log(TWO_PI)
    return logsumexp(lw + lg, axis=1)


def nll_grad(p, f, t, w):
    """Mean negative log-likelihood of (t, w) under the network's mixture and
    its gradient with respect to every parameter (float64 backprop)."""
    out, cache = forward(p, f)
    B = len(f)
    o = out.reshape(B, N_COMP, 13)
    mp = mixture(out)
    t3 = np.asarray(t, np.float64)[:, None, :]
    w3 = np.asarray(w, np.float64)[:, None, :]
    lw = mp["logit"] - logsumexp(mp["logit"], axis=1, keepdims=True)
    zt = (t3 - mp["mu_t"]) / mp["s_t"]
    zw = (w3 - mp["mu_w"]) / mp["s_w"]
    lg = -0.5 * (zt ** 2).sum(-1) - np.log(mp["s_t"]).sum(-1) \
        - 0.5 * (zw ** 2).sum(-1) - np.log(mp["s_w"]).sum(-1) \
        - 3 * math.log(TWO_PI)
    a = lw + lg
    ll = logsumexp(a, axis=1)
    loss = -ll.mean()
    r = np.exp(a - ll[:, None])               # responsibilities (B, 8)
    pi = np.exp(lw)
    d = np.zeros_like(o)                      # d loss / d out, per sample
    d[..., 0] = -(r - pi)
    # d lg / d mu = z / s ; d lg / d s = (z^2 - 1) / s
    d[..., 1:4] = -r[..., None] * zt / mp["s_t"]
    dmu_w = -r[..., None] * zw / mp["s_w"]
    th = np.tanh(o[..., 4:7])
    d[..., 4:7] = dmu_w * math.pi * (1 - th ** 2)
    ds_t = -r[..., None] * (zt ** 2 - 1) / mp["s_t"]
    sg = _sig(o[..., 7:10])
    d[..., 7:10] = ds_t * (S_T[1] - S_T[0]) * sg * (1 - sg)
    ds_w = -r[..., None] * (zw ** 2 - 1) / mp["s_w"]
    sg = _sig(o[..., 10:13])
    d[..., 10:13] = ds_w * (S_W[1] - S_W[0]) * sg * (1 - sg)
    dout = d.reshape(B, N_OUT) / B
    return loss, backward(p, cache, dout), dout


# --------------------------------------------------------------------------
# density on SE(3), sampling
# --------------------------------------------------------------------------

def log_q_se3(mp_row, t, R):
    """ln q(t, R) w.r.t. Lebesgue x Haar (J d^3 omega) for one mixture."""
    w0 = log_rotation(R)
    th = np.linalg.norm(w0)
    if th < 1e-9:
        # identity: only the m = 0 preimage is a point; J -> 1 there
        mp1 = {k: v[None] for k, v in mp_row.items()}
        return float(log_pmix(mp1, t[None], np.zeros((1, 3)))[0])
    n = w0 / th
    terms = []
    ws = []
    for m in range(-M_FOLD, M_FOLD + 1):
        a = th + TWO_PI * m
        ws.append(a * n)
        terms.append(2.0 * math.log(abs(a)) - math.log(2.0 * (1 - math.cos(th))))
    mp1 = {k: np.repeat(v[None], len(ws), axis=0) for k, v in mp_row.items()}
    lp = log_pmix(mp1, np.repeat(np.asarray(t)[None], len(ws), 0),
                  np.array(ws))
    return float(logsumexp(lp + np.array(terms)))


def sample(mp_row, u_comp, z_t, z_w):
    """Draw (t, omega) from one mixture given a uniform and six normals."""
    pw = np.exp(mp_row["logit"] - logsumexp(mp_row["logit"]))
    cum = np.cumsum(pw)
    j = int(np.searchsorted(cum, u_comp * cum[-1], side="left"))
    j = min(j, N_COMP - 1)
    t = mp_row["mu_t"][j] + mp_row["s_t"][j] * np.asarray(z_t)
    w = mp_row["mu_w"][j] + mp_row["s_w"][j] * np.asarray(z_w)
    return j, t, w


def pose_move(x, mass, frame_atoms, c0, mp_row, energy, beta, u_comp, z_t,
              z_w, u_acc):
    """One independence Metropolis-Hastings pose move of one replica.

    energy(x) returns the state's potential energy E_k(x); the internal
    coordinates (and with them the bonded energy) are unchanged.  Returns
    (x_new, accepted, ln_alpha)."""
    t, R, y = pose(x, mass, frame_atoms, c0)
    _, t2, w2 = sample(mp_row, u_comp, z_t, z_w)
    R2 = rodrigues(w2)
    x2 = rebuild(t2, R2, y, c0)
    lq_old = log_q_se3(mp_row, t, R)
    lq_new = log_q_se3(mp_row, t2, R2)
    ln_a = -beta * (energy(x2) - energy(x)) + lq_old - lq_new
    acc = bool(np.isfinite(ln_a) and math.log(u_acc) < ln_a)
    return (x2 if acc else np.asarray(x, np.float64)), acc, ln_a
