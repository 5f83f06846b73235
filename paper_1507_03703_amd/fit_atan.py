"""Coefficients of the polynomial behind the angle term's arctangent.

atan(t) = t P(t^2) on [0, 1], P of degree 8, fitted by least squares on
20000 points (denser towards both ends) with weights updated from the
residuals until the error is nearly equioscillating.  Prints the
coefficients (lowest order first) and the largest absolute error in exact
arithmetic; the device code (angle_atan2 in csrc/device.h) holds them."""
import numpy as np


def fit(degree=8, n=20000, rounds=60):
    t = (1.0 - np.cos(np.linspace(0.0, np.pi, n))) / 2.0
    f = np.arctan(t)
    A = np.stack([t ** (2 * k + 1) for k in range(degree + 1)], axis=1)
    w = np.ones(n)
    for _ in range(rounds):
        c, *_ = np.linalg.lstsq(A * w[:, None], f * w, rcond=None)
        err = A @ c - f
        w = w * (np.abs(err) / np.abs(err).max() + 1e-3) ** 0.5
        w /= w.mean()
    return c, float(np.abs(A @ c - f).max())


if __name__ == "__main__":
    c, e = fit()
    print(", ".join("%.9e" % v for v in c))
    print("max abs error %.3g" % e)
