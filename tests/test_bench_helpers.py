"""The benchmark's statistics against the oracle's definitions (CPU): the
FFT statistical inefficiency equals the direct truncated autocorrelation
sum, batch means recover the AR(1) inefficiency, and a request for more than
one GPU is refused before anything touches a device."""
import os
import subprocess
import sys

import numpy as np

import bench
from oracle.estimators import statistical_inefficiency

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ar1(phi, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.normal(size=n)
    z = np.zeros(n)
    for t in range(1, n):
        z[t] = phi * z[t - 1] + e[t]
    return z


def test_fft_inefficiency_equals_the_direct_sum():
    for phi, n, seed in ((0.0, 500, 1), (0.5, 2000, 2), (0.9, 3000, 3),
                         (-0.3, 800, 4)):
        a = _ar1(phi, n, seed)
        g_fft = bench.stat_inefficiency(a)
        g_dir = statistical_inefficiency(a)
        assert abs(g_fft - g_dir) <= 1e-9 * g_dir, (phi, g_fft, g_dir)
    assert bench.stat_inefficiency(np.ones(10)) == 1.0


def test_batch_means_recover_the_ar1_inefficiency():
    phi = 0.9
    a = _ar1(phi, 300000, 5)
    g = bench.batch_means_inefficiency(a)
    g_ref = (1 + phi) / (1 - phi)
    assert abs(g - g_ref) < 0.35 * g_ref, (g, g_ref)
    assert bench.batch_means_inefficiency(np.ones(100)) == 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
