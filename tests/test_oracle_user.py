"""Pins of the oracle's path for caller-defined integrands (points from the
oracle's own sampler, integrand in numpy, exact-rounded sums).

* The harmonic family written as a caller function must reproduce the oracle's
  built-in harmonic sums on the same seeds (same samples, same formula).
* A quadratic integrand's estimate must lie within a few standard errors of
  its closed form, and the SE must match the closed-form variance.
* Brute force on a tiny N: the sums equal fsum over points taken one by one.
"""

import math

import numpy as np

import user_families as U
from oracle import oracle as O
from paper_2104_10073_amd import workloads as W


def _harmonic_np(x, p):
    theta = np.zeros(x.shape[0])
    for j in range(x.shape[1]):
        theta = theta + p[2 + j] * x[:, j]
    return p[0] * np.cos(theta) + p[1] * np.sin(theta)


def test_user_path_reproduces_builtin_harmonic():
    t = W.mixed_batch(40, dim_range=(1, 12), log10_samples=(2.0, 4.0), gen_seed=11)
    t = t[t["family"] == W.HARMONIC]
    assert len(t) >= 5
    ref, _ = O.integrate(t, 4)
    got = O.default().integrate_user(t, _harmonic_np)
    assert np.array_equal(got["n"], ref["n"])
    assert np.all(np.abs(got["sum_f"] - ref["sum_f"]) <= 1e-13 * ref["sum_abs"])
    assert np.all(np.abs(got["sum_f2"] - ref["sum_f2"]) <= 1e-13 * ref["sum_f2"])


def test_quadratic_closed_form():
    """f = p0 + sum_j p_j x_j^2 (p1 = 0): E f = p0 + sum p_j (hi^3-lo^3)/(3w);
    Var f = sum p_j^2 Var(x_j^2), Var(x^2) = (hi^5-lo^5)/(5w) - ((hi^3-lo^3)/(3w))^2."""
    t = U.user_table(12, 16, gen_seed=21, log10_samples=(4.0, 4.7), dim_range=(1, 6))
    t["params"][:, 1] = 0.0
    got = O.default().integrate_user(t, U.quad_sine_np)
    zs = []
    for i in range(len(t)):
        d = int(t["dim"][i])
        lo, hi, p = t["lo"][i, :d], t["hi"][i, :d], t["params"][i]
        w = hi - lo
        m2 = (hi ** 3 - lo ** 3) / (3 * w)
        m4 = (hi ** 5 - lo ** 5) / (5 * w)
        mean_f = p[0] + np.sum(p[2:2 + d] * m2)
        var_f = np.sum(p[2:2 + d] ** 2 * (m4 - m2 ** 2))
        V = float(np.prod(w))
        n = int(t["n_samples"][i])
        se_exact = V * math.sqrt(var_f / n)
        zs.append((got["mean"][i] - V * mean_f) / se_exact)
        assert abs(got["stderr"][i] / se_exact - 1.0) < 0.1
    zs = np.array(zs)
    assert np.all(np.abs(zs) < 4.5), zs
    assert abs(np.mean(zs)) < 1.5


def test_tiny_n_brute_force():
    t = U.user_table(4, 16, gen_seed=31, log10_samples=(0.5, 1.2))
    got = O.default().integrate_user(t, U.rational_np)
    orc = O.default()
    for i in range(len(t)):
        n = int(t["n_samples"][i])
        vals = [float(U.rational_np(orc.sample_point(t, i, k)[None, :], t["params"][i])[0]) for k in range(n)]
        assert got["sum_f"][i] == math.fsum(vals)
        assert got["sum_f2"][i] == math.fsum(v * v for v in vals)
