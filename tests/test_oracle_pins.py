"""The CPU oracle against facts outside itself (see tests/oracle_pins.py)."""

import math

import numpy as np
import pytest

import oracle_pins as P
from closed_forms import exact_integral
from paper_2104_10073_amd import workloads as W


def test_uniform(orc):
    P.check_uniform(orc)


def test_sample_points_exact(orc, rocrand_ref):
    P.check_sample_points(orc, rocrand_ref)


def test_point_values_vs_mpmath(orc):
    P.check_point_values(orc)


def test_brute_force_sums(orc, rocrand_ref):
    P.check_brute_force_sums(orc, rocrand_ref)


def test_compensated_sums(orc):
    P.check_compensated_sums(orc)


def test_finalize_textbook(orc):
    P.check_finalize_textbook(orc)


def test_special_cases(orc):
    P.check_special_cases(orc)


def test_closed_forms_within_4_sigma(orc):
    P.check_closed_forms_4sigma(orc)


def test_z_batches(orc):
    P.check_z_batch(orc)


def test_eq2_worked_values(orc):
    P.check_eq2_worked_values(orc)


def test_spread_over_independent_runs(orc):
    P.check_run_spread(orc)


def test_eq1_closed_form_matches_compact_formula():
    """Eq. (1) on [0,1]^4 with equal k: F_n = (2 sin(k/2)/k)^4 (cos 2k + sin 2k) -- pins the product form."""
    import mpmath
    t = W.eq1_series()
    for i in (0, 1, 24, 49, 74, 99):
        k = mpmath.mpf(i + 51) / (2 * mpmath.pi)
        compact = (2 * mpmath.sin(k / 2) / k) ** 4 * (mpmath.cos(2 * k) + mpmath.sin(2 * k))
        assert abs(exact_integral(t, i) - float(compact)) < 1e-15


def _float_point_value(t, i, x):
    """Plain double evaluation of f for quadrature (accurate to ~1e-15, far below the 1e-8 bar)."""
    d = int(t["dim"][i])
    p = t["params"][i]
    fam = int(t["family"][i])
    x = np.asarray(x, dtype=np.float64)
    if fam == W.HARMONIC:
        th = float(np.dot(p[W.V0:W.V0 + d], x))
        return p[0] * math.cos(th) + p[1] * math.sin(th)
    if fam == W.ABS_LINEAR:
        return p[0] * abs(p[1] + float(np.dot(p[W.V0:W.V0 + d], x)))
    if fam == W.GAUSSIAN:
        return p[0] * math.exp(-float(np.sum((x - p[W.V0:W.V0 + d]) ** 2)) / (2 * p[1] ** 2))
    return float(np.prod(1 + p[W.V0:W.V0 + d] * x ** p[W.W0:W.W0 + d]))


def test_closed_forms_vs_quadrature():
    """The closed forms themselves against adaptive quadrature in 1-2 dimensions."""
    from scipy import integrate
    import closed_forms as C
    t = P.small_mixed(16, dims=(1, 2), gen_seed=67)
    for i in range(len(t)):
        d = int(t["dim"][i])
        lo, hi = t["lo"][i, :d], t["hi"][i, :d]
        if int(t["family"][i]) == W.HARMONIC:
            # keep quadrature cheap: moderate frequencies
            t["params"][i, W.V0:W.V0 + d] = np.minimum(t["params"][i, W.V0:W.V0 + d], 8.0)

        def f(*x):
            return _float_point_value(t, i, x)

        def f2(*x):
            return _float_point_value(t, i, x) ** 2

        ranges = [(float(lo[j]), float(hi[j])) for j in range(d)]
        opts = {"limit": 200, "epsabs": 1e-11, "epsrel": 1e-11}
        q1, _ = integrate.nquad(f, ranges, opts=[opts] * d)
        q2, _ = integrate.nquad(f2, ranges, opts=[opts] * d)
        I1, I2, V = C.exact_moments(t, i)
        assert abs(q1 - float(I1)) < 1e-8 * (1 + abs(q1)), (i, q1, float(I1))
        assert abs(q2 - float(I2)) < 1e-8 * (1 + abs(q2)), (i, q2, float(I2))


def test_threads_do_not_change_results(orc):
    t = P.small_mixed(30, dims=(1, 7), n_samples=3000, gen_seed=71)
    r1, u1 = orc.integrate(t, 1)
    r8, u8 = orc.integrate(t, 8)
    assert u1 == 1 and u8 >= 1
    assert r1.tobytes() == r8.tobytes()


def test_validation_codes(orc):
    t = W.eq1_series(n_funcs=1)
    assert orc.validate(t, 0) == 0
    bad = t.copy(); bad["family"][0] = 9
    assert orc.validate(bad, 0) == -2
    bad = t.copy(); bad["dim"][0] = 13
    assert orc.validate(bad, 0) == -3
    bad = t.copy(); bad["hi"][0, 2] = bad["lo"][0, 2]
    assert orc.validate(bad, 0) == -4
    bad = t.copy(); bad["n_samples"][0] = 1
    assert orc.validate(bad, 0) == -1
    bad = t.copy(); bad["params"][0, 5] = np.nan
    assert orc.validate(bad, 0) == -5
