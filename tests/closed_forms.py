"""Exact box integrals of the four integrand families (test-side ground truth).

These pin the oracle's *estimates* statistically: for a function f on a box B,
the direct MC estimate with N samples has mean F = int_B f and standard error
V * sqrt(Var_u(f) / N), where Var_u(f) = int_B f^2 / V - (int_B f / V)^2.
Both integrals have closed forms for every family used here:

* HARMONIC (Eq. 1)  int e^{i k.x} over a box = prod_j (e^{i k_j hi_j} - e^{i k_j lo_j}) / (i k_j)
  (the factor is the width when k_j = 0); cos and sin are its real and
  imaginary parts, and f^2 expands into a constant plus the same product at 2k.
* ABS_LINEAR (Eq. 2) int (L)_+ over a box for L = c0 + c.x, all c_j != 0, is the
  alternating vertex sum sum_s (-1)^{d-|s|} L(v_s)_+^{d+1} / ((d+1)! prod c_j);
  int |L| = 2 int L_+ - int L.  Evaluated in exact rationals because the 2^d
  terms cancel heavily.
* GAUSSIAN          a product of erf differences.
* POLY_PRODUCT      a product of one-dimensional polynomial integrals, exact in rationals.

Nothing here is shared with the oracle or the GPU library.
"""

from __future__ import annotations

import itertools
import math
from fractions import Fraction

import mpmath

from paper_2104_10073_amd import workloads as W

mpmath.mp.dps = 40


def _row(t, i):
    d = int(t["dim"][i])
    fam = int(t["family"][i])
    lo = [float(v) for v in t["lo"][i, :d]]
    hi = [float(v) for v in t["hi"][i, :d]]
    p = [float(v) for v in t["params"][i]]
    return fam, d, lo, hi, p


def _harmonic_product(k, lo, hi, scale=1):
    prod = mpmath.mpc(1)
    for kj, l, h in zip(k, lo, hi):
        kk = mpmath.mpf(kj) * scale
        if kk == 0:
            prod *= (mpmath.mpf(h) - mpmath.mpf(l))
        else:
            prod *= (mpmath.expj(kk * mpmath.mpf(h)) - mpmath.expj(kk * mpmath.mpf(l))) / (1j * kk)
    return prod


def _abs_linear_pos(c0, c, lo, hi):
    """int over the box of max(c0 + c.x, 0), exact (Fractions), handling c_j == 0."""
    c0 = Fraction(c0)
    width_factor = Fraction(1)
    cs, ls, hs = [], [], []
    for cj, l, h in zip(c, lo, hi):
        if cj == 0:
            width_factor *= Fraction(h) - Fraction(l)
        else:
            cs.append(Fraction(cj))
            ls.append(Fraction(l))
            hs.append(Fraction(h))
    d = len(cs)
    if d == 0:
        return width_factor * max(c0, Fraction(0))
    denom = Fraction(math.factorial(d + 1))
    for cj in cs:
        denom *= cj
    acc = Fraction(0)
    for s in itertools.product((0, 1), repeat=d):
        val = c0 + sum(cj * (hj if sj else lj) for cj, lj, hj, sj in zip(cs, ls, hs, s))
        if val > 0:
            sign = -1 if (d - sum(s)) % 2 else 1
            acc += sign * val ** (d + 1)
    return width_factor * acc / denom


def exact_moments(t, i):
    """(int f, int f^2, V) for function i of table t, as mpmath numbers."""
    fam, d, lo, hi, p = _row(t, i)
    V = mpmath.mpf(1)
    for l, h in zip(lo, hi):
        V *= mpmath.mpf(h) - mpmath.mpf(l)
    if fam == W.HARMONIC:
        a, b = mpmath.mpf(p[0]), mpmath.mpf(p[1])
        k = p[W.V0:W.V0 + d]
        P1 = _harmonic_product(k, lo, hi, 1)
        P2 = _harmonic_product(k, lo, hi, 2)
        I1 = a * P1.real + b * P1.imag
        # f^2 = (a^2+b^2)/2 + (a^2-b^2)/2 cos(2 theta) + a b sin(2 theta)
        I2 = (a * a + b * b) / 2 * V + (a * a - b * b) / 2 * P2.real + a * b * P2.imag
        return I1, I2, V
    if fam == W.ABS_LINEAR:
        a, c0 = Fraction(p[0]), Fraction(p[1])
        c = p[W.V0:W.V0 + d]
        Vq = Fraction(1)
        mean_L = c0
        var_L = Fraction(0)
        for cj, l, h in zip(c, lo, hi):
            w = Fraction(h) - Fraction(l)
            Vq *= w
            mean_L += Fraction(cj) * (Fraction(l) + Fraction(h)) / 2
            var_L += Fraction(cj) ** 2 * w * w / 12
        int_L = Vq * mean_L
        int_pos = _abs_linear_pos(p[1], c, lo, hi)
        int_abs = 2 * int_pos - int_L
        int_L2 = Vq * (mean_L ** 2 + var_L)
        I1 = a * int_abs
        I2 = a * a * int_L2
        return mpmath.mpf(I1.numerator) / I1.denominator, mpmath.mpf(I2.numerator) / I2.denominator, V
    if fam == W.GAUSSIAN:
        A, sigma = mpmath.mpf(p[0]), mpmath.mpf(p[1])
        mu = p[W.V0:W.V0 + d]

        def one(sig, amp):
            val = amp
            for m, l, h in zip(mu, lo, hi):
                s2 = sig * mpmath.sqrt(2)
                val *= sig * mpmath.sqrt(mpmath.pi / 2) * (
                    mpmath.erf((mpmath.mpf(h) - m) / s2) - mpmath.erf((mpmath.mpf(l) - m) / s2))
            return val

        return one(sigma, A), one(sigma / mpmath.sqrt(2), A * A), V
    if fam == W.POLY_PRODUCT:
        pp = p[W.V0:W.V0 + d]
        dg = [int(v) for v in p[W.W0:W.W0 + d]]
        I1 = Fraction(1)
        I2 = Fraction(1)
        for pj, e, l, h in zip(pp, dg, lo, hi):
            P, L, H = Fraction(pj), Fraction(l), Fraction(h)
            m1 = (H ** (e + 1) - L ** (e + 1)) / (e + 1)
            m2 = (H ** (2 * e + 1) - L ** (2 * e + 1)) / (2 * e + 1)
            I1 *= (H - L) + P * m1
            I2 *= (H - L) + 2 * P * m1 + P * P * m2
        return mpmath.mpf(I1.numerator) / I1.denominator, mpmath.mpf(I2.numerator) / I2.denominator, V
    raise ValueError(fam)


def exact_integral(t, i) -> float:
    return float(exact_moments(t, i)[0])


def exact_se(t, i, n=None) -> float:
    """Standard error of the direct MC estimate with n samples (default: the table's)."""
    I1, I2, V = exact_moments(t, i)
    n = int(t["n_samples"][i]) if n is None else n
    var_u = I2 / V - (I1 / V) ** 2
    if var_u < 0:
        var_u = mpmath.mpf(0)
    return float(V * mpmath.sqrt(var_u / n))


def point_value(t, i, x) -> mpmath.mpf:
    """f(x) at the exact double coordinates x, in 40-digit arithmetic."""
    fam, d, lo, hi, p = _row(t, i)
    xs = [mpmath.mpf(float(v)) for v in x[:d]]
    if fam == W.HARMONIC:
        th = sum(mpmath.mpf(p[W.V0 + j]) * xs[j] for j in range(d))
        return mpmath.mpf(p[0]) * mpmath.cos(th) + mpmath.mpf(p[1]) * mpmath.sin(th)
    if fam == W.ABS_LINEAR:
        s = mpmath.mpf(p[1]) + sum(mpmath.mpf(p[W.V0 + j]) * xs[j] for j in range(d))
        return mpmath.mpf(p[0]) * abs(s)
    if fam == W.GAUSSIAN:
        q = sum((xs[j] - mpmath.mpf(p[W.V0 + j])) ** 2 for j in range(d))
        return mpmath.mpf(p[0]) * mpmath.exp(-q / (2 * mpmath.mpf(p[1]) ** 2))
    if fam == W.POLY_PRODUCT:
        val = mpmath.mpf(1)
        for j in range(d):
            val *= 1 + mpmath.mpf(p[W.V0 + j]) * xs[j] ** int(p[W.W0 + j])
        return val
    raise ValueError(fam)


def theta_scale(t, i, x) -> float:
    """Magnitude that bounds FP64 rounding of f(x): the size of the inner sums before the last op."""
    fam, d, lo, hi, p = _row(t, i)
    if fam == W.HARMONIC:
        return (abs(p[0]) + abs(p[1])) * (1 + sum(abs(p[W.V0 + j] * x[j]) for j in range(d)))
    if fam == W.ABS_LINEAR:
        return abs(p[0]) * (abs(p[1]) + sum(abs(p[W.V0 + j] * x[j]) for j in range(d)) + 1e-300)
    return 0.0
