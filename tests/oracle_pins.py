"""Checks that pin the CPU oracle to facts outside itself.

Each check raises AssertionError on failure.  They are run against the real
oracle (test_oracle_pins.py) and against deliberately broken copies of it
(test_oracle_mutants.py), to show that a plausible mistake anywhere in the
oracle -- a dropped term, a wrong sign or index, a swapped operand -- fails at
least one of them.

Sources of truth used here, none of them the oracle's own code:
* rocRAND's Philox4x32-10 run on the host (an independent implementation),
* exact rational arithmetic for the uniform construction and the box mapping,
* 40-digit mpmath evaluation of each integrand at a point,
* math.fsum brute force of the sums on tiny sample counts, and exactly
  rounded sums where a plain running sum drifts (N up to 10^7),
* closed-form box integrals (tests/closed_forms.py): the estimate must sit
  within a few standard errors of the exact value, the standard errors must
  match the exact ones, and batches of z-scores must look standard normal,
* textbook special cases (constant integrands, linearity in the amplitudes).
"""

from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

from paper_2104_10073_amd import workloads as W

from closed_forms import exact_integral, exact_se, point_value

EPS = 2.0 ** -52


def word_index(dim: int, i: int, j: int) -> int:
    """Stream position of coordinate j of sample i: word s = i mod 4 of block (i // 4) * dim + j."""
    return 4 * ((i // 4) * dim + j) + (i % 4)


def stream_words(rocrand_ref, seed: int, dim: int, samples) -> dict:
    """rocRAND's words for the given samples (all coordinates), keyed by (i, j)."""
    samples = list(samples)
    quads = sorted({i // 4 for i in samples})
    lines = [f"w {seed} {4 * q * dim} {4 * dim}" for q in quads]
    got = rocrand_ref(lines)
    out = {}
    for q, words in zip(quads, got):
        for i in samples:
            if i // 4 == q:
                for j in range(dim):
                    out[(i, j)] = words[word_index(dim, i, j) - 4 * q * dim]
    return out


def exact_uniform(r: int) -> Fraction:
    return Fraction(2 * (r & 0x7FFFFF) + 1, 1 << 24)


def exact_point(t, i, words) -> list[float]:
    """Sample coordinates from raw words: x_j = round(lo_j + (hi_j - lo_j) * u_j)."""
    d = int(t["dim"][i])
    xs = []
    for j in range(d):
        lo, hi = float(t["lo"][i, j]), float(t["hi"][i, j])
        w = hi - lo
        xs.append(float(Fraction(lo) + Fraction(w) * exact_uniform(words[j])))
    return xs


def small_mixed(n=40, dims=(1, 4), n_samples=20_000, gen_seed=31, base=0):
    return W.mixed_batch(n, dim_range=dims, log10_samples=(4.0, 4.0001), gen_seed=gen_seed,
                         base=base, sample_scale=n_samples / 10_000)


# ---------------------------------------------------------------------------

def check_philox_blocks(orc, rocrand_ref, n=24):
    rng = np.random.Generator(np.random.PCG64(5))
    cases = [(0, 0, 0, 0, 0, 0)]
    for _ in range(n):
        c = [int(v) for v in rng.integers(0, 2**32, 4)]
        c[1] &= 0x0FFFFFFF
        k = [int(v) for v in rng.integers(0, 2**32, 2)]
        cases.append(tuple(c + k))
    ref = rocrand_ref(["b " + " ".join(str(v) for v in cs) for cs in cases])
    for cs, r in zip(cases, ref):
        assert orc.philox(cs[:4], cs[4:]) == r, ("philox block", cs)


def check_stream_layout(orc, rocrand_ref):
    for seed in (3, W.stream_seed(9, 2)):
        for dim in (1, 3, 5, 12):
            for i0 in (0, 3, 12345):
                samples = range(i0, i0 + 6)
                ref = stream_words(rocrand_ref, seed, dim, samples)
                for i in samples:
                    for j in range(dim):
                        assert orc.word(seed, dim, i, j) == ref[(i, j)], ("stream layout", seed, dim, i, j)


def check_uniform(orc):
    rng = np.random.Generator(np.random.PCG64(6))
    rs = [0, 1, 0x7FFFFF, 0x800000, 0xFFFFFFFF, 0x3F800000] + [int(v) for v in rng.integers(0, 2**32, 500)]
    for r in rs:
        u = orc.uniform(r)
        assert 0.0 < u < 1.0, ("uniform range", r)
        assert Fraction(u) == exact_uniform(r), ("uniform value", r)


def check_sample_points(orc, rocrand_ref):
    t = small_mixed(12, dims=(1, 12), gen_seed=41)
    for i in range(len(t)):
        d = int(t["dim"][i])
        seed = int(t["seed"][i])
        samples = (0, 1, 2, 5, 1001)
        ref = stream_words(rocrand_ref, seed, d, samples)
        for s in samples:
            want = exact_point(t, i, [ref[(s, j)] for j in range(d)])
            got = orc.sample_point(t, i, s)
            assert list(got) == want, ("sample point", i, s)


def check_point_values(orc, n_points=25):
    rng = np.random.Generator(np.random.PCG64(7))
    t = small_mixed(24, dims=(1, 7), gen_seed=43)
    for i in range(len(t)):
        d = int(t["dim"][i])
        fam = int(t["family"][i])
        lo, hi = t["lo"][i, :d], t["hi"][i, :d]
        for _ in range(n_points):
            x = rng.uniform(lo, hi)
            got = orc.evaluate(t, i, x)
            ex = point_value(t, i, x)
            p = t["params"][i]
            if fam == W.HARMONIC:
                scale = (abs(p[0]) + abs(p[1])) * (1.0 + float(np.sum(np.abs(p[W.V0:W.V0 + d] * x))))
                tol = 8 * EPS * scale
            elif fam == W.ABS_LINEAR:
                scale = abs(p[0]) * (abs(p[1]) + float(np.sum(np.abs(p[W.V0:W.V0 + d] * x))))
                tol = 8 * EPS * scale
            elif fam == W.GAUSSIAN:
                q = float(np.sum((x - p[W.V0:W.V0 + d]) ** 2)) / (2 * p[1] ** 2)
                tol = EPS * (8 + 4 * q) * abs(float(ex)) + 1e-300
            else:
                tol = 64 * EPS * float(np.prod(1 + np.abs(p[W.V0:W.V0 + d] * x ** p[W.W0:W.W0 + d])))
            assert abs(got - float(ex)) <= tol, ("point value", i, fam, got, float(ex))


def check_brute_force_sums(orc, rocrand_ref):
    """S1, S2 over N <= 16 samples equal fsum of exactly-evaluated f at exactly-mapped points."""
    t = small_mixed(16, dims=(1, 6), gen_seed=47)
    for i in range(len(t)):
        d = int(t["dim"][i])
        seed = int(t["seed"][i])
        n = 1 + (i % 16)
        ref = stream_words(rocrand_ref, seed, d, range(n))
        fs = []
        for s in range(n):
            x = exact_point(t, i, [ref[(s, j)] for j in range(d)])
            fs.append(point_value(t, i, x))
        s1_ref = math.fsum(float(v) for v in fs)
        s2_ref = math.fsum(float(v * v) for v in fs)
        sabs = math.fsum(abs(float(v)) for v in fs)
        s1, s2, sa = orc.partial_sums(t, i, 0, n)
        # each f carries a few ulp of evaluation error (harmonic phases up to ~200 rad)
        tol1 = 1e-13 * (sabs + 1.0)
        assert abs(s1 - s1_ref) <= tol1, ("S1 brute force", i, s1, s1_ref)
        assert abs(s2 - s2_ref) <= 1e-13 * (s2_ref + 1.0), ("S2 brute force", i, s2, s2_ref)
        assert abs(sa - sabs) <= tol1, ("sum|f| brute force", i)
        if n >= 2:
            # finalize: textbook unbiased variance of the same f values
            mean, se = orc.finalize(orc.volume(t, i), n, s1, s2)
            fl = [float(v) for v in fs]
            mu = math.fsum(fl) / n
            var = math.fsum((v - mu) ** 2 for v in fl) / (n - 1)
            V = float(np.prod(t["hi"][i, :d] - t["lo"][i, :d]))
            assert abs(mean - V * mu) <= 1e-12 * V * (sabs / n + 1e-300), ("finalize mean", i)
            se_ref = V * math.sqrt(var / n)
            assert abs(se - se_ref) <= 1e-6 * se_ref + 1e-12 * V * math.sqrt(s2_ref / n) / n, ("finalize se", i)


def check_compensated_sums(orc):
    """The oracle's sums are the accurate side of every parity bar (paper, "Solution
    method": one direct Monte Carlo sum per integrand over up to ~10^7 samples).

    Two cases where an uncompensated running sum visibly drifts, each against an
    exactly rounded sum computed outside the oracle:
    * a constant integrand with a non-dyadic value (Eq. (1) with k = 0: f = a
      exactly) over N = 10^7 + 3 samples -- S1 and sum|f| must equal N * fl(0.1)
      rounded once, S2 likewise N * fl(fl(0.1)^2) (a plain running sum is off by
      about 1.6e-10 relative here);
    * a high-frequency Eq. (1) term, f = cos(k x) on [0, 1] with k = 1000.5, over
      2^20 samples: positive and negative values cancel so that |S1| is about
      sqrt(N) while sum|f| is about 0.64 N.  The values are recomputed here from
      the oracle's sample points with Python's float arithmetic and libm cos (the
      same operations, each rounded once) and summed exactly with math.fsum (a
      plain running sum is off by ~10^3 ulp of S1)."""
    t = W.empty(2)
    n_const = 10_000_003
    W.set_harmonic(t, 0, 1, 0.1, 0.7, [0.0], [0.0], [1.0])
    W.set_harmonic(t, 1, 1, 1.0, 0.0, [1000.5], [0.0], [1.0])
    t["n_samples"][:] = [n_const, 1 << 20]
    t["seed"][:] = [11, 12]

    s1, s2, sa = orc.partial_sums(t, 0, 0, n_const)
    want1 = float(Fraction(0.1) * n_const)
    want2 = float(Fraction(0.1 * 0.1) * n_const)
    assert abs(s1 - want1) <= math.ulp(want1), ("compensated S1, constant", s1, want1)
    assert abs(sa - want1) <= math.ulp(want1), ("compensated sum|f|, constant", sa, want1)
    assert abs(s2 - want2) <= math.ulp(want2), ("compensated S2, constant", s2, want2)

    n = int(t["n_samples"][1])
    xs = orc.sample_points(t, 1, 0, n)[:, 0]
    fs = [math.cos(1000.5 * float(x)) for x in xs]
    want1 = math.fsum(fs)
    want2 = math.fsum(v * v for v in fs)
    wanta = math.fsum(abs(v) for v in fs)
    s1, s2, sa = orc.partial_sums(t, 1, 0, n)
    assert abs(want1) < 4.0 * math.sqrt(n) and wanta > 0.5 * n, "the case must cancel"
    assert abs(s1 - want1) <= 2.0 * math.ulp(want1), ("compensated S1, cancelling", s1, want1)
    assert abs(s2 - want2) <= 2.0 * math.ulp(want2), ("compensated S2, cancelling", s2, want2)
    assert abs(sa - wanta) <= 2.0 * math.ulp(wanta), ("compensated sum|f|, cancelling", sa, wanta)


def check_finalize_textbook(orc):
    """f = 1, 2, 3, 4 on a box of volume 2: mean 5, sample variance 5/3."""
    mean, se = orc.finalize(2.0, 4, 10.0, 30.0)
    assert mean == 5.0
    assert abs(se - 2.0 * math.sqrt((5.0 / 3.0) / 4.0)) <= 1e-15


def _z_scores(orc, t):
    res, _ = orc.integrate(t, threads=8)
    z = []
    ratios = []
    for i in range(len(t)):
        ex = exact_integral(t, i)
        se_ex = exact_se(t, i)
        assert res["status"][i] == 0
        if se_ex == 0.0:
            assert res["mean"][i] == ex or abs(res["mean"][i] - ex) <= 1e-12 * abs(ex)
            continue
        z.append((res["mean"][i] - ex) / se_ex)
        # The oracle's own SE estimates the exact one; its relative spread is about
        # sqrt((kurtosis - 1) / (4 N)), large for narrow Gaussians and high powers,
        # so single functions get a loose bound and the batch a tight one.
        r = res["stderr"][i] / se_ex
        assert abs(r - 1.0) < 0.5, ("stderr vs exact", i, res["stderr"][i], se_ex)
        ratios.append(r)
    ratios = np.array(ratios)
    assert abs(np.median(ratios) - 1.0) < 0.03, ("median SE ratio", np.median(ratios))
    assert abs(np.mean(ratios ** 2) - 1.0) < 0.1, ("mean variance ratio", np.mean(ratios ** 2))
    return np.array(z)


def check_closed_forms_4sigma(orc):
    """Every estimate within 4 sigma of its exact integral on tiny inputs (d <= 4, N = 2e4)."""
    t = small_mixed(40, dims=(1, 4), n_samples=20_000, gen_seed=53)
    z = _z_scores(orc, t)
    assert np.all(np.abs(z) < 4.0), ("4 sigma", np.max(np.abs(z)))


def check_z_batch(orc, n_funcs=100):
    """Batch z-scores look standard normal: Eq. (1) series and a mixed batch."""
    for t in (W.eq1_series(n_samples=10_000, n_funcs=n_funcs),
              small_mixed(n_funcs, dims=(1, 5), n_samples=10_000, gen_seed=59)):
        z = _z_scores(orc, t)
        m = len(z)
        assert abs(z.mean()) < 4.0 / math.sqrt(m), ("z mean", z.mean())
        assert abs((z * z).mean() - 1.0) < 4.0 * math.sqrt(2.0 / m), ("z^2 mean", (z * z).mean())


def check_run_spread(orc, runs=10, n_samples=2_000):
    """The paper's error bar (Fig. 1) is the sample standard deviation of the
    estimates over independent runs.  Over the Eq. (1) series, run r drawing the
    streams of base r: per function, (spread / exact SE)^2 is chi^2 with runs - 1
    degrees of freedom over runs - 1 (mean 1, sd sqrt(2 / (runs - 1))), and the
    mean over runs sits around the exact integral with sd SE / sqrt(runs)."""
    t0 = W.eq1_series(n_samples=n_samples)
    m = len(t0)
    est = []
    for r in range(runs):
        t = t0.copy()
        for i in range(m):
            t["seed"][i] = W.stream_seed(r, i)
        res, _ = orc.integrate(t, threads=8)
        est.append(res["mean"])
    est = np.array(est)
    fbar = est.mean(axis=0)
    spread = est.std(axis=0, ddof=1)
    ex = np.array([exact_integral(t0, i) for i in range(m)])
    se = np.array([exact_se(t0, i) for i in range(m)])
    ratio = (spread / se) ** 2
    assert abs(ratio.mean() - 1.0) < 4.0 * math.sqrt(2.0 / (runs - 1)) / math.sqrt(m), ("spread^2 / SE^2",
                                                                                       ratio.mean())
    z = (fbar - ex) / (se / math.sqrt(runs))
    assert abs(z.mean()) < 4.0 / math.sqrt(m), ("F-bar z mean", z.mean())
    assert abs((z * z).mean() - 1.0) < 4.0 * math.sqrt(2.0 / m), ("F-bar z^2 mean", (z * z).mean())


def check_special_cases(orc):
    # k = 0: f is the constant a; every sum is exact
    t = W.empty(3)
    W.set_harmonic(t, 0, 3, 1.5, -0.25, [0.0, 0.0, 0.0], [0, -1, 2], [1, 0.5, 2.25])
    W.set_poly(t, 1, 5, [0.0] * 5, [1, 2, 3, 4, 2], [-1] * 5, [0.5] * 5)
    W.set_abs_linear(t, 2, 2, -2.0, 10.0, [1.0, -1.0], [0, 0], [1, 1])  # L > 0 everywhere: f = -2 L
    t["n_samples"][:] = 1000
    t["seed"][:] = [1, 2, 3]
    res, _ = orc.integrate(t, threads=1)
    V0 = 1.0 * 1.5 * 0.25
    assert res["sum_f"][0] == 1000 * 1.5 and res["stderr"][0] == 0.0
    assert res["mean"][0] == V0 * 1.5
    assert res["mean"][1] == 1.5 ** 5 and res["stderr"][1] == 0.0
    # abs-linear with L > 0: the estimate is the sample mean of -2 (10 + x1 - x2)
    s1 = 0.0
    pts = [orc.sample_point(t, 2, s) for s in range(1000)]
    s1 = math.fsum(-2.0 * (10.0 + x[0] - x[1]) for x in pts)
    assert abs(res["sum_f"][2] - s1) <= 1e-12 * abs(s1)
    # linearity in (a, b) on the same samples
    base = W.harmonic_batch(4, n_samples=5000, gen_seed=61)
    ta, tb = base.copy(), base.copy()
    ta["params"][:, 1] = 0.0
    ta["params"][:, 0] = 1.0
    tb["params"][:, 0] = 0.0
    tb["params"][:, 1] = 1.0
    r, _ = orc.integrate(base, 1)
    ra, _ = orc.integrate(ta, 1)
    rb, _ = orc.integrate(tb, 1)
    a, b = base["params"][:, 0], base["params"][:, 1]
    lin = a * ra["sum_f"] + b * rb["sum_f"]
    assert np.all(np.abs(r["sum_f"] - lin) <= 1e-12 * r["sum_abs"]), "linearity in (a, b)"


def check_eq2_worked_values(orc):
    """Eq. (2) on unit boxes: int |x1+x2| = 1 and int |x1+x2-x3| = 7/12; estimates within 4 sigma."""
    t = W.eq2_series(n_samples=40_000)
    assert abs(exact_integral(t, 0) - 1.0) < 1e-15
    assert abs(exact_integral(t, 60) - 7.0 / 12.0) < 1e-15
    sub = np.ascontiguousarray(t[[0, 10, 48, 49, 60, 99]])
    res, _ = orc.integrate(sub, 2)
    for i in range(len(sub)):
        ex = exact_integral(sub, i)
        assert abs(res["mean"][i] - ex) < 4 * exact_se(sub, i), ("Eq. 2", i)


ALL_CHECKS = [
    ("philox_blocks", lambda o, r: check_philox_blocks(o, r)),
    ("stream_layout", lambda o, r: check_stream_layout(o, r)),
    ("uniform", lambda o, r: check_uniform(o)),
    ("sample_points", lambda o, r: check_sample_points(o, r)),
    ("point_values", lambda o, r: check_point_values(o, n_points=6)),
    ("brute_force", lambda o, r: check_brute_force_sums(o, r)),
    ("finalize", lambda o, r: check_finalize_textbook(o)),
    ("special_cases", lambda o, r: check_special_cases(o)),
    ("closed_forms", lambda o, r: check_closed_forms_4sigma(o)),
    ("eq2", lambda o, r: check_eq2_worked_values(o)),
    ("run_spread", lambda o, r: check_run_spread(o)),
    ("compensated_sums", lambda o, r: check_compensated_sums(o)),
]
