"""FP32-evaluation requests over wide parameter ranges (every family, dims 1..12,
boxes from 1e-3 to 1e2 wide and up to 1e2 from the origin, Eq. (1) phases up
to the FP32 limit and beyond, narrow and wide Gaussians, centres outside the
box, polynomial degrees 0..8, 2 to 3e5 samples): every result meets the bar of
the precision it reports -- FP32: within 0.01 SE of the FP64 path, FP64 (re-run
or chosen at submit): the FP64 path's sums to 1e-12 -- and the FP64 path
matches the oracle on every one of them."""

import math

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _wide_table(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = W.empty(n)
    for i in range(n):
        d = int(rng.integers(1, 13))
        far = rng.random() < 0.3
        lo = rng.uniform(-100, 100, d) if far else rng.uniform(-1, 1, d)
        w = 10 ** rng.uniform(-3, 2, d)
        hi = lo + w
        fam = int(rng.integers(0, 4))
        if fam == W.HARMONIC:
            # phase bound 10^U(0, 5) revolutions, split over the dimensions
            theta = 10 ** rng.uniform(0, 5)
            k = rng.choice([-1.0, 1.0], d) * (theta / (2 * d)) * 2 * math.pi / w * rng.uniform(0.5, 1.0, d)
            W.set_harmonic(t, i, d, rng.uniform(-5, 5), rng.uniform(-5, 5), k, lo, hi)
        elif fam == W.ABS_LINEAR:
            W.set_abs_linear(t, i, d, rng.uniform(-3, 3), rng.uniform(-10, 10), rng.uniform(-5, 5, d), lo, hi)
        elif fam == W.GAUSSIAN:
            mu = rng.uniform(lo - w, hi + w)
            sigma = float(np.mean(w)) * 10 ** rng.uniform(-1.5, 1.5)
            W.set_gaussian(t, i, d, rng.uniform(0.1, 10), sigma, mu, lo, hi)
        else:
            W.set_poly(t, i, d, rng.uniform(-2, 2, d), rng.integers(0, 9, d), lo, hi)
        t["n_samples"][i] = int(10 ** rng.uniform(math.log10(2), 5.5))
        t["seed"][i] = W.stream_seed(91, i)
    return t


def test_fp32_requests_over_wide_parameter_ranges():
    import paper_2104_10073_amd as Z
    t = _wide_table(400, seed=2024)
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
        r64 = c.integrate(t, Z.PREC_FP64)
    assert np.all(r32["status"] == 0) and np.all(r64["status"] == 0)
    f32 = r32["precision"] == 0
    # FP32 results: within 0.01 SE of the FP64 path (exact zero spread: equal means)
    se = r64["std_error"]
    err = np.abs(r32["mean"] - r64["mean"])
    ok = np.where(se > 0, err <= 0.01 * se, err <= 1e-6 * np.abs(r64["mean"]) + 1e-300)
    bad = np.nonzero(f32 & ~ok)[0]
    assert bad.size == 0, [(int(i), float(err[i] / max(se[i], 1e-300)), int(t["family"][i])) for i in bad[:8]]
    # results that came back in FP64 equal the FP64 path bit for bit (same records, same tree)
    f64 = ~f32
    for k in ("sum_f", "sum_f2", "mean", "std_error"):
        assert np.array_equal(r32[k][f64], r64[k][f64]), k
    # and the FP64 path agrees with the oracle on every function
    G.check_fp64(r64, G.oracle_results(t), "wide ranges, FP64 path")
