"""Helpers shared by the GPU parity tests: run the HIP path, run the oracle, compare."""

from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2104_10073_amd import workloads as W

FP64_REL = 1e-12      # FP64 paths: |S_gpu - S_oracle| <= 1e-12 * sum|f|  (S2: <= 1e-12 * S2)
FP32_SE_FRAC = 1e-2   # FP32-eval path: |F_gpu - F_oracle| <= 0.01 * SE_oracle


def oracle_results(table, threads=16):
    res, _ = O.integrate(np.ascontiguousarray(table), threads)
    assert np.all(res["status"] == 0)
    return res


def check_fp64(gpu, orc, label=""):
    assert np.all(gpu["status"] == 0), label
    assert np.array_equal(gpu["n"], orc["n"]), label
    d1 = np.abs(gpu["sum_f"] - orc["sum_f"])
    d2 = np.abs(gpu["sum_f2"] - orc["sum_f2"])
    tol1 = FP64_REL * orc["sum_abs"] + 1e-300
    tol2 = FP64_REL * orc["sum_f2"] + 1e-300
    bad1 = np.nonzero(d1 > tol1)[0]
    bad2 = np.nonzero(d2 > tol2)[0]
    assert bad1.size == 0, f"{label} S1 mismatch at {bad1[:10]}: rel {(d1 / tol1 * FP64_REL)[bad1[:10]]}"
    assert bad2.size == 0, f"{label} S2 mismatch at {bad2[:10]}"
    # mean and SE follow from the sums by the same formulas
    dm = np.abs(gpu["mean"] - orc["mean"])
    tolm = FP64_REL * orc["sum_abs"] / orc["n"] * orc["volume"] * 4 + 1e-300
    assert np.all(dm <= tolm), label
    return float(np.max(d1 / (orc["sum_abs"] + 1e-300)))


def check_fp32(gpu, orc, label=""):
    assert np.all(gpu["status"] == 0), label
    assert np.array_equal(gpu["n"], orc["n"]), label
    err = np.abs(gpu["mean"] - orc["mean"])
    se = orc["stderr"]
    exact_zero = se == 0.0
    ratio = np.where(exact_zero, 0.0, err / np.where(exact_zero, 1.0, se))
    bad = np.nonzero(ratio > FP32_SE_FRAC)[0]
    assert bad.size == 0, f"{label}: |F32 - F64| / SE above 0.01 at {bad[:10]}: {ratio[bad[:10]]}"
    # constant integrands (SE = 0) must come out exact to FP32 evaluation of a constant
    if np.any(exact_zero):
        assert np.all(np.abs(err[exact_zero]) <= 1e-6 * np.abs(orc["mean"][exact_zero]) + 1e-300), label
    se_ratio = np.where(exact_zero, 1.0, gpu["std_error"] / np.where(exact_zero, 1.0, se))
    assert np.all(np.abs(se_ratio - 1.0) < 1e-3), f"{label}: SE ratio {se_ratio[np.abs(se_ratio - 1) >= 1e-3][:5]}"
    return float(np.max(ratio))


def edge_table():
    """Ragged and degenerate cases: tiny N, partial quads, segment and tile boundaries,
    every dimension, every family, high polynomial degrees, a centre outside the box."""
    rows = []
    rng = np.random.Generator(np.random.PCG64(77))
    sizes = [2, 3, 4, 5, 7, 63, 64, 65, 255, 257, 4095, 4096, 4097, 16383, 16384, 16385, 65537, 100_003]
    fam_cycle = [W.HARMONIC, W.ABS_LINEAR, W.GAUSSIAN, W.POLY_PRODUCT]
    t = W.empty(len(sizes) * 4 + 12 + 4)
    i = 0
    for n in sizes:
        for fam in fam_cycle:
            dim = 1 + (i % 12)
            lo = rng.uniform(-1, 1, dim)
            hi = lo + rng.uniform(0.5, 2, dim)
            if fam == W.HARMONIC:
                W.set_harmonic(t, i, dim, rng.uniform(-2, 2), rng.uniform(-2, 2), rng.uniform(-30, 30, dim), lo, hi)
            elif fam == W.ABS_LINEAR:
                W.set_abs_linear(t, i, dim, rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(-2, 2, dim), lo, hi)
            elif fam == W.GAUSSIAN:
                W.set_gaussian(t, i, dim, rng.uniform(0.5, 2), rng.uniform(0.1, 1), rng.uniform(lo, hi), lo, hi)
            else:
                W.set_poly(t, i, dim, rng.uniform(-1, 1, dim), rng.integers(0, 9, dim), lo, hi)
            t["n_samples"][i] = n
            t["seed"][i] = W.stream_seed(9, i) ^ (0xABCDEF << 40)
            i += 1
    # every dimension at a mid size
    for d in range(1, 13):
        lo = np.zeros(d)
        hi = np.ones(d)
        W.set_harmonic(t, i, d, 1.0, 0.5, rng.uniform(0.5, 5, d), lo, hi)
        t["n_samples"][i] = 50_000 + d
        t["seed"][i] = W.stream_seed(10, i)
        i += 1
    # degenerate: k = 0, p = 0, Gaussian centre outside the box, huge sigma
    W.set_harmonic(t, i, 3, 1.5, -0.25, [0, 0, 0], [0, -1, 2], [1, 0.5, 2.25]); i += 1
    W.set_poly(t, i, 5, [0.0] * 5, [1, 2, 3, 4, 2], [-1] * 5, [0.5] * 5); i += 1
    W.set_gaussian(t, i, 2, 1.0, 0.3, [3.0, -2.0], [0, 0], [1, 1]); i += 1
    W.set_gaussian(t, i, 4, 2.0, 1e3, [0.5] * 4, [0] * 4, [1] * 4); i += 1
    for k in range(i - 4, i):
        t["n_samples"][k] = 30_001
        t["seed"][k] = W.stream_seed(11, k)
    assert i == len(t)
    return t
