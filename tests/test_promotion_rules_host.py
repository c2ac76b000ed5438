"""The GPU tests' predictor of FP32 -> FP64 promotion, checked on the CPU.

The FP32 parity checks grade every row by the precision it reports and require
the promoted rows to be exactly those the library's documented rules call for
(`gpu_common.expected_promotion`).  Here the predictor itself is checked on
cases whose answer is known by construction.
"""

import numpy as np

import gpu_common as G
from oracle import oracle as O
from paper_2104_10073_amd import workloads as W


def test_range_and_constant_rows():
    t = W.empty(10)
    W.set_harmonic(t, 0, 3, 1e25, -2e25, [3.0, 4.0, 5.0], [0, -1, 0.5], [1, 0.5, 2])  # amplitude only
    W.set_harmonic(t, 1, 3, 1e-25, 2e-25, [3.0, 4.0, 5.0], [0, -1, 0.5], [1, 0.5, 2])
    W.set_gaussian(t, 2, 2, 1e-40, 0.5, [0.3, 0.6], [0, 0], [1, 1])
    W.set_abs_linear(t, 3, 4, 1e-50, 0.1, [1.0, -1.0, 1.0, 1.0], [0] * 4, [1] * 4)
    W.set_abs_linear(t, 4, 2, 2.0, 0.0, [3e20, -1e20], [0, 0], [1, 1])       # g^2 overflows
    W.set_poly(t, 5, 2, [0.5, 0.5], [8, 8], [-1e5, -1e5], [1e5, 1e5])        # g overflows
    W.set_abs_linear(t, 6, 2, 1.0, 0.0, [1e-25, 2e-25], [0, 0], [1, 1])      # g^2 underflows
    W.set_gaussian(t, 7, 2, 1.0, 0.3015, [3.0, 3.0], [0, 0], [1, 1])         # far tail
    W.set_harmonic(t, 8, 2, 0.0, 0.0, [1.0, 1.0], [0, 0], [1, 1])            # f == 0
    W.set_harmonic(t, 9, 4, 1.0, 0.5, [20.0] * 4, [0] * 4, [1] * 4)
    t["n_samples"][:] = 20_003
    t["seed"][:] = [W.stream_seed(41, i) for i in range(len(t))]
    orc, _ = O.default().integrate(t, 4)
    must, may = G.expected_promotion(t, orc)
    assert np.nonzero(must)[0].tolist() == [4, 5, 6, 7]
    assert np.array_equal(must, may)


def test_degenerate_edge_rows():
    t = G.edge_table()
    orc, _ = O.default().integrate(t, 8)
    must, may = G.expected_promotion(t, orc)
    assert np.nonzero(must)[0].tolist() == list(range(len(t) - 4, len(t)))
    assert np.array_equal(must, may)


def test_submit_time_rules():
    """Phase bound, absolute-coordinate offset and sample count: decided from the
    table alone (the sums are not consulted for these rows)."""
    t = W.empty(6)
    W.set_harmonic(t, 0, 2, 1.0, 1.0, [6500.0, 6500.0], [0, 0], [1, 1])      # theta ~ 4138 rev
    W.set_harmonic(t, 1, 2, 1.0, 1.0, [6400.0, 6400.0], [0, 0], [1, 1])      # theta ~ 4075 rev
    W.set_poly(t, 2, 1, [0.5], [2], [100.0], [100.01])                       # K ~ 1e4
    W.set_poly(t, 3, 1, [0.5], [2], [0.0], [1.0])                            # K = 1
    W.set_harmonic(t, 4, 1, 1.0, 0.0, [3.0], [0], [1])
    W.set_harmonic(t, 5, 1, 1.0, 0.0, [3.0], [0], [1])
    t["n_samples"][:] = [10_000, 10_000, 10_000, 10_000, 2_000_000_000, 100_000_000]
    fake = np.zeros(len(t), dtype=O.RESULT_DTYPE)
    fake["sum_f"] = 0.0
    fake["sum_f2"] = 0.5 * t["n_samples"]        # sigma / rms = 1: no post-run rule
    must, may = G.expected_promotion(t, fake)
    assert must.tolist() == [True, False, True, False, True, False]
    assert np.array_equal(must, may)
