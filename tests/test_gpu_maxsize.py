"""Very large functions on an MI355X, checked by properties that hold at any
size (the oracle cannot run 6.9e10 samples): FP64 and raw FP32 estimates
within 5 standard errors of the exact integrals, standard errors within 1 % of
the exact ones, and an FP32 request promoted to FP64 at this size.  At 2^36 samples and d = 12 the Philox
block index runs far past 2^32, so the counter's high word is exercised by the
batched kernels themselves (its sample-by-sample exactness is in
test_gpu_samples.py)."""

import numpy as np
import pytest

import closed_forms as CF
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _table():
    rows = W.high_dim_batch(6, gen_seed=4)[:2].copy()  # one harmonic, one Gaussian, d 8..12
    rows["dim"] = 12
    for i in range(len(rows)):
        rows["lo"][i, :12] = 0.0
        rows["hi"][i, :12] = 1.0
    rows["params"][0, W.V0:W.V0 + 12] = np.linspace(0.5, 3.0, 12)
    rows["params"][1, 1] = 0.6          # Gaussian sigma
    rows["params"][1, W.V0:W.V0 + 12] = 0.5
    rows["n_samples"] = 1 << 36
    return rows


def test_max_size_functions_match_exact_integrals():
    import paper_2104_10073_amd as Z
    t = _table()
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        print("max size: 2 functions x 2^36 samples, d = 12", flush=True)
        r64 = c.integrate(t, Z.PREC_FP64)
        # at 6.9e10 samples FP32 evaluation cannot reach 0.01 SE: the FP32 request
        # runs in FP64 (decided at submit; MC_NO_PROMOTE keeps FP32)
        r32p = c.integrate(t, Z.PREC_FP32)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH | Z.MC_NO_PROMOTE) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
    assert np.all(r32p["precision"] == Z.PREC_FP64) and np.all(r32["precision"] == Z.PREC_FP32)
    for k in ("mean", "std_error", "sum_f", "sum_f2"):
        assert np.array_equal(r32p[k], r64[k]), k
    # the resident engine: the same tiles and trees, so the same bits (a function
    # of 2^16 tiles, chunks of up to 8)
    print("max size through a resident context", flush=True)
    with Z.Context(device=0, flags=Z.MC_RESIDENT | Z.MC_NO_PROMOTE) as c:
        q64 = c.integrate(t, Z.PREC_FP64)
        q32 = c.integrate(t, Z.PREC_FP32)
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
        assert np.array_equal(q64[k], r64[k]), k
        assert np.array_equal(q32[k], r32[k]), k
    for i in range(len(t)):
        F = float(CF.exact_integral(t, i))
        se = float(CF.exact_se(t, i))
        for r in (r64, r32):
            assert r["n"][i] == 1 << 36
            assert abs(r["mean"][i] - F) <= 5 * se, (i, r["mean"][i], F, se)
            assert abs(r["std_error"][i] / se - 1) < 0.01, (i, r["std_error"][i], se)
