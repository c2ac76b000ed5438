"""The benchmark-sized workloads, in the launch configuration bench.py times, against the
oracle on sampled functions (the oracle computes each sampled function in full)."""

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bench_ctx(Z, table):
    probe = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    probe.submit(table, Z.PREC_FP32)
    tiles = probe.validate_tiles()
    probe.close()
    return Z.Context(workspace="torch", policy=Z.MC_SCHED_FIFO, max_tiles_per_run=tiles,
                     max_functions=65536)


def test_harmonic_batch_full_size():
    """1000 functions x 10^6 samples (the benchmark workload), seed base 0."""
    import paper_2104_10073_amd as Z
    t = W.harmonic_batch(1000, n_samples=1_000_000, base=0)
    with _bench_ctx(Z, t) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
        r64 = c.integrate(t, Z.PREC_FP64)
        st = c.stats()
    assert st["bad_records"] == 0
    sub = np.array([0, 1, 137, 500, 998, 999])
    orc = G.oracle_results(t[sub])
    G.check_fp32(r32[sub], orc, "harmonic batch fp32")
    G.check_fp64(r64[sub], orc, "harmonic batch fp64")
    # all 1000: FP32 against the FP64 GPU path at the same bar
    err = np.abs(r32["mean"] - r64["mean"]) / r64["std_error"]
    assert err.max() < 1e-2, err.max()


def test_mixed_batch_full_size():
    """2000 mixed functions, dims 1..7, 10^4..10^7 samples: sampled against the oracle."""
    import paper_2104_10073_amd as Z
    t = W.mixed_batch(2000, dim_range=(1, 7), gen_seed=3)
    with _bench_ctx(Z, t) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
        r64 = c.integrate(t, Z.PREC_FP64)
    order = np.argsort(t["n_samples"])
    sub = np.concatenate([order[:12], order[-2:], np.arange(0, 2000, 250)])
    sub = np.unique(sub)
    orc = G.oracle_results(t[sub])
    G.check_fp32(r32[sub], orc, "mixed fp32", table=t[sub])
    G.check_fp64(r64[sub], orc, "mixed fp64")
    err = np.abs(r32["mean"] - r64["mean"]) / np.maximum(r64["std_error"], 1e-300)
    assert err.max() < 1e-2, (err.max(), int(np.argmax(err)))


def test_high_dim_full_size_sampled():
    """500 functions, dims 8..12, 10^7 samples each, every 10th with |F| < 1e-4."""
    import paper_2104_10073_amd as Z
    t = W.high_dim_batch(500, n_samples=10_000_000)
    with _bench_ctx(Z, t) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
        r64 = c.integrate(t, Z.PREC_FP64)
    sub = np.array([0, 1, 9, 19])   # harmonic, Gaussian, two near-zero
    orc = G.oracle_results(t[sub])
    G.check_fp32(r32[sub], orc, "high-dim fp32", table=t[sub])
    G.check_fp64(r64[sub], orc, "high-dim fp64")
    err = np.abs(r32["mean"] - r64["mean"]) / np.maximum(r64["std_error"], 1e-300)
    assert err.max() < 1e-2, (err.max(), int(np.argmax(err)))
