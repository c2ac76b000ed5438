"""Parameter-grid requests (functional mode) on an MI355X: the device builds the
records from the grid spec; the results equal those of the expanded table bit
for bit (the device packs every coefficient with the host's operations, in both
precisions) and match the oracle on that table."""

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_grid_equals_table_and_oracle():
    import paper_2104_10073_amd as Z
    base, axes = W.functional_grid(n_k=12, n_ab=4, n_samples=20_001)
    table = W.expand_grid(base, axes)
    orc = G.oracle_results(table)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        print("grid: functions", len(table), flush=True)
        for prec in (Z.PREC_FP64, Z.PREC_FP32):
            g = c.integrate_grid(base, axes, prec)
            t = c.integrate(table, prec)
            assert np.array_equal(g["n"], t["n"])
            # the records the device packs from the spec are the host's bits
            for k in ("mean", "std_error", "sum_f", "sum_f2", "status", "precision"):
                assert np.array_equal(g[k], t[k]), (prec, k)
            if prec == Z.PREC_FP64:
                G.check_fp64(g, orc, "grid fp64")
            else:
                G.check_fp32(g, orc, "grid fp32", table=table)


def _base(family):
    b = W.empty(1)
    if family == "abs_linear":
        W.set_abs_linear(b, 0, 3, 1.0, 0.2, [1.0, -1.0, 0.5], [-0.5, 0.0, 0.2], [0.5, 1.5, 1.0])
        axes = [(0, 3, 0.5, 0.75), (W.V0 + 1, 4, -2.0, 1.3)]
    elif family == "gaussian":
        W.set_gaussian(b, 0, 2, 1.5, 0.4, [0.3, 0.6], [0.0, 0.0], [1.0, 1.2])
        axes = [(1, 3, 0.2, 0.3), (W.V0, 5, 0.1, 0.2)]
    elif family == "poly":
        W.set_poly(b, 0, 3, [0.5, -0.4, 0.9], [2, 1, 3], [-1.0, 0.0, 0.5], [1.0, 2.0, 1.5])
        axes = [(W.V0, 4, -1.0, 0.6), (W.W0 + 2, 3, 1.0, 2.0)]            # degrees 1, 3, 5
    else:
        W.set_harmonic(b, 0, 4, 1.0, 0.5, [3.0, 5.0, 7.0, 2.0], [0.0] * 4, [1.0] * 4)
        axes = [(0, 2, 0.5, 1.0), (1, 2, -1.0, 2.0), (W.V0 + 3, 3, 2.0, 5.0)]
    b["n_samples"][0] = 20_001
    b["seed"][0] = W.stream_seed(12, 0)
    return b, axes


@pytest.mark.parametrize("family", ["abs_linear", "gaussian", "poly", "harmonic_three_axes"])
def test_grids_of_every_family(family):
    """Grids with axes on scalar, per-dimension and degree parameters: results equal
    the expanded table's bit for bit in both precisions and match the oracle (FP32
    at the FP32 bar); through a resident context too."""
    import paper_2104_10073_amd as Z
    base, axes = _base(family)
    table = W.expand_grid(base, axes)
    orc = G.oracle_results(table)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        g64 = c.integrate_grid(base, axes, Z.PREC_FP64)
        t64 = c.integrate(table, Z.PREC_FP64)
        g32 = c.integrate_grid(base, axes, Z.PREC_FP32)
        t32 = c.integrate(table, Z.PREC_FP32)
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as c:
        q32 = c.integrate_grid(base, axes, Z.PREC_FP32)
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "precision"):
        assert np.array_equal(g64[k], t64[k]), k
        assert np.array_equal(g32[k], t32[k]), k
        assert np.array_equal(q32[k], g32[k]), k
    G.check_fp64(g64, orc, f"{family} grid fp64")
    f32 = g32["precision"] == 0
    assert f32.any()
    G.check_fp32(g32[f32], orc[f32], f"{family} grid fp32")
    if (~f32).any():
        G.check_fp64(g32[~f32], orc[~f32], f"{family} grid promoted")
