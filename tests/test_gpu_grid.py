"""Parameter-grid requests (functional mode) on an MI355X: the device builds the
records from the grid spec; the results equal those of the expanded table
(FP64: bitwise) and match the oracle on that table."""

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
            if prec == Z.PREC_FP64:
                # the FP64 record fields are exact functions of the inputs: same bits
                for k in ("mean", "std_error", "sum_f", "sum_f2"):
                    assert np.array_equal(g[k], t[k]), k
                G.check_fp64(g, orc, "grid fp64")
            else:
                # FP32 coefficients come from the device's libm instead of the
                # host's (hypot, atan2 may differ in the last bit before rounding
                # to float): far inside the FP32 bar
                assert np.all(np.abs(g["mean"] - t["mean"]) <= 1e-3 * orc["stderr"])
                G.check_fp32(g, orc, "grid fp32")
