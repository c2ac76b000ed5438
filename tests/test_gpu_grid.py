"""Parameter-grid requests (functional mode) on an MI355X: a grid gives the
same bits as the table it stands for, and matches the oracle on that table."""

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
            for k in ("mean", "std_error", "sum_f", "sum_f2", "n"):
                assert np.array_equal(g[k], t[k]), k
            if prec == Z.PREC_FP64:
                G.check_fp64(g, orc, "grid fp64")
            else:
                G.check_fp32(g, orc, "grid fp32")
