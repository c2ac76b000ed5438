"""The paper's error statistic on the GPU: Eq. (1) over independent runs (Fig. 1).

Ten runs of the 100-function series, each drawing its own streams, in one
launch; the mean over runs must sit around the exact integral and the
spread over runs must estimate the exact standard error, on both batched
paths.  Each run equals the same table integrated alone.
"""

import math

import numpy as np
import pytest

from paper_2104_10073_amd import runs as R
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name", ["PREC_FP32", "PREC_FP64"])
def test_spread_over_runs_against_closed_forms(prec_name):
    import closed_forms as CF
    import paper_2104_10073_amd as Z
    prec = getattr(Z, prec_name)
    runs = 10
    t0 = W.eq1_series(n_samples=100_000)
    m = len(t0)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as ctx:
        res, s = R.integrate_runs(ctx, t0, runs=runs, precision=prec, base=3)
        alone = ctx.integrate(R.reseeded(t0, 3 + runs - 1), prec)
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n"):
        assert np.array_equal(res[-1][k], alone[k]), k
    ex = np.array([CF.exact_integral(t0, i) for i in range(m)])
    se = np.array([CF.exact_se(t0, i) for i in range(m)])
    ratio = (s["spread"] / se) ** 2
    assert abs(ratio.mean() - 1.0) < 4.0 * math.sqrt(2.0 / (runs - 1)) / math.sqrt(m), ratio.mean()
    z = (s["mean"] - ex) / (se / math.sqrt(runs))
    assert abs(z.mean()) < 4.0 / math.sqrt(m), z.mean()
    assert abs((z * z).mean() - 1.0) < 4.0 * math.sqrt(2.0 / m), (z * z).mean()
    assert np.all(np.abs(s["rms_se"] / se - 1.0) < 0.01)
