"""Captured HIP-graph launches give the same bits as direct launches, replay after replay."""

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_graph_replays_match_direct_launches():
    import torch
    import paper_2104_10073_amd as Z
    t = W.mixed_batch(80, dim_range=(1, 12), log10_samples=(3.0, 5.5), gen_seed=313)
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        ref32 = c.integrate(t, Z.PREC_FP32)
        ref64 = c.integrate(t, Z.PREC_FP64)
    with Z.Context() as c:
        for rep in range(5):
            got32 = c.integrate(t, Z.PREC_FP32)
            # eager work and a synchronisation between replays
            x = torch.arange(1000, device="cuda", dtype=torch.float32).sum()
            torch.cuda.synchronize()
            got64 = c.integrate(t, Z.PREC_FP64)
            for k in ("mean", "std_error", "sum_f", "sum_f2"):
                assert np.array_equal(got32[k], ref32[k]), (rep, k)
                assert np.array_equal(got64[k], ref64[k]), (rep, k)
            assert float(x) == 499500.0
