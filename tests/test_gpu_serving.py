"""The open-loop serving driver over the continuous-batching context: requests
arriving (Poisson) while others run are admitted and share launches under each
scheduling policy; every result equals the request integrated alone, and every
latency is the time from arrival to results on the host."""

import numpy as np
import pytest

from paper_2104_10073_amd import serving
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b, label):
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
        assert np.array_equal(a[k], b[k]), f"{label}: field {k} differs"


@pytest.mark.parametrize("policy", ["MC_SCHED_SRPT", "MC_SCHED_FAIR", "MC_SCHED_FIFO"])
def test_serve_open_loop(policy):
    import paper_2104_10073_amd as Z
    n = 60
    reqs = W.serving_requests(n, gen_seed=17, max_funcs=40, log10_samples=(3.0, 5.5))
    arrivals = W.poisson_arrivals(n, 3000.0, seed=3)   # arrivals overlap running work
    with Z.Context(flags=Z.MC_NO_GRAPH, policy=getattr(Z, policy), max_tiles_per_run=1 << 10) as c:
        out = serving.serve(c, reqs, arrivals, keep_results=True)
        alone = [c.integrate(r, Z.PREC_FP32) for r in reqs]
    lat = out["latency_s"]
    assert np.all(np.isfinite(lat)) and np.all(lat > 0.0)
    assert np.allclose(out["done_s"] - arrivals, lat)
    assert out["evals"] == sum(int(r["n_samples"].sum()) for r in reqs)
    for i in range(n):
        _same(out["results"][i], alone[i], f"request {i}")
    s = serving.summarize(out, arrivals)
    assert s["measured"] == n - n // 10 and s["p50_ms"] <= s["p99_ms"]
