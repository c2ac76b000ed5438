"""The open-loop serving driver's own logic on the CPU, against a stand-in context
that completes each request a fixed time after it was submitted: requests are
submitted at their arrival times (never before), each latency is completion
minus arrival, results are kept per request, and both the busy-polling and the
sleeping loop finish."""

import time

import numpy as np
import pytest

from paper_2104_10073_amd import serving
from paper_2104_10073_amd import workloads as W
from paper_2104_10073_amd._native import RESULT_DTYPE


class StandInContext:
    def __init__(self, service_s):
        self.service = service_s
        self.t0 = time.perf_counter()
        self.submitted = {}
        self.taken = set()
        self.reported = set()
        self.runs = 0

    def submit(self, table, precision):
        rid = len(self.submitted) + 1
        self.submitted[rid] = (time.perf_counter(), len(table))
        return rid

    def run(self, stream=None):
        self.runs += 1
        return True

    def poll(self):
        now = time.perf_counter()
        done = [rid for rid, (ts, _) in self.submitted.items()
                if rid not in self.reported and now - ts >= self.service]
        self.reported.update(done)
        return done

    def results(self, rid, n, blocking=True):
        assert rid in self.reported and rid not in self.taken and n == self.submitted[rid][1]
        self.taken.add(rid)
        out = np.zeros(n, dtype=RESULT_DTYPE)
        out["mean"] = rid
        return out


@pytest.mark.parametrize("idle_sleep", [0.0, 200e-6])
def test_serve_driver_bookkeeping(idle_sleep):
    reqs = W.serving_requests(40, gen_seed=3, max_funcs=20, log10_samples=(3.0, 4.0))
    arrivals = np.sort(W.poisson_arrivals(40, 400.0, seed=9))
    ctx = StandInContext(service_s=2e-3)
    out = serving.serve(ctx, reqs, arrivals, keep_results=True, idle_sleep=idle_sleep)
    lat = out["latency_s"]
    assert np.all(np.isfinite(lat)) and np.all(lat >= 2e-3 - 1e-9)
    assert np.all(lat < 2e-3 + 0.25)                  # noticed promptly (generous for a loaded host)
    assert np.allclose(out["done_s"] - arrivals, lat)
    assert len(ctx.taken) == len(reqs) and ctx.runs >= len(reqs)
    # request i was submitted no earlier than its arrival, and results map back to it
    for i, (ts, n) in enumerate(sorted(ctx.submitted.values())):
        assert ts - ctx.t0 >= arrivals[i] - 0.01 and n == len(reqs[i])
    assert [int(r["mean"][0]) for r in out["results"]] == list(range(1, len(reqs) + 1))
    assert out["evals"] == sum(int(r["n_samples"].sum()) for r in reqs)
    s = serving.summarize(out, arrivals)
    assert s["measured"] == 36 and s["p50_ms"] <= s["p99_ms"]
