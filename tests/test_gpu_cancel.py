"""Cancelling single requests on an MI355X (mc_cancel), in both engines: a
request cancelled while its work runs comes back aborted except for results
already in, which equal an uninterrupted run's bit for bit; the request beside
it and a request that takes the cancelled one's device slots afterwards come
back exactly as they would alone."""

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")


def _same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


@pytest.mark.parametrize("engine", ["launch", "resident"])
def test_cancel_running_request(engine):
    import paper_2104_10073_amd as Z
    big = W.mixed_batch(60, dim_range=(1, 12), log10_samples=(5.0, 6.5), gen_seed=801)
    small = W.mixed_batch(20, dim_range=(1, 8), log10_samples=(3.0, 5.5), gen_seed=802)
    after = W.mixed_batch(60, dim_range=(1, 12), log10_samples=(3.0, 5.5), gen_seed=803)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref_big, ref_small, ref_after = (c.integrate(t, Z.PREC_FP32) for t in (big, small, after))
    flags = Z.MC_RESIDENT if engine == "resident" else 0
    with Z.Context(device=0, flags=flags, policy=Z.MC_SCHED_FIFO, max_tiles_per_run=64, max_functions=100) as c:
        rb = c.submit(big, Z.PREC_FP32)
        rs = c.submit(small, Z.PREC_FP32)
        for _ in range(4):
            c.run()
        print(f"{engine}: cancel", flush=True)
        c.cancel(rb)
        got = c.results(rb, len(big), allow_aborted=True)
        kept = got["status"] == 0
        assert np.all(got["status"][~kept] == -10)  # MC_ERR_ABORTED
        assert np.all(got["n"] == big["n_samples"])
        for f in FIELDS:
            assert np.array_equal(got[f][kept], ref_big[f][kept]), f
        assert not np.all(kept), "the request finished before it was cancelled"
        print(f"{engine}: {int(kept.sum())} of {len(big)} results were in", flush=True)
        _same(c.results(rs, len(small)), ref_small, "beside the cancelled request")
        # the cancelled request's slots are free again (100 slots: 60 + 60 fit only without it)
        _same(c.integrate(after, Z.PREC_FP32), ref_after, "in the cancelled request's slots")


@pytest.mark.parametrize("engine", ["launch", "resident"])
def test_cancels_while_serving(engine):
    """Requests arrive at 2000/s and a seeded script picks about one in six of
    them to cancel a few loop turns after it arrives (queued, running or done by
    then): every request that was not cancelled comes back as it does alone,
    bit for bit, and every cancelled one keeps exactly the results that were in."""
    import time
    import paper_2104_10073_amd as Z
    reqs = W.serving_requests(150, gen_seed=811, max_funcs=200, log10_samples=(3.0, 6.0))
    arrivals = W.poisson_arrivals(len(reqs), 2000.0, seed=811)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref = [c.integrate(t, Z.PREC_FP32) for t in reqs]
    rng = np.random.Generator(np.random.PCG64(812))
    flags = Z.MC_RESIDENT if engine == "resident" else 0
    with Z.Context(device=0, flags=flags, policy=Z.MC_SCHED_SRPT) as c:
        rid_of, idx_of, plan, cancelled, out = {}, {}, {}, set(), {}
        nxt = 0
        t0 = time.perf_counter()
        while len(out) < len(reqs):
            assert time.perf_counter() - t0 < 60.0, f"{len(out)} of {len(reqs)} requests in after 60 s"
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arrivals[nxt] <= now:
                rid = c.submit(reqs[nxt], Z.PREC_FP32)
                rid_of[nxt], idx_of[rid] = rid, nxt
                if rng.random() < 1.0 / 6.0:
                    plan[nxt] = int(rng.integers(0, 40))  # loop turns before the cancel
                nxt += 1
            c.run()
            for k in list(plan):
                if plan[k] > 0:
                    plan[k] -= 1
                    continue
                del plan[k]
                if k not in out:
                    c.cancel(rid_of[k])
                    cancelled.add(k)
            for rid in c.poll():
                k = idx_of[rid]
                out[k] = c.results(rid, len(reqs[k]), allow_aborted=True)
    print(f"{engine}: {len(cancelled)} of {len(reqs)} requests cancelled", flush=True)
    assert len(cancelled) >= 5
    for k in range(len(reqs)):
        if k not in cancelled:
            _same(out[k], ref[k], f"request {k}")
            continue
        kept = out[k]["status"] == 0
        assert np.all(out[k]["status"][~kept] == -10), k  # MC_ERR_ABORTED
        for f in FIELDS:
            assert np.array_equal(out[k][f][kept], ref[k][f][kept]), (k, f)
