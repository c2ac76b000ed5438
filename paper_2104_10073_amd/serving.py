"""Open-loop serving driver for the continuous-batching context.

Requests (function tables) arrive at given times; each is submitted when its
arrival time has passed, the context admits it into device slots as soon as
function slots and tile-partial memory allow, and every `mc_run` shares one
launch among all admitted requests (by the context's scheduling policy).  A request's latency is the
time from its arrival to the moment its results are on the host.  The loop only
marshals calls into the library; all integration work runs in its kernels.
"""

from __future__ import annotations

import time

import numpy as np

from ._native import PREC_FP32, Context


def serve(ctx: Context, requests, arrivals, stream=None, precision: int = PREC_FP32,
          keep_results: bool = False, idle_sleep: float = 0.0):
    """Run `requests` (list of tables) arriving at `arrivals` (seconds from start).

    The loop busy-polls for arrivals and completions by default (one host core,
    as a latency-sensitive server thread would); a positive `idle_sleep` sleeps
    that long when nothing happened instead (the OS rounds short sleeps up to
    about 60 us, which adds that much to the time a completion is noticed).

    Returns a dict with per-request latency (s), completion times, total
    evaluations, wall time and, if asked, the results of every request.
    """
    n = len(requests)
    arrivals = np.asarray(arrivals, dtype=np.float64)
    assert len(arrivals) == n and np.all(np.diff(arrivals) >= 0)
    lat = np.full(n, np.nan)
    done_t = np.full(n, np.nan)
    sizes = [len(r) for r in requests]
    results = [None] * n if keep_results else None
    id_to_idx = {}
    next_i = 0
    completed = 0
    t0 = time.perf_counter()
    while completed < n:
        now = time.perf_counter() - t0
        progressed = False
        while next_i < n and arrivals[next_i] <= now:
            rid = ctx.submit(requests[next_i], precision)
            id_to_idx[rid] = next_i
            next_i += 1
            progressed = True
            # launch as soon as there is work, so the GPU starts while later
            # arrivals are still being submitted
            ctx.run(stream)
        ctx.run(stream)
        for rid in ctx.poll():
            i = id_to_idx.pop(rid, None)
            if i is None:
                continue
            res = ctx.results(rid, sizes[i], blocking=True)
            t = time.perf_counter() - t0
            done_t[i] = t
            lat[i] = t - arrivals[i]
            if keep_results:
                results[i] = res
            completed += 1
            progressed = True
        if not progressed:
            # nothing arrived or finished: wait a little, but never past the next arrival
            wait = idle_sleep
            if next_i < n:
                wait = min(wait, max(0.0, arrivals[next_i] - (time.perf_counter() - t0)))
            if wait > 0:
                time.sleep(wait)
    wall = time.perf_counter() - t0
    evals = int(sum(int(r["n_samples"].sum()) for r in requests))
    return {"latency_s": lat, "done_s": done_t, "wall_s": wall, "evals": evals, "results": results}


def summarize(out: dict, arrivals, warmup_frac: float = 0.1) -> dict:
    """p50/p99 latency over the requests after the warm-up fraction, and sustained rates."""
    n = len(out["latency_s"])
    k0 = int(n * warmup_frac)
    lat = out["latency_s"][k0:]
    span = float(np.nanmax(out["done_s"]) - np.asarray(arrivals)[k0]) if n > k0 else out["wall_s"]
    return {
        "requests": n, "measured": n - k0,
        "p50_ms": float(np.nanpercentile(lat, 50) * 1e3),
        "p99_ms": float(np.nanpercentile(lat, 99) * 1e3),
        "mean_ms": float(np.nanmean(lat) * 1e3),
        "achieved_qps": (n - k0) / span if span > 0 else float("nan"),
        "sustained_evals_per_s": out["evals"] / out["wall_s"],
    }
