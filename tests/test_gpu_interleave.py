"""Checkpoint, resume and cancellation interleaved with running work, on an
MI355X, in both engines: a seeded script submits requests (tables and grids,
FP32 and FP64), runs, polls, snapshots requests while their work is on the GPU,
restores the snapshots into the same context and into a context of the other
engine while that one runs other requests, cancels some requests, now and then
aborts a context, and takes results as they complete.  Whatever the timing,
every request and every restored copy must come back with the results of an
uninterrupted run bit for bit, and every cancelled or aborted one with exactly
the results that were in."""

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")


def _pool(Z):
    jobs = []
    for k in range(10):
        t = W.mixed_batch(int(5 + 17 * k % 60), dim_range=(1, 12), log10_samples=(3.0, 6.3), gen_seed=700 + k)
        jobs.append(("table", t, Z.PREC_FP64 if k % 4 == 3 else Z.PREC_FP32, len(t)))
    base = W.harmonic_batch(1, 400_000, base=9)[0]
    jobs.append(("grid", (base, [(W.V0, 5, 4.0, 2.5), (0, 3, 0.5, 0.75)]), Z.PREC_FP32, 15))
    flat = W.harmonic_batch(1, 150_000, gen_seed=8)
    flat["params"][0, W.V0:W.V0 + 4] = 0.0  # constant integrands: the FP32 check sends them to FP64
    jobs.append(("grid", (flat[0], [(0, 3, 0.5, 0.25)]), Z.PREC_FP32, 3))
    return jobs


def _submit(c, job):
    kind, t, prec, _ = job
    if kind == "grid":
        return c.submit_grid(t[0], t[1], prec)
    return c.submit(t, prec)


def _same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


def _kept(a, b, label):
    """A cancelled request: the results that came in equal the reference, the rest are aborted."""
    kept = a["status"] == 0
    assert np.all(a["status"][~kept] == -10), label  # MC_ERR_ABORTED
    for f in FIELDS:
        assert np.array_equal(a[f][kept], b[f][kept]), (label, f)


# (seed 105 with a resident first context cancelled a restored request before
# its runs opened, which left its saved tile counts in the slots the next
# request took, until cancelling cleared them)
@pytest.mark.parametrize("first,seed,aborts", [("launch", 31, False), ("resident", 32, False), ("launch", 105, False),
                                               ("resident", 105, False), ("launch", 113, False),
                                               ("resident", 118, False), ("launch", 201, True),
                                               ("resident", 202, True), ("launch", 203, True), ("resident", 204, True)])
def test_snapshots_interleaved_with_running_work(first, seed, aborts):
    import paper_2104_10073_amd as Z
    jobs = _pool(Z)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref = [c.results(_submit(c, j), j[3]) for j in jobs]
    flags = {"launch": 0, "resident": Z.MC_RESIDENT}
    other = "resident" if first == "launch" else "launch"
    rng = np.random.Generator(np.random.PCG64(seed))
    with Z.Context(device=0, flags=flags[first], max_tiles_per_run=48) as a, \
            Z.Context(device=0, flags=flags[other], max_tiles_per_run=96) as b:
        live = {}      # (context, request id) -> job index
        cancelled = set()
        checked = 0
        order = list(rng.permutation(len(jobs)))
        for step in range(160):
            op = rng.integers(0, 7)
            if op == 0 and order:
                k = int(order.pop())
                live[(a, _submit(a, jobs[k]))] = k
            elif op == 1 and set(live) - cancelled:
                # snapshot a request while its work runs; resume the copy in one of the contexts
                keys = [key for key in live if key not in cancelled]
                ctx, rid = keys[int(rng.integers(0, len(keys)))]
                blob = ctx.snapshot(rid)
                dst = a if rng.random() < 0.5 else b
                live[(dst, dst.restore(blob))] = live[(ctx, rid)]
            elif op == 2:
                a.run()
                b.run()
            elif op == 3:
                for ctx in (a, b):
                    for rid in ctx.poll():
                        k = live.pop((ctx, rid))
                        got = ctx.results(rid, jobs[k][3], allow_aborted=True)
                        (_kept if (ctx, rid) in cancelled else _same)(got, ref[k], f"step {step}: job {k}")
                        checked += 1
            elif op == 4 and aborts and rng.random() < 0.125:
                # abort one context: every request in it so far keeps what came in
                ctx = a if rng.random() < 0.5 else b
                ctx.abort()
                cancelled.update(key for key in live if key[0] is ctx)
            elif op == 5 and len(set(live) - cancelled) > 2 and rng.random() < 0.5:
                keys = [key for key in live if key not in cancelled]
                ctx, rid = keys[int(rng.integers(0, len(keys)))]
                ctx.cancel(rid)
                cancelled.add((ctx, rid))
            else:
                a.run()
        for (ctx, rid), k in list(live.items()):
            got = ctx.results(rid, jobs[k][3], allow_aborted=True)
            (_kept if (ctx, rid) in cancelled else _same)(got, ref[k], f"end: job {k}")
            checked += 1
        for k in order:
            _same(a.results(_submit(a, jobs[k]), jobs[k][3]), ref[k], f"late: job {k}")
            checked += 1
    print(f"{checked} requests checked, {len(cancelled)} of them cancelled", flush=True)
    assert checked >= len(jobs)
