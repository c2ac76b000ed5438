"""Separate contexts are independent: two contexts driven from two host threads at
once (each on its own stream), and two contexts interleaved on one thread, give
every request bitwise the result it has alone."""

import threading

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _same(a, b, label):
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
        assert np.array_equal(a[k], b[k]), f"{label}: field {k} differs"


def _tables():
    return [W.mixed_batch(60, dim_range=(1, 12), log10_samples=(3.0, 5.5), gen_seed=101 + k, base=k)
            for k in range(6)]


def test_two_contexts_on_two_threads():
    import torch
    import paper_2104_10073_amd as Z
    tables = _tables()
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        alone = [c.integrate(t, Z.PREC_FP32) for t in tables]
    out = [None] * len(tables)
    errors = []

    def worker(part):
        try:
            stream = torch.cuda.Stream()
            with Z.Context(flags=Z.MC_NO_GRAPH, max_tiles_per_run=256) as c:
                ids = [(i, c.submit(tables[i], Z.PREC_FP32)) for i in part]
                c.run(stream)
                for i, rid in ids:
                    out[i] = c.results(rid, len(tables[i]))
            stream.synchronize()
        except Exception as e:   # reported on the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(part,)) for part in ([0, 2, 4], [1, 3, 5])]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads), "a worker did not finish"
    assert not errors, errors
    for i in range(len(tables)):
        _same(alone[i], out[i], f"table {i}")


def test_two_contexts_interleaved_on_one_thread():
    import paper_2104_10073_amd as Z
    tables = _tables()
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        alone = [c.integrate(t, Z.PREC_FP32) for t in tables]
    with Z.Context(flags=Z.MC_NO_GRAPH, max_tiles_per_run=128) as a, \
            Z.Context(flags=Z.MC_NO_GRAPH, max_tiles_per_run=512, policy=Z.MC_SCHED_SRPT) as b:
        ids = []
        for i, t in enumerate(tables):
            ctx = a if i % 2 == 0 else b
            ids.append((ctx, ctx.submit(t, Z.PREC_FP32)))
            a.run()
            b.run()
        got = [None] * len(tables)
        for i in reversed(range(len(tables))):
            ctx, rid = ids[i]
            got[i] = ctx.results(rid, len(tables[i]))
    for i in range(len(tables)):
        _same(alone[i], got[i], f"table {i}")
