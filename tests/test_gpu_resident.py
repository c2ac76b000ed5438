"""The resident engine (MC_RESIDENT) on an MI355X.

One persistent kernel serves every request: the host appends chunks of tiles to
a ring in pinned memory, workgroups take tickets, the workgroup that counts a
function's last tile finalizes it and stores the result and a done word in
host memory.  The tiles, partials and reduction trees are those of the launch
path, so every result must equal the launch path's bit for bit; FP32 rows the
precision check sends to FP64 run a second time with a new record.  Every wait
in the kernel is bounded: it leaves by itself after about 0.1 s without work
(the next request relaunches it), and a stop word from the host ends it at
destroy, abort and when its record arena has to be recycled.
"""

import time

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")


def _same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


def _launch_results(Z, jobs):
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        return [c.integrate(t, p) for t, p in jobs]


def _drive(ctx, ids, sizes, limit_s=60.0):
    """mc_run / mc_poll until every request is in; results by id."""
    out = {}
    t0 = time.perf_counter()
    while len(out) < len(ids):
        assert time.perf_counter() - t0 < limit_s, f"{len(out)} of {len(ids)} requests in after {limit_s} s"
        ctx.run()
        for rid in ctx.poll():
            out[rid] = ctx.results(rid, sizes[rid], blocking=False)
            assert out[rid] is not None
    return out


def test_resident_against_oracle_and_launch_path():
    import paper_2104_10073_amd as Z
    jobs = [(W.mixed_batch(120, dim_range=(1, 12), log10_samples=(2.0, 5.5), gen_seed=501), Z.PREC_FP32),
            (G.edge_table(), Z.PREC_FP32),
            (W.mixed_batch(40, dim_range=(1, 8), log10_samples=(2.0, 5.0), gen_seed=502), Z.PREC_FP64)]
    ref = _launch_results(Z, jobs)
    print("resident: three requests submitted together, direct path", flush=True)
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as c:
        ids = [c.submit(t, p) for t, p in jobs]
        got = _drive(c, ids, {rid: len(t) for rid, (t, _) in zip(ids, jobs)})
        st = c.stats()
    for k, rid in enumerate(ids):
        _same(got[rid], ref[k], f"request {k}")
    assert st["bad_records"] == 0 and st["launches"] >= 1
    # pinned to the oracle directly as well
    t32, _ = jobs[0]
    G.check_fp32(got[ids[0]], G.oracle_results(t32), "resident fp32", table=t32)
    edge = jobs[1][0]
    r = G.check_fp32(got[ids[1]], G.oracle_results(edge), "resident edge", table=edge)
    assert r["fp64"] == 4
    G.check_fp64(got[ids[2]], G.oracle_results(jobs[2][0]), "resident fp64")


def test_resident_serving_mix_equals_alone():
    import paper_2104_10073_amd as Z
    from paper_2104_10073_amd import serving
    reqs = W.serving_requests(200, gen_seed=77, max_funcs=300, log10_samples=(3.0, 6.0))
    arrivals = W.poisson_arrivals(len(reqs), 2000.0, seed=77)
    print(f"resident serving: {len(reqs)} requests, {sum(len(r) for r in reqs)} functions", flush=True)
    for policy in (Z.MC_SCHED_SRPT, Z.MC_SCHED_FAIR):
        with Z.Context(device=0, flags=Z.MC_RESIDENT, policy=policy) as c:
            run = serving.serve(c, reqs, arrivals, keep_results=True)
            st = c.stats()
        assert st["bad_records"] == 0
        print(f"policy {policy}: p50 {np.nanpercentile(run['latency_s'], 50) * 1e3:.3f} ms, "
              f"{st['launches']} launches", flush=True)
        picks = np.random.Generator(np.random.PCG64(3)).choice(len(reqs), 25, replace=False)
        alone = _launch_results(Z, [(reqs[i], Z.PREC_FP32) for i in picks])
        for i, a in zip(picks, alone):
            _same(run["results"][i], a, f"request {i}")


def test_resident_relaunch_after_idle_and_destroy_while_running():
    import paper_2104_10073_amd as Z
    t1 = W.mixed_batch(50, dim_range=(1, 6), log10_samples=(3.0, 5.0), gen_seed=511)
    t2 = W.mixed_batch(50, dim_range=(1, 6), log10_samples=(3.0, 5.0), gen_seed=512)
    ref = _launch_results(Z, [(t1, Z.PREC_FP32), (t2, Z.PREC_FP64)])
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as c:
        _same(c.integrate(t1, Z.PREC_FP32), ref[0], "first")
        assert c.stats()["launches"] == 1
        print("resident: idle for 0.5 s", flush=True)
        time.sleep(0.5)  # the kernel leaves after ~0.1 s without work
        _same(c.integrate(t2, Z.PREC_FP64), ref[1], "second")
        assert c.stats()["launches"] == 2
        big = W.mixed_batch(400, dim_range=(1, 12), log10_samples=(6.0, 7.0), gen_seed=513)
        c.submit(big, Z.PREC_FP32)
        c.run()
        print("resident: destroy with a request running", flush=True)
    # (destroyed: the kernel saw the stop word and left)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        _same(c.integrate(t1, Z.PREC_FP32), ref[0], "a context after it")


def test_resident_abort_then_continue():
    import paper_2104_10073_amd as Z
    big = W.mixed_batch(600, dim_range=(1, 12), log10_samples=(6.0, 7.0), gen_seed=521)
    small = W.mixed_batch(30, dim_range=(1, 5), log10_samples=(3.0, 5.0), gen_seed=522)
    ref, ref_big = _launch_results(Z, [(small, Z.PREC_FP32), (big, Z.PREC_FP32)])
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as c:
        rid = c.submit(big, Z.PREC_FP32)
        c.run()
        time.sleep(0.002)
        print("resident: abort", flush=True)
        c.abort()
        rid_later = c.submit(small, Z.PREC_FP32)  # after the abort call: served normally
        r = c.results(rid, len(big), blocking=True, allow_aborted=True)
        # results that came in before the abort stay, bit for bit; the rest are aborted
        kept = r["status"] == 0
        assert np.all(r["status"][~kept] == -10) and not np.all(kept)
        for f in ("mean", "std_error", "sum_f", "sum_f2", "n", "precision"):
            assert np.array_equal(r[f][kept], ref_big[f][kept]), f
        _same(c.results(rid_later, len(small)), ref, "submitted after the abort")
        _same(c.integrate(small, Z.PREC_FP32), ref, "after abort")


def test_resident_arena_recycled_across_launches():
    import paper_2104_10073_amd as Z
    # more runs than the record arena (8192 positions with 1024 function slots) within one launch
    reqs = [W.mixed_batch(1000, dim_range=(1, 4), log10_samples=(2.0, 4.0), gen_seed=530 + k) for k in range(10)]
    ref = _launch_results(Z, [(t, Z.PREC_FP32) for t in reqs])
    print("resident: 10 x 1000 functions through an 8192-record arena", flush=True)
    with Z.Context(device=0, flags=Z.MC_RESIDENT, max_functions=1024) as c:
        ids = [c.submit(t, Z.PREC_FP32) for t in reqs]
        got = _drive(c, ids, {rid: len(t) for rid, t in zip(ids, reqs)})
        st = c.stats()
    for k, rid in enumerate(ids):
        _same(got[rid], ref[k], f"request {k}")
    print(f"{st['launches']} launches, {st['functions']} functions", flush=True)
    assert st["launches"] >= 2 and st["bad_records"] == 0


def test_resident_in_a_torch_workspace_on_a_side_stream():
    """A resident context whose device memory is a caller's torch tensor (every
    device buffer of the context, the ring's device words and the record arena
    included), driven while torch works on a stream of its own: bitwise the
    launch engine's results."""
    import torch
    import paper_2104_10073_amd as Z
    t = W.mixed_batch(120, dim_range=(1, 12), log10_samples=(3.0, 6.0), gen_seed=531)
    ref = _launch_results(Z, [(t, Z.PREC_FP32)])[0]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = torch.randn(2048, 2048, device="cuda")
        for _ in range(4):
            a = a @ a.T / 2048.0
    with Z.Context(device=0, flags=Z.MC_RESIDENT, workspace="torch") as c:
        got = c.integrate(t, Z.PREC_FP32)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all()
    _same(got, ref, "torch workspace")
