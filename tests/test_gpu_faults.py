"""Failed HIP calls on an MI355X (MC_FAULT_HIP): no wrong result, no hang.

Each run creates a context with MC_FAULT_HIP=n, so the n-th checked HIP call
the library makes reports failure without being made (the GPU itself never
faults: the call is simply not issued), and drives three requests -- mixed
forms in FP32, the edge table (with its promoted rows), a mixed FP64 table --
through launches of 8 tiles, or through a resident context (every third n)
whose ring holds 8 unread tiles; after the first run the first request is
snapshotted and restored into the same context as a fourth.  Every request must come back either bitwise as
in a run without failures or with MC_ERR_HIP / MC_ERR_OUT_OF_MEMORY; every
call returns.  The CPU emulation sweeps every n (test_host_runtime_emulated);
this runs the same kind of sweep against the real runtime, graphs included.
"""

import os

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")


def _run(Z, flags, tables):
    """{request index: results array or error status}, and the failed mc_run count;
    (None, status) when the context could not be created."""
    try:
        ctx = Z.Context(device=0, flags=flags, max_tiles_per_run=8, max_functions=256, max_partials=1 << 14)
    except Z.McError as e:
        assert e.status in (-6, -8), e
        return None, e.status
    out, ids, run_errors = {}, {}, 0
    sizes = {k: len(t) for k, (t, _) in enumerate(tables)}
    try:
        for k, (t, prec) in enumerate(tables):
            ids[k] = ctx.submit(t, prec)
        for it in range(20000):
            if len(out) == len(tables) + 1:
                break
            try:
                ctx.run()
            except Z.McError as e:
                assert e.status in (-6, -8), e
                run_errors += 1
            if it == 0:
                # the first request, snapshotted while its work runs, restored into the same context
                k = len(tables)
                sizes[k] = sizes[0]
                try:
                    ids[k] = ctx.restore(ctx.snapshot(ids[0]))
                except Z.McError as e:
                    assert e.status in (-1, -6, -8), e  # (-1: the request was lost to a failed launch)
                    out[k] = e.status
            for k, rid in ids.items():
                if k in out:
                    continue
                try:
                    r = ctx.results(rid, sizes[k], blocking=it > 10000)
                except Z.McError as e:
                    assert e.status in (-6, -8), e
                    out[k] = e.status
                    continue
                if r is not None:
                    out[k] = r
        assert len(out) == len(tables) + 1, "requests left unfinished"
    finally:
        ctx.close()
    return out, run_errors


def test_failed_hip_calls_never_give_wrong_results():
    import paper_2104_10073_amd as Z
    tables = [(W.mixed_batch(30, dim_range=(1, 12), log10_samples=(2.0, 5.5), gen_seed=301), Z.PREC_FP32),
              (G.edge_table(), Z.PREC_FP32),
              (W.mixed_batch(10, dim_range=(1, 6), log10_samples=(3.0, 5.0), gen_seed=302), Z.PREC_FP64)]
    os.environ.pop("MC_FAULT_HIP", None)
    ref, errors = _run(Z, Z.MC_NO_GRAPH, tables)
    assert errors == 0 and all(isinstance(v, np.ndarray) for v in ref.values())
    for f in FIELDS:  # the restored copy completes as the request itself
        assert np.array_equal(ref[3][f], ref[0][f]), f
    res_ref, errors = _run(Z, Z.MC_RESIDENT, tables)
    assert errors == 0
    for k in ref:
        for f in FIELDS:
            assert np.array_equal(res_ref[k][f], ref[k][f]), (k, f)
    seen_errors = 0
    try:
        for n in range(1, 600):
            os.environ["MC_FAULT_HIP"] = str(n)
            # direct launches, graphs, and the resident engine in turn
            flags = (Z.MC_NO_GRAPH, 0, Z.MC_RESIDENT)[n % 3]
            out, errors = _run(Z, flags, tables)
            if out is None:
                seen_errors += 1
                continue
            for k, v in out.items():
                if isinstance(v, np.ndarray):
                    for f in FIELDS:
                        assert np.array_equal(v[f], ref[k][f]), (n, k, f)
                else:
                    seen_errors += 1
            seen_errors += errors
    finally:
        os.environ.pop("MC_FAULT_HIP", None)
    print(f"failed HIP calls 1..599: {seen_errors} errors reported, no wrong result", flush=True)
    assert seen_errors > 50
