"""Error paths of the C ABI on a device context: unknown or already-taken request
ids, a wrong result count, a non-blocking query before the work has run, mc_run
with every launch slot in flight, and a caller workspace that is too small or
misaligned -- each returns its status (and a message) and leaves the context
usable."""

import ctypes

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

MC_ERR_INVALID_ARG = -1
MC_ERR_UNKNOWN_REQUEST = -11


def test_result_queries():
    import paper_2104_10073_amd as Z
    t = W.eq1_series(n_samples=20_000, n_funcs=8)
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        rid = c.submit(t, Z.PREC_FP32)
        assert c.results(rid, len(t), blocking=False) is None      # not launched yet
        with pytest.raises(Z.McError) as e:
            c.results(rid, len(t) + 1)
        assert e.value.status == MC_ERR_INVALID_ARG and "functions" in str(e.value)
        with pytest.raises(Z.McError) as e:
            c.results(rid + 1000, len(t))
        assert e.value.status == MC_ERR_UNKNOWN_REQUEST
        r = c.results(rid, len(t))                                  # blocking: runs and waits
        assert np.all(r["status"] == 0)
        with pytest.raises(Z.McError) as e:
            c.results(rid, len(t))                                  # results are taken once
        assert e.value.status == MC_ERR_UNKNOWN_REQUEST
        again = c.integrate(t, Z.PREC_FP32)                         # the context still works
        assert np.array_equal(again["sum_f"], r["sum_f"])


def test_run_with_every_slot_in_flight():
    """Three launches of ~10^9 samples in 8..12 dimensions (several ms each) fill the
    ring of launch slots; a fourth mc_run right after them finds no free slot and
    returns MC_NOT_READY (False)."""
    import paper_2104_10073_amd as Z
    t = W.high_dim_batch(500, n_samples=10_000_000)
    with Z.Context(flags=Z.MC_NO_GRAPH, max_tiles_per_run=1 << 16) as c:
        rid = c.submit(t, Z.PREC_FP32)
        launched = [c.run() for _ in range(4)]
        assert launched[:3] == [True, True, True] and launched[3] is False, launched
        r = c.results(rid, len(t))
        assert np.all(r["status"] == 0)


def test_caller_workspace_too_small_or_misaligned():
    import torch
    import paper_2104_10073_amd as Z
    from paper_2104_10073_amd import _native
    L = Z.load()
    cfg = _native.McConfig()
    L.mc_config_init(ctypes.byref(cfg))
    cfg.flags = Z.MC_NO_GRAPH
    need = ctypes.c_uint64()
    assert L.mc_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == 0
    buf = torch.empty(int(need.value) + 512, dtype=torch.uint8, device="cuda:0")
    base = int(buf.data_ptr()) + ((-int(buf.data_ptr())) % 256)
    h = ctypes.c_void_p()
    cfg.workspace, cfg.workspace_bytes = base, int(need.value) - 1
    assert L.mc_create(ctypes.byref(cfg), ctypes.byref(h)) == MC_ERR_INVALID_ARG
    assert b"smaller" in L.mc_last_error(None)
    cfg.workspace, cfg.workspace_bytes = base + 8, int(need.value)
    assert L.mc_create(ctypes.byref(cfg), ctypes.byref(h)) == MC_ERR_INVALID_ARG
    assert b"aligned" in L.mc_last_error(None)
    cfg.workspace, cfg.workspace_bytes = base, int(need.value)
    assert L.mc_create(ctypes.byref(cfg), ctypes.byref(h)) == 0
    assert L.mc_destroy(h) == 0
    torch.cuda.synchronize()
