"""mc_autotune on an MI355X: it returns within its time budget, changes no result
bit (the reduction tree of a function does not depend on the launch shape or
the tile size), and with MC_TUNE_CACHE set a second context takes the tuned
choice from the cache instead of timing again."""

import time

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")


def test_autotune_budget_results_and_cache(tmp_path, monkeypatch):
    import paper_2104_10073_amd as Z
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MC_TUNE_CACHE", str(cache))
    t = W.mixed_batch(200, dim_range=(1, 12), log10_samples=(3.0, 6.0), gen_seed=401)
    with Z.Context(device=0) as c:
        r32 = c.integrate(t, Z.PREC_FP32)
        r64 = c.integrate(t, Z.PREC_FP64)
        for prec, budget in ((Z.PREC_FP32, 2.0), (Z.PREC_FP64, 1.0)):
            t0 = time.perf_counter()
            c.autotune(prec, budget_seconds=budget)
            dt = time.perf_counter() - t0
            print(f"autotune precision {prec}: {dt:.2f} s of a {budget} s budget", flush=True)
            assert dt < budget + 1.5
        blocks, seg = c.get_tuning()
        assert 1 <= blocks <= 32 and seg.max() <= 6
        a32 = c.integrate(t, Z.PREC_FP32)
        a64 = c.integrate(t, Z.PREC_FP64)
    for f in FIELDS:
        assert np.array_equal(a32[f], r32[f]), f
        assert np.array_equal(a64[f], r64[f]), f
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("zmc-tune 1 gfx950") for ln in lines)
    with Z.Context(device=0) as c2:
        t0 = time.perf_counter()
        c2.autotune(Z.PREC_FP32, budget_seconds=2.0)
        c2.autotune(Z.PREC_FP64, budget_seconds=1.0)
        dt = time.perf_counter() - t0
        b2, seg2 = c2.get_tuning()
        assert dt < 0.2, dt
        assert b2 == blocks and np.array_equal(seg2, seg)
        for f in FIELDS:
            assert np.array_equal(c2.integrate(t, Z.PREC_FP32)[f], r32[f]), f
    assert len(cache.read_text().splitlines()) == 2
