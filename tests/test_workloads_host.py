"""Seeded workload generator and host-side planning (CPU only)."""

import math
import os

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W


def test_tables_are_deterministic_and_well_formed():
    a = W.mixed_batch(300, dim_range=(1, 7), gen_seed=3)
    b = W.mixed_batch(300, dim_range=(1, 7), gen_seed=3)
    assert a.tobytes() == b.tobytes()
    assert set(np.unique(a["family"])) == {0, 1, 2, 3}
    assert a["dim"].min() >= 1 and a["dim"].max() <= 7
    assert np.all(a["n_samples"] >= 10_000) and np.all(a["n_samples"] <= 10_000_000)
    for i in range(len(a)):
        d = int(a["dim"][i])
        w = a["hi"][i, :d] - a["lo"][i, :d]
        assert np.all(w >= 0.5) and np.all(w <= 2.0)
        assert np.all(a["lo"][i, d:] == 0) and np.all(a["hi"][i, d:] == 0)
    # distinct streams per function, base in the high word
    assert len(set(a["seed"].tolist())) == len(a)
    assert W.stream_seed(7, 3) == (7 << 32) | 3


def test_harmonic_batch_bases_share_parameters():
    a = W.harmonic_batch(50, base=0)
    b = W.harmonic_batch(50, base=3)
    assert np.array_equal(a["params"], b["params"])
    assert not np.array_equal(a["seed"], b["seed"])
    k = a["params"][:, W.V0:W.V0 + 4]
    assert k.min() >= 5 and k.max() <= 30


def test_eq1_series_matches_paper_definition():
    t = W.eq1_series()
    n = np.arange(1, 101)
    assert np.allclose(t["params"][:, W.V0], (n + 50) / (2 * np.pi))
    assert np.all(t["params"][:, 0] == 1) and np.all(t["params"][:, 1] == 1)
    assert np.all(t["dim"] == 4)


def test_high_dim_near_zero_selection_is_real():
    """Every 10th function is near-zero by the tests' own exact closed forms."""
    from closed_forms import exact_integral
    t = W.high_dim_batch(40, n_samples=1000)
    for i in range(9, 40, 10):
        assert abs(exact_integral(t, i)) < 1e-4, i
    assert t["dim"].min() >= 8 and t["dim"].max() <= 12


def test_serving_requests_shapes():
    reqs = W.serving_requests(50, gen_seed=5)
    sizes = [len(r) for r in reqs]
    assert min(sizes) >= 1 and max(sizes) <= 1000
    for r_i, r in enumerate(reqs):
        assert np.all(r["seed"] >> 32 == r_i)
        assert r["dim"].min() >= 1 and r["dim"].max() <= 12
    arr = W.poisson_arrivals(1000, 200.0)
    assert np.all(np.diff(arr) > 0)
    assert abs(1000 / arr[-1] - 200.0) < 30.0


def test_tile_planning_counts():
    """Tiles per function = ceil(segments / 4) with segments of 4096 samples (default tuning)."""
    import paper_2104_10073_amd as Z
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    t = W.eq1_series(n_funcs=6)
    t["n_samples"][:] = [2, 4096, 4097, 16384, 16385, 10_000_000]
    c.submit(t)
    segs = np.ceil(np.ceil(t["n_samples"] / 4) / 1024)
    assert c.pending()[1] == int(np.sum(np.ceil(segs / 4)))
    assert Z.segment_samples() == 4096
    c.close()


def test_serving_summary_math():
    from paper_2104_10073_amd.serving import summarize
    lat = np.linspace(0.001, 0.1, 100)
    out = {"latency_s": lat, "done_s": np.arange(100) * 0.01 + lat, "wall_s": 1.0, "evals": 10**9}
    s = summarize(out, np.arange(100) * 0.01, warmup_frac=0.1)
    assert s["measured"] == 90
    assert abs(s["p50_ms"] - np.percentile(lat[10:], 50) * 1e3) < 1e-9
    assert s["sustained_evals_per_s"] == 1e9


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; asking for more exits with a message (no GPU touched)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_very_large_functions_take_larger_tiles():
    """Tiles grow (up to 256 segments of 4096 samples) so that a function needs
    at most 2^16 tile partials where it can: 2^36 samples -> 2^16 tiles, 2^40
    samples -> 2^20 (the largest tile), both within the default partial space."""
    import paper_2104_10073_amd as Z
    for log2n, tiles in ((36, 1 << 16), (40, 1 << 20), (20, 64)):
        row = W.harmonic_batch(1, n_samples=1 << log2n)
        with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
            c.submit(row, Z.PREC_FP32)
            assert c.validate_tiles() == tiles, log2n


def test_runs_reseed_and_spread():
    """Run r of a table draws the streams of base r; the spread is the per-function
    mean and sample standard deviation (n - 1) over runs."""
    from paper_2104_10073_amd import runs as R
    from paper_2104_10073_amd._native import RESULT_DTYPE
    t = W.harmonic_batch(5, n_samples=1000, base=0)
    u = R.reseeded(t, 7)
    assert list(u["seed"]) == [W.stream_seed(7, i) for i in range(5)]
    assert list(t["seed"]) == [W.stream_seed(0, i) for i in range(5)]
    for k in ("family", "dim", "n_samples", "lo", "hi", "params"):
        assert np.array_equal(t[k], u[k])
    rs = []
    for r, vals in enumerate(([1.0, 2.0], [3.0, 2.0], [5.0, 2.0])):
        a = np.zeros(2, dtype=RESULT_DTYPE)
        a["mean"] = vals
        a["std_error"] = [r + 1.0, 0.0]
        rs.append(a)
    s = R.spread(rs)
    assert s["runs"] == 3
    assert list(s["mean"]) == [3.0, 2.0]
    assert list(s["spread"]) == [2.0, 0.0]
    assert abs(s["rms_se"][0] - math.sqrt(14.0 / 3.0)) < 1e-15 and s["rms_se"][1] == 0.0
    with pytest.raises(ValueError):
        R.spread(rs[:1])


def test_bench_roofline_helpers(monkeypatch):
    """The roofline's algorithmic work (77 lane-slots per d = 4 harmonic evaluation:
    Philox 60, uniforms 4, phase and cos 9, sums 4) and the committed HBM counter
    summary, which is used only while the kernel sources match its hash."""
    import bench
    assert bench.algorithmic_slots_per_eval("harmonic", 4) == 77.0
    assert bench.algorithmic_slots_per_eval("harmonic", 8) == 60 * 2 + 8 + 13 + 4
    traffic = bench.measured_traffic("zmc_batched_fp32")
    assert traffic is None or 3e6 < traffic < 1e8           # None once the sources differ from the profile's
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("zmc_batched_fp32") is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_bench_help_lists_the_contract_options():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--serve-policy", "--blocks-per-cu", "--graph"):
        assert opt in p.stdout, opt


def test_bench_full_oracle_check_grades_by_precision():
    """bench.full_oracle_check: results equal to the oracle's pass; an FP32 row off by
    0.02 SE or an FP64 sum off by 1e-11 relative fails; promoted rows are graded by
    the FP64 bar."""
    import importlib.util
    from oracle import oracle as O
    from paper_2104_10073_amd import _native
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = W.mixed_batch(24, dim_range=(1, 5), log10_samples=(3.0, 3.5), gen_seed=17)
    o, _ = O.default().integrate(t, 4)

    def as_gpu(prec):
        r = np.zeros(len(t), dtype=_native.RESULT_DTYPE)
        for f in ("mean", "sum_f", "sum_f2", "n"):
            r[f] = o[f]
        r["std_error"] = o["stderr"]
        r["precision"] = prec
        return r

    r32, r64 = as_gpu(0), as_gpu(1)
    r32["precision"][3] = 1
    res = bench.full_oracle_check(O.default(), t, r32, r64, 4)
    assert res["pass"] and res["promoted_rows"] == 1 and res["fp32_rows"] == len(t) - 1
    bad = r32.copy()
    bad["mean"][5] += 0.02 * o["stderr"][5]
    assert not bench.full_oracle_check(O.default(), t, bad, r64, 4)["pass"]
    bad = r64.copy()
    bad["sum_f"][7] += 1e-11 * o["sum_abs"][7]
    assert not bench.full_oracle_check(O.default(), t, r32, bad, 4)["pass"]
    bad = r32.copy()
    bad["sum_f"][3] += 1e-11 * o["sum_abs"][3]
    assert not bench.full_oracle_check(O.default(), t, bad, r64, 4)["pass"]
