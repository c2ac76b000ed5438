"""The C ABI library loads on a CPU-only host, exports every declared symbol,
and validates inputs without touching a device (MC_VALIDATE_ONLY)."""

import os
import re

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Z():
    import paper_2104_10073_amd as Z
    if not os.path.exists(os.path.join(ROOT, "paper_2104_10073_amd", "libzmc.so")):
        from paper_2104_10073_amd import build
        build.build()
    Z.load()
    return Z


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "zmc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:mc_status|const char\*|uint32_t)\s+(mc_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(Z):
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2104_10073_amd", "libzmc.so"))
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    from paper_2104_10073_amd import _native
    assert sorted(_native.EXPORTS) == syms


def test_struct_sizes(Z):
    import ctypes
    from paper_2104_10073_amd import _native
    assert W.FUNC_DTYPE.itemsize == 472
    assert _native.RESULT_DTYPE.itemsize == 48
    assert ctypes.sizeof(_native.McConfig) == 56
    assert ctypes.sizeof(_native.McStats) == 88


def test_validate_only_accepts_workloads(Z):
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    for t in (W.eq1_series(), W.eq2_series(), W.harmonic_batch(50), W.mixed_batch(200, dim_range=(1, 12)),
              W.high_dim_batch(20, near_zero_every=0)):
        assert c.submit(t) > 0
        assert c.submit(t, Z.PREC_FP64) > 0
    c.close()


@pytest.mark.parametrize("field,value,code", [
    ("family", 7, -2), ("dim", 0, -3), ("dim", 13, -3), ("n_samples", 1, -1), ("n_samples", 2**41, -1),
])
def test_validate_only_rejects(Z, field, value, code):
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    t = W.eq1_series(n_funcs=5)
    t[field][3] = value
    with pytest.raises(Z.McError) as e:
        c.submit(t)
    assert e.value.status == code
    assert "function 3" in str(e.value)
    c.close()


def test_validate_only_rejects_bounds_and_params(Z):
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    t = W.eq1_series(n_funcs=2)
    b = t.copy(); b["hi"][1, 2] = b["lo"][1, 2]
    with pytest.raises(Z.McError) as e:
        c.submit(b)
    assert e.value.status == -4
    b = t.copy(); b["lo"][0, 0] = np.inf
    with pytest.raises(Z.McError) as e:
        c.submit(b)
    assert e.value.status == -4
    b = t.copy(); b["params"][0, 30] = np.nan
    with pytest.raises(Z.McError) as e:
        c.submit(b)
    assert e.value.status == -5
    g = W.empty(1); W.set_gaussian(g, 0, 2, 1.0, 0.0, [0, 0], [0, 0], [1, 1]); g["n_samples"] = 10
    with pytest.raises(Z.McError) as e:
        c.submit(g)
    assert e.value.status == -5
    p = W.empty(1); W.set_poly(p, 0, 2, [1, 1], [1, 9], [0, 0], [1, 1]); p["n_samples"] = 10
    with pytest.raises(Z.McError) as e:
        c.submit(p)
    assert e.value.status == -5
    p["params"][0, W.W0 + 1] = 2.5
    with pytest.raises(Z.McError) as e:
        c.submit(p)
    assert e.value.status == -5
    with pytest.raises(Z.McError) as e:
        c.submit(t, precision=7)
    assert e.value.status == -1
    c.close()


def test_validate_only_has_no_device_calls(Z):
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    with pytest.raises(Z.McError) as e:
        c.run()
    assert e.value.status == -9
    with pytest.raises(Z.McError) as e:
        c.plain_fp64(W.eq1_series(n_funcs=2))
    assert e.value.status == -9
    with pytest.raises(Z.McError) as e:
        c.plain_fp64_noalloc(W.eq1_series(n_funcs=2))
    assert e.value.status == -9
    c.close()


def test_admission_limits(Z):
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY, max_functions=10, max_partials=8)
    with pytest.raises(Z.McError) as e:
        c.submit(W.eq1_series(n_funcs=11))
    assert e.value.status == -7
    big = W.harmonic_batch(2, n_samples=10_000_000)
    with pytest.raises(Z.McError) as e:
        c.submit(big)
    assert e.value.status == -7
    c.close()


def test_workspace_size_monotone(Z):
    import ctypes
    from paper_2104_10073_amd import _native
    L = Z.load()
    sizes = []
    for mf in (1000, 100_000):
        cfg = _native.McConfig()
        L.mc_config_init(ctypes.byref(cfg))
        cfg.max_functions = mf
        out = ctypes.c_uint64()
        assert L.mc_workspace_size(ctypes.byref(cfg), ctypes.byref(out)) == 0
        sizes.append(out.value)
    assert sizes[1] > sizes[0] > 0


@pytest.mark.parametrize("kw", [{"max_partials": 1 << 32}, {"max_functions": (1 << 24) + 1},
                                {"max_tiles_per_run": (1 << 28) + 1}])
def test_config_limits_of_32bit_indices(Z, kw):
    with pytest.raises(Z.McError) as e:
        Z.Context(flags=Z.MC_VALIDATE_ONLY, **kw)
    assert e.value.status == -1


def test_c_client_links_and_checks_its_input(tmp_path):
    """The tests' plain C client compiles against include/zmc.h, links libzmc.so, and
    rejects a wrong command line or a file that is not whole 472-byte records before
    it touches a device."""
    import subprocess
    import __graft_entry__ as g
    exe = os.path.join(g.ROOT, "tests", "c_client", "zmc_c_client")
    if not os.path.exists(exe):
        g._build_c_client()
    p = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert p.returncode == 2 and "usage" in p.stderr
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"\0" * 471)
    p = subprocess.run([exe, str(bad), str(tmp_path / "out.bin")], capture_output=True, text=True, timeout=60)
    assert p.returncode == 2 and "472-byte records" in p.stderr


def test_unknown_policy_and_empty_request(Z):
    with pytest.raises(Z.McError) as e:
        Z.Context(flags=Z.MC_VALIDATE_ONLY, policy=3)
    assert e.value.status == -1 and "policy" in str(e.value)
    c = Z.Context(flags=Z.MC_VALIDATE_ONLY)
    with pytest.raises(Z.McError) as e:
        c.submit(W.eq1_series(n_funcs=1)[:0])
    assert e.value.status == -1
    c.close()
