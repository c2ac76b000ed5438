"""The C ABI used from plain C (tests/c_client/zmc_c_client.c, a separate process):
the same function records give bitwise the results of the Python binding on the
batched FP32 and FP64 paths and the plain FP64 path, a resident context gives
the batched FP32 results, and an invalid function is rejected with its status
and a message."""

import os
import subprocess

import numpy as np
import pytest

from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_client", "zmc_c_client")


def test_c_client_matches_python_binding(tmp_path):
    import paper_2104_10073_amd as Z
    if not os.path.exists(EXE):
        pytest.skip("the C client binary is not built (__graft_entry__.build() compiles it)")
    t = np.concatenate([W.eq1_series(n_samples=100_000),
                        W.mixed_batch(40, dim_range=(1, 12), log10_samples=(3.0, 5.0), gen_seed=61)])
    assert t.dtype.itemsize == 472
    fin, fout = tmp_path / "functions.bin", tmp_path / "results.bin"
    t.tofile(fin)
    p = subprocess.run([EXE, str(fin), str(fout)], capture_output=True, text=True, timeout=180)
    assert p.returncode == 0, p.stdout + p.stderr
    got = np.fromfile(fout, dtype=Z.RESULT_DTYPE).reshape(4, len(t))
    with Z.Context(flags=Z.MC_NO_GRAPH) as c:
        want = [c.integrate(t, Z.PREC_FP32), c.integrate(t, Z.PREC_FP64), c.plain_fp64(t)]
    want.append(want[0])
    for k, label in enumerate(("batched FP32", "batched FP64", "plain FP64", "resident FP32")):
        for f in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
            assert np.array_equal(got[k][f], want[k][f]), f"{label}: field {f} differs"
