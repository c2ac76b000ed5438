"""The plain FP64 path without allocation (mc_integrate_plain_fp64_noalloc), on an MI355X.

Its working set lives in the library's fixed per-GPU array, which keeps the
previous call's contents; two calls in a row, the second smaller, must each
give what mc_integrate_plain_fp64 gives for the same table (bitwise: same
kernels, same records), and meet the FP64 bar against the oracle.
"""

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2104_10073_amd as Z
    c = Z.Context(device=0, flags=Z.MC_NO_GRAPH)
    yield c
    c.close()


def _same(a, b, label):
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
        assert np.array_equal(a[k], b[k]), (label, k)


def test_noalloc_matches_plain_twice(ctx):
    import torch
    stream = torch.cuda.current_stream()
    big = np.concatenate([G.edge_table(),
                          W.mixed_batch(200, dim_range=(1, 12), log10_samples=(2.0, 5.5), gen_seed=211)])
    small = W.mixed_batch(17, dim_range=(1, 12), log10_samples=(1.0, 3.0), gen_seed=212)
    for label, t in (("first call, large", big), ("second call, smaller", small)):
        print(f"no-alloc plain path: {label}, {len(t)} functions", flush=True)
        got = ctx.plain_fp64_noalloc(t, stream=stream)
        ref = ctx.plain_fp64(t, stream=stream)
        _same(got, ref, label)
        G.check_fp64(got, G.oracle_results(t), "no-alloc " + label)


def test_noalloc_largest_function(ctx):
    """One function at the largest sample count the fixed array holds (2^30), next
    to a tiny one: equal to the allocating path bit for bit."""
    t = W.mixed_batch(2, dim_range=(3, 3), log10_samples=(2.0, 2.0), gen_seed=213)
    t["n_samples"][0] = 1 << 30
    print("no-alloc plain path: 2^30 samples", flush=True)
    _same(ctx.plain_fp64_noalloc(t), ctx.plain_fp64(t), "2^30 samples")


def test_noalloc_limits_rejected(ctx):
    import paper_2104_10073_amd as Z
    over_n = W.mixed_batch(4097, dim_range=(1, 2), log10_samples=(1.0, 1.0), gen_seed=214)
    with pytest.raises(Z.McError) as e:
        ctx.plain_fp64_noalloc(over_n)
    assert e.value.status == -1
    over_samples = W.mixed_batch(2, dim_range=(1, 2), log10_samples=(1.0, 1.0), gen_seed=215)
    over_samples["n_samples"][1] = (1 << 30) + 1
    with pytest.raises(Z.McError) as e:
        ctx.plain_fp64_noalloc(over_samples)
    assert e.value.status == -1
    # the context and the array still work after a refused call
    t = W.eq1_series(n_samples=10_000, n_funcs=8)
    _same(ctx.plain_fp64_noalloc(t), ctx.plain_fp64(t), "after refused calls")
