"""The library's sample points against the oracle's, bit for bit, across the
whole index range (an MI355X): the generator and FP64 mapping the batched
kernels use, read out through mc_sample_points.  Covers every dimension, the
first samples, partial quads, the 2^32 crossing of the Philox block index (the
counter's high word) and the last samples of a 2^40-sample function."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    t = W.mixed_batch(24, dim_range=(1, 12), log10_samples=(4.0, 5.0), gen_seed=41)
    out = []
    for i in range(len(t)):
        row = t[i:i + 1].copy()
        d = int(row["dim"][0])
        row["n_samples"] = 1 << 40
        starts = [0, 3, 4097]
        # sample index at which block q*d + j first reaches 2^32
        q = (1 << 32) // d
        starts.append(4 * q - 8)
        starts.append((1 << 40) - 64)
        out.append((row, starts))
    return out


def test_sample_points_bit_exact_across_the_range():
    import paper_2104_10073_amd as Z
    orc = O.default()
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        for row, starts in _cases():
            for s0 in starts:
                gpu = c.sample_points(row, s0, 64)
                ref = orc.sample_points(row, 0, s0, 64)
                assert np.array_equal(gpu, ref), (int(row["dim"][0]), s0)


def test_sample_points_range_errors():
    import paper_2104_10073_amd as Z
    row = W.harmonic_batch(1, n_samples=1000)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        for first, count in ((1000, 1), (990, 11)):
            with pytest.raises(Z.McError) as e:
                c.sample_points(row, first, count)
            assert e.value.status == -1
        assert c.sample_points(row, 999, 1).shape == (1, 4)
