"""Pins of the oracle's random-number stream against AMD's rocRAND Philox4x32-10.

rocRAND is an independent implementation of Philox4x32-10 (Salmon et al., SC'11).
Its host-side generator, seeded with the 64-bit function seed and read from
subsequence 0, produces word g of the stream from counter (g/4 lo, g/4 hi, 0, 0)
and key (seed lo, seed hi) -- exactly the layout the oracle defines (coordinate
j of sample i uses word g = i*d + j).  The tests compare bit for bit.
"""

import numpy as np

from paper_2104_10073_amd import workloads as W


def test_philox_blocks_match_rocrand(orc, rocrand_ref):
    rng = np.random.Generator(np.random.PCG64(11))
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 1, 0, 0, 0, 0),
             (0, 0, 1, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 1, 0), (0, 0, 0, 0, 0, 1)]
    for _ in range(200):
        c = [int(v) for v in rng.integers(0, 2**32, 4)]
        c[1] &= 0x0FFFFFFF  # rocRAND's skip-ahead takes the block offset in words (4 per block)
        k = [int(v) for v in rng.integers(0, 2**32, 2)]
        cases.append(tuple(c + k))
    ref = rocrand_ref(["b " + " ".join(str(v) for v in cs) for cs in cases])
    for cs, r in zip(cases, ref):
        assert orc.philox(cs[:4], cs[4:]) == r, cs


def test_stream_layout_matches_rocrand(orc, rocrand_ref):
    """Word g of function seed s is rocRAND's g-th output for seed s (subsequence 0)."""
    lines, expect = [], []
    for seed in (0, 7, W.stream_seed(3, 17), W.stream_seed(0xFFFFFFFF, 0xFFFFFFFF), 2**63 + 5):
        for dim in (1, 3, 4, 7, 12):
            for i0 in (0, 1, 5, 1_000_003):
                n = 6
                lines.append(f"w {seed} {i0 * dim} {n * dim}")
                expect.append([orc.word(seed, dim, i, j) for i in range(i0, i0 + n) for j in range(dim)])
    ref = rocrand_ref(lines)
    for ln, r, e in zip(lines, ref, expect):
        assert r == e, ln


def test_high_counter_word(orc, rocrand_ref):
    """Block index past 2^32 carries into counter word 1."""
    seed, dim = 12345, 12
    i = (1 << 32) // 3 + 77  # g = i*12 > 2^34, block > 2^32
    line = f"w {seed} {i * dim} {dim}"
    ref = rocrand_ref([line])[0]
    assert ref == [orc.word(seed, dim, i, j) for j in range(dim)]
