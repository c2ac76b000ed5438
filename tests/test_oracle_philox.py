"""Pins of the oracle's random-number stream against AMD's rocRAND Philox4x32-10.

rocRAND is an independent implementation of Philox4x32-10 (Salmon et al., SC'11).
Its host-side generator, seeded with the 64-bit function seed and read from
subsequence 0, produces word g of the stream from counter (g/4 lo, g/4 hi, 0, 0)
and key (seed lo, seed hi).  The oracle takes samples in quads: coordinate j
of sample i is word i mod 4 of block (i / 4) * d + j, i.e. stream word
g = 4 * ((i / 4) * d + j) + (i mod 4).  The tests compare bit for bit.
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
    """Coordinate j of sample i is word 4*((i//4)*d + j) + i%4 of rocRAND's stream for seed s."""
    from oracle_pins import stream_words
    for seed in (0, 7, W.stream_seed(3, 17), W.stream_seed(0xFFFFFFFF, 0xFFFFFFFF), 2**63 + 5):
        for dim in (1, 3, 4, 7, 12):
            for i0 in (0, 1, 5, 1_000_003):
                samples = range(i0, i0 + 9)
                ref = stream_words(rocrand_ref, seed, dim, samples)
                for i in samples:
                    for j in range(dim):
                        assert orc.word(seed, dim, i, j) == ref[(i, j)], (seed, dim, i, j)


def test_quad_uses_consecutive_blocks(orc, rocrand_ref):
    """A quad of samples consumes exactly d consecutive Philox blocks, nothing wasted."""
    seed, dim = 99, 5
    words = rocrand_ref([f"w {seed} 0 {4 * dim * 3}"])[0]
    got = []
    for q in range(3):
        for j in range(dim):
            got.extend(orc.word(seed, dim, 4 * q + s, j) for s in range(4))
    assert got == words


def test_high_counter_word(orc, rocrand_ref):
    """Block index past 2^32 carries into counter word 1."""
    from oracle_pins import stream_words
    seed, dim = 12345, 12
    i = 4 * ((1 << 32) // 12 + 77)  # first block of the quad > 2^32
    ref = stream_words(rocrand_ref, seed, dim, range(i, i + 4))
    for s in range(4):
        for j in range(dim):
            assert orc.word(seed, dim, i + s, j) == ref[(i + s, j)]
