"""Plant plausible mistakes in copies of the oracle (on the CPU) and show the pins catch each.

Every mutant below is a one-line edit of ``oracle/zmc_oracle.c`` of the kind a
reader of the paper could make while writing it: a wrong constant, a dropped
term, a flipped sign, a transposed index or operand.  Each is compiled into a
temporary library and run through the pin checks; at least one check must
fail.  The real oracle passes all of them (test_oracle_pins.py).
"""

import os

import pytest

import oracle_pins as P
from oracle import oracle as O

MUTANTS = [
    ("philox multiplier", "PHILOX_M0 = 0xD2511F53u", "PHILOX_M0 = 0xD2511F55u"),
    ("philox hi/lo swap", "uint32_t n1 = lo1;", "uint32_t n1 = hi1;"),
    ("philox key bump dropped", "k1 += PHILOX_W1;", "k1 += 0u;"),
    ("philox nine rounds", "r < 10; ++r", "r < 9; ++r"),
    ("philox xor operand", "uint32_t n2 = hi0 ^ c[3] ^ k1;", "uint32_t n2 = hi0 ^ c[1] ^ k1;"),
    ("uniform high bits", "uint32_t m = r & 0x7FFFFFu;", "uint32_t m = r >> 9;"),
    ("uniform left endpoint", "(double)(2u * m + 1u)", "(double)(2u * m)"),
    ("stream block stride", "uint64_t b = q * (uint64_t)dim + (uint64_t)j;",
     "uint64_t b = q * (uint64_t)(dim + 1) + (uint64_t)j;"),
    ("quad member ignored", "return out[s];", "return out[j & 3u];"),
    ("quad index is the sample index", "uint64_t q = i / 4u;                       /* quad */",
     "uint64_t q = i;"),
    ("counter words in 2-3", "{(uint32_t)b, (uint32_t)(b >> 32), 0u, 0u}", "{0u, 0u, (uint32_t)b, (uint32_t)(b >> 32)}"),
    ("key halves swapped", "{(uint32_t)seed, (uint32_t)(seed >> 32)}", "{(uint32_t)(seed >> 32), (uint32_t)seed}"),
    ("key high word dropped", "{(uint32_t)seed, (uint32_t)(seed >> 32)}", "{(uint32_t)seed, 0u}"),
    ("mapping drops lo", "x[j] = fma(w, u, fn->lo[j]);", "x[j] = w * u;"),
    ("harmonic sin sign", "fma(p[0], cos(theta), p[1] * sin(theta))", "fma(p[0], cos(theta), -p[1] * sin(theta))"),
    ("harmonic a/b swapped", "fma(p[0], cos(theta), p[1] * sin(theta))", "fma(p[1], cos(theta), p[0] * sin(theta))"),
    ("harmonic last dim dropped", "for (uint32_t j = 0; j < d; ++j) theta = fma",
     "for (uint32_t j = 0; j + 1 < d; ++j) theta = fma"),
    ("abs-linear offset dropped", "double s = p[1];", "double s = 0.0;"),
    ("gaussian width", "double h = 0.5 / (p[1] * p[1]);", "double h = 0.5 / p[1];"),
    ("gaussian centre sign", "double t = x[j] - p[ORC_V0 + j];", "double t = x[j] + p[ORC_V0 + j];"),
    ("poly degree off by one", "for (int e = 0; e < deg; ++e)", "for (int e = 0; e <= deg; ++e)"),
    ("S2 sums f", "nsum_add(&a2, f * f);", "nsum_add(&a2, f);"),
    ("compensation dropped", "static double nsum_value(const orc_sum* a) { return a->s + a->c; }",
     "static double nsum_value(const orc_sum* a) { return a->s; }"),
    ("compensation branch swapped", "if (fabs(a->s) >= fabs(x))", "if (fabs(a->s) < fabs(x))"),
    ("compensation term sign", "a->c += (a->s - t) + x;", "a->c -= (a->s - t) + x;"),
    ("variance denominator N", "/ (dn - 1.0);", "/ dn;"),
    ("SE without volume", "*se = volume * sqrt(var / dn);", "*se = sqrt(var / dn);"),
    ("mean without volume", "*mean = volume * (s1 / dn);", "*mean = s1 / dn;"),
    ("volume from hi only", "v *= (fn->hi[j] - fn->lo[j]);", "v *= fn->hi[j];"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path, rocrand_ref):
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/present: {old}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = O.compile_source(str(mut), str(tmp_path / f"libmutant_{abs(hash(name))}.so"))
    orc = O.Oracle(lib)
    failed = []
    for check_name, check in P.ALL_CHECKS:
        try:
            check(orc, rocrand_ref)
        except AssertionError:
            failed.append(check_name)
            break
    assert failed, f"mutant '{name}' passed every pin"
