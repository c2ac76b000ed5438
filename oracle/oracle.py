"""ctypes front end of the serial FP64 CPU oracle (``oracle/zmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg load this module; the GPU library never does.  It imports
nothing from the GPU package; the function table it reads is the shared input
format produced by the seeded workload generator.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "zmc_oracle.c")
LIB = os.path.join(HERE, "libzmc_oracle.so")

RESULT_DTYPE = np.dtype([
    ("mean", "<f8"), ("stderr", "<f8"), ("sum_f", "<f8"), ("sum_f2", "<f8"),
    ("sum_abs", "<f8"), ("volume", "<f8"), ("n", "<u8"), ("status", "<i4"), ("pad", "<i4"),
])
FUNC_SIZE = 472
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file with gcc (strict IEEE: no contraction, no fast-math)."""
    subprocess.run(["gcc", *CFLAGS, "-o", out + ".tmp", src, "-lm", "-lpthread"], check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        compile_source(SRC, LIB)
    return LIB


class Oracle:
    """One loaded build of the oracle (the default build, or a test's variant of it)."""

    def __init__(self, path: str = LIB):
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [ctypes.c_uint32]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_word.restype = ctypes.c_uint32
        L.orc_sample_point.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        L.orc_sample_point.restype = None
        L.orc_sample_points.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        L.orc_sample_points.restype = None
        L.orc_eval.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_eval.restype = ctypes.c_double
        L.orc_validate.argtypes = [ctypes.c_void_p]
        L.orc_validate.restype = ctypes.c_int
        L.orc_partial_sums.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, dp, dp, dp]
        L.orc_partial_sums.restype = None
        L.orc_volume.argtypes = [ctypes.c_void_p]
        L.orc_volume.restype = ctypes.c_double
        L.orc_finalize.argtypes = [ctypes.c_double, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_finalize.restype = None
        L.orc_integrate.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_integrate.restype = ctypes.c_int
        L.orc_integrate_batch.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int]
        L.orc_integrate_batch.restype = ctypes.c_int
        L.orc_sizeof_function.restype = ctypes.c_size_t
        L.orc_sizeof_result.restype = ctypes.c_size_t
        assert L.orc_sizeof_function() == FUNC_SIZE
        assert L.orc_sizeof_result() == RESULT_DTYPE.itemsize
        self.L = L
        self.path = path

    @staticmethod
    def _row(table: np.ndarray, i: int = 0) -> int:
        assert table.dtype.itemsize == FUNC_SIZE and table.flags["C_CONTIGUOUS"]
        return table.ctypes.data + i * FUNC_SIZE

    def philox(self, ctr, key):
        c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
        k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
        o = (ctypes.c_uint32 * 4)()
        self.L.orc_philox4x32_10(c, k, o)
        return [int(o[i]) for i in range(4)]

    def uniform(self, r: int) -> float:
        return self.L.orc_uniform(int(r) & 0xFFFFFFFF)

    def word(self, seed: int, dim: int, i: int, j: int) -> int:
        return int(self.L.orc_word(seed, dim, i, j))

    def sample_point(self, table: np.ndarray, idx: int, i: int) -> np.ndarray:
        x = np.zeros(12, dtype=np.float64)
        self.L.orc_sample_point(self._row(table, idx), i, x.ctypes.data)
        return x[: int(table["dim"][idx])]

    def sample_points(self, table: np.ndarray, idx: int, i0: int, count: int) -> np.ndarray:
        """Points of samples [i0, i0 + count) of function idx, shape (count, dim)."""
        d = int(table["dim"][idx])
        x = np.zeros((count, d), dtype=np.float64)
        self.L.orc_sample_points(self._row(table, idx), i0, count, x.ctypes.data)
        return x

    def integrate_user(self, table: np.ndarray, f, chunk: int = 1 << 16):
        """Direct MC of caller-defined integrands on the oracle's own samples.

        ``f(x, p)`` evaluates the integrand in float64 on points x (n, d) with the
        function's params p (32,); each function's sums are exact-rounded
        (math.fsum over all its samples) and finalized like the built-in
        families (paper, "Solution method": direct Monte Carlo per integrand)."""
        import math
        table = np.ascontiguousarray(table)
        out = np.zeros(len(table), dtype=RESULT_DTYPE)
        for i in range(len(table)):
            n = int(table["n_samples"][i])
            vals = []
            for i0 in range(0, n, chunk):
                x = self.sample_points(table, i, i0, min(chunk, n - i0))
                vals.append(np.asarray(f(x, np.array(table["params"][i], dtype=np.float64)), dtype=np.float64))
            v = np.concatenate(vals)
            s1, s2, sa = math.fsum(v), math.fsum(v * v), math.fsum(np.abs(v))
            vol = self.volume(table, i)
            m, se = self.finalize(vol, n, s1, s2)
            out[i] = (m, se, s1, s2, sa, vol, n, 0, 0)
        return out

    def evaluate(self, table: np.ndarray, idx: int, x) -> float:
        xx = np.zeros(12, dtype=np.float64)
        x = np.asarray(x, dtype=np.float64)
        xx[: len(x)] = x
        return float(self.L.orc_eval(self._row(table, idx), xx.ctypes.data))

    def validate(self, table: np.ndarray, idx: int) -> int:
        return int(self.L.orc_validate(self._row(table, idx)))

    def partial_sums(self, table: np.ndarray, idx: int, i0: int, i1: int):
        s1, s2, sa = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self.L.orc_partial_sums(self._row(table, idx), i0, i1, ctypes.byref(s1), ctypes.byref(s2),
                                ctypes.byref(sa))
        return s1.value, s2.value, sa.value

    def volume(self, table: np.ndarray, idx: int) -> float:
        return float(self.L.orc_volume(self._row(table, idx)))

    def finalize(self, volume: float, n: int, s1: float, s2: float):
        m, se = ctypes.c_double(), ctypes.c_double()
        self.L.orc_finalize(volume, n, s1, s2, ctypes.byref(m), ctypes.byref(se))
        return m.value, se.value

    def integrate(self, table: np.ndarray, threads: int | None = None):
        """Integrate every function of ``table``; returns (results, threads used)."""
        table = np.ascontiguousarray(table)
        out = np.zeros(len(table), dtype=RESULT_DTYPE)
        if threads is None:
            threads = os.cpu_count() or 1
        used = self.L.orc_integrate_batch(table.ctypes.data, len(table), out.ctypes.data, int(threads))
        return out, int(used)


_default = None


def default() -> Oracle:
    """The oracle built from ``zmc_oracle.c`` (compiled on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build(force=True)
        _default = Oracle(LIB)
    return _default


def integrate(table: np.ndarray, threads: int | None = None):
    return default().integrate(table, threads)
