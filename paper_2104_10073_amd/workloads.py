"""Seeded synthetic function tables for multi-function direct Monte Carlo.

This module only *draws* integrands: families, dimensions, box domains,
parameters, sample counts and seeds.  It holds none of the estimator's
arithmetic (no random-number stream, no sample mapping, no integrand
evaluation, no reduction), so both the CPU oracle and the GPU library can be
fed from it without sharing any of the method.

The table layout is the one the C ABI reads (``mc_function`` in
``include/zmc.h``): 472 bytes per function, little-endian, no padding::

    uint32 family; uint32 dim; uint64 n_samples; uint64 seed;
    double lo[12]; double hi[12]; double params[32];

Parameter layout per family (``s0 = params[0]``, ``s1 = params[1]``,
``v = params[2:14]``, ``w = params[14:26]``):

* HARMONIC      f = a cos(k.x) + b sin(k.x)           s0=a, s1=b, v=k     (Eq. 1)
* ABS_LINEAR    f = a |c0 + c.x|                      s0=a, s1=c0, v=c    (Eq. 2)
* GAUSSIAN      f = A exp(-|x-mu|^2 / (2 sigma^2))    s0=A, s1=sigma, v=mu
* POLY_PRODUCT  f = prod_j (1 + p_j x_j^{d_j})        v=p, w=d (integers stored as doubles)

The workload shapes follow the paper's experiment (Eq. 1 on [0,1]^4 with
k_n = (n+50)/(2 pi) in every component, "Test on GPUs" and the Fig. 1
caption), its mixed-dimension example (Eq. 2), and the scaled batches used
for measurement.  Every draw uses numpy's PCG64 with a fixed seed.
"""

from __future__ import annotations

import cmath
import math

import numpy as np

MAX_DIM = 12
N_PARAMS = 32

HARMONIC = 0
ABS_LINEAR = 1
GAUSSIAN = 2
POLY_PRODUCT = 3
FAMILY_NAMES = {HARMONIC: "harmonic", ABS_LINEAR: "abs_linear",
                GAUSSIAN: "gaussian", POLY_PRODUCT: "poly_product"}

FUNC_DTYPE = np.dtype([
    ("family", "<u4"),
    ("dim", "<u4"),
    ("n_samples", "<u8"),
    ("seed", "<u8"),
    ("lo", "<f8", (MAX_DIM,)),
    ("hi", "<f8", (MAX_DIM,)),
    ("params", "<f8", (N_PARAMS,)),
])
assert FUNC_DTYPE.itemsize == 472

V0 = 2            # first index of the per-dimension vector v
W0 = 2 + MAX_DIM  # first index of the per-dimension vector w


def empty(n: int) -> np.ndarray:
    return np.zeros(n, dtype=FUNC_DTYPE)


def stream_seed(base: int, index: int) -> int:
    """Per-function 64-bit seed: base run id in the high word, function index in the low word.

    The Philox key of a function is (seed mod 2^32, seed >> 32), so functions of
    one run draw from distinct streams and run ``base`` selects an independent
    repetition of the whole batch (the paper's 10 independent evaluations).
    """
    return ((int(base) & 0xFFFFFFFF) << 32) | (int(index) & 0xFFFFFFFF)


def set_harmonic(t, i, dim, a, b, k, lo, hi):
    t["family"][i] = HARMONIC
    t["dim"][i] = dim
    t["params"][i, 0] = a
    t["params"][i, 1] = b
    t["params"][i, V0:V0 + dim] = k
    t["lo"][i, :dim] = lo
    t["hi"][i, :dim] = hi


def set_abs_linear(t, i, dim, a, c0, c, lo, hi):
    t["family"][i] = ABS_LINEAR
    t["dim"][i] = dim
    t["params"][i, 0] = a
    t["params"][i, 1] = c0
    t["params"][i, V0:V0 + dim] = c
    t["lo"][i, :dim] = lo
    t["hi"][i, :dim] = hi


def set_gaussian(t, i, dim, amp, sigma, mu, lo, hi):
    t["family"][i] = GAUSSIAN
    t["dim"][i] = dim
    t["params"][i, 0] = amp
    t["params"][i, 1] = sigma
    t["params"][i, V0:V0 + dim] = mu
    t["lo"][i, :dim] = lo
    t["hi"][i, :dim] = hi


def set_poly(t, i, dim, p, deg, lo, hi):
    t["family"][i] = POLY_PRODUCT
    t["dim"][i] = dim
    t["params"][i, V0:V0 + dim] = p
    t["params"][i, W0:W0 + dim] = np.asarray(deg, dtype=np.float64)
    t["lo"][i, :dim] = lo
    t["hi"][i, :dim] = hi


# ---------------------------------------------------------------------------
# Quick float64 integrals, used only to *select* near-zero integrands when a
# workload asks for them.  Tests pin the estimator with their own
# high-precision closed forms; nothing here is used to check a result.
# ---------------------------------------------------------------------------

def _harmonic_box_integral(a, b, k, lo, hi):
    prod = 1.0 + 0.0j
    for kj, l, h in zip(k, lo, hi):
        if kj == 0.0:
            prod *= (h - l)
        else:
            prod *= (cmath.exp(1j * kj * h) - cmath.exp(1j * kj * l)) / (1j * kj)
    return a * prod.real + b * prod.imag


def _gaussian_box_integral(amp, sigma, mu, lo, hi):
    s = sigma * math.sqrt(2.0)
    val = amp
    for m, l, h in zip(mu, lo, hi):
        val *= sigma * math.sqrt(math.pi / 2.0) * (math.erf((h - m) / s) - math.erf((l - m) / s))
    return val


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def eq1_series(n_samples: int = 10_000, base: int = 0, n_funcs: int = 100) -> np.ndarray:
    """Eq. (1) with a_n = b_n = 1 on [0,1]^4, k_n = (n+50)/(2 pi) in all four components.

    This is the paper's illustrative example ("Test on GPUs", Fig. 1: n = 1..100,
    10^6 samples per n there); the default sample count is the small FP64 case.
    """
    t = empty(n_funcs)
    for i in range(n_funcs):
        n = i + 1
        kn = (n + 50) / (2.0 * math.pi)
        set_harmonic(t, i, 4, 1.0, 1.0, [kn] * 4, [0.0] * 4, [1.0] * 4)
        t["n_samples"][i] = n_samples
        t["seed"][i] = stream_seed(base, i)
    return t


def eq2_series(n_samples: int = 10_000, base: int = 0) -> np.ndarray:
    """Eq. (2): |x1+x2| for n = 1..49 (2-D) and |x1+x2-x3| for n = 50..100 (3-D).

    Amplitudes a_n = b_n = 1 and unit boxes, as in the Eq. (1) example.
    """
    t = empty(100)
    for i in range(100):
        n = i + 1
        if n < 50:
            set_abs_linear(t, i, 2, 1.0, 0.0, [1.0, 1.0], [0.0, 0.0], [1.0, 1.0])
        else:
            set_abs_linear(t, i, 3, 1.0, 0.0, [1.0, 1.0, -1.0], [0.0] * 3, [1.0] * 3)
        t["n_samples"][i] = n_samples
        t["seed"][i] = stream_seed(base, i)
    return t


def harmonic_batch(n_funcs: int = 1000, n_samples: int = 1_000_000, base: int = 0,
                   gen_seed: int = 2) -> np.ndarray:
    """Paper-scale harmonic batch: a_n, b_n ~ U(0.5, 2), k components ~ U(5, 30), [0,1]^4.

    Parameters are drawn once from ``gen_seed``; ``base`` only changes the
    sample streams, so bases 0..9 are ten independent evaluations of the
    same 1000 integrals.
    """
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    t = empty(n_funcs)
    a = rng.uniform(0.5, 2.0, n_funcs)
    b = rng.uniform(0.5, 2.0, n_funcs)
    k = rng.uniform(5.0, 30.0, (n_funcs, 4))
    for i in range(n_funcs):
        set_harmonic(t, i, 4, a[i], b[i], k[i], [0.0] * 4, [1.0] * 4)
        t["n_samples"][i] = n_samples
        t["seed"][i] = stream_seed(base, i)
    return t


def _draw_mixed(rng, t, i, dim, fam=None):
    """One function of the mixed-form batch: family uniform over the four families
    (or the given one), parameters and box drawn as for that batch."""
    if fam is None:
        fam = int(rng.integers(0, 4))
    lo = rng.uniform(-1.0, 1.0, dim)
    w = rng.uniform(0.5, 2.0, dim)
    hi = lo + w
    if fam == HARMONIC:
        set_harmonic(t, i, dim, rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0),
                     rng.uniform(1.0, 30.0, dim), lo, hi)
    elif fam == ABS_LINEAR:
        c = np.where(rng.integers(0, 2, dim) == 1, 1.0, -1.0)
        set_abs_linear(t, i, dim, 1.0, 0.0, c, lo, hi)
    elif fam == GAUSSIAN:
        mu = rng.uniform(lo, hi)
        set_gaussian(t, i, dim, 1.0, rng.uniform(0.1, 1.0), mu, lo, hi)
    else:
        set_poly(t, i, dim, rng.uniform(-1.0, 1.0, dim), rng.integers(1, 5, dim), lo, hi)


def _log_uniform_count(rng, lo_exp: float, hi_exp: float) -> int:
    return int(math.floor(10.0 ** rng.uniform(lo_exp, hi_exp)))


def mixed_batch(n_funcs: int = 2000, dim_range=(1, 7), log10_samples=(4.0, 7.0), base: int = 0,
                gen_seed: int = 3, sample_scale: float = 1.0) -> np.ndarray:
    """Mixed-form, mixed-dimension batch (harmonic / |c.x| / Gaussian / product polynomial).

    dim ~ U{dim_range}, per-dimension box [lo, lo+w] with lo ~ U(-1,1), w ~ U(0.5,2),
    samples log-uniform over 10^4..10^7 (``sample_scale`` shrinks them for the
    oracle-sized parity cases, keeping at least 2 samples).
    """
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    t = empty(n_funcs)
    for i in range(n_funcs):
        dim = int(rng.integers(dim_range[0], dim_range[1] + 1))
        _draw_mixed(rng, t, i, dim)
        n = _log_uniform_count(rng, *log10_samples)
        t["n_samples"][i] = max(2, int(n * sample_scale))
        t["seed"][i] = stream_seed(base, i)
    return t


def family_batch(family: int, dim: int, n_funcs: int = 256, n_samples: int = 1 << 22, base: int = 0,
                 gen_seed: int = 9) -> np.ndarray:
    """Functions of one family and one dimension, parameters and boxes drawn as in
    the mixed-form batch, all with the same sample count (for per-(family, d)
    throughput)."""
    rng = np.random.Generator(np.random.PCG64(gen_seed + 97 * family + dim))
    t = empty(n_funcs)
    for i in range(n_funcs):
        _draw_mixed(rng, t, i, dim, family)
        t["n_samples"][i] = n_samples
        t["seed"][i] = stream_seed(base, i)
    return t


def high_dim_batch(n_funcs: int = 500, n_samples: int = 10_000_000, base: int = 0,
                   gen_seed: int = 4, near_zero_every: int = 10,
                   near_zero_limit: float = 1e-4) -> np.ndarray:
    """High-dimensional precision stress: harmonic and Gaussian alternate, dim ~ U{8..12} on [0,1]^d.

    Harmonic: a, b ~ U(0.5, 2), k components ~ U(0.5, 5).  Gaussian: A = 1,
    sigma ~ U(0.1, 1), mu ~ U(box).  Every ``near_zero_every``-th function is
    redrawn until its exact integral is below ``near_zero_limit`` in magnitude.
    """
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    t = empty(n_funcs)
    for i in range(n_funcs):
        want_small = near_zero_every > 0 and (i % near_zero_every) == near_zero_every - 1
        for _attempt in range(100_000):
            dim = int(rng.integers(8, 13))
            lo = np.zeros(dim)
            hi = np.ones(dim)
            if i % 2 == 0:
                a, b = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
                k = rng.uniform(0.5, 5.0, dim)
                val = _harmonic_box_integral(a, b, k, lo, hi)
                if not want_small or abs(val) < near_zero_limit:
                    set_harmonic(t, i, dim, a, b, k, lo, hi)
                    break
            else:
                sigma = rng.uniform(0.1, 1.0)
                mu = rng.uniform(lo, hi)
                val = _gaussian_box_integral(1.0, sigma, mu, lo, hi)
                if not want_small or abs(val) < near_zero_limit:
                    set_gaussian(t, i, dim, 1.0, sigma, mu, lo, hi)
                    break
        else:  # pragma: no cover - the acceptance rate is ~1 %, 10^5 draws never all fail
            raise RuntimeError("near-zero draw did not converge")
        t["n_samples"][i] = n_samples
        t["seed"][i] = stream_seed(base, i)
    return t


def serving_requests(n_requests: int = 3000, gen_seed: int = 5, max_funcs: int = 1000,
                     dim_range=(1, 12), log10_samples=(4.0, 7.0), sample_scale: float = 1.0):
    """Requests for the serving loop: each carries floor(10^U(0, log10 max_funcs)) functions.

    Functions are drawn as in :func:`mixed_batch` with dim ~ U{1..12}; request r
    uses base r for its sample streams.  Returns a list of tables.
    """
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    reqs = []
    top = math.log10(max_funcs)
    for r in range(n_requests):
        count = max(1, int(math.floor(10.0 ** rng.uniform(0.0, top))))
        t = empty(count)
        for i in range(count):
            dim = int(rng.integers(dim_range[0], dim_range[1] + 1))
            _draw_mixed(rng, t, i, dim)
            n = _log_uniform_count(rng, *log10_samples)
            t["n_samples"][i] = max(2, int(n * sample_scale))
            t["seed"][i] = stream_seed(r, i)
        reqs.append(t)
    return reqs


def expand_grid(base: np.ndarray, axes) -> np.ndarray:
    """The table a parameter grid stands for: row i is ``base`` with each axis
    (param, count, start, step) set to start + k*step at the mixed-radix digit k
    of i (axis 0 fastest) and seed base.seed + i."""
    b = np.atleast_1d(base)
    n = int(np.prod([int(a[1]) for a in axes]))
    t = np.repeat(b[:1], n)
    for i in range(n):
        rest = i
        for param, count, start, step in axes:
            k = rest % int(count)
            rest //= int(count)
            t["params"][i, int(param)] = float(start) + float(k) * float(step)
        t["seed"][i] = int(b["seed"][0]) + i
    return t


def functional_grid(n_k: int = 64, n_ab: int = 16, n_samples: int = 100_000, dim: int = 4, base: int = 0):
    """The functional-mode workload: one harmonic form a cos(k.x) + b sin(k.x) on
    [0,1]^dim, k_0 swept over n_k points in [5, 30] and a over n_ab points in
    [0.5, 2]; b = 1 and k_j = 10 for j > 0.  Returns (base row, axes)."""
    t = empty(1)
    t["family"][0] = HARMONIC
    t["dim"][0] = dim
    t["n_samples"][0] = n_samples
    t["seed"][0] = stream_seed(base, 0)
    t["hi"][0, :dim] = 1.0
    t["params"][0, 0] = 1.0
    t["params"][0, 1] = 1.0
    t["params"][0, V0:V0 + dim] = 10.0
    axes = [(V0, n_k, 5.0, 25.0 / max(1, n_k - 1)), (0, n_ab, 0.5, 1.5 / max(1, n_ab - 1))]
    return t, axes


def poisson_arrivals(n: int, qps: float, seed: int = 5) -> np.ndarray:
    """Open-loop Poisson arrival times (seconds from start) at rate ``qps``."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return np.cumsum(rng.exponential(1.0 / qps, n))


def total_evals(t: np.ndarray) -> int:
    return int(t["n_samples"].astype(np.uint64).sum())
