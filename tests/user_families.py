"""Run-time integrand families used by the tests: device source and the same
integrand in numpy (float64) for the oracle.  The two are written separately;
only the formula is shared."""

from __future__ import annotations

import numpy as np

from paper_2104_10073_amd import workloads as W

# f = p0 + sum_j p_{2+j} x_j^2 + p1 sin(x_0 x_{d-1})
QUAD_SINE_SRC = r"""
template <class T>
__device__ T mc_user_integrand(const T* x, const T* p, uint32_t d)
{
    T q = p[0];
    for (uint32_t j = 0; j < d; ++j) q += p[2 + j] * x[j] * x[j];
    return q + p[1] * sin(x[0] * x[d - 1]);
}
"""


def quad_sine_np(x, p):
    d = x.shape[1]
    q = np.full(x.shape[0], p[0])
    for j in range(d):
        q = q + p[2 + j] * x[:, j] * x[:, j]
    return q + p[1] * np.sin(x[:, 0] * x[:, d - 1])


# f = 1 / (1 + sum_j (p_{2+j} x_j)^2)
RATIONAL_SRC = r"""
template <class T>
__device__ T mc_user_integrand(const T* x, const T* p, uint32_t d)
{
    T s = T(1);
    for (uint32_t j = 0; j < d; ++j) {
        const T t = p[2 + j] * x[j];
        s += t * t;
    }
    return T(1) / s;
}
"""


def rational_np(x, p):
    s = np.ones(x.shape[0])
    for j in range(x.shape[1]):
        t = p[2 + j] * x[:, j]
        s = s + t * t
    return 1.0 / s


def user_table(n: int, family: int, gen_seed: int, log10_samples=(2.0, 5.0), dim_range=(1, 12), base: int = 0):
    """Seeded functions of a run-time family: boxes lo~U(-1,1), w~U(0.5,2),
    p0~U(-1,1), p1~U(0.5,2), p_{2+j}~U(-2,2); ragged sample counts."""
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    t = np.zeros(n, dtype=W.FUNC_DTYPE)
    for i in range(n):
        d = int(rng.integers(dim_range[0], dim_range[1] + 1))
        lo = rng.uniform(-1.0, 1.0, d)
        w = rng.uniform(0.5, 2.0, d)
        t["family"][i] = family
        t["dim"][i] = d
        t["n_samples"][i] = int(10 ** rng.uniform(*log10_samples))
        t["seed"][i] = W.stream_seed(base, i)
        t["lo"][i, :d] = lo
        t["hi"][i, :d] = lo + w
        t["params"][i, 0] = rng.uniform(-1.0, 1.0)
        t["params"][i, 1] = rng.uniform(0.5, 2.0)
        t["params"][i, 2:2 + d] = rng.uniform(-2.0, 2.0, d)
    return t
