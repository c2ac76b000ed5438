"""Repeated independent runs and the spread statistic of the paper's results.

The paper's test on GPUs (Fig. 1 and its caption) reports each integral as
the mean over independent runs with the standard deviation over those runs as
its error bar.  Each run
of one table differs only in the sample streams: function i of run r takes
the seed ``workloads.stream_seed(base + r, i)``.  Per run, the library's
own per-function standard error estimates the same spread, so over many
runs the variance across runs divided by the mean squared SE is about 1.
"""

import numpy as np

from . import workloads as _W


def reseeded(table: np.ndarray, base: int) -> np.ndarray:
    """A copy of ``table`` whose function i draws the stream of run ``base``
    (seed = base in the high word, i in the low word)."""
    t = np.array(table, copy=True)
    for i in range(len(t)):
        t["seed"][i] = _W.stream_seed(base, i)
    return t


def spread(results) -> dict:
    """Per-function mean over runs and sample standard deviation (n - 1) over
    runs, from a list of result arrays of the same table (one per run).

    Returns ``mean`` (F-bar), ``spread`` (Delta F), ``runs`` and ``rms_se`` (root
    mean square of the per-run standard errors, the quantity ``spread``
    estimates)."""
    runs = len(results)
    if runs < 2:
        raise ValueError("the spread over runs needs at least two runs")
    m = np.stack([np.asarray(r["mean"], dtype=np.float64) for r in results])
    se = np.stack([np.asarray(r["std_error"], dtype=np.float64) for r in results])
    return {"runs": runs, "mean": m.mean(axis=0), "spread": m.std(axis=0, ddof=1),
            "rms_se": np.sqrt((se * se).mean(axis=0))}


def integrate_runs(ctx, table, runs: int = 10, precision: int | None = None, base: int = 0, stream=None):
    """Integrate ``runs`` independent runs of ``table`` on ``ctx`` (run r draws the
    streams of base + r), all submitted before one launch so they share the GPU.
    Returns (list of per-run result arrays, ``spread`` of them)."""
    from ._native import PREC_FP32
    prec = PREC_FP32 if precision is None else precision
    ids = [ctx.submit(reseeded(table, base + r), prec) for r in range(runs)]
    ctx.run(stream)
    res = [ctx.results(rid, len(table)) for rid in ids]
    return res, spread(res)
