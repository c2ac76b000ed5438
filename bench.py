"""Benchmark of the batched multi-function direct Monte Carlo path on one MI355X.

Default workload: the paper-scale harmonic batch -- 1000 integrands
a_n cos(k_n.x) + b_n sin(k_n.x) on [0,1]^4, a_n, b_n ~ U(0.5, 2), k components
~ U(5, 30), 10^6 samples each -- evaluated for independent seeds (the paper's
independent evaluations, Fig. 1 caption).  One step = one seed's whole batch
through the hot path: admission and work list, the persistent FP32-evaluation
kernel (Philox samples, box mapping, integrand, compensated sums, segment and
tile reductions), the FP64 finalize pass and the copy of the 1000 results.

Prints one JSON line.  `value` is integrand evaluations per second over the
timed steps (inputs resident before the clock starts).  `roofline` prices the
persistent kernel's algorithmic VALU work against the chip's VALU issue peak
(with the FP32 FLOP and transcendental fractions beside it and the HBM bytes
of the committed counter summary); `run_spread` is the paper's error bar over
the timed seeds.  Beside them: `comparators` (the batched FP64 path, the plain
one-launch-per-function FP64 path, graph replays of the same steps),
`other_configs` (the paper's Eq. (1) cases including the Fig. 1 job, a
parameter grid, a run-time compiled family, the mixed and high-dimensional
batches with their FP32 errors), `serving` (open-loop Poisson arrivals at a
fixed rate under SRPT, FAIR at the same rates, alone-vs-mix equality),
`cpu_baseline` (the serial FP64 CPU oracle on a bounded sample of the same
workload, all host cores) and `oracle_check` (the timed FP32 results against
that oracle, and every function of the mixed and high-dimensional batches in
both precisions).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs, 2.4 GHz peak engine clock, 128 lanes of full-rate 32-bit VALU
# issue per CU per clock (this is what the 157.3 TFLOP/s FP32-vector figure counts:
# 128 FMA lanes x 2 flops).  32x32->64 integer products issue at half that rate.
VALU_SLOT_PEAK = 256 * 128 * 2.4e9   # lane-slots per second


# Sources that determine the persistent kernel's code; HBM counter figures are
# used only while these are unchanged since the counters were taken.
KERNEL_SOURCES = ["paper_2104_10073_amd/csrc/zmc_batched.hip", "paper_2104_10073_amd/csrc/zmc_device_code.hpp",
                  "paper_2104_10073_amd/csrc/zmc_device.hpp"]
WORKLOAD_TAG = "harmonic1000x1e6"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` on the default workload, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (each counter scaled by what it reads
    for a plain copy of known size); None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{WORKLOAD_TAG}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel-sources-sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm-bytes-per-launch"])
    except (KeyError, ValueError):
        return None


def log(msg: str) -> None:
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_slots_per_eval(family: str, d: int, degrees=None) -> float:
    """Full-rate VALU lane-slots one sample of the FP32 path needs (the method's own
    work, no overheads).

    Philox4x32-10: 10 rounds x (2 products at half rate = 4 slots + 2 three-input
    xors = 2 slots) = 60 slots per block, d/4 blocks per sample.  Uniform: 1 slot
    per coordinate.  Accumulation: 4 slots (pairwise quad sums, square,
    compensated add).  A transcendental (cos, exp) issues at a quarter of the
    full rate: 4 slots.  Per family:
      harmonic      d FMAs + fract + cos                      d + 5
      |linear|      d FMAs + the offset's low part            d + 1
      Gaussian      per coordinate sub, mul, FMA; exp         3 d + 4
      polynomial    per coordinate sub, FMA (x), n_j - 1 multiplies (x^n),
                    FMA (1 + p x^n), multiply into the product  sum_j (4 + n_j)
    """
    philox = 60.0 * d / 4.0
    uniform = float(d)
    if family == "harmonic":
        fam = d + 1 + 4
    elif family == "abs_linear":
        fam = d + 1
    elif family == "gaussian":
        fam = 3 * d + 4
    elif family == "poly_product":
        degs = [2.5] * d if degrees is None else list(degrees)[:d]
        fam = sum(4.0 + n for n in degs)
    else:
        raise ValueError(family)
    return philox + uniform + fam + 4.0


FAMILY_NAMES = ("harmonic", "abs_linear", "gaussian", "poly_product")


def algorithmic_slots(table) -> float:
    """Sum over a table's functions of N x the algorithmic slots per sample."""
    total = 0.0
    for i in range(len(table)):
        d = int(table["dim"][i])
        fam = FAMILY_NAMES[int(table["family"][i])]
        degs = table["params"][i, 14:14 + d] if fam == "poly_product" else None
        total += float(table["n_samples"][i]) * algorithmic_slots_per_eval(fam, d, degs)
    return total


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(table, budget_s: float = 10.0):
    from oracle import oracle as O
    orc = O.default()
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    # one core: the first 20 functions (each is serial in the oracle anyway)
    sub = np.ascontiguousarray(table[:20])
    t1 = time.perf_counter()
    orc.integrate(sub, 1)
    one_core = float(sub["n_samples"].sum()) / (time.perf_counter() - t1)
    done = 0
    evals = 0
    used = 1
    most = 1
    parts = []
    t0 = time.perf_counter()
    chunk = max(threads, 16)
    while done < len(table) and time.perf_counter() - t0 < budget_s:
        sub = np.ascontiguousarray(table[done:done + chunk])
        res, used = orc.integrate(sub, threads)
        parts.append(res)
        most = max(most, used)
        done += len(sub)
        evals += int(sub["n_samples"].sum())
    dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": "integrand evals/s", "cores": int(most), "kind": "oracle",
            "sample": f"first {done} of {len(table)} functions of the first timed step's batch in full "
                      f"({evals:.3g} evals, {dt:.1f} s wall, threads over functions)",
            "one_core_value": one_core, "one_core_sample": "first 20 functions of the first timed step's batch",
            "cpu_model": cpu_model(), "cpus_available": int(threads)}, orc, np.concatenate(parts)


def timed_steps(ctx, batches, n, K, Wm, stream):
    """Submit every batch, run Wm untimed launches (which also capture launch
    graphs), then time K launches, one batch each.  Launches are enqueued two
    steps ahead of the results being collected, so the host's work-list building
    and result handling overlap the GPU.  Returns (stats before, seconds,
    results of the K timed batches, stats after)."""
    import torch
    import paper_2104_10073_amd as Z
    ids = [ctx.submit(b, Z.PREC_FP32) for b in batches]
    for i in range(Wm):
        ctx.run(stream)
        ctx.results(ids[i], n)
    torch.cuda.synchronize()
    log(f"warmup done; timing {K} steps")
    st0 = ctx.stats()
    t0 = time.perf_counter()
    results = []
    nxt = Wm
    for _ in range(min(2, K)):
        ctx.run(stream)
        nxt += 1
    for i in range(Wm, Wm + K):
        if nxt < Wm + K:
            ctx.run(stream)
            nxt += 1
        results.append(ctx.results(ids[i], n))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return st0, dt, results, ctx.stats()


def serving_leg(Z, W, stream, args):
    """Continuous batching under open-loop Poisson arrivals at a fixed QPS.

    Requests of floor(10^U(0,3)) functions (mixed forms, dims 1..12, 10^4..10^7
    samples each).  The saturated rate is measured first with every request
    arriving at t = 0 under the headline scheduling policy; the offered QPS is
    `serve_load` times it.  Latency is arrival to results-on-host; the first
    10 % of requests are warm-up.  The other policies are measured at the same
    absolute arrival rates, then the same requests and rates go through a
    resident context (one persistent kernel fed through a ring, no launch per
    batch), and both engines serve a twentieth of the saturated rate (nearly
    alone).
    """
    from paper_2104_10073_amd import serving

    n = args.serve_requests
    reqs = W.serving_requests(n, gen_seed=5)
    flags = 0 if args.graph else Z.MC_NO_GRAPH
    loads = sorted(set([args.serve_load] + [float(x) for x in args.serve_loads.split(",") if x]))
    head = args.serve_policy
    others = [p for p in args.serve_compare.split(",") if p and p != head]

    def make_ctx(name):
        return Z.Context(device=0, flags=flags, policy=SERVE_POLICIES[name](Z), max_tiles_per_run=1 << 15,
                         max_functions=1 << 17, max_partials=1 << 24)

    with make_ctx(head) as ctx:
        sat = serving.serve(ctx, reqs, np.zeros(n), stream)
    sat_qps = n / sat["wall_s"]
    # the mix's algorithmic VALU work per evaluation (the roofline count of the headline)
    mix_slots_per_eval = sum(algorithmic_slots(t) for t in reqs) / float(sat["evals"])
    summ = None
    compare = {}
    for name in [head] + others:
        per_load = []
        with make_ctx(name) as ctx:
            for lf in loads:
                if name == head and lf == args.serve_load:
                    continue
                arr = W.poisson_arrivals(n, lf * sat_qps, seed=5)
                o = serving.serve(ctx, reqs, arr, stream)
                sm = serving.summarize(o, arr)
                sm.update({"load_fraction": lf, "offered_qps": lf * sat_qps})
                per_load.append(sm)
                log(f"serving ({name}) at {lf:.2f} x saturated: p50 {sm['p50_ms']:.2f} ms, p99 {sm['p99_ms']:.2f} ms")
            if name != head:
                compare[name] = per_load
                continue
            qps = args.serve_load * sat_qps
            arrivals = W.poisson_arrivals(n, qps, seed=5)
            run = serving.serve(ctx, reqs, arrivals, stream, keep_results=True)
            summ = serving.summarize(run, arrivals)
            log(f"serving ({name}) at {args.serve_load:.2f} x saturated: p50 {summ['p50_ms']:.2f} ms, "
                f"p99 {summ['p99_ms']:.2f} ms")
            # each result alone equals its result inside the mix
            rng = np.random.Generator(np.random.PCG64(23))
            picks = rng.choice(n, size=min(20, n), replace=False)
            same = True
            for i in picks:
                alone = ctx.integrate(reqs[i], Z.PREC_FP32, stream=stream)
                mixed = run["results"][i]
                same = same and all(np.array_equal(alone[k], mixed[k]) for k in ("mean", "std_error", "sum_f", "sum_f2"))
            head_other = per_load
    summ.update({"engine": "launches", "policy": head, "offered_qps": qps, "saturated_qps": sat_qps,
                 "saturated_evals_per_s": sat["evals"] / sat["wall_s"],
                 "saturated_valu_frac": sat["evals"] / sat["wall_s"] * mix_slots_per_eval / VALU_SLOT_PEAK,
                 "mix_slots_per_eval": mix_slots_per_eval,
                 "load_fraction": args.serve_load, "alone_equals_mix_bitwise": bool(same),
                 "requests_checked_alone": int(len(picks)),
                 "other_loads": head_other,
                 "other_policies_same_arrivals": compare,
                 "workload": "requests of floor(10^U(0,3)) functions, forms mixed, dims U{1..12}, "
                             "10^U(4,7) samples each, Poisson arrivals"})
    if args.serve_resident:
        summ["resident"] = resident_serving(Z, W, serving, reqs, sat_qps, loads, head, others, picks, run, args)
        summ["resident"]["saturated_valu_frac"] = (summ["resident"]["saturated_evals_per_s"] * mix_slots_per_eval /
                                                   VALU_SLOT_PEAK)
    # nearly alone: a twentieth of the saturated rate, both engines (the latency a request
    # sees with the GPU to itself, for comparison with the loaded medians)
    m = min(n, 400)
    arr = W.poisson_arrivals(m, 0.05 * sat_qps, seed=5)
    low = {}
    for engine in ("launches", "resident") if args.serve_resident else ("launches",):
        flags_e = Z.MC_RESIDENT if engine == "resident" else flags
        with Z.Context(device=0, flags=flags_e, policy=SERVE_POLICIES[head](Z),
                       max_tiles_per_run=0 if engine == "resident" else 1 << 15,
                       max_functions=1 << 17, max_partials=1 << 24) as ctx:
            o = serving.serve(ctx, reqs[:m], arr)
        sm = serving.summarize(o, arr)
        sm.update({"load_fraction": 0.05, "offered_qps": 0.05 * sat_qps})
        low[engine] = sm
        log(f"serving ({engine}, {head}) at 0.05 x saturated: p50 {sm['p50_ms']:.3f} ms, p99 {sm['p99_ms']:.2f} ms")
    summ["nearly_alone"] = low
    return summ


def resident_serving(Z, W, serving, reqs, sat_qps, loads, head, others, picks, launch_run, args):
    """The same requests through a resident context (MC_RESIDENT: one persistent kernel fed
    through a ring in pinned memory, no launch per batch), at the same absolute arrival
    rates as the launch engine.  Every result of the headline load is compared bitwise with
    the launch engine's result of the same request, and the sampled requests re-run alone."""
    n = len(reqs)

    def make_ctx(name):
        return Z.Context(device=0, flags=Z.MC_RESIDENT, policy=SERVE_POLICIES[name](Z),
                         max_functions=1 << 17, max_partials=1 << 24)

    with make_ctx(head) as ctx:
        sat = serving.serve(ctx, reqs, np.zeros(n))
    out = {"engine": "resident", "policy": head, "saturated_qps": n / sat["wall_s"],
           "saturated_evals_per_s": sat["evals"] / sat["wall_s"], "per_load": {}, "other_policies": {}}
    log(f"serving (resident, {head}) saturated: {out['saturated_qps']:.0f} requests/s, "
        f"{out['saturated_evals_per_s']:.3g} evals/s")
    for name in [head] + others:
        with make_ctx(name) as ctx:
            for lf in loads:
                arr = W.poisson_arrivals(n, lf * sat_qps, seed=5)
                keep = name == head and lf == args.serve_load
                o = serving.serve(ctx, reqs, arr, keep_results=keep)
                sm = serving.summarize(o, arr)
                sm.update({"load_fraction": lf, "offered_qps": lf * sat_qps})
                log(f"serving (resident, {name}) at {lf:.2f} x saturated: p50 {sm['p50_ms']:.2f} ms, "
                    f"p99 {sm['p99_ms']:.2f} ms")
                if name == head:
                    out["per_load"][f"{lf:.2f}"] = sm
                else:
                    out["other_policies"].setdefault(name, []).append(sm)
                if keep:
                    same_launch = all(np.array_equal(o["results"][i][k], launch_run["results"][i][k])
                                      for i in range(n) for k in ("mean", "std_error", "sum_f", "sum_f2", "n"))
                    same_alone = True
                    for i in picks:
                        alone = ctx.integrate(reqs[i], Z.PREC_FP32)
                        same_alone = same_alone and all(np.array_equal(alone[k], o["results"][i][k])
                                                        for k in ("mean", "std_error", "sum_f", "sum_f2"))
                    out["all_results_equal_launch_engine_bitwise"] = bool(same_launch)
                    out["alone_equals_mix_bitwise"] = bool(same_alone)
                    out["stats"] = {k: v for k, v in ctx.stats().items() if k in ("launches", "functions", "promoted",
                                                                                   "bad_records", "tiles32", "tiles64")}
                    log(f"serving (resident): every result equals the launch engine's: {same_launch}; "
                        f"alone equals mix: {same_alone}")
    return out


SERVE_POLICIES = {
    "fair": lambda Z: Z.MC_SCHED_FAIR,
    "fifo": lambda Z: Z.MC_SCHED_FIFO,
    "srpt": lambda Z: Z.MC_SCHED_SRPT,
}


USER_RATIONAL_SRC = r"""
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


def family_table(Z, W, stream, dims=(1, 2, 4, 8, 12), n_funcs=256, n_samples=1 << 22):
    """FP32 persistent-kernel throughput per (family, dimension): 256 functions of
    one family and dimension, 2^22 samples each (parameters and boxes drawn as in
    the mixed-form batch), one launch; kernel time from HIP events (the second of
    two runs), algorithmic VALU slots from `algorithmic_slots`."""
    rows = []
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH, max_tiles_per_run=1 << 20) as ctx:
        for fam, name in enumerate(FAMILY_NAMES):
            for d in dims:
                t = W.family_batch(fam, d, n_funcs, n_samples)
                ctx.integrate(t, Z.PREC_FP32, stream=stream)
                st0 = ctx.stats()
                ctx.integrate(t, Z.PREC_FP32, stream=stream)
                st1 = ctx.stats()
                ms = st1["fp32_ms"] - st0["fp32_ms"]
                ev = W.total_evals(t)
                slots = algorithmic_slots(t)
                rows.append({"family": name, "dim": d, "evals": ev, "kernel_ms": ms,
                             "evals_per_s": ev / (ms * 1e-3), "slots_per_eval": slots / ev,
                             "valu_frac": slots / (ms * 1e-3) / VALU_SLOT_PEAK,
                             "promoted": st1["promoted"] - st0["promoted"]})
                log(f"family table: {name} d={d}: {ev / (ms * 1e-3):.3g} evals/s, "
                    f"VALU fraction {rows[-1]['valu_frac']:.3f}")
    return rows


def other_configs(Z, W, stream, keep=None):
    """Throughput of the other workloads (each run twice, the second timed): the
    paper's Eq. (1) series (plain FP64 and batched FP32), a parameter grid
    (functional mode), a run-time compiled integrand, the mixed-form batch and
    the high-dimensional batch (batched FP32 with FP64 promotion).  `keep`
    receives the mixed and high-dimensional tables with their FP32 and FP64
    results, for the check against the oracle."""
    import torch
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    # one GPU's share of the headline batch spread over 8 GPUs: 125 of its 1000
    # functions, the same number of tiles per GPU as a cost-balanced eighth of its
    # tile list (the rest of a multi-GPU step, one gather of partials, is not built)
    K = 10
    share = [W.harmonic_batch(125, n_samples=1_000_000, base=2000 + b) for b in range(K + 2)]
    with Z.Context(device=0, flags=Z.MC_VALIDATE_ONLY) as probe:
        probe.submit(share[0], Z.PREC_FP32)
        share_tiles = probe.validate_tiles()  # one batch per launch, as in the headline's steps
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH, policy=Z.MC_SCHED_FIFO, max_tiles_per_run=share_tiles) as sctx:
        st0, dt, _, st1 = timed_steps(sctx, share, 125, K, 2, stream)
        kernel_ms = (st1["fp32_ms"] - st0["fp32_ms"]) / K
        ev = 125 * 1_000_000
        out["harmonic_share_1_of_8"] = {
            "functions": 125, "evals_per_step": ev, "ms_per_step": dt / K * 1e3, "fp32_kernel_ms": kernel_ms,
            "evals_per_s": ev * K / dt, "kernel_fraction_of_step": kernel_ms / (dt / K * 1e3)}
        log(f"harmonic_share_1_of_8: {ev * K / dt:.3g} evals/s, {dt / K * 1e3:.3f} ms per step, "
            f"FP32 kernel {kernel_ms:.3f} ms")
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as ctx:
        # the headline batch end to end from a host table: validation, packing, the
        # PCIe upload of 1000 records, the launch and the results back (the
        # PCIe-inclusive rate; the headline value has the records resident)
        hb = W.harmonic_batch(1000, n_samples=1_000_000, base=77)
        ev = W.total_evals(hb)
        _, th = timed(lambda: ctx.integrate(hb, Z.PREC_FP32, stream=stream))
        out["harmonic_1000x1e6_from_host_table"] = {"evals": ev, "wall_ms": th * 1e3, "evals_per_s": ev / th}
        log(f"harmonic_1000x1e6_from_host_table: {ev / th:.3g} evals/s")
        eq1 = W.eq1_series(n_samples=10_000)
        ev = W.total_evals(eq1)
        _, tp = timed(lambda: ctx.plain_fp64(eq1, stream=stream))
        _, tb = timed(lambda: ctx.integrate(eq1, Z.PREC_FP32, stream=stream))
        out["eq1_100x1e4"] = {"evals": ev, "plain_fp64_ms": tp * 1e3, "batched_fp32_ms": tb * 1e3,
                              "plain_fp64_evals_per_s": ev / tp, "batched_fp32_evals_per_s": ev / tb}
        # the paper's Fig. 1 job: the Eq. (1) series at 10^6 samples, ten independent
        # runs, each function reported as mean and spread over the runs
        fig1 = W.eq1_series(n_samples=1_000_000)
        ev = 10 * W.total_evals(fig1)
        row = {"evals": ev, "runs": 10,
               "paper_context": "about one minute per run (all 100 integrals) on one V100, precision not stated"}
        for pname, prec in (("fp32", Z.PREC_FP32), ("fp64", Z.PREC_FP64)):
            (_, sp), tf = timed(lambda: Z.runs.integrate_runs(ctx, fig1, runs=10, precision=prec, stream=stream))
            row[pname] = {"wall_ms": tf * 1e3, "ms_per_run": tf * 1e3 / 10, "evals_per_s": ev / tf,
                          "mean_spread2_over_se2": float(np.mean((sp["spread"] / sp["rms_se"]) ** 2))}
        out["eq1_fig1_100x1e6_10runs"] = row
        log(f"eq1_fig1_100x1e6_10runs: {row['fp32']['ms_per_run']:.3f} ms per run (fp32), "
            f"{row['fp64']['ms_per_run']:.3f} ms (fp64)")
        # functional mode: one harmonic form over a 64 x 16 parameter grid, records built on the device
        base, axes = W.functional_grid(n_k=64, n_ab=16, n_samples=1_000_000)
        ev = 64 * 16 * 1_000_000
        _, tg = timed(lambda: ctx.integrate_grid(base, axes, Z.PREC_FP32, stream=stream))
        out["grid_64x16_harmonic_1e6"] = {"evals": ev, "wall_ms": tg * 1e3, "evals_per_s": ev / tg}
        log(f"grid_64x16_harmonic_1e6: {ev / tg:.3g} evals/s")
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as ctx:
        # a caller-supplied integrand compiled at run time: 1 / (1 + sum_j (p_j x_j)^2)
        fam = ctx.register_family(USER_RATIONAL_SRC)
        table = W.mixed_batch(1000, dim_range=(1, 12), log10_samples=(6.0, 6.0), gen_seed=7)
        table["family"] = fam
        ev = W.total_evals(table)
        _, tu = timed(lambda: ctx.integrate(table, Z.PREC_FP32, stream=stream))
        out["user_family_1000x1e6_dims1to12"] = {"evals": ev, "wall_ms": tu * 1e3, "evals_per_s": ev / tu}
        log(f"user_family_1000x1e6_dims1to12: {ev / tu:.3g} evals/s")
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as ctx:
        for name, table in (("mixed_2000_dims1to7", W.mixed_batch(2000)),
                            ("highdim_500x1e7_dims8to12", W.high_dim_batch(500))):
            ev = W.total_evals(table)
            # warm-up: the engine clock climbs over the first runs after the GPU has
            # been idle (the mixed batch's FP32 kernel: 4.6, 4.3, 4.1, 4.0 ms)
            for _ in range(3):
                ctx.integrate(table, Z.PREC_FP32, stream=stream)
            torch.cuda.synchronize()
            # kernel times and counts of the timed run only
            st0 = ctx.stats()
            t0 = time.perf_counter()
            r32 = ctx.integrate(table, Z.PREC_FP32, stream=stream)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st1 = ctx.stats()
            runk = {k: st1[k] - st0[k] for k in ("fp32_ms", "fp64_ms", "finalize_ms", "promoted", "launches")}
            r64 = ctx.integrate(table, Z.PREC_FP64, stream=stream)
            if keep is not None:
                keep[name] = (table, r32, r64)
            # FP32-evaluation error per function against the FP64 path (itself equal
            # to the oracle's sums within 1e-12 of sum|f|), in units of the SE
            err = np.abs(r32["mean"] - r64["mean"]) / np.maximum(r64["std_error"], 1e-300)
            near_zero = np.abs(r64["mean"]) < 1e-4
            out[name] = {"evals": ev, "wall_ms": t * 1e3, "evals_per_s": ev / t,
                         "kernel_ms": runk["fp32_ms"] + runk["fp64_ms"] + runk["finalize_ms"],
                         "fp32_kernel_ms": runk["fp32_ms"],
                         "fp32_kernel_valu_frac": algorithmic_slots(table) / (runk["fp32_ms"] * 1e-3) / VALU_SLOT_PEAK,
                         "promoted_to_fp64_per_run": runk["promoted"], "launches_per_run": runk["launches"],
                         "fp32_vs_fp64_max_dF_over_SE": float(err.max()),
                         "fp32_vs_fp64_median_dF_over_SE": float(np.median(err)),
                         "near_zero_functions": int(near_zero.sum()),
                         "near_zero_max_dF_over_SE": float(err[near_zero].max()) if near_zero.any() else None}
            log(f"{name}: {ev / t:.3g} evals/s, FP32 vs FP64 max |dF|/SE {err.max():.2e}, "
                f"FP32 kernel VALU fraction {out[name]['fp32_kernel_valu_frac']:.3f}")
    out["family_table"] = family_table(Z, W, stream)
    return out


def full_oracle_check(orc, table, r32, r64, threads):
    """Every function of a batch against the CPU oracle on the same samples.

    FP32 request: rows that stayed FP32 against the FP32 bar (|dF| <= 0.01 SE of
    the oracle, and the SE ratio), rows the library promoted to FP64 against the
    FP64 bar; FP64 request: S1 within 1e-12 of sum|f| and S2 within 1e-12 of
    itself.  Near-zero integrals (|F_oracle| < 1e-4) are reported apart."""
    t0 = time.perf_counter()
    parts, used = [], 1
    chunk = 8 * threads
    for i0 in range(0, len(table), chunk):
        res, u = orc.integrate(np.ascontiguousarray(table[i0:i0 + chunk]), threads)
        parts.append(res)
        used = max(used, u)
        log(f"  oracle: {min(i0 + chunk, len(table))} of {len(table)} functions, {time.perf_counter() - t0:.0f} s")
    o = np.concatenate(parts)
    dt = time.perf_counter() - t0
    promoted = r32["precision"] == 1
    se = o["stderr"]
    exact = se == 0.0
    f32 = ~promoted & ~exact
    err = np.abs(r32["mean"] - o["mean"]) / np.where(exact, 1.0, se)
    se_dev = np.abs(r32["std_error"] / np.where(exact, 1.0, se) - 1.0)
    near_zero = np.abs(o["mean"]) < 1e-4
    sabs = np.maximum(o["sum_abs"], 1e-300)
    s2 = np.maximum(o["sum_f2"], 1e-300)
    d1_64 = np.abs(r64["sum_f"] - o["sum_f"]) / sabs
    d2_64 = np.abs(r64["sum_f2"] - o["sum_f2"]) / s2
    d1_p = (np.abs(r32["sum_f"] - o["sum_f"]) / sabs)[promoted]
    d2_p = (np.abs(r32["sum_f2"] - o["sum_f2"]) / s2)[promoted]

    def mx(a):
        return float(np.max(a)) if a.size else None

    res = {
        "functions": int(len(table)), "oracle_s": dt, "oracle_threads": int(used),
        "fp32_rows": int(f32.sum()), "promoted_rows": int(promoted.sum()), "constant_rows": int(exact.sum()),
        "fp32_max_dF_over_SE": mx(err[f32]), "fp32_median_dF_over_SE": float(np.median(err[f32])) if f32.any() else None,
        "fp32_max_SE_ratio_dev": mx(se_dev[f32]),
        "near_zero_functions": int(near_zero.sum()), "near_zero_fp32_max_dF_over_SE": mx(err[f32 & near_zero]),
        "promoted_max_dS1_over_sum_abs": mx(d1_p), "promoted_max_dS2_over_S2": mx(d2_p),
        "fp64_max_dS1_over_sum_abs": mx(d1_64), "fp64_max_dS2_over_S2": mx(d2_64),
        "bars": {"fp32_dF_over_SE": 0.01, "fp32_SE_ratio_dev": 1e-3, "fp64_rel": 1e-12},
    }
    worst64 = max([v for v in (mx(d1_64), mx(d2_64), mx(d1_p), mx(d2_p)) if v is not None] or [0.0])
    res["pass"] = bool((res["fp32_max_dF_over_SE"] or 0.0) <= 0.01 and (res["fp32_max_SE_ratio_dev"] or 0.0) < 1e-3
                       and worst64 <= 1e-12 and np.all(r32["status"] == 0) and np.all(r64["status"] == 0))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-funcs", type=int, default=1000)
    ap.add_argument("--n-samples", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="with --autotune 0: persistent-kernel workgroups per CU for the timed contexts")
    ap.add_argument("--autotune", type=float, default=5.0,
                    help="seconds of autotuning (timed apart, before the timed steps); 0 keeps the defaults")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured HIP graphs (then only whole-launch times are measured)")
    ap.add_argument("--serve-loads", default="0.25,0.75",
                    help="further offered loads (fractions of saturated) reported beside the headline one")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' throughput lines")
    ap.add_argument("--no-oracle-full", action="store_true",
                    help="skip the check of every mixed and high-dimensional function against the CPU oracle")
    ap.add_argument("--serve-requests", type=int, default=3000,
                    help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--serve-policy", default="srpt", choices=sorted(SERVE_POLICIES),
                    help="scheduling policy of the headline serving measurement")
    ap.add_argument("--serve-compare", default="fair,srpt",
                    help="policies also measured at the same arrival rates (comma-separated)")
    ap.add_argument("--serve-load", type=float, default=0.5,
                    help="offered load as a fraction of the measured saturated request rate")
    ap.add_argument("--no-serve-resident", dest="serve_resident", action="store_false",
                    help="skip the serving measurement through a resident context (MC_RESIDENT)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a device buffer of this many MiB 5 times (scale for HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-GPU path (tiles sharded across GPUs, one gather "
              "of tile partials) is not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2104_10073_amd as Z
    from paper_2104_10073_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # A plain device-to-device copy of known size: FETCH_SIZE / WRITE_SIZE of its
        # dispatches calibrate the counters read on the integration kernels.
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 5}))
        return
    stream = torch.cuda.current_stream()
    K, Wm = args.steps, args.warmup
    if args.graph:
        # every launch slot captures its graph on first use: warm all three
        Wm = max(Wm, 3)
    log(f"building {K + Wm} batches of {args.n_funcs} functions")
    batches = [W.harmonic_batch(args.n_funcs, n_samples=args.n_samples, base=b) for b in range(K + Wm)]
    evals_per_step = W.total_evals(batches[0])

    # Autotuning on a context of its own (timed apart); its choices are applied
    # to the probe that sizes a launch and to the timed context.
    flags = 0 if args.graph else Z.MC_NO_GRAPH
    tuning = None
    tuned = None
    if args.autotune > 0:
        ta = time.perf_counter()
        with Z.Context(device=0, flags=flags) as tctx:
            tctx.autotune(Z.PREC_FP32, stream=stream, budget_seconds=args.autotune)
            tuned = tctx.get_tuning()
        b, seg = tuned
        tuning = {"autotune_s": time.perf_counter() - ta, "blocks_per_cu": b,
                  "tile_segments_log2_fp32_harmonic_d4": int(seg[0][0][3])}
        log(f"autotuned: {tuning}")
    elif args.blocks_per_cu > 0:
        # a fixed launch shape (for profiles of the tuned configuration without the
        # autotuner's own launches in the trace); tile sizes keep their defaults
        with Z.Context(device=0, flags=Z.MC_VALIDATE_ONLY) as vctx:
            tuned = (args.blocks_per_cu, vctx.get_tuning()[1])
        tuning = {"blocks_per_cu": args.blocks_per_cu, "fixed": True}
    # One launch per step: FIFO scheduling with the per-launch tile cap set to one
    # batch's tile count, so each mc_run takes exactly the next seed's batch.
    probe = Z.Context(device=0, flags=Z.MC_VALIDATE_ONLY)
    if tuned is not None:
        probe.set_tuning(0, tuned[1])
    probe.submit(batches[0], Z.PREC_FP32)
    tiles_per_batch = probe.validate_tiles()
    probe.close()
    ctx = Z.Context(device=0, workspace="torch", flags=flags, policy=Z.MC_SCHED_FIFO,
                    max_tiles_per_run=tiles_per_batch, max_functions=max(65536, 2 * args.n_funcs))
    if tuned is not None:
        ctx.set_tuning(tuned[0], tuned[1])
    n = args.n_funcs
    st0, dt, results, st1 = timed_steps(ctx, batches, n, K, Wm, stream)
    value = evals_per_step * K / dt
    launches = st1["launches"] - st0["launches"]
    assert launches == K and st1["samples"] - st0["samples"] == evals_per_step * K, (st0, st1)
    assert st1["bad_records"] == 0

    # roofline of the persistent kernel from its HIP-event time (graph launches are
    # timed as a whole: FP32 kernel + empty FP64 kernel + finalize)
    key = "graph_ms" if args.graph else "fp32_ms"
    avg_main_s = (st1[key] - st0[key]) / launches * 1e-3
    slots = algorithmic_slots_per_eval("harmonic", 4) * evals_per_step
    achieved = slots / avg_main_s
    # secondary fractions of the same kernel time: FP32 FLOPs (d = 4 harmonic: 4 phase
    # FMAs = 8 flops, fract, cos, 4 for the pairwise and compensated sums: ~14 per
    # evaluation) against the 157.3 TFLOP/s FP32-vector peak, and one v_cos_f32 per
    # evaluation against the transcendental issue rate (a quarter of the full
    # 32-bit lane rate)
    evals_per_s_kernel = evals_per_step / avg_main_s
    secondary = {"fp32_flop_frac": 14.0 * evals_per_s_kernel / 157.3e12,
                 "transcendental_frac": evals_per_s_kernel / (VALU_SLOT_PEAK / 4.0),
                 "flops_per_eval": 14.0, "transcendentals_per_eval": 1.0}
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_SLOT_PEAK / 1e12,
            "unit": "T lane-slots/s (full-rate VALU issue)", "frac": achieved / VALU_SLOT_PEAK,
            "traffic": measured_traffic("zmc_batched_fp32"), "kernel": "zmc_batched_fp32", "kernel_ms": avg_main_s * 1e3,
            "slots_per_eval": algorithmic_slots_per_eval("harmonic", 4), "secondary": secondary}

    out = {
        "metric": "integrand evals/sec + % FP32 VALU peak; serving p50/p99 latency at fixed QPS",
        "value": value, "unit": "integrand evals/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": dt / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded PCG64 parameters, Philox samples)",
        "config": {"workload": f"harmonic batch: {args.n_funcs} integrands a cos(k.x)+b sin(k.x) on [0,1]^4, "
                               f"a,b~U(0.5,2), k~U(5,30), {args.n_samples:.0e} samples each, one seed per step",
                   "functions": args.n_funcs, "samples_per_function": args.n_samples, "dim": 4,
                   "precision": "fp32 evaluation, fp64 reductions and finalize", "tuning": tuning or "default"},
        "roofline": roof,
    }

    log(f"timed: {value:.4g} evals/s, fp32 kernel {avg_main_s * 1e3:.3f} ms/launch")
    if K >= 2:
        # the paper's error statistic over the timed steps (each step one seed of the
        # same functions): the spread over runs against the per-run standard errors
        sp = Z.runs.spread(results)
        q = (sp["spread"] / sp["rms_se"]) ** 2
        out["run_spread"] = {
            "runs": K, "functions": n,
            "statistic": "per function: mean and sample std (n-1) of the estimate over the timed runs",
            "mean_spread2_over_se2": float(np.mean(q)),
            "expected_sd_of_that_mean": float(np.sqrt(2.0 / (K - 1) / n)),
            "median_spread_over_se": float(np.median(np.sqrt(q))),
        }
    if not args.no_comparators:
        # batched FP64 and the plain one-launch-per-function FP64 path on the first timed step's batch
        b0 = batches[Wm]
        torch.cuda.synchronize()
        fp64_ms0 = ctx.stats()["fp64_ms"]
        t1 = time.perf_counter()
        r64 = ctx.integrate(b0, Z.PREC_FP64, stream=stream)
        torch.cuda.synchronize()
        t_b64 = time.perf_counter() - t1
        # the FP64 kernel's own time, from the launches' HIP events
        k64_ms = ctx.stats()["fp64_ms"] - fp64_ms0
        t1 = time.perf_counter()
        rp = ctx.plain_fp64(b0, stream=stream)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t1
        r32 = results[0]
        se = r64["std_error"]
        out["comparators"] = {
            "batched_fp64_evals_per_s": evals_per_step / t_b64,
            "batched_fp64_kernel_ms": k64_ms,
            "batched_fp64_kernel_evals_per_s": evals_per_step / (k64_ms * 1e-3) if k64_ms > 0 else None,
            "plain_fp64_evals_per_s": evals_per_step / t_plain,
            "fp32_over_plain_fp64": value / (evals_per_step / t_plain),
            "fp32_vs_fp64_max_dF_over_SE": float(np.max(np.abs(r32["mean"] - r64["mean"]) / se)),
            "plain_vs_batched_fp64_max_rel_dS1": float(np.max(np.abs(rp["sum_f"] - r64["sum_f"]) /
                                                              np.sqrt(r64["n"] * r64["sum_f2"]))),
        }
    ctx.close()
    if not args.no_comparators and not args.graph:
        # the same steps replayed as captured launch graphs (the context default)
        with Z.Context(device=0, workspace="torch", flags=0, policy=Z.MC_SCHED_FIFO,
                       max_tiles_per_run=tiles_per_batch, max_functions=max(65536, 2 * args.n_funcs)) as gctx:
            if tuned is not None:
                gctx.set_tuning(tuned[0], tuned[1])
            # three warm-up launches, so every launch slot has captured its graph
            # before the clock starts; then the same K seeds as the direct run
            warm = [W.harmonic_batch(args.n_funcs, n_samples=args.n_samples, base=1000 + b) for b in range(3)]
            _, gdt, gres, _ = timed_steps(gctx, warm + batches[Wm:], n, K, 3, stream)
        same = all(np.array_equal(a[f], b[f]) for a, b in zip(results, gres)
                   for f in ("mean", "std_error", "sum_f", "sum_f2"))
        out["comparators"]["graph_replay"] = {"evals_per_s": evals_per_step * K / gdt, "ms_per_step": gdt / K * 1e3,
                                              "results_equal_direct_bitwise": bool(same)}
        log(f"graph replay: {evals_per_step * K / gdt:.4g} evals/s, results equal: {same}")

    kept = {}
    if not args.no_configs:
        log("other workloads")
        out["other_configs"] = other_configs(Z, W, stream, kept)

    if args.serve_requests > 0:
        log("serving leg")
        out["serving"] = serving_leg(Z, W, stream, args)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb, orc, ores = cpu_baseline(batches[Wm])
        out["cpu_baseline"] = cb
        # parity of the timed FP32 results against the oracle: every function the
        # baseline computed of the first timed step, and a fixed tenth of the
        # functions (index = step mod 10) of each later step
        worst = float(np.max(np.abs(results[0]["mean"][:len(ores)] - ores["mean"]) / ores["stderr"]))
        checked = len(ores)
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        for k in range(1, K):
            idx = np.arange(k % 10, n, 10)
            o, _ = orc.integrate(np.ascontiguousarray(batches[Wm + k][idx]), threads)
            worst = max(worst, float(np.max(np.abs(results[k]["mean"][idx] - o["mean"]) / o["stderr"])))
            checked += len(idx)
        out["oracle_check"] = {"functions": int(checked), "first_step_functions": int(len(ores)),
                               "later_steps": int(K - 1), "later_step_fraction": 0.1,
                               "max_dF_over_SE": worst, "bar": 0.01}
        if not args.no_oracle_full:
            # the mixed-form and high-dimensional batches, every function
            for name, key in (("mixed_2000_dims1to7", "mixed"), ("highdim_500x1e7_dims8to12", "highdim")):
                if name in kept:
                    log(f"oracle check of every function: {name}")
                    out["oracle_check"][key] = full_oracle_check(orc, *kept[name], threads)
                    log(f"  {key}: {json.dumps(out['oracle_check'][key])}")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
