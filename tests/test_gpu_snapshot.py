"""Checkpoint and resume on an MI355X (mc_snapshot / mc_restore).

Requests are snapshotted part way through -- functions spanning launches of a
few tiles or a resident launch's chunks, FP32 rows whose results were sent to
FP64, a grid -- and restored into another context (with another tiling for new
work, launch or resident) and into another process; every result must equal a
run without the interruption bit for bit,
because a tile's samples depend only on the function's seed and the tile's
index and the partials saved are the ones the tree would have summed.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

import gpu_common as G
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _jobs(Z):
    base = W.harmonic_batch(1, 300_000)[0]
    axes = [(W.V0, 6, 5.0, 3.0), (0, 4, 0.5, 0.5)]
    # a grid of constant integrands (every k = 0): the FP32 check sends each row to FP64
    flat = W.harmonic_batch(1, 200_000, gen_seed=7)
    flat["params"][0, W.V0:W.V0 + 4] = 0.0
    return [("table", W.mixed_batch(150, dim_range=(1, 12), log10_samples=(3.0, 6.3), gen_seed=601), Z.PREC_FP32),
            ("table", G.edge_table(), Z.PREC_FP32),
            ("table", W.mixed_batch(40, dim_range=(1, 8), log10_samples=(3.0, 5.5), gen_seed=602), Z.PREC_FP64),
            ("grid", (base, axes), Z.PREC_FP32),
            ("grid", (flat, [(0, 4, 0.5, 0.25)]), Z.PREC_FP32)]


def _submit(c, job):
    kind, t, prec = job
    if kind == "grid":
        return c.submit_grid(t[0], t[1], prec), int(np.prod([a[1] for a in t[1]]))
    return c.submit(t, prec), len(t)


def _same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), (label, f)


RESTORE_SCRIPT = r"""
import sys
import numpy as np
import paper_2104_10073_amd as Z
blobs = [open(p, "rb").read() for p in sys.argv[2:]]
with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
    ids = [c.restore(b) for b in blobs]
    for k, (rid, n) in enumerate(zip(ids, map(int, sys.argv[1].split(",")))):
        np.save(sys.argv[2 + k] + ".npy", c.results(rid, n))
"""


def test_snapshot_restore_bitwise(tmp_path):
    import paper_2104_10073_amd as Z
    jobs = _jobs(Z)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref = []
        for job in jobs:
            rid, n = _submit(c, job)
            ref.append(c.results(rid, n))
    print("snapshot after a few launches of 64 tiles", flush=True)
    with Z.Context(device=0, max_tiles_per_run=64) as a:
        ids = [_submit(a, job) for job in jobs]
        for _ in range(6):
            a.run()
        blobs = [a.snapshot(rid) for rid, _ in ids]
        assert a.pending()[1] > 0, "nothing left to resume"
    print("restore into another context", flush=True)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as b:
        b.set_tuning(seg_log2=np.full(96, 2, dtype=np.uint8))  # new work would tile differently
        rids = [b.restore(blob) for blob in blobs]
        for k, (rid, (_, n)) in enumerate(zip(rids, ids)):
            _same(b.results(rid, n), ref[k], f"request {k}")
    # FP32 rows graded against the oracle as well (the edge table's promoted rows at the FP64 bar)
    edge = jobs[1][1]
    G.check_fp32(ref[1], G.oracle_results(edge), "edge", table=edge)
    assert np.all(ref[4]["precision"] == G.PREC_FP64)  # the constant grid ran in FP64
    print("restore in another process", flush=True)
    paths = []
    for k, blob in enumerate(blobs):
        p = tmp_path / f"snap{k}.bin"
        p.write_bytes(blob)
        paths.append(str(p))
    env = dict(os.environ)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    proc = subprocess.run([sys.executable, "-c", RESTORE_SCRIPT, ",".join(str(n) for _, n in ids), *paths],
                          capture_output=True, text=True, env=env, cwd=ROOT, timeout=240)
    assert proc.returncode == 0, proc.stderr[-3000:]
    for k, p in enumerate(paths):
        _same(np.load(p + ".npy"), ref[k], f"request {k} (other process)")


GRID_SPEC_BYTES = 584  # the parameter grid's description in a snapshot (sizeof(GridSpec))


def _partly_run(blob):
    """Functions of a snapshot that had run some but not all of their tiles."""
    n, n_partials = (int(x) for x in np.frombuffer(blob, dtype="<u8", count=2, offset=24))
    grid = int(np.frombuffer(blob, dtype="<u4", count=1, offset=52)[0])
    fn_bytes = W.FUNC_DTYPE.itemsize
    spec = GRID_SPEC_BYTES if grid else 0
    # (header, grid, functions, progress, results, partials, then the family sources: 8 bytes without any)
    assert len(blob) == 64 + spec + n * (fn_bytes + 16 + 48) + n_partials * 16 + 8
    sf = np.frombuffer(blob, dtype="<u4", count=4 * n, offset=64 + spec + n * fn_bytes).reshape(-1, 4)
    return int(np.count_nonzero((sf[:, 2] > 0) & (sf[:, 2] < sf[:, 1])))


def test_resident_snapshot_restore_bitwise():
    """A resident context's requests snapshotted while its launch runs (the
    launch stops, the snapshot is taken, it starts again) restore into a launch
    and a resident context; a launch context's snapshot restores into a
    resident one; the source contexts finish with the uninterrupted results."""
    import paper_2104_10073_amd as Z
    jobs = _jobs(Z)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref = []
        for job in jobs:
            rid, n = _submit(c, job)
            ref.append(c.results(rid, n))
    print("snapshot a resident context part way through", flush=True)
    with Z.Context(device=0, flags=Z.MC_RESIDENT, max_tiles_per_run=64) as a:
        ids = [_submit(a, job) for job in jobs]
        for _ in range(3):
            a.run()
        res_blobs = [a.snapshot(rid) for rid, _ in ids]
        for k, (rid, n) in enumerate(ids):
            _same(a.results(rid, n), ref[k], f"resident source request {k}")
    print("partly run functions:", [_partly_run(b) for b in res_blobs], flush=True)
    assert sum(_partly_run(b) for b in res_blobs) > 0, "no function was saved part way through"
    print("snapshot a launch context part way through", flush=True)
    with Z.Context(device=0, max_tiles_per_run=64) as a:
        ids = [_submit(a, job) for job in jobs]
        for _ in range(6):
            a.run()
        launch_blobs = [a.snapshot(rid) for rid, _ in ids]
    for label, blobs, flags in (("resident -> launch", res_blobs, Z.MC_NO_GRAPH),
                                ("resident -> resident", res_blobs, Z.MC_RESIDENT),
                                ("launch -> resident", launch_blobs, Z.MC_RESIDENT)):
        print("restore", label, flush=True)
        with Z.Context(device=0, flags=flags) as b:
            rids = [b.restore(blob) for blob in blobs]
            for k, (rid, (_, n)) in enumerate(zip(rids, ids)):
                _same(b.results(rid, n), ref[k], f"{label}: request {k}")


def test_snapshot_of_finished_and_queued_requests():
    import paper_2104_10073_amd as Z
    t = W.mixed_batch(30, dim_range=(1, 6), log10_samples=(3.0, 5.0), gen_seed=611)
    with Z.Context(device=0, flags=Z.MC_NO_GRAPH) as c:
        ref = c.integrate(t)
    # one slot group too few: the second request waits in the queue
    with Z.Context(device=0, max_functions=40) as a:
        r1 = a.submit(t)
        r2 = a.submit(t)
        assert a.pending()[0] == 2
        while r1 not in a.poll():
            a.run()
        done_blob = a.snapshot(r1)
        queued_blob = a.snapshot(r2)
    with Z.Context(device=0) as b:
        q1 = b.restore(done_blob)
        assert q1 in b.poll()  # finished at once
        _same(b.results(q1, len(t)), ref, "finished")
        q2 = b.restore(queued_blob)
        _same(b.results(q2, len(t)), ref, "queued")
