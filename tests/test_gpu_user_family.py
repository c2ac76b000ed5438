"""Run-time compiled integrand families (hipRTC) against the oracle, on an MI355X.

A request mixes built-in families with two caller-defined ones, so one launch
runs the built-in kernels and both families' kernels over their own parts of
the tile list.  Built-in rows are checked against the oracle's formulas, the
caller's rows against the oracle's samples evaluated by the numpy form of the
same integrand; the bars are those of the built-in families.
"""

import numpy as np
import pytest

import gpu_common as G
import user_families as U
from oracle import oracle as O
from paper_2104_10073_amd import workloads as W

pytestmark = pytest.mark.gpu


def _table(fam_a, fam_b):
    builtin = W.mixed_batch(30, dim_range=(1, 12), log10_samples=(2.0, 5.0), gen_seed=901)
    ua = U.user_table(20, fam_a, gen_seed=902, base=1)
    ub = U.user_table(20, fam_b, gen_seed=903, base=2)
    # edge sizes and dims on the caller's family: partial quads, a single segment, dim 12
    ue = U.user_table(6, fam_a, gen_seed=904, base=3, dim_range=(12, 12))
    ue["n_samples"] = [2, 3, 5, 4095, 4097, 70_001]
    t = np.concatenate([builtin, ua, ub, ue])
    return t, slice(0, 30), [(slice(30, 50), U.quad_sine_np), (slice(50, 70), U.rational_np),
                             (slice(70, 76), U.quad_sine_np)]


def _oracle(t, parts):
    orc = np.zeros(len(t), dtype=O.RESULT_DTYPE)
    b, users = parts
    orc[b] = G.oracle_results(t[b])
    for sl, f in users:
        orc[sl] = O.default().integrate_user(t[sl], f)
    return orc


@pytest.fixture(scope="module")
def setup():
    import paper_2104_10073_amd as Z
    c = Z.Context(device=0, flags=Z.MC_NO_GRAPH)
    fa = c.register_family(U.QUAD_SINE_SRC)
    fb = c.register_family(U.RATIONAL_SRC)
    t, b, users = _table(fa, fb)
    orc = _oracle(t, (b, users))
    yield c, t, orc, (fa, fb)
    c.close()


def test_user_families_fp64(setup):
    import paper_2104_10073_amd as Z
    c, t, orc, _ = setup
    print("user families fp64: functions", len(t), flush=True)
    G.check_fp64(c.integrate(t, Z.PREC_FP64), orc, "user fp64")


def test_user_families_fp32(setup):
    import paper_2104_10073_amd as Z
    c, t, orc, _ = setup
    print("user families fp32: functions", len(t), flush=True)
    info = G.check_fp32(c.integrate(t, Z.PREC_FP32), orc, "user fp32", table=t)
    must, may = G.expected_promotion(t, orc)
    assert int(np.count_nonzero(must)) <= info["fp64"] <= int(np.count_nonzero(may)), info


def test_user_family_alone_equals_mixed(setup):
    import paper_2104_10073_amd as Z
    c, t, _, _ = setup
    mixed = c.integrate(t, Z.PREC_FP32)
    alone = c.integrate(t[30:50], Z.PREC_FP32)
    for k in ("mean", "std_error", "sum_f", "sum_f2"):
        assert np.array_equal(alone[k], mixed[k][30:50]), k


def test_user_family_on_graph_context_matches(setup):
    """A context that would replay graphs launches directly once families are
    registered; results are the same bits."""
    import paper_2104_10073_amd as Z
    c, t, _, _ = setup
    ref = c.integrate(t, Z.PREC_FP32)
    with Z.Context(device=0) as g:
        assert g.register_family(U.QUAD_SINE_SRC) == Z.MC_FAMILY_USER0
        assert g.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0 + 1
        for _ in range(2):
            got = g.integrate(t, Z.PREC_FP32)
            for k in ("mean", "std_error", "sum_f", "sum_f2"):
                assert np.array_equal(got[k], ref[k]), k


def test_user_families_on_a_resident_context(setup):
    """A resident context compiles its kernel again at each registration; the
    second registration replaces the kernel while the first one's launch is
    serving a request.  Results are those of the launch context, bit for bit,
    in FP32 (with its promotions) and FP64."""
    import paper_2104_10073_amd as Z
    c, t, _, _ = setup
    ref32, ref64 = c.integrate(t, Z.PREC_FP32), c.integrate(t, Z.PREC_FP64)
    fields = ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision")
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as r:
        assert r.register_family(U.QUAD_SINE_SRC) == Z.MC_FAMILY_USER0
        first = t[:50]  # built-in rows and the first family's
        rid = r.submit(first, Z.PREC_FP32)
        r.run()
        print("resident: second family registered while a request runs", flush=True)
        assert r.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0 + 1
        got_first = r.results(rid, len(first))
        got32, got64 = r.integrate(t, Z.PREC_FP32), r.integrate(t, Z.PREC_FP64)
        assert r.stats()["bad_records"] == 0
    for k in fields:
        assert np.array_equal(got_first[k], ref32[k][:50]), ("first", k)
        assert np.array_equal(got32[k], ref32[k]), ("fp32", k)
        assert np.array_equal(got64[k], ref64[k]), ("fp64", k)


def test_user_family_snapshot_resumes_under_other_ids(setup):
    """A request that uses both caller families, snapshotted part way through in
    a launch context, resumes in a resident context that registered the same
    sources in the other order (the snapshot carries the sources; the request
    takes the resident context's ids): results bit for bit as uninterrupted."""
    import paper_2104_10073_amd as Z
    c, t, _, _ = setup
    ref = c.integrate(t, Z.PREC_FP32)
    with Z.Context(device=0, max_tiles_per_run=16) as a:
        a.register_family(U.QUAD_SINE_SRC)
        a.register_family(U.RATIONAL_SRC)
        rid = a.submit(t, Z.PREC_FP32)
        for _ in range(3):
            a.run()
        blob = a.snapshot(rid)
        assert a.pending()[1] > 0, "nothing left to resume"
    with Z.Context(device=0, flags=Z.MC_RESIDENT) as b:
        assert b.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0
        assert b.register_family(U.QUAD_SINE_SRC) == Z.MC_FAMILY_USER0 + 1
        got = b.results(b.restore(blob), len(t))
    for k in ("mean", "std_error", "sum_f", "sum_f2", "n", "status", "precision"):
        assert np.array_equal(got[k], ref[k]), k


def test_plain_path_rejects_user_family(setup):
    import paper_2104_10073_amd as Z
    c, t, _, _ = setup
    with pytest.raises(Z.McError) as e:
        c.plain_fp64(t[30:32])
    assert e.value.status == -2


def test_user_family_far_narrow_box_runs_in_fp64(setup):
    """A run-time family sees x in FP32 absolute coordinates, so a box far from the
    origin relative to its width (K sqrt(N) > 24200) runs in FP64 from submit and
    matches the oracle at the FP64 bar; the same function near the origin stays FP32."""
    import paper_2104_10073_amd as Z
    c, _, _, (fa, fb) = setup
    t = U.user_table(2, fb, gen_seed=905, log10_samples=(5.0, 5.0), dim_range=(2, 2), base=4)
    t["lo"][0, :2] = [200.0, -0.5]
    t["hi"][0, :2] = [200.05, 0.5]                      # K = 4001, K sqrt(N) ~ 1.3e6
    r = c.integrate(t, Z.PREC_FP32)
    assert r["precision"].tolist() == [1, 0]
    orc = O.default().integrate_user(t, U.rational_np)
    G.check_fp64(r[:1], orc[:1], "far box, run-time family")
    G.check_fp32(r[1:], orc[1:], "box near the origin, run-time family")
