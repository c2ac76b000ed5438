"""Run-time family registration on the host (no GPU): hipRTC compiles the
caller's source into the library's kernels on a validate-only context; ids,
limits, compile errors and validation of family ids."""

import numpy as np
import pytest

import user_families as U
import paper_2104_10073_amd as Z
from paper_2104_10073_amd import workloads as W


def test_register_compiles_and_assigns_ids():
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        a = c.register_family(U.QUAD_SINE_SRC)
        b = c.register_family(U.RATIONAL_SRC)
        assert (a, b) == (Z.MC_FAMILY_USER0, Z.MC_FAMILY_USER0 + 1)
        t = np.concatenate([U.user_table(5, a, 1), U.user_table(5, b, 2), W.mixed_batch(5, gen_seed=3)])
        c.submit(t, Z.PREC_FP32)
        assert c.validate_tiles() >= len(t)


def test_unregistered_family_rejected():
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        t = U.user_table(3, Z.MC_FAMILY_USER0, 1)
        with pytest.raises(Z.McError) as e:
            c.submit(t, Z.PREC_FP32)
        assert e.value.status == -2
        c.register_family(U.RATIONAL_SRC)
        c.submit(t, Z.PREC_FP32)
        t["family"] = Z.MC_FAMILY_USER0 + 1
        with pytest.raises(Z.McError):
            c.submit(t, Z.PREC_FP32)


def test_compile_error_reports_log():
    bad = "template <class T> __device__ T mc_user_integrand(const T* x, const T* p, uint32_t d) { return nope; }"
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.register_family(bad)
        assert e.value.status == -12
        assert "nope" in str(e.value) and "integrand" in str(e.value)
        # a failed compile takes no id
        assert c.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0


def test_missing_entry_point_is_a_compile_error():
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.register_family("__device__ float other(float x) { return x; }")
        assert e.value.status == -12


@pytest.mark.slow
def test_family_limit():
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        for k in range(Z.MC_MAX_USER_FAMILIES):
            assert c.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0 + k
        with pytest.raises(Z.McError) as e:
            c.register_family(U.RATIONAL_SRC)
        assert e.value.status == -1


def test_resident_context_compiles_its_kernel_with_the_family():
    """A resident context compiles its resident kernel again with the caller's
    family (hipRTC; on a validate-only context nothing is loaded) and then
    accepts the family's id."""
    with Z.Context(flags=Z.MC_VALIDATE_ONLY | Z.MC_RESIDENT) as c:
        t = U.user_table(4, Z.MC_FAMILY_USER0, 1)
        with pytest.raises(Z.McError):
            c.submit(t, Z.PREC_FP32)
        assert c.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0
        c.submit(np.concatenate([t, W.mixed_batch(4, gen_seed=5)]), Z.PREC_FP32)


def test_snapshot_carries_family_sources():
    """A snapshot of a request that uses a run-time family holds the family's
    source; it restores into a context that registered the same source, under
    that context's id, and nowhere else."""
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as a:
        a.register_family(U.QUAD_SINE_SRC)
        fb = a.register_family(U.RATIONAL_SRC)
        assert fb == Z.MC_FAMILY_USER0 + 1
        t = np.concatenate([U.user_table(3, fb, 2), W.mixed_batch(3, gen_seed=4)])
        blob = a.snapshot(a.submit(t, Z.PREC_FP32))
    assert U.RATIONAL_SRC.encode() in blob and U.QUAD_SINE_SRC.encode() not in blob
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.restore(blob)
        assert e.value.status == -2  # MC_ERR_UNSUPPORTED_FAMILY: not registered here
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as b:
        assert b.register_family(U.RATIONAL_SRC) == Z.MC_FAMILY_USER0
        blob2 = b.snapshot(b.restore(blob))
    fams = np.frombuffer(blob2, dtype=W.FUNC_DTYPE, count=len(t), offset=64)["family"]
    assert list(fams) == [Z.MC_FAMILY_USER0] * 3 + list(t["family"][3:])
