"""Parameter-grid submission (functional mode) on the host: expansion order,
seeds, validation and errors, on a validate-only context."""

import numpy as np
import pytest

import paper_2104_10073_amd as Z
from paper_2104_10073_amd import workloads as W


def test_grid_takes_the_tiles_of_its_table():
    base, axes = W.functional_grid(n_k=7, n_ab=3, n_samples=300_000)
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        c.submit_grid(base, axes)
        grid_tiles = c.validate_tiles()
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        c.submit(W.expand_grid(base, axes))
        assert c.validate_tiles() == grid_tiles > 21


def test_expand_grid_order_and_seeds():
    base, _ = W.functional_grid(n_k=2, n_ab=2)
    axes = [(2, 3, 1.0, 0.5), (0, 2, -1.0, 2.0)]
    t = W.expand_grid(base, axes)
    assert len(t) == 6
    assert list(t["params"][:, 2]) == [1.0, 1.5, 2.0, 1.0, 1.5, 2.0]
    assert list(t["params"][:, 0]) == [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    assert list(t["seed"]) == [int(base["seed"][0]) + i for i in range(6)]


@pytest.mark.parametrize("axes,status", [
    ([], -1),
    ([(32, 2, 0.0, 1.0)], -1),
    ([(2, 0, 0.0, 1.0)], -1),
    ([(2, 2, 0.0, 1.0), (2, 3, 0.0, 1.0)], -1),
    ([(2, 2, 0.0, 1.0)] * 5, -1),
    ([(1, 3, -1.0, 1.0)], -5),                # sigma <= 0 on a Gaussian: the bad point's index is reported
    ([(2, 300, 0.0, 1.0), (3, 300, 0.0, 1.0)], -7),  # more functions than the context's slots
])
def test_grid_errors(axes, status):
    base = W.mixed_batch(40, gen_seed=3)
    g = base[base["family"] == W.GAUSSIAN][:1]
    assert len(g) == 1
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.submit_grid(g, axes)
        assert e.value.status == status
        if status == -5:
            assert "function 0" in str(e.value)


def test_grid_seed_wrap_rejected():
    base, axes = W.functional_grid(n_k=4, n_ab=1)
    base["seed"] = np.uint64(2 ** 64 - 2)
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.submit_grid(base, axes)
        assert e.value.status == -1


def test_grid_validation_names_the_failing_point():
    """Each constraint involves one parameter, so the grid is validated axis by
    axis without expanding it; the first failing point is reported by its index."""
    t = W.mixed_batch(40, gen_seed=3)
    poly = t[t["family"] == W.POLY_PRODUCT][:1].copy()
    assert len(poly) == 1
    deg0 = W.W0  # degree of coordinate 0
    # axis 0 over a harmless parameter (3 points), axis 1 over the degree: 1, 2.5 (bad), 3.5 (bad)
    axes = [(W.V0, 3, 0.1, 0.1), (deg0, 3, 1.0, 1.5)]
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        with pytest.raises(Z.McError) as e:
            c.submit_grid(poly, axes)
        assert e.value.status == -5
        assert "function 3:" in str(e.value)  # point k = 1 of axis 1 is function 1 * 3


def test_grid_axis_may_override_an_invalid_base_parameter():
    t = W.mixed_batch(40, gen_seed=3)
    g = t[t["family"] == W.GAUSSIAN][:1].copy()
    g["params"][0, 1] = 0.0  # sigma 0 in the base, but every grid point sets it
    with Z.Context(flags=Z.MC_VALIDATE_ONLY) as c:
        c.submit_grid(g, [(1, 4, 0.2, 0.1)])
        assert c.validate_tiles() >= 4
