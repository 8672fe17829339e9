"""The sampled-column oracle (tests/oracle_windows.py) against the whole oracle (no GPU needed):
on a block the oracle can step whole, every sampled column of the windowed runs equals the
whole run's column exactly, inlet and outlet nodes included."""

import numpy as np
import pytest

import oracle
import oracle_windows as ow
from paper_1809_01600_amd import inputs


def _percolating(seed0, lat="D3Q19"):
    seed = seed0
    while True:
        c = inputs.random_small(40, 12, 11, lat, seed=seed, solid_frac=0.2, tau_ref=3.0)
        if oracle.label(lat, c.mask())[1] > 0:
            return c
        seed += 1


@pytest.mark.parametrize("lat,mode", [("D3Q19", oracle.LOCAL_FLUX), ("D3Q7", oracle.LOCAL_FLUX),
                                      ("D3Q7", oracle.STOICH)])
@pytest.mark.parametrize("steps", [1, 2])
def test_windows_reproduce_the_whole_oracle(steps, lat, mode):
    case = _percolating(30, lat)
    X0 = inputs.random_field(case.shape, seed=31, lo=0.2, hi=0.8)
    whole = oracle.Oracle(case, ms_mode=mode)
    whole.init_field(X0)
    whole.step(steps)
    Xw = whole.moments()
    mask, Q, eps = ow.full_inputs(case)
    assert np.array_equal(mask, whole.solid)
    columns = [(0, 0), (5, 3), (11, 10), (6, 7)]  # edges of the periodic block included
    rows = ow.column_rows(case, X0, steps, columns, mask, Q, eps, ms_mode=mode)
    for (y, z), row in zip(columns, rows):
        assert np.array_equal(row, Xw[:, z, y, :]), (y, z, np.max(np.abs(row - Xw[:, z, y, :])))


def test_a_window_too_small_would_differ():
    """The radius is needed: from the equilibrium start two steps reach three nodes out, and
    windows of half-width 2 change every sampled column, so the equality above is not vacuous."""
    case = _percolating(30)
    X0 = inputs.random_field(case.shape, seed=31, lo=0.2, hi=0.8)
    whole = oracle.Oracle(case)
    whole.init_field(X0)
    whole.step(2)
    Xw = whole.moments()
    mask, Q, eps = ow.full_inputs(case)
    columns = [(0, 0), (5, 3), (11, 10), (6, 7)]
    rows = ow.column_rows(case, X0, 2, columns, mask, Q, eps, radius=2)
    assert all(np.max(np.abs(row - Xw[:, z, y, :])) > 1e-6 for (y, z), row in zip(columns, rows))
