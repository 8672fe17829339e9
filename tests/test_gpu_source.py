"""The volumetric source of Eq. 27 (F_a = w_a S on a reaction layer next to the electrolyte),
GPU through the C ABI against the oracle, whose source is pinned on the CPU (exact conservation,
second-order convergence to the continuum): short runs in every storage family from a random
start, one-step conservation, the steady reaction-layer slab, and the API's limits."""

import numpy as np
import pytest

import oracle
from paper_1809_01600_amd import inputs
from test_oracle import run_to_steady

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import lbm_ms  # noqa: E402


def _percolating(lat, shape, seed0, **kw):
    nz, ny, nx = shape
    seed = seed0
    while True:
        c = inputs.random_small(nx, ny, nz, lat, seed=seed, solid_frac=0.2, **kw)
        if oracle.label(lat, c.mask())[1] > 0:
            return c
        seed += 1


def _pair(case, x_first, j_src_A_cm2, precision="fp64", shift=lbm_ms.SHIFT_GLOBAL, ms_mode=lbm_ms.LOCAL_FLUX):
    s = lbm_ms.Solver(case, precision=precision, shift_mode=shift, ms_mode=ms_mode)
    s.set_source(x_first, j_src_A_cm2 * 1.0e4)
    o = oracle.Oracle(case, ms_mode=ms_mode)
    o.set_source(x_first, j_src_A_cm2)
    info = s.get_info()
    assert info.n_source == o.n_source > 0 and info.source_x0 == x_first
    assert np.allclose(np.array(info.S[:2]), [o.p.S[0], o.p.S[1]], rtol=1e-14, atol=0)
    return s, o


@pytest.mark.parametrize("lat,shape,precision,shift,tol", [
    ("D2Q9", (1, 40, 96), "fp64", lbm_ms.SHIFT_GLOBAL, 1e-12),
    ("D3Q19", (9, 11, 40), "fp64", lbm_ms.SHIFT_GLOBAL, 1e-12),
    ("D2Q9", (1, 40, 96), "fp32", lbm_ms.SHIFT_GLOBAL, 2e-6),
    ("D2Q9", (1, 40, 96), "bf16", lbm_ms.SHIFT_NODE, 2e-3),
    ("D3Q19", (9, 11, 40), "fp32", lbm_ms.SHIFT_NODE, 2e-6),
])
def test_source_short_run_matches_oracle(lat, shape, precision, shift, tol):
    """Stoichiometric flux ratio: from a random start the local flux-norm ratio of Eq. 24
    amplifies rounding by orders of magnitude within 100 steps, which would hide the source."""
    case = _percolating(lat, shape, 80, j_A_cm2=0.5, tau_ref=5.0)
    s, o = _pair(case, shape[2] - 10, 1.0, precision, shift, ms_mode=lbm_ms.STOICH)
    X0 = inputs.random_field(case.shape, seed=81, lo=0.2, hi=0.8)
    s.init(X0)
    o.init_field(X0)
    s.step(100)
    o.step(100)
    err = float(np.max(np.abs(s.get_fields() - o.moments())))
    print("%s %s shift %d: max |dX| after 100 steps with the source = %.3e" % (lat, precision, shift, err))
    assert err <= tol
    s.close()


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 40, 96)), ("D3Q19", (9, 11, 40))])
def test_source_conserves_species(lat, shape):
    case = _percolating(lat, shape, 90, j_A_cm2=0.5, tau_ref=5.0)
    s, _ = _pair(case, shape[2] - 10, 1.0)
    info = s.get_info()
    s.init(inputs.random_field(case.shape, seed=91, lo=0.2, hi=0.8))
    for _ in range(3):
        inv, inflow, outflow = s.mass_balance()
        s.step(1)
        inv2, _, _ = s.mass_balance()
        src = info.n_source * np.array(info.S[:2])
        assert np.allclose(inv2 - inv, inflow - outflow + src, rtol=0, atol=1e-13 * np.max(inv))
    s.close()


def test_steady_reaction_layer_slab_matches_oracle():
    """Reaction over the last quarter of a y-invariant slab with a closed outlet face."""
    case = inputs.Case(name="reaction layer", lattice="D2Q9", nx=64, ny=4, nz=1, dx=1.0e-3 / 63.5,
                       tau_ref=10.0, X_in=(0.6, 0.3, 0.1), j_A_cm2=0.0)
    s, o = _pair(case, 48, 2.0, ms_mode=lbm_ms.STOICH)
    s.init()
    o.init_uniform()
    s.converge(1e-14, 3_000_000, check_every=1000)
    Xo, _ = run_to_steady(o, window=2000, tol=1e-14)
    err = float(np.max(np.abs(s.get_fields() - Xo)))
    print("steady reaction-layer slab: max |dX| = %.3e" % err)
    assert err <= 1e-11
    s.close()


def test_source_limits_and_clearing():
    case = _percolating("D2Q9", (1, 20, 48), 95, j_A_cm2=0.5, tau_ref=5.0)
    s = lbm_ms.Solver(case, precision="fp64")
    for bad in (-1, case.nx + 1):
        with pytest.raises(lbm_ms.LbmMsError):
            s.set_source(bad, 1.0e4)
    with pytest.raises(lbm_ms.LbmMsError):
        s.set_source(10, -1.0)
    s.set_source(40, 1.0e4)
    assert s.get_info().n_source > 0
    s.set_source(case.nx, 1.0e4)  # removes it
    info = s.get_info()
    assert info.n_source == 0 and info.S[0] == 0.0 and info.source_x0 == case.nx
    s.set_source(40, 1.0e4)
    s.set_geometry(case.mask())  # a new geometry clears the layer
    assert s.get_info().n_source == 0
    s.close()
