"""The paper's homogenized anode case on the GPU (Sec. 4.1-4.2): the path unchanged, fed by the
Eq. 40-42 diffusivities.  The full 100 x 1000 slab against the oracle step by step; the steady
state of the y-invariant slab against the scheme's exact discrete steady state (a chain of
per-link flux relations) and the continuum Stefan profile; the dilution sweep's eta - eta0
against the continuum."""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_1809_01600_amd import paper_case as pc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import lbm_ms  # noqa: E402


@pytest.mark.parametrize("reading", ["printed", "mean"])
def test_full_slab_matches_oracle(reading):
    case = pc.make_case(0.4, 1.0, reading)  # 100 x 1000
    s = lbm_ms.Solver(case, precision="fp64", ms_mode=lbm_ms.STOICH)
    o = oracle.Oracle(case, ms_mode=oracle.STOICH)
    s.init()
    o.init_uniform()
    s.step(200)
    o.step(200)
    err = float(np.max(np.abs(s.get_fields() - o.moments())))
    print("%s: 100x1000 after 200 steps max |dX| = %.3e" % (reading, err))
    assert err <= 1e-12
    s.close()


def test_steady_slab_is_the_discrete_chain_and_near_the_continuum():
    case = pc.make_case(0.3, 1.0, "printed", ny=4)
    s = lbm_ms.Solver(case, precision="fp64", ms_mode=lbm_ms.STOICH)
    s.init()
    steps, r = s.converge(1e-15, 3_000_000, check_every=1000)
    X = s.get_fields()[:, 0]  # [3, ny, nx]
    lp = oracle.lattice_params(case, case.ny)
    chain = cf.discrete_chain_stoich(lp["Dl"], case.X_in, lp["Q"], case.nx)
    err = float(np.max(np.abs(X[:2] - chain[:, None, :])))
    eta = s.overpotential()
    eta_chain = cf.overpotential(case.T, 2, case.X_in, chain[:, -1])
    N = np.array([1.0, -1.0, 0.0]) * case.j_A_m2 / (2 * cf.FARADAY)
    cont = cf.stefan_continuum(case.D_matrix(), case.T, case.p, case.X_in, N, [(case.nx - 1) * case.dx])
    eta_cont = cf.overpotential(case.T, 2, case.X_in, cont[:2, 0])
    print("steps %d r %.1e: |X - chain| %.2e, eta %.6f mV, chain %.6f mV, continuum %.6f mV"
          % (steps, r, err, 1e3 * eta, 1e3 * eta_chain, 1e3 * eta_cont))
    assert err <= 1e-10
    assert abs(eta - eta_chain) <= 1e-10
    # the scheme is second order in dx: with 100 nodes across the slab the continuum is within a
    # few parts in 1e4 of eta
    assert abs(eta - eta_cont) <= 1e-3 * abs(eta_cont)
    s.close()


def test_dilution_sweep_follows_the_continuum():
    res = pc.sweep(currents=(0.3, 1.0), x_h2=(0.8, 0.5, 0.2), ny=4, log=lambda m: None)
    assert all(v == lbm_ms.OK for v in res["status"])
    for j, rows in res["by_current"].items():
        base = [q for q in rows if q["X_H2"] == 0.8][0]
        assert base["eta_minus_eta0_mV"] == 0.0
        for q in rows:
            if q["X_H2"] == 0.8:
                continue
            # dilution raises the overpotential; the lattice follows the continuum closely
            assert q["eta_minus_eta0_mV"] > 0.0
            assert abs(q["eta_minus_eta0_mV"] - q["continuum_eta_minus_eta0_mV"]) <= 2e-3 * q["eta_mV"] + 1e-3
