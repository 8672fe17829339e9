"""Pins of the oracle's porous-geometry behaviour, its regularizer reading and Eq. 43.

* Composition trajectory (App. of the reading: with the stoichiometric electrode fluxes of Eq. 39
  the steady Maxwell-Stefan fluxes are N_2 = -N_1, N_3 = 0 everywhere in any pore geometry, so
  every node's composition lies on the 1D Stefan-tube curve that starts at the inlet
  composition).  The curve is integrated here from Eq. 19 directly (closed_forms), independent of
  the oracle.  Under the two-relaxation-time collision the walls no longer depend on tau, and the
  steady compositions of a porous slab lie within a few 1e-6 of the curve, shrinking under
  refinement.  Under the paper's BGK collision each species' bounce-back walls sit at a
  tau-dependent place, and the two species have different tau, so the distance is about 1e-3 and
  shrinks at first order.  A wrong sign in Eq. 24 or a gradient that reads solid nodes as zero
  puts nodes 1e-1 or more off the curve.
* The regularizer eps of the flux-norm ratio in Eq. 24 (a reading: the paper is silent on
  vanishing fluxes) moves the steady field by a few 1e-6 and eta by about 2e-7 V between the
  default 1e-2 max|Q| and 1e-4 max|Q|.
* Eq. 43 rederived from the Nernst potentials of the anode reaction written with chemical
  potentials mu_i = mu_i0 + R T ln X_i.
"""

import numpy as np
import pytest

import closed_forms as cf
import oracle
from paper_1809_01600_amd import inputs

# coarse layout of the slab (rows = y, columns = x, 1 = solid); refined by whole factors so that
# every resolution has exactly the same obstacles
BASE = np.array([
    [0, 0, 1, 0, 0, 0, 0, 0],
    [0, 0, 1, 0, 0, 1, 1, 0],
    [0, 0, 0, 0, 0, 1, 1, 0],
    [0, 1, 0, 0, 0, 0, 0, 0],
], dtype=np.uint8)
LENGTH = 20e-3  # m: the composition changes by about 0.25 across the slab at 1 A/cm^2


def _slab(r, tau_ref):
    mask = np.kron(BASE, np.ones((r, r), dtype=np.uint8))[None]
    _, ny, nx = mask.shape
    return inputs.Case(name="slab", lattice="D2Q9", nx=nx, ny=ny, nz=1, dx=LENGTH / nx,
                       tau_ref=tau_ref, X_in=(0.6, 0.3, 0.1), j_A_cm2=1.0, solid=mask)


def _electrode_flux(case):
    """Eq. 39, N_s = -nu_s I / (n F), I in A/m^2."""
    I = case.j_A_cm2 * 1e4
    return np.array([-case.nu[s] * I / (case.n_electrons * cf.FARADAY) for s in range(3)])


def _curve(case, xi):
    return cf.stefan_continuum(case.D_matrix(), case.T, case.p, case.X_in, _electrode_flux(case), xi)


def _steady(case, mode, trt=None, eps=None, tol=1e-12, chunk=1000, max_steps=500_000):
    o = oracle.Oracle(case, ms_mode=mode, eps=eps)
    if trt is not None:
        o.set_trt(trt)
    # start from the open-channel curve along x (closer to the steady state than uniform)
    C = _curve(case, np.arange(case.nx) * case.dx)
    X0 = np.zeros((3,) + case.shape)
    for s in range(3):
        X0[s] = C[s][None, None, :]
    o.init_field(X0)
    prev = o.moments()
    t = 0
    while t < max_steps:
        o.step(chunk)
        t += chunk
        X = o.moments()
        r = oracle.residual(X, prev, o.fluid(), chunk)
        prev = X
        if r < tol:
            return o, X
    raise AssertionError("no steady state within %d steps (r = %g)" % (max_steps, r))


def _distance_to_curve(case, X, fluid):
    """Euclidean distance in (X_1, X_2) from each fluid node to the curve: nearest of a dense
    sampling, refined between the neighbouring samples."""
    pts = np.stack([X[0][fluid], X[1][fluid]], 1)
    xi = np.linspace(-0.3 * LENGTH, 3.0 * LENGTH, 4001)
    C = _curve(case, xi)
    k = np.argmin(np.hypot(pts[:, None, 0] - C[0][None], pts[:, None, 1] - C[1][None]), 1)
    out = np.empty(len(pts))
    for i, p in enumerate(pts):
        fine = np.linspace(xi[max(k[i] - 1, 0)], xi[min(k[i] + 1, len(xi) - 1)], 401)
        Cf = _curve(case, fine)
        out[i] = np.min(np.hypot(p[0] - Cf[0], p[1] - Cf[1]))
    return out


@pytest.mark.parametrize("mode", [oracle.LOCAL_FLUX, oracle.STOICH], ids=["local", "stoich"])
def test_porous_steady_compositions_lie_on_the_stefan_curve_trt(mode):
    dmax = []
    for r in (2, 4):
        case = _slab(r, tau_ref=5.0)
        o, X = _steady(case, mode, trt=0.25)
        d = _distance_to_curve(case, X, o.fluid())
        # the slab does deplete: the nodes spread along a good part of the curve
        assert X[0][o.fluid()].min() < 0.45
        dmax.append(d.max())
    print("TRT distance to the curve, nx = 16, 32:", dmax)
    assert dmax[1] <= 4e-6
    assert dmax[1] < dmax[0]


def test_porous_steady_compositions_approach_the_stefan_curve_bgk():
    dmax = []
    for r in (2, 4):
        case = _slab(r, tau_ref=1.5)
        o, X = _steady(case, oracle.LOCAL_FLUX)
        dmax.append(_distance_to_curve(case, X, o.fluid()).max())
    print("BGK distance to the curve, nx = 16, 32:", dmax)
    assert dmax[1] <= 5e-3
    # first order: the tau-dependent bounce-back walls of the two species
    assert dmax[0] / dmax[1] >= 1.8


def test_flux_ratio_regularizer_barely_moves_the_steady_state():
    case = _slab(4, tau_ref=1.5)
    n_open = oracle.label("D2Q9", case.mask())[1]
    Qmax = np.max(np.abs(oracle.lattice_params(case, n_open)["Q"]))
    o1, X1 = _steady(case, oracle.LOCAL_FLUX, eps=1e-2 * Qmax + 1e-14)
    o2, X2 = _steady(case, oracle.LOCAL_FLUX, eps=1e-4 * Qmax + 1e-14)
    fl = o1.fluid()
    dX = np.max(np.abs(X1[:2] - X2[:2])[:, fl])
    deta = abs(o1.overpotential() - o2.overpotential())
    print("eps 1e-2 Q vs 1e-4 Q: max |dX| %.2e, |d eta| %.2e V" % (dX, deta))
    assert dX <= 1e-5
    assert deta <= 1e-6


def test_overpotential_from_nernst_potentials():
    """Eq. 43 is the difference of the anode's Nernst potentials at the channel and at the
    electrode: for H2 + O^2- -> H2O + 2 e-, E(X) = -(mu_H2O - mu_H2 - mu_O) / (n F) + const with
    mu_i = mu_i0 + R T ln X_i, and eta = E(X_in) - E(X_out).  Arbitrary standard potentials
    cancel."""
    rng = np.random.default_rng(4)
    case = inputs.stefan_tube()
    mu0 = {"H2": -1.3e5, "H2O": -4.2e5, "O": 2.7e5}  # J/mol, arbitrary
    RT = cf.R_GAS * case.T

    def nernst(X):
        mu_h2 = mu0["H2"] + RT * np.log(X[0])
        mu_h2o = mu0["H2O"] + RT * np.log(X[1])
        return -(mu_h2o - mu_h2 - mu0["O"]) / (case.n_electrons * cf.FARADAY)

    for _ in range(20):
        X_in = rng.dirichlet((6, 3, 1))
        X_out = rng.dirichlet((4, 5, 1))
        c = inputs.Case(**{**case.__dict__, "X_in": tuple(X_in)})
        want = nernst(X_in) - nernst(X_out)
        got = oracle.overpotential(c, X_out[:2])
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)) + 1e-15
    # depleting H2 and enriching H2O at the electrode costs voltage
    c = inputs.Case(**{**case.__dict__, "X_in": (0.6, 0.3, 0.1)})
    assert oracle.overpotential(c, np.array([0.5, 0.4])) > 0


def test_oracle_outlet_mean_and_overpotential_on_a_porous_face():
    """X_out in Eq. 43 is the mean over the open outlet-column nodes (a reading); the oracle's
    eta uses exactly those nodes (solid outlet nodes carry no composition)."""
    case = _slab(2, tau_ref=1.5)
    mask = case.mask().copy()
    mask[0, 2:4, -2:] = 1  # close part of the outlet face
    case.solid = mask
    o = oracle.Oracle(case)
    o.init_uniform()
    o.step(300)
    X = o.moments()
    col = o.fluid()[0, :, -1]
    assert 0 < col.sum() < case.ny
    X_out = np.array([X[0][0, :, -1][col].mean(), X[1][0, :, -1][col].mean()])
    assert np.allclose(o.outlet_mean(), X_out, rtol=1e-15, atol=0)
    RT = cf.R_GAS * case.T
    want = RT / (case.n_electrons * cf.FARADAY) * (np.log(X_out[1] / case.X_in[1]) - np.log(X_out[0] / case.X_in[0]))
    assert abs(o.overpotential() - want) <= 1e-12 * abs(want)
