"""The C oracle against a literal per-node transcription of the step (tests/literal_step.py) on
tiny porous grids, with solid next to the inlet and outlet columns so that diagonal boundary links
meet solid neighbours, from a random initial field, 50 steps.  The transcription derives its own
lattice units and outlet flux and solves the Maxwell-Stefan systems by another route, so this pins
the oracle's porous rules (one-sided and zero gradients next to solid, bounce-back, the corner
precedence of boundary links over solid) against a second reading of the same statements
(Eq. 24-25, 28-29, 32-37, Sec. 3.3)."""

import dataclasses

import numpy as np
import pytest

import oracle
from literal_step import LiteralStep
from paper_1809_01600_amd import inputs

# 6 x 5, D2Q9: solid at (x=0, y=1) and (x=5, y=2), each between fluid nodes of its column
MASK_2D = np.array([
    [0, 0, 1, 0, 0, 0],
    [1, 0, 0, 0, 1, 0],
    [0, 0, 1, 0, 0, 1],
    [0, 1, 0, 0, 0, 0],
    [0, 0, 0, 1, 0, 0],
], dtype=np.uint8)[None]


def _mask_3d():
    m = np.zeros((3, 4, 4), dtype=np.uint8)
    m[0, 1, 0] = 1      # inlet column
    m[1, 2, 0] = 1
    m[2, 0, 3] = 1      # outlet column
    m[1, 1, 3] = 1
    m[1, 1, 1] = 1      # interior
    m[2, 2, 2] = 1
    m[0, 3, 2] = 1
    return m


def _case(lattice, mask):
    nz, ny, nx = mask.shape
    return inputs.Case(name="literal", lattice=lattice, nx=nx, ny=ny, nz=nz, dx=5e-4,
                       tau_ref=3.0, X_in=(0.55, 0.3, 0.15), j_A_cm2=1.0, solid=mask)


def _random_X(case, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.zeros((3,) + case.shape)
    for s in range(2):
        X[s] = case.X_in[s] + 0.05 * rng.uniform(-1.0, 1.0, case.shape)
    X[2] = 1.0 - X[0] - X[1]
    return X


def _perm(lattice, lit):
    eo, _ = oracle.velocities(lattice)
    return [eo.tolist().index(v) for v in lit.e]


CASES = [("D2Q9", MASK_2D), ("D2Q5", MASK_2D), ("D3Q19", _mask_3d()), ("D3Q7", _mask_3d())]


@pytest.mark.parametrize("lattice,mask", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", [oracle.LOCAL_FLUX, oracle.STOICH], ids=["local", "stoich"])
def test_oracle_equals_literal_transcription(lattice, mask, mode):
    case = _case(lattice, mask)
    o = oracle.Oracle(case, ms_mode=mode)
    # the chosen masks need no clean-up: every fluid node is linked to the inlet column
    assert np.array_equal(o.solid, mask)
    lit = LiteralStep(case, o.solid, mode == oracle.STOICH, eps=o.p.eps)
    assert np.allclose(lit.Q, o.lp["Q"], rtol=1e-14, atol=0)
    X0 = _random_X(case, 7)
    o.init_field(X0)
    f = lit.equilibrium(X0)
    perm = _perm(lattice, lit)
    worst = 0.0
    for t in range(50):
        f, inflow, outflow = lit.step(f)
        st = o.step(1)
        fa = lit.to_array(f)
        err = np.max(np.abs(fa - o.f[:, perm]))
        worst = max(worst, err)
        assert err <= 1e-14, "step %d: max |f_literal - f_oracle| = %g" % (t + 1, err)
        assert np.allclose(inflow, st.inflow[:2], rtol=0, atol=1e-14)
        assert np.allclose(outflow, st.outflow[:2], rtol=0, atol=1e-14)
    # the run moved the state well away from the start, so the rules were exercised
    X = o.moments()
    assert np.max(np.abs(X[:2] - X0[:2])[:, o.fluid()]) > 1e-3
    print("%s mode %d: worst |df| over 50 steps %.2e" % (lattice, mode, worst))


def test_boundary_links_meet_solid_in_the_chosen_masks():
    """The masks do put solid next to fluid in both x-face columns (the corner precedence of
    boundary links over solid is therefore exercised above)."""
    for mask in (MASK_2D, _mask_3d()):
        for col in (0, -1):
            c = mask[:, :, col]
            assert c.any() and not c.all()


def test_literal_relaxation_times_equal_the_oracles():
    case = _case("D2Q9", MASK_2D)
    o = oracle.Oracle(case, ms_mode=oracle.LOCAL_FLUX)
    lit = LiteralStep(case, o.solid, False, eps=o.p.eps)
    X0 = _random_X(case, 3)
    o.init_field(X0)
    _, tau_o, _, _ = o.collide()
    _, tau_l, _ = lit.collide(lit.equilibrium(X0))
    tl = np.array(tau_l).reshape((2,) + case.shape)
    fl = o.fluid()
    assert np.max(np.abs(tl[:, fl] - tau_o[:, fl])) <= 1e-13 * np.max(tau_o[:, fl])
