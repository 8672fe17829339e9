"""GPU (HIP, gfx950) parity with the FP64 CPU oracle, through the C ABI.

Tolerances: FP64 storage 1e-12 absolute on mole fractions (values are O(1)) and populations;
reduced precision against the oracle as stated per test.
"""

import numpy as np
import pytest

import oracle
import oracle_windows as ow
from paper_1809_01600_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import lbm_ms  # noqa: E402

FP64_TOL = 1e-12


def _percolating_2d(n, ny, seed0=0, **kw):
    seed = seed0
    while True:
        c = inputs.porous_2d(n=n, ny=ny, seed=seed, **kw)
        if oracle.label("D2Q9", c.mask())[1] > 0:
            return c
        seed += 1


def _pair(case, precision="fp64", ms_mode=lbm_ms.LOCAL_FLUX, inlet_wall=False, **kw):
    s = lbm_ms.Solver(case, precision=precision, ms_mode=ms_mode,
                      inlet_mode=lbm_ms.INLET_WALL if inlet_wall else lbm_ms.INLET_DIRICHLET, **kw)
    # the oracle derives its own regularizer unless the test sets one for both sides
    eps = kw.get("eps_flux", -1.0)
    o = oracle.Oracle(case, ms_mode=ms_mode, inlet_wall=inlet_wall, eps=eps if eps > 0 else None)
    return s, o


def _perm(lattice):
    """index of each product velocity in the oracle's order"""
    e, _ = lbm_ms.lattice_info(lbm_ms.D2Q9 if lattice == "D2Q9" else lbm_ms.D3Q19)
    eo, _ = oracle.velocities(lattice)
    return [eo.tolist().index(v) for v in e.tolist()]


def _check_setup(s, o):
    assert np.array_equal(s.get_geometry(), o.solid)
    info = s.get_info()
    assert info.n_open_outlet == o.n_open
    assert np.allclose(np.array(info.Q[:]), o.lp["Q"], rtol=1e-15, atol=0)
    Dl = np.array(info.Dl[:]).reshape(3, 3)
    assert np.allclose(Dl, o.lp["Dl"], rtol=1e-15, atol=0)
    assert abs(info.eps_flux - oracle.default_eps(o.lp["Q"])) <= 1e-15 * info.eps_flux


def _compare(s, o, tol=FP64_TOL, pops=True):
    X = s.get_fields()
    Xo = o.moments()
    err = np.max(np.abs(X - Xo))
    assert err <= tol, "max |dX| = %g" % err
    if pops:
        f = s.get_populations()
        fo, _, _, _ = o.collide()
        fo = fo[:, _perm(o.lattice)]
        errf = np.max(np.abs(f - fo))
        assert errf <= tol, "max |df*| = %g" % errf
    return err


@pytest.mark.parametrize("mode", [lbm_ms.LOCAL_FLUX, lbm_ms.STOICH])
def test_stefan_tube_fp64_5000_steps(mode):
    case = inputs.stefan_tube()  # 128 x 8, T = 1073 K, 1 atm, j = 0.5 A/cm^2
    s, o = _pair(case, ms_mode=mode)
    _check_setup(s, o)
    s.init()
    o.init_uniform()
    s.step(5000)
    o.step(5000)
    _compare(s, o)
    assert abs(s.overpotential() - o.overpotential()) <= 1e-10 * abs(o.overpotential())


@pytest.mark.parametrize("mode", [lbm_ms.LOCAL_FLUX, lbm_ms.STOICH])
def test_porous_2d_fp64_every_tile_shape(mode):
    case = _percolating_2d(150, 70, seed0=3, tau_ref=5.0)  # ragged in x (150 = 2*64 + 22) and y
    o = None
    for ty, rows in lbm_ms.tile_options(lbm_ms.D2Q9):
        s, o2 = _pair(case, ms_mode=mode, tile_y=ty, chunk_z=rows)
        if o is None:
            o = o2
            _check_setup(s, o)
            o.init_uniform()
            o.step(300)
        s.init()
        s.step(300)
        err = _compare(s, o)
        print("tile %d: max |dX| vs oracle %.3e" % (ty, err))
        s.close()


def test_porous_3d_fp64_every_tile_shape():
    case = inputs.random_small(70, 20, 36, "D3Q19", seed=5, solid_frac=0.25, tau_ref=4.0)
    o = None
    for ty, cz in lbm_ms.tile_options(lbm_ms.D3Q19, lbm_ms.FP64):
        s, o2 = _pair(case, tile_y=ty, chunk_z=cz)
        if o is None:
            o = o2
            _check_setup(s, o)
            o.init_uniform()
            o.step(40)
        s.init()
        s.step(40)
        err = _compare(s, o)
        print("tile (%d, %d): max |dX| vs oracle %.3e" % (ty, cz, err))
        s.close()


def test_3d_stoich_and_short_z():
    # nz smaller than a z chunk, ny smaller than the tile
    case = inputs.random_small(33, 3, 5, "D3Q19", seed=8, solid_frac=0.15, tau_ref=2.0)
    s, o = _pair(case, ms_mode=lbm_ms.STOICH)
    s.init()
    o.init_uniform()
    s.step(80)
    o.step(80)
    _compare(s, o)


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 20, 70)), ("D3Q19", (9, 7, 66))])
@pytest.mark.parametrize("mode,eps", [(lbm_ms.STOICH, -1.0), (lbm_ms.LOCAL_FLUX, 1e-4)])
def test_closed_box_conserves_on_gpu(lat, shape, mode, eps):
    """Closed box (wall inlet, j = 0) from a random field.  With the flux-norm ratio and only the
    1e-14 floor as regularizer this start is chaotic (a one-ulp change of the input grows to 4e-9
    in 200 steps on the CPU alone), so that reading runs with eps = 1e-4 here."""
    nz, ny, nx = shape
    case = inputs.random_small(nx, ny, nz, lat, seed=13, solid_frac=0.2, j_A_cm2=0.0)
    s, o = _pair(case, ms_mode=mode, inlet_wall=True, eps_flux=eps)
    X0 = inputs.random_field(shape, seed=14)
    s.init(X0)
    o.init_field(X0)
    inv0, _, _ = s.mass_balance()
    s.step(200)
    o.step(200)
    inv1, inflow, outflow = s.mass_balance()
    assert np.all(np.abs(inv1 - inv0) <= 1e-13 * inv0)
    assert np.all(np.abs(inflow) < 1e-15) and np.all(np.abs(outflow) < 1e-15)
    _compare(s, o, pops=False)


def test_mass_balance_matches_oracle():
    case = _percolating_2d(96, 40, seed0=1, tau_ref=3.0)
    s, o = _pair(case)
    s.init()
    o.init_uniform()
    s.step(20)
    o.step(20)
    for _ in range(3):
        inv, inflow, outflow = s.mass_balance()
        assert np.allclose(inv, o.inventory(), rtol=1e-13, atol=0)
        oin, oout, _ = o.step_stats()
        s.step(1)
        assert np.allclose(inflow, oin, rtol=1e-11, atol=1e-15)
        assert np.allclose(outflow, oout, rtol=1e-11, atol=1e-15)
        assert np.allclose(outflow, s.get_info().Q[:2] * np.array([1.0, 1.0]) * s.get_info().n_open_outlet,
                           rtol=1e-11, atol=1e-15)
        inv2, _, _ = s.mass_balance()
        assert np.allclose(inv2 - inv, inflow - outflow, rtol=0, atol=1e-12)


def test_residual_and_overpotential_match_definitions():
    case = _percolating_2d(80, 48, seed0=2, tau_ref=3.0)
    s, o = _pair(case)
    s.init()
    o.init_uniform()
    s.step(100)
    o.step(100)
    Xa = o.moments()
    s.residual()  # new window
    s.step(50)
    o.step(50)
    r = s.residual()
    ro = oracle.residual(o.moments(), Xa, o.fluid(), 50)
    assert abs(r - ro) <= 1e-10 * ro
    assert np.allclose(s.outlet_mean()[:2], o.outlet_mean(), rtol=0, atol=1e-13)
    assert abs(s.overpotential() - o.overpotential()) <= 1e-9 * abs(o.overpotential())


def test_paper_profile_init():
    case = inputs.stefan_tube(nx=64, ny=4, dx=0.1 / 64, j_A_cm2=1.0, tau_ref=5.0)
    s, o = _pair(case)
    s.init_paper_profile()
    X = s.get_fields()
    P = oracle.paper_profile(case, case.nx)
    for s_ in range(3):
        assert np.max(np.abs(X[s_, 0] - P[s_][None, :])) < 1e-12


def test_init_from_device_and_host_fields_agree():
    case = _percolating_2d(64, 32, seed0=4, tau_ref=3.0)
    s, _ = _pair(case)
    X0 = inputs.random_field(case.shape, seed=3)
    s.init(X0)
    s.step(10)
    a = s.get_fields()
    s.init(torch.tensor(X0, dtype=torch.float64, device="cuda").contiguous())
    s.step(10)
    b = s.get_fields()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision,shift", [("fp64", lbm_ms.SHIFT_GLOBAL), ("fp32", lbm_ms.SHIFT_GLOBAL),
                                             ("bf16", lbm_ms.SHIFT_GLOBAL), ("bf16", lbm_ms.SHIFT_NODE)])
def test_checkpoint_restart_is_bitwise(precision, shift):
    case = _percolating_2d(70, 30, seed0=6, tau_ref=3.0)
    s, _ = _pair(case, precision=precision, shift_mode=shift)
    s.init()
    s.step(30)
    blob = s.save_state()
    s.step(25)
    ref = s.get_populations()
    s2, _ = _pair(case, precision=precision, shift_mode=shift)
    s2.load_state(blob)
    s2.step(25)
    assert np.array_equal(s2.get_populations(), ref)


@pytest.mark.parametrize("precision,shift,tol", [
    ("fp32", lbm_ms.SHIFT_GLOBAL, 2e-6),
    ("fp16", lbm_ms.SHIFT_GLOBAL, 2e-4),
    ("bf16", lbm_ms.SHIFT_GLOBAL, 2e-3),
    ("fp32", lbm_ms.SHIFT_NODE, 2e-6),
    ("fp16", lbm_ms.SHIFT_NODE, 2e-4),
    ("bf16", lbm_ms.SHIFT_NODE, 2e-3),
])
def test_reduced_precision_short_run(precision, shift, tol):
    case = _percolating_2d(96, 40, seed0=5, tau_ref=5.0)
    s, o = _pair(case, precision=precision, shift_mode=shift)
    s.init()
    o.init_uniform()
    s.step(200)
    o.step(200)
    err = np.max(np.abs(s.get_fields() - o.moments()))
    print("precision %s shift %d: max |dX| after 200 steps = %.3e" % (precision, shift, err))
    assert err <= tol


@pytest.mark.parametrize("precision,shift,tol", [
    ("fp32", lbm_ms.SHIFT_GLOBAL, 2e-6),
    ("fp32", lbm_ms.SHIFT_NODE, 2e-6),
    ("bf16", lbm_ms.SHIFT_GLOBAL, 2e-3),
    ("fp16", lbm_ms.SHIFT_NODE, 2e-4),
    ("bf16", lbm_ms.SHIFT_NODE, 2e-3),
])
def test_reduced_precision_short_run_3d(precision, shift, tol):
    """D3Q19 storage modes against the FP64 oracle (same bounds as the 2D run), on a block that
    spans several tiles in x and y, two z chunks and ragged tails, with both x faces open."""
    case = inputs.random_small(70, 11, 37, "D3Q19", seed=12, solid_frac=0.2, tau_ref=4.0)
    s, o = _pair(case, precision=precision, shift_mode=shift, ms_mode=lbm_ms.STOICH)
    s.init()
    o.init_uniform()
    s.step(100)
    o.step(100)
    err = np.max(np.abs(s.get_fields() - o.moments()))
    print("3D precision %s shift %d: max |dX| after 100 steps = %.3e" % (precision, shift, err))
    assert err <= tol


def test_full_size_porous_2d_fp64_and_fp32():
    """The 1024^2 porous slice in the benchmark's launch shape: a few steps against the oracle."""
    case = inputs.porous_2d()  # 1024 x 1024, seed 2
    o = None
    # FP32 storage rounds each stored population by <= 2^-24 of its value, so the node sum moves
    # by <= ~6e-8 per store; collision arithmetic adds a few ulps: allow 1e-6 per step
    for precision, tol in (("fp64", FP64_TOL), ("fp32", 3e-6)):
        s, o2 = _pair(case, precision=precision)
        if o is None:
            o = o2
            _check_setup(s, o)
            X0 = inputs.random_field(case.shape, seed=9, lo=0.2, hi=0.8)
            o.init_field(X0)
            o.step(3)
        s.init(X0)
        s.step(3)
        err = np.max(np.abs(s.get_fields() - o.moments()))
        print("full size %s: max |dX| after 3 steps = %.3e" % (precision, err))
        assert err <= tol
        s.close()


@pytest.mark.parametrize("precision,x_tol,eta_tol", [
    ("fp32", 1e-7, 1e-8),
    ("bf16", 1e-5, 1e-6),
    ("fp16", 1e-5, 1e-6),
])
def test_node_shift_steady_state_matches_fp64(precision, x_tol, eta_tol):
    """Steady state of the reduced-precision NODE-shift storage against the FP64 path (itself
    pinned to the oracle's steady state in test_gpu_steady.py).  The moment stays in FP64, so
    the rounding of the stored deviations does not stall the slowest mode: the converged fields
    agree to 1e-5 in mole fraction, far below the distance to steady state that a residual of
    1e-8 leaves."""
    case = _percolating_2d(64, 40, seed0=31, tau_ref=3.0, j_A_cm2=1.5)
    ref = lbm_ms.Solver(case, precision="fp64", ms_mode=lbm_ms.STOICH)
    ref.init()
    n_ref, r_ref = ref.converge(1e-12, 2_000_000, check_every=1000)
    s = lbm_ms.Solver(case, precision=precision, shift_mode=lbm_ms.SHIFT_NODE, ms_mode=lbm_ms.STOICH)
    s.init()
    # a 16-bit state may stop short of 1e-12 at its rounding floor; it runs as long as FP64 did
    n, r, rc = s.converge(1e-12, n_ref, check_every=1000, raise_on_fail=False)
    assert rc in (lbm_ms.OK, lbm_ms.E_NOT_CONVERGED)
    dX = np.max(np.abs(s.get_fields() - ref.get_fields()))  # solid nodes read 0 in both
    deta = abs(s.overpotential() - ref.overpotential())
    print("%s node shift: %d steps (FP64 %d), r %.2e, max |dX| %.3e, |d eta| %.3e V"
          % (precision, n, n_ref, r, dX, deta))
    assert dX <= x_tol and deta <= eta_tol
    s.close()
    ref.close()



@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", 3e-6)])
def test_full_size_porous_3d_sampled_columns(precision, tol):
    """The 256^3 porous block in the benchmark's launch shape (default tile), two steps from a
    random start, element by element on sampled x-columns against the oracle stepped on windows
    that reproduce those columns exactly (tests/oracle_windows.py; the whole block is beyond
    the oracle's reach in a test).  Half the columns are open at both the inlet and the outlet."""
    case = inputs.porous_3d()  # 256^3, seed 3
    X0 = inputs.random_field(case.shape, seed=9, lo=0.2, hi=0.8)
    mask, Q, eps = ow.full_inputs(case)
    rng = np.random.Generator(np.random.PCG64(12))
    open_ends = np.argwhere((mask[:, :, 0] == 0) & (mask[:, :, -1] == 0))  # (z, y)
    pick = open_ends[rng.choice(len(open_ends), 6, replace=False)]
    columns = [(int(y), int(z)) for z, y in pick]
    columns += [(int(rng.integers(case.ny)), int(rng.integers(case.nz))) for _ in range(6)]
    rows = ow.column_rows(case, X0, 2, columns, mask, Q, eps)
    s = lbm_ms.Solver(case, precision=precision)
    info = s.get_info()
    assert np.array_equal(s.get_geometry(), mask)
    assert np.allclose(np.array(info.Q[:2]), Q, rtol=1e-15, atol=0)
    s.init(X0)
    s.step(2)
    X = s.get_fields()
    err = max(float(np.max(np.abs(X[:, z, y, :] - row))) for (y, z), row in zip(columns, rows))
    print("256^3 %s tile (%d, %d): max |dX| on %d sampled columns after 2 steps = %.3e"
          % (precision, info.tile_y, info.chunk_z, len(columns), err))
    assert err <= tol
    s.close()


def test_full_size_batch_instances_match_oracle():
    """The benchmark's 64-slice batch (sides 256..1024, FP32, default tile) advanced two steps
    from a random start in one launch per step: the smallest, a middle and the largest instance
    against the oracle stepped on that instance alone."""
    cases = inputs.batch_2d(tau_ref=3.0, accept=lambda solid: lbm_ms.clean_geometry("D2Q9", solid)[1] > 0)
    X0 = [inputs.random_field(c.shape, seed=40 + k, lo=0.2, hi=0.8) for k, c in enumerate(cases)]
    b = lbm_ms.Batch(cases, precision="fp32")
    b.init(np.concatenate([x.reshape(-1) for x in X0]))
    b.step(2)
    sides = [c.nx for c in cases]
    for k in sorted({int(np.argmin(sides)), len(cases) // 2, int(np.argmax(sides))}):
        o = oracle.Oracle(cases[k])
        o.init_field(X0[k])
        o.step(2)
        err = float(np.max(np.abs(b.instance(k).get_fields() - o.moments())))
        print("batch instance %d (side %d): max |dX| after 2 steps = %.3e" % (k, sides[k], err))
        assert err <= 3e-6, k
    b.close()


def test_population_buffer_size_limit_fp64_3d():
    """Largest sizes: an all-fluid FP64 D3Q19 box of 241^3 (14.0 M fluid nodes) puts the last
    population of a buffer about 4.26 GB from its base, just inside the 32-bit offsets; one step
    from a random start conserves each species there.  At 242^3 one buffer would exceed 4 GiB,
    and set_geometry refuses the geometry."""
    case = inputs.Case(name="all fluid 241^3", lattice="D3Q19", nx=241, ny=241, nz=241, tau_ref=3.0)
    s = lbm_ms.Solver(case, precision="fp64")
    info = s.get_info()
    assert info.n_fluid == 241 ** 3
    s.init(inputs.random_field(case.shape, seed=23, lo=0.2, hi=0.8))
    inv, inflow, outflow = s.mass_balance()
    s.step(1)
    inv2, _, _ = s.mass_balance()
    err = np.abs((inv2 - inv) - (inflow - outflow))
    print("241^3 all fluid FP64: |change - (in - out)| = %s" % err)
    assert np.all(err <= _conservation_tol("fp64", 19, info.n_fluid, inv))
    assert np.all(np.isfinite(s.get_fields()))
    s.close()
    big = inputs.Case(name="all fluid 242^3", lattice="D3Q19", nx=242, ny=242, nz=242, tau_ref=3.0)
    with pytest.raises(lbm_ms.LbmMsError) as e:
        lbm_ms.Solver(big, precision="fp64")
    assert "4 GiB" in str(e.value)


def _conservation_tol(precision, q, n_fluid, inv):
    """Bound on |change of inventory - (inflow - outflow)| over one step from rounding alone.
    FP64: two tree reductions of the inventory, each within ~log2(N) eps of it.  FP32 storage: each
    of the q n_fluid stored values (deviations from the reference, below 1/3 in size) is rounded
    once per step to half an ulp, at most 2^-26; the rounding errors are taken as independent, so
    their sum stays within 8 standard deviations of sqrt(q n_fluid) 2^-26 / sqrt(3)."""
    if precision == "fp64":
        return 2.0 * np.log2(n_fluid) * 2.0 ** -52 * inv
    return np.full(2, 8.0 * np.sqrt(q * n_fluid) * 2.0 ** -26 / np.sqrt(3.0))


def _outflow_tol(precision, info):
    """Bound on |outflow - Q_s n_open| from rounding: the populations that cross an outlet node's
    face sum in size to at most 1/3 (their weights sum to 1/6 in either direction, X <= 1); FP32
    storage and arithmetic move that sum by at most a few ulps, taken as 4 ulps of 1/3 per node."""
    scale = np.abs(np.array(info.Q[:2])) * info.n_open_outlet
    if precision == "fp64":
        return 1e-9 * scale
    return np.full(2, 4.0 * 2.0 ** -24 / 3.0 * info.n_open_outlet)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_full_size_porous_3d_conserves_species(precision):
    """The 256^3 porous block in the benchmark's launch configuration: one step changes each
    species' inventory by the inlet inflow minus the outlet outflow, to rounding (the oracle cannot
    step this size within a test; conservation holds at any size), and the outflow is the imposed
    flux Q_s on every open outlet node."""
    case = inputs.porous_3d()  # 256^3, seed 3
    s = lbm_ms.Solver(case, precision=precision)
    info = s.get_info()
    # a random start, so that the inlet face carries a nonzero inflow from the first step
    s.init(inputs.random_field(case.shape, seed=21, lo=0.2, hi=0.8))
    s.step(5)
    for _ in range(2):
        inv, inflow, outflow = s.mass_balance()
        s.step(1)
        inv2, _, _ = s.mass_balance()
        dout = np.abs(outflow - np.array(info.Q[:2]) * info.n_open_outlet)
        err = np.abs((inv2 - inv) - (inflow - outflow))
        tol = _conservation_tol(precision, 19, info.n_fluid, inv)
        print("256^3 %s: inventory %s, in %s, out %s, |out - Q n_open| %s (bound %s), "
              "|error| %s (bound %s)" % (precision, inv, inflow, outflow, dout,
                                         _outflow_tol(precision, info), err, tol), flush=True)
        assert np.all(dout <= _outflow_tol(precision, info))
        assert np.all(err <= tol)
    s.close()


def test_full_size_batch_conserves_species_per_instance():
    """The 64-slice batch of the benchmark (sides 256..1024, FP32) advanced by batched steps from a
    random start: for the smallest, a middle and the largest instance, one step changes the
    inventory by the inflow minus the imposed outflow, to rounding."""
    cases = inputs.batch_2d(tau_ref=3.0, accept=lambda solid: lbm_ms.clean_geometry("D2Q9", solid)[1] > 0)
    b = lbm_ms.Batch(cases, precision="fp32")
    b.init(np.concatenate([inputs.random_field(c.shape, seed=22 + k, lo=0.2, hi=0.8).reshape(-1)
                           for k, c in enumerate(cases)]))
    b.step(5)
    sides = [c.nx for c in cases]
    picks = sorted({int(np.argmin(sides)), len(cases) // 2, int(np.argmax(sides))})
    before = {k: b.instance(k).mass_balance() for k in picks}
    b.step(1)
    for k in picks:
        inv, inflow, outflow = before[k]
        inv2, _, _ = b.instance(k).mass_balance()
        info = b.instance(k).get_info()
        dout = np.abs(outflow - np.array(info.Q[:2]) * info.n_open_outlet)
        err = np.abs((inv2 - inv) - (inflow - outflow))
        tol = _conservation_tol("fp32", 9, info.n_fluid, inv)
        print("batch instance %d (side %d): in %s, out %s, |out - Q n_open| %s (bound %s), "
              "|error| %s (bound %s)" % (k, sides[k], inflow, outflow, dout,
                                         _outflow_tol("fp32", info), err, tol), flush=True)
        assert np.all(dout <= _outflow_tol("fp32", info)), k
        assert np.all(err <= tol), k
    b.close()


_SHAPE_ORACLE = {}


@pytest.mark.parametrize("lat", ["D3Q19", "D3Q7"])
@pytest.mark.parametrize("precision,shift,tol", [("fp32", lbm_ms.SHIFT_GLOBAL, 2e-6),
                                                 ("bf16", lbm_ms.SHIFT_GLOBAL, 2e-3),
                                                 ("fp32", lbm_ms.SHIFT_NODE, 2e-6),
                                                 ("bf16", lbm_ms.SHIFT_NODE, 2e-3)])
def test_3d_launch_shapes_in_every_storage_mode(lat, precision, shift, tol):
    """Every 3D launch shape, 64-plane chunks included (nz = 80 leaves a ragged last chunk), in
    every storage mode against the FP64 oracle (stoichiometric ratio, uniform start; the
    tolerances of the short-run storage tests).  Shapes are not compared bit for bit with each
    other: the compiler may contract FP32 multiply-adds differently in each instantiation."""
    case = inputs.random_small(70, 20, 80, lat, seed=17, solid_frac=0.2, tau_ref=4.0)
    if lat not in _SHAPE_ORACLE:
        o = oracle.Oracle(case, ms_mode=oracle.STOICH)
        o.init_uniform()
        o.step(30)
        _SHAPE_ORACLE[lat] = o.moments()
    Xo = _SHAPE_ORACLE[lat]
    for ty, cz in lbm_ms.tile_options(lbm_ms.LATTICES[lat], precision, shift):
        s = lbm_ms.Solver(case, precision=precision, shift_mode=shift, tile_y=ty, chunk_z=cz,
                          ms_mode=lbm_ms.STOICH)
        s.init()
        s.step(30)
        err = float(np.max(np.abs(s.get_fields() - Xo)))
        s.close()
        print("%s %s shift %d tile (%d, %d): max |dX| %.3e" % (lat, precision, shift, ty, cz, err))
        assert err <= tol, (ty, cz, err)


COMPACTED = [(12, 32), (12, 64), (16, 16), (16, 32), (16, 64)]


@pytest.mark.parametrize("lat", ["D3Q19", "D3Q7"])
@pytest.mark.parametrize("shape,solid,steps", [((130, 17, 40), 0.05, 40), ((33, 3, 5), 0.15, 60),
                                               ((70, 29, 37), 0.45, 40)],
                         ids=["dense", "narrow", "porous"])
def test_3d_compacted_columns_local_flux(lat, shape, solid, steps):
    """The fluid-compacted 3D columns with the paper's local flux ratio (gradients enter tau), in
    FP32 against the FP64 oracle and against the one-voxel-per-lane kernel: a nearly all-fluid
    block (every plane of a column overflows its 512 lanes into a second pass), a box narrower
    than a column with fewer planes than a chunk, and a porous block with ragged columns."""
    nx, ny, nz = shape
    seed = 21
    while True:
        case = inputs.random_small(nx, ny, nz, lat, seed=seed, solid_frac=solid, tau_ref=4.0)
        if oracle.label(lat, case.mask())[1] > 0:
            break
        seed += 1
    o = oracle.Oracle(case)
    o.init_uniform()
    o.step(steps)
    Xo = o.moments()
    ref = lbm_ms.Solver(case, precision="fp32", tile_y=8, chunk_z=32)
    ref.init()
    ref.step(steps)
    Xr = ref.get_fields()
    ref.close()
    err_ref = float(np.max(np.abs(Xr - Xo)))
    print("%s %s: one voxel per lane, max |dX| vs oracle %.3e" % (lat, shape, err_ref))
    assert err_ref <= 2e-6
    for ty, cz in COMPACTED:
        s = lbm_ms.Solver(case, precision="fp32", tile_y=ty, chunk_z=cz)
        s.init()
        s.step(steps)
        X = s.get_fields()
        s.close()
        err = float(np.max(np.abs(X - Xo)))
        d = float(np.max(np.abs(X - Xr)))
        print("  tile (%d, %d): max |dX| vs oracle %.3e, vs one voxel per lane %.3e" % (ty, cz, err, d))
        assert err <= 2e-6 and d <= 1e-6, (ty, cz, err, d)


def test_3d_compacted_columns_rejected_where_not_built():
    case = inputs.random_small(20, 9, 7, "D3Q19", seed=5, solid_frac=0.2, tau_ref=4.0)
    for kw in (dict(precision="fp64"), dict(precision="fp32", shift_mode=lbm_ms.SHIFT_NODE)):
        with pytest.raises(lbm_ms.LbmMsError):
            lbm_ms.Solver(case, tile_y=16, chunk_z=32, **kw)
        s = lbm_ms.Solver(case, tile_y=8, chunk_z=32, **kw)
        with pytest.raises(lbm_ms.LbmMsError):
            s.set_tile(12, 32)
        s.close()
