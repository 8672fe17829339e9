"""Batched launches (one kernel per step over many ragged instances) and hipGraph replay."""

import numpy as np
import pytest

import oracle
from paper_1809_01600_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import lbm_ms  # noqa: E402


def _cases(seed0=100, sizes=((70, 33), (129, 64), (64, 64), (200, 17)), js=(0.4, 1.2, 0.0, 2.0),
           tau_ref=5.0):
    out = []
    seed = seed0
    for (nx, ny), j in zip(sizes, js):
        while True:
            c = inputs.porous_2d(n=nx, ny=ny, seed=seed, j_A_cm2=j, tau_ref=tau_ref, r_lo=3.0, r_hi=8.0)
            seed += 1
            if oracle.label("D2Q9", c.mask())[1] > 0:
                break
        out.append(c)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_equals_single_instances(precision):
    cases = _cases()
    b = lbm_ms.Batch(cases, precision=precision, tile_y=8)
    b.init()
    b.step(120)
    for k, c in enumerate(cases):
        s = lbm_ms.Solver(c, precision=precision, tile_y=8)
        s.init()
        s.step(120)
        assert np.array_equal(b.instance(k).get_fields(), s.get_fields()), k
        s.close()
    a, nf, t = b.stats()
    assert a == len(cases) and t > 0
    b.close()


def test_batch_fp64_matches_oracle():
    cases = _cases(seed0=300, sizes=((90, 40), (66, 20)), js=(1.0, 0.5))
    b = lbm_ms.Batch(cases, precision="fp64", tile_y=4)
    b.init()
    b.step(150)
    for k, c in enumerate(cases):
        o = oracle.Oracle(c)
        o.init_uniform()
        o.step(150)
        assert np.max(np.abs(b.instance(k).get_fields() - o.moments())) < 1e-12
    b.close()


def test_graph_replays_equal_eager_steps():
    """Graph replays with eager work and synchronizations between them equal eager launches."""
    cases = _cases(seed0=500)
    g = lbm_ms.Batch(cases, precision="fp32", tile_y=8)
    e = lbm_ms.Batch(cases, precision="fp32", tile_y=8)
    g.init()
    e.init()
    e.use_graphs(False)
    for rep in range(4):
        g.converge(0.0, 50, check_every=50, raise_on_fail=False)  # one captured 50-step chunk
        e.step(50)
        for k in range(len(cases)):
            assert np.array_equal(g.instance(k).get_fields(), e.instance(k).get_fields()), (rep, k)
    g.close()
    e.close()


def test_converged_instances_retire():
    """Instances leave the work list when their residual falls below tol; the rest go on."""
    cases = [inputs.stefan_tube(nx=24, ny=8, tau_ref=20.0, j_A_cm2=0.0, dx=1e-4),
             inputs.stefan_tube(nx=32, ny=8, tau_ref=20.0, j_A_cm2=1.0, dx=1e-4),
             inputs.stefan_tube(nx=64, ny=4, tau_ref=20.0, j_A_cm2=0.5, dx=1e-4)]
    b = lbm_ms.Batch(cases, precision="fp64", tile_y=4)
    b.init()
    steps, r, rc = b.converge(1e-10, 40000, check_every=100, raise_on_fail=False)
    assert rc == lbm_ms.OK, (rc, steps, r)
    # j = 0 keeps the inlet composition: converged at the first check
    assert steps[0] == 100 and steps[1] > steps[0] and steps[2] > steps[1]
    assert np.all(r < 1e-10)
    eta = b.overpotential()
    assert eta[0] == 0.0 and eta[1] > 0.0 and eta[2] > 0.0
    X0 = b.instance(0).get_fields()
    assert np.max(np.abs(X0[0] - cases[0].X_in[0])) < 1e-15
    # each retired instance equals its own single-instance run stopped at the same step
    for k in (1, 2):
        s = lbm_ms.Solver(cases[k], precision="fp64", tile_y=4)
        s.init()
        s.step(int(steps[k]))
        assert np.array_equal(s.get_fields(), b.instance(k).get_fields()), k
        s.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_residuals_equal_single_instance_residuals(precision):
    """The batch reduces every instance's residual window in one pass over the batch; each value
    is bit for bit the one the instance's own check computes after the same steps."""
    cases = _cases(js=(0.4, 1.2, 0.8, 1.5))  # no j = 0 instance: none converges by step 300
    b = lbm_ms.Batch(cases, precision=precision)
    b.init()
    steps, r, rc = b.converge(1e-300, 300, check_every=100, raise_on_fail=False)
    assert rc == lbm_ms.E_NOT_CONVERGED and np.all(steps == 300)
    for k, c in enumerate(cases):
        s = lbm_ms.Solver(c, precision=precision)
        s.init()
        n, rs, rcs = s.converge(1e-300, 300, check_every=100, raise_on_fail=False)
        assert n == 300 and rcs == lbm_ms.E_NOT_CONVERGED
        assert rs == r[k], (k, rs, r[k])
        s.close()
    b.close()


def test_instance_retired_in_the_last_check_stays_put():
    """An instance that converges at the last check of a converge call leaves the work list before
    the call returns: later steps of the batch do not move it."""
    cases = [inputs.stefan_tube(nx=24, ny=8, tau_ref=20.0, j_A_cm2=0.0, dx=1e-4),
             inputs.stefan_tube(nx=32, ny=8, tau_ref=20.0, j_A_cm2=1.0, dx=1e-4)]
    b = lbm_ms.Batch(cases, precision="fp64", tile_y=4)
    b.init()
    steps, r, rc = b.converge(1e-10, 100, check_every=100, raise_on_fail=False)
    assert steps[0] == 100 and r[0] < 1e-10  # the inlet composition: converged at once
    X0 = b.instance(0).get_fields()
    X1 = b.instance(1).get_fields()
    b.step(200)
    assert np.array_equal(b.instance(0).get_fields(), X0)
    assert not np.array_equal(b.instance(1).get_fields(), X1)
    b.close()


def test_failed_instance_retires_with_its_status():
    """An instance past its limiting current (a fraction turns negative: the oracle shows it by
    step 100 at 100 A/cm^2 over 2.4 mm) retires with E_NEG_FRACTION; the others still converge."""
    cases = [inputs.stefan_tube(nx=24, ny=8, tau_ref=20.0, j_A_cm2=0.0, dx=1e-4),
             inputs.stefan_tube(nx=24, ny=8, tau_ref=20.0, j_A_cm2=100.0, dx=1e-4),
             inputs.stefan_tube(nx=64, ny=4, tau_ref=20.0, j_A_cm2=0.5, dx=1e-4)]
    b = lbm_ms.Batch(cases, precision="fp64", ms_mode=lbm_ms.STOICH, tile_y=4)
    b.init()
    steps, r, rc = b.converge(1e-10, 40000, check_every=100, raise_on_fail=False)
    assert rc == lbm_ms.E_NEG_FRACTION
    assert list(b.status) == [lbm_ms.OK, lbm_ms.E_NEG_FRACTION, lbm_ms.OK], (b.status, steps, r)
    assert steps[1] == 100 and r[2] < 1e-10
    eta = b.overpotential()
    assert np.isnan(eta[1]) and eta[2] > 0.0
    s = lbm_ms.Solver(cases[2], precision="fp64", ms_mode=lbm_ms.STOICH, tile_y=4)
    s.init()
    s.step(int(steps[2]))
    assert np.array_equal(s.get_fields(), b.instance(2).get_fields())
    s.close()
    b.close()


def test_autotune_keeps_results_bitwise(tmp_path, monkeypatch):
    from paper_1809_01600_amd import autotune
    monkeypatch.setenv("LBM_MS_TUNE_CACHE", str(tmp_path / "tune.json"))
    c = _cases(seed0=900, sizes=((150, 70),), js=(1.0,))[0]
    ref = lbm_ms.Solver(c, precision="fp32", tile_y=8)
    ref.init()
    ref.step(60)
    s = lbm_ms.Solver(c, precision="fp32")
    s.init()
    best = autotune.tune(s, steps=20, warmup=2)
    assert best in lbm_ms.tile_options(lbm_ms.D2Q9)
    s.step(60)
    assert np.array_equal(s.get_fields(), ref.get_fields())
    # second call hits the cache
    assert autotune.tune(s) == best
    b = lbm_ms.Batch(_cases(seed0=950, sizes=((80, 40), (64, 30)), js=(0.5, 1.0)), precision="fp32")
    tb = autotune.tune_batch(b, steps=5, warmup=1)
    assert tb in lbm_ms.tile_options(lbm_ms.D2Q9)
    b.close()


def test_create_names_the_instance_without_a_path():
    """A failed batch create returns no handle; its reason, naming the instance whose outlet the
    inlet cannot reach, comes from lbm_ms_batch_last_error(NULL)."""
    import dataclasses
    cases = _cases(seed0=500, sizes=((70, 33), (64, 40)), js=(1.0, 1.0))
    wall = cases[1].mask().copy()
    wall[:, :, 30] = 1  # a solid column across the slice
    blocked = dataclasses.replace(cases[1], solid=wall)
    with pytest.raises(lbm_ms.LbmMsError) as e:
        lbm_ms.Batch([cases[0], blocked], precision="fp32")
    assert e.value.status == lbm_ms.E_GEOM
    assert "instance 1" in str(e.value)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_packed_tiles_batch_equals_single_and_oracle(precision):
    """Packed tiles (rows grown up to 12 or 256 fluid nodes per 64-wide tile): a batch equals
    single solves with the same tiling bitwise, and FP64 equals the oracle."""
    cases = _cases(seed0=700, sizes=((150, 70), (64, 64), (200, 17)), js=(0.8, 1.5, 0.3))
    b = lbm_ms.Batch(cases, precision=precision, tile_y=8, rows=12, ms_mode=lbm_ms.STOICH)
    b.init()
    b.step(120)
    for k, c in enumerate(cases):
        s = lbm_ms.Solver(c, precision=precision, tile_y=8, chunk_z=12, ms_mode=lbm_ms.STOICH)
        info = s.get_info()
        assert (info.tile_y, info.chunk_z) == (8, 12)
        s.init()
        s.step(120)
        assert np.array_equal(b.instance(k).get_fields(), s.get_fields()), k
        s.close()
        if precision == "fp64":
            o = oracle.Oracle(c, ms_mode=oracle.STOICH)
            o.init_uniform()
            o.step(120)
            assert np.max(np.abs(b.instance(k).get_fields() - o.moments())) < 1e-12, k
    b.close()
