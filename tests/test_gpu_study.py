"""End-to-end runs of the batched steady-state workflows at tiny sizes: a polarization curve from
one job, and the warm-start pipeline (labels from the method, HIP training, evaluation of every
starting point against a tighter FP64 reference)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1809_01600_amd import cnn, lbm_ms, polarization, warmstart  # noqa: E402


def test_polarization_curve_in_one_job():
    res = polarization.curve(count=6, side_lo=32, side_hi=48, tol=1e-8, log=lambda m: None)
    rows = res["curve"]
    assert res["converged"] == 6 and len(rows) == 6
    js = [r["j_A_cm2"] for r in rows]
    assert js == sorted(js)
    # H2 is consumed: the concentration overpotential is positive and finite
    assert all(np.isfinite(r["eta_V"]) and r["eta_V"] > 0.0 for r in rows)
    assert all(r["steps"] > 0 and r["status"] == lbm_ms.OK for r in rows)


def test_warm_start_pipeline_small():
    feat, tgt, fluid = warmstart.generate(8, 32, 50000, chunk=8, tol=1e-9, log=lambda m: None)
    assert feat.shape[1:] == (cnn.CIN, 32, 32) and tgt.shape[1:] == (cnn.OUT, 32, 32)
    assert feat.shape[0] == tgt.shape[0] == fluid.shape[0] >= 6
    net = cnn.WarmStartNet(seed=0)
    hist = warmstart.train(net, feat, tgt, fluid, epochs=3, batch=4, log=lambda m: None)
    assert np.all(np.isfinite(hist))
    cases = warmstart.make_cases(4, 32, 70000)
    out = warmstart.evaluate(net, cases, tol=1e-8, ref_tol=1e-10, reduced=("bf16",),
                             plain=True, reference=True, log=lambda m: None)
    for name in ("plain", "batch", "batch_profile", "batch_cnn", "batch_cnn_bf16_node"):
        r = out[name]
        assert all(s == lbm_ms.OK for s in r["status"]), (name, r["status"])
        assert r["seconds"] > 0 and r["max_abs_eta_err_V"] < 1e-3, (name, r)
    # same FP32 arithmetic one instance at a time or batched: the same steps
    assert out["plain"]["steps"] == out["batch"]["steps"]


def test_trained_network_saves_steps_on_held_out_draws():
    """What the learned start gains over the method without it: a network trained by the HIP
    kernels on steady fields the method generated (256 draws of 48^2) starts 12 unseen draws
    closer to their steady states than the uniform inlet composition (the zero-initialised
    fallback): fewer steps to r = 1e-8, and, converged on from either start to r = 1e-11, the
    same overpotential to 1e-4 V (in fact to rounding: the steady state does not depend on the
    start)."""
    print("warm-start gain: generating labels", flush=True)
    feat, tgt, fluid = warmstart.generate(256, 48, 50000, chunk=128, tol=1e-9, log=lambda m: None)
    assert feat.shape[0] >= 200
    net = cnn.WarmStartNet(seed=0)
    hist = warmstart.train(net, feat, tgt, fluid, epochs=12, batch=16, lr=2e-3, log=lambda m: None)
    assert hist[-1] < hist[0]
    cases = warmstart.make_cases(12, 48, 70000)
    b_u, st_u, _ = warmstart.solve(cases, tol=1e-8, precision="fp64")
    b_c, st_c, _ = warmstart.solve(cases, X0=warmstart.cnn_start(net, cases), tol=1e-8,
                                   precision="fp64")
    ok = [k for k in range(len(cases)) if b_u.status[k] == 0 and b_c.status[k] == 0]
    assert len(ok) >= 10
    su, sc = st_u[ok].astype(float), st_c[ok].astype(float)
    print("mean steps to r = 1e-8: uniform %.0f, network %.0f (%d of %d instances fewer)"
          % (su.mean(), sc.mean(), int(np.sum(sc < su)), len(ok)))
    assert sc.mean() < 0.9 * su.mean()
    assert np.sum(sc < su) >= 0.75 * len(ok)
    b_u.close()
    b_c.close()
    # the same steady state from either start (converged instances retire, so solve again)
    b_u, _, _ = warmstart.solve(cases, tol=1e-11, precision="fp64", max_steps=3_000_000)
    b_c, _, _ = warmstart.solve(cases, X0=warmstart.cnn_start(net, cases), tol=1e-11,
                                precision="fp64", max_steps=3_000_000)
    assert all(b_u.status[k] == 0 and b_c.status[k] == 0 for k in ok)
    eu, ec = b_u.overpotential()[ok], b_c.overpotential()[ok]
    print("max |eta(network start) - eta(uniform start)| = %.2e V" % np.max(np.abs(eu - ec)))
    assert np.max(np.abs(eu - ec)) <= 1e-4
    b_u.close()
    b_c.close()
