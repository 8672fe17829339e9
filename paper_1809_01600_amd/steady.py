"""One steady solve of a named single-domain workload: steps, time, residual, status and the
overpotential (Eq. 43), with progress lines while it runs.

    python -m paper_1809_01600_amd.steady --workload porous_2d --tol 1e-8 --tau-ref 100
    python -m paper_1809_01600_amd.steady --workload porous_2d --tol 1e-8 --tau-ref 3 --shift node

The 1024^2 porous slice (overlapping disks, void fraction 0.40, seed 2, X_in ~ Dirichlet(6, 3, 1),
j = 1 A/cm^2) or the 256^3 porous block; FP32 storage by default.  A check that finds a mole
fraction below -1e-12 (the limiting current reached in a pore) ends the solve with that status.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

from . import inputs, lbm_ms


def solve(workload="porous_2d", tol=1e-8, tau_ref=100.0, precision="fp32", shift="global",
          max_steps=20_000_000, check_every=1000, chunk=200_000, log=print):
    import torch
    case = inputs.porous_2d(tau_ref=tau_ref) if workload == "porous_2d" else inputs.porous_3d(tau_ref=tau_ref)
    s = lbm_ms.Solver(case, precision=precision,
                      shift_mode=lbm_ms.SHIFT_NODE if shift == "node" else lbm_ms.SHIFT_GLOBAL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.init()
    steps, r, rc = 0, float("inf"), lbm_ms.E_NOT_CONVERGED
    while steps < max_steps and rc == lbm_ms.E_NOT_CONVERGED:
        n, r, rc = s.converge(tol, min(chunk, max_steps - steps), check_every=check_every,
                              raise_on_fail=False)
        steps += n
        log("  %d steps, r %.3e, status %d, %.1f s" % (steps, r, rc, time.perf_counter() - t0))
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    eta = s.overpotential() if rc in (lbm_ms.OK, lbm_ms.E_NOT_CONVERGED) else None
    info = s.get_info()
    out = {"workload": workload, "nx": case.nx, "ny": case.ny, "nz": case.nz,
           "fluid_nodes": int(info.n_fluid), "tau_ref": tau_ref, "precision": precision,
           "shift": shift, "tol": tol, "steps": int(steps), "residual": r, "status": int(rc),
           "status_text": lbm_ms.lib().lbm_ms_status_string(rc).decode(), "seconds": sec,
           "eta_V": eta, "X_out": s.outlet_mean().tolist() if eta is not None else None,
           "node_mlups": info.n_fluid * steps / sec / 1e6}
    s.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="porous_2d", choices=["porous_2d", "porous_3d"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--tau-ref", type=float, default=100.0)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--shift", default="global", choices=["global", "node"])
    ap.add_argument("--max-steps", type=int, default=20_000_000)
    ap.add_argument("--check-every", type=int, default=1000)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    res = solve(args.workload, args.tol, args.tau_ref, args.precision, args.shift, args.max_steps,
                args.check_every, log=lambda m: print(m, flush=True))
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
