"""A concentration-overpotential curve eta(j) from one batched job: ragged porous slices of one
inlet composition at current densities drawn over [0, j_max], every instance converged in the same
batch (one launch per step, hipGraph chunks, converged instances leave the work list, an instance
past its limiting current leaves with E_NEG_FRACTION).

    python -m paper_1809_01600_amd.polarization --count 64 --side-lo 64 --side-hi 256 \\
        --tol 1e-9 --out polarization.json
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import autotune, inputs, lbm_ms


def curve(count=64, side_lo=64, side_hi=256, j_hi=2.0, tau_ref=3.0, tol=1e-9, precision="fp32",
          shift="node", max_steps=8_000_000, check_every=1000, chunk=500_000, subset=0, log=print):
    """subset > 0 keeps that many of the `count` drawn instances, evenly spaced in side length
    (the drawn batch sorted by side), so a shorter job still spans the size range."""
    import torch
    cases = inputs.batch_2d(count=count, side_lo=side_lo, side_hi=side_hi, j_hi=j_hi, tau_ref=tau_ref,
                            accept=lambda solid: lbm_ms.clean_geometry("D2Q9", solid)[1] > 0)
    if 0 < subset < count:
        by_side = sorted(range(count), key=lambda k: (cases[k].nx, k))
        cases = [cases[by_side[(i * count) // subset + count // (2 * subset)]] for i in range(subset)]
        count = subset
    b = lbm_ms.Batch(cases, precision=precision, ms_mode=lbm_ms.STOICH,
                     shift_mode=lbm_ms.SHIFT_NODE if shift == "node" else lbm_ms.SHIFT_GLOBAL)
    tile = autotune.tune_batch(b)
    b.use_graphs(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.init()
    steps = np.zeros(count, dtype=np.int64)
    done = 0
    while done < max_steps:
        n = min(chunk, max_steps - done)
        st, r, rc = b.converge(tol, n, check_every=check_every, raise_on_fail=False)
        steps += st
        done += n
        running = int(np.sum(b.status == lbm_ms.E_NOT_CONVERGED))
        log("  %d steps: %d of %d still running" % (done, running, count))
        if running == 0:
            break
    eta = b.overpotential()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    order = np.argsort([c.j_A_cm2 for c in cases])
    rows = [{"j_A_cm2": cases[k].j_A_cm2, "side": cases[k].nx, "eta_V": float(eta[k]),
             "steps": int(steps[k]), "status": int(b.status[k])} for k in order]
    b.close()
    return {"instances": count, "sides": [side_lo, side_hi], "tol": tol, "tau_ref": tau_ref,
            "storage": "%s-%s-shift" % (precision, shift), "tile": list(tile), "seconds": sec,
            "converged": int(sum(1 for r in rows if r["status"] == 0)), "curve": rows}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--side-lo", type=int, default=64)
    ap.add_argument("--side-hi", type=int, default=256)
    ap.add_argument("--j-hi", type=float, default=2.0)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--shift", default="node", choices=["node", "global"])
    ap.add_argument("--subset", type=int, default=0,
                    help="keep this many of the drawn instances, evenly spaced in side")
    ap.add_argument("--max-steps", type=int, default=8_000_000)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    res = curve(args.count, args.side_lo, args.side_hi, args.j_hi, tol=args.tol,
                precision=args.precision, shift=args.shift, max_steps=args.max_steps,
                subset=args.subset, log=lambda m: print(m, flush=True))
    print(json.dumps({k: v for k, v in res.items() if k != "curve"}), flush=True)
    for r in res["curve"]:
        print("j %.4f A/cm2  side %4d  eta %.6f V  steps %8d  status %d"
              % (r["j_A_cm2"], r["side"], r["eta_V"], r["steps"], r["status"]), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
