"""The paper's anode case (Sec. 4.1, Tables 1-2), homogenized: a porous anode slab 2 mm thick in the
diffusion direction and 20 mm wide, 100 x 1000 D2Q9 nodes (dx = 20 um), fed with H2/H2O = 4:1
diluted by Ar at the channel side (Dirichlet, Eq. 36) and drawing the electrode flux of Eq. 39 at
the anode/electrolyte interface.  The binary diffusivities come from Fuller's correlation (Eq. 40,
Table 1) with the porosity, tortuosity and Knudsen corrections of Eq. 41-42 (Table 2).  The
sweep reports the concentration overpotential (Eq. 43) relative to the undiluted feed,
X_H2 = 0.8 (Sec. 4.2), at 0.3, 0.7 and 1.0 A/cm^2, together with the continuum prediction of the
paper's own 1D profile (Sec. 4.1, initial settings), which for this y-invariant slab is the exact
steady state of the continuum equations.

Eq. 40 is printed with sqrt(1/M_i + 1/M_j); the constant 0.00143 belongs to the form with the mean
sqrt((1/M_i + 1/M_j) / 2), which is smaller by sqrt(2).  Both readings are available
("printed", "mean").  The paper's measured data and figures are not reproduced here.

    python -m paper_1809_01600_amd.paper_case --reading both --out paper_case.json
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs

R_GAS = 8.3145      # J/(mol K)
FARADAY = 96485.0   # C/mol

# Table 1: molar mass M (kg/kmol) and Fuller diffusion volume V_F of H2, H2O, Ar
TABLE1 = (("H2", 2.016, 6.12), ("H2O", 18.015, 13.1), ("Ar", 39.948, 16.2))

# Table 2: operating point and anode substrate
TABLE2 = {"T": 1023.15, "p": 1.013e5, "porosity": 0.46, "tortuosity": 4.5, "d_p": 2.6e-6}

# Sec. 4.1: 2 mm x 20 mm on 100 x 1000 nodes, 2 s of physical time in 100000 steps
NX, NY, DX, DT = 100, 1000, 20.0e-6, 2.0e-5

CURRENTS = (0.3, 0.7, 1.0)                         # A/cm^2 (Sec. 4.1)
X_H2_SWEEP = (0.8, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2)   # H2/(H2 + H2O + Ar); 0.8 is the undiluted basis


def fuller(T: float, p_pa: float, Mi: float, Mj: float, Vi: float, Vj: float,
           reading: str = "printed") -> float:
    """Eq. 40: binary diffusivity [m^2/s] from T [K], p [Pa], molar masses [kg/kmol] and Fuller
    volumes.  The correlation is in cm^2/s with p in bar."""
    if reading not in ("printed", "mean"):
        raise ValueError("reading must be 'printed' or 'mean'")
    m = 1.0 / Mi + 1.0 / Mj
    if reading == "mean":
        m *= 0.5
    p_bar = p_pa / 1.0e5
    d_cm2 = 0.00143 * T ** 1.75 * math.sqrt(m) / (p_bar * (Vi ** (1.0 / 3.0) + Vj ** (1.0 / 3.0)) ** 2)
    return d_cm2 * 1.0e-4


def knudsen(d_p: float, T: float, M: float) -> float:
    """Eq. 42: Knudsen diffusivity [m^2/s] in pores of mean diameter d_p [m]; M in kg/kmol."""
    return d_p / 3.0 * math.sqrt(8.0 * R_GAS * T / (math.pi * M * 1.0e-3))


def effective(Dij: float, DiM: float, DjM: float, porosity: float, tortuosity: float) -> float:
    """Eq. 41: effective binary diffusivity of a porous electrode, symmetric in i and j."""
    return porosity / (2.0 * tortuosity) * (1.0 / (1.0 / Dij + 1.0 / DiM) + 1.0 / (1.0 / Dij + 1.0 / DjM))


def diffusivities(reading: str = "printed", **table2) -> tuple:
    """Effective (D_12, D_13, D_23) [m^2/s] of H2 (1), H2O (2), Ar (3) at the Table 2 point."""
    t = dict(TABLE2)
    t.update(table2)
    out = []
    for i, j in ((0, 1), (0, 2), (1, 2)):
        (_, Mi, Vi), (_, Mj, Vj) = TABLE1[i], TABLE1[j]
        Dij = fuller(t["T"], t["p"], Mi, Mj, Vi, Vj, reading)
        out.append(effective(Dij, knudsen(t["d_p"], t["T"], Mi), knudsen(t["d_p"], t["T"], Mj),
                             t["porosity"], t["tortuosity"]))
    return tuple(out)


def feed(x_h2: float) -> tuple:
    """Inlet composition with H2/H2O = 4:1 and Ar making up the rest (Sec. 4.1)."""
    if not 0.0 < x_h2 <= 0.8:
        raise ValueError("X_H2 must lie in (0, 0.8] for H2/H2O = 4:1")
    x_h2o = 0.25 * x_h2
    return (x_h2, x_h2o, max(0.0, 1.0 - x_h2 - x_h2o))


def tau_ref_for(D: tuple, dx: float = DX, dt: float = DT) -> float:
    """tau of the fastest pair that gives the paper's time step: dt = (tau - 1/2) dx^2 / (3 D_max)
    (Eq. 25 with c_s^2 = 1/3)."""
    return 3.0 * max(D) * dt / dx ** 2 + 0.5


def make_case(x_h2: float, j_A_cm2: float, reading: str = "printed", ny: int = NY,
              tau_ref: float = 0.0) -> inputs.Case:
    """One point of the sweep: the homogenized slab (no resolved solid), nx = 100 nodes across
    the 2 mm thickness, ny nodes along the 20 mm width (periodic; the problem is y-invariant)."""
    D12, D13, D23 = diffusivities(reading)
    return inputs.Case(name="paper anode %s X_H2=%.2f j=%.2f" % (reading, x_h2, j_A_cm2),
                       lattice="D2Q9", nx=NX, ny=ny, nz=1, T=TABLE2["T"], p=TABLE2["p"],
                       D12=D12, D13=D13, D23=D23, dx=DX,
                       tau_ref=tau_ref if tau_ref > 0 else tau_ref_for((D12, D13, D23)),
                       X_in=feed(x_h2), j_A_cm2=j_A_cm2, nu=(-1, 1, 0), n_electrons=2)


def overpotential(T: float, X_in, X_out, n_electrons: int = 2) -> float:
    """Eq. 43 with species 1 = H2 and 2 = H2O."""
    return R_GAS * T / (n_electrons * FARADAY) * math.log(X_in[0] * X_out[1] / (X_out[0] * X_in[1]))


def sweep(currents=CURRENTS, x_h2=X_H2_SWEEP, reading: str = "printed", ny: int = NY,
          precision: str = "fp64", tol: float = 1e-12, max_steps: int = 2_000_000,
          check_every: int = 1000, log=print) -> dict:
    """Every (current, X_H2) point of one reading converged in one batched job (STOICH fluxes,
    which the steady state satisfies exactly).  Returns per current the rows X_H2, eta,
    eta - eta0, the continuum eta - eta0 and the steps, with eta0 at X_H2 = 0.8."""
    import torch
    from . import lbm_ms
    if 0.8 not in x_h2:
        raise ValueError("the sweep needs the basis point X_H2 = 0.8")
    cases = [make_case(x, j, reading, ny) for j in currents for x in x_h2]
    b = lbm_ms.Batch(cases, precision=precision, ms_mode=lbm_ms.STOICH)
    b.use_graphs(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.init()
    steps, r, rc = b.converge(tol, max_steps, check_every=check_every, raise_on_fail=False)
    eta = b.overpotential()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    # continuum steady state: the 1D generalized-Fick profile at the outlet node
    cont = []
    for k, c in enumerate(cases):
        prof = b.instance(k).paper_profile()
        cont.append(overpotential(c.T, c.X_in, (prof[0, -1], prof[1, -1])))
    out = {"reading": reading, "D_eff_m2_s": list(diffusivities(reading)), "tau_ref": cases[0].tau_ref,
           "dx_m": DX, "dt_s": DT, "shape": [NX, ny], "precision": precision, "tol": tol,
           "seconds": sec, "status": [int(v) for v in b.status], "by_current": {}}
    n = len(x_h2)
    for a, j in enumerate(currents):
        base = a * n + list(x_h2).index(0.8)
        rows = []
        for m, x in enumerate(x_h2):
            k = a * n + m
            rows.append({"X_H2": x, "eta_mV": 1e3 * float(eta[k]),
                         "eta_minus_eta0_mV": 1e3 * float(eta[k] - eta[base]),
                         "continuum_eta_minus_eta0_mV": 1e3 * (cont[k] - cont[base]),
                         "steps": int(steps[k]), "status": int(b.status[k])})
        out["by_current"]["%.1f" % j] = rows
    log("%s reading: %d instances of %dx%d, %.1f s, status %s" % (reading, len(cases), NX, ny, sec,
                                                                   sorted(set(out["status"]))))
    b.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--reading", default="both", choices=["printed", "mean", "both"])
    ap.add_argument("--ny", type=int, default=NY)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    res = {}
    for reading in (("printed", "mean") if args.reading == "both" else (args.reading,)):
        r = sweep(reading=reading, ny=args.ny, precision=args.precision, tol=args.tol, log=log)
        res[reading] = r
        log("D_eff (H2-H2O, H2-Ar, H2O-Ar) = %s m^2/s, tau_ref %.3f" % (
            ", ".join("%.3e" % d for d in r["D_eff_m2_s"]), r["tau_ref"]))
        for j, rows in r["by_current"].items():
            log("  j = %s A/cm^2: " % j + "  ".join(
                "X_H2 %.1f: %.2f mV (continuum %.2f)" % (q["X_H2"], q["eta_minus_eta0_mV"],
                                                         q["continuum_eta_minus_eta0_mV"]) for q in rows))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
