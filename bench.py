"""Benchmark of the LBM / Maxwell-Stefan hot path on one MI355X.

Workload (default): the batch of 64 ragged porous anode slices (D2Q9, sides 256..1024, void
fraction U[0.3, 0.5], overlapping disks r ~ U[3, 12], one inlet composition, current densities
U[0, 2] A/cm^2): 10.1 M fluid nodes, a 1.5 GB double-buffered FP32 state that does not fit the
256 MB last-level cache, so the step kernel's rate is an HBM rate.  A step is one time step of the
whole path (stream, boundaries, moments, gradients, Maxwell-Stefan solve, relaxation time,
collision) over every instance, one kernel launch; hipGraph chunks of --check-every steps with
the per-instance residual check between them, and the overpotential of every instance at the end.
--workload porous_2d (the 1024^2 slice, 56 MB: cache-resident) and porous_3d (the 256^3 block)
select the single-domain workloads.

Prints one JSON line: species-MLUPS (fluid nodes x 2 evolved species x steps / s / 1e6) as the
value, the step kernel's roofline (algorithmic bytes per launch over its mean duration from HIP
events on the launch stream), and the FP64 CPU oracle's rate on a bounded sample of the same
workload, taken before the GPU is touched: for the batch one worker process per host core (up
to 16), each stepping its own instance; for a single domain one thread.
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "species-MLUPS & HBM GB/s (% roofline); steady solves/s vs plain at 1e-8 residual"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid-node update: each of Q populations of the 2 evolved species read
# once and written once (pull scheme)
BYTES_PER_NODE = {("D2Q9", "fp64"): 288, ("D2Q9", "fp32"): 144, ("D2Q9", "fp16"): 72,
                  ("D2Q9", "bf16"): 72, ("D3Q19", "fp64"): 608, ("D3Q19", "fp32"): 304,
                  ("D3Q19", "fp16"): 152, ("D3Q19", "bf16"): 152, ("D2Q5", "fp64"): 160,
                  ("D2Q5", "fp32"): 80, ("D2Q5", "fp16"): 40, ("D2Q5", "bf16"): 40,
                  ("D3Q7", "fp64"): 224, ("D3Q7", "fp32"): 112, ("D3Q7", "fp16"): 56,
                  ("D3Q7", "bf16"): 56}
# the lattice each workload is defined on, and the alternative velocity set it accepts
WORKLOAD_LATTICES = {"porous_2d": ("D2Q9", "D2Q5"), "porous_3d": ("D3Q19", "D3Q7"),
                     "batch_2d": ("D2Q9",), "steady": ("D2Q9",)}
NODE_SHIFT_BYTES = 2 * 8 * 2
# --advection: a reaction that changes the number of moles (nu = -1, 2, 0), so a net molar flux
# drives u_M, carried by the second lattice Boltzmann model (relaxation time ADV_TAU_FLOW)
ADV_NU = (-1, 2, 0)
ADV_TAU_FLOW = 1.0


def adv_bytes_per_node(lattice: str, precision: str) -> int:
    """Algorithmic bytes of one advective step per fluid node: both species' populations and the
    velocity model's read and written once (6 Q entries), and the node velocity of the previous
    step read and of this step written (2 x 3 doubles).  The two-pass kernels also write and read
    back X (2 doubles) and pull the species twice; that traffic is theirs, not the method's."""
    q = {"D2Q9": 9, "D2Q5": 5, "D3Q19": 19, "D3Q7": 7}[lattice]
    es = 8 if precision == "fp64" else 4
    return 6 * q * es + 48
KERNEL_SOURCES = ["paper_1809_01600_amd/csrc/lbm_ms_device.hpp",
                  "paper_1809_01600_amd/csrc/lbm_ms_kernels.hip",
                  "paper_1809_01600_amd/csrc/lbm_ms_runtime.hip"]  # the node numbering


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        rec = data.get(workload_key)
        if not rec or rec.get("kernel_hash") != kernel_hash():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _oracle_sample(case, steps: int, advection: bool = False):
    """Oracle steps on one problem (or the first 32 z-planes of a 3D block as a periodic slab);
    returns (fluid nodes, steps, seconds)."""
    import dataclasses
    import numpy as np
    import oracle
    sample = case
    if case.nz > 32:
        sample = dataclasses.replace(case, nz=32, solid=np.ascontiguousarray(case.mask()[:32]))
    o = oracle.Oracle(sample, advection=advection, tau_flow=ADV_TAU_FLOW)
    o.init_uniform()
    o.step(1)  # warm-up (allocations, page faults)
    t0 = time.perf_counter()
    o.step(steps)
    return int(o.fluid().sum()), steps, time.perf_counter() - t0


def _oracle_timed(case, seconds: float):
    """Oracle steps on one problem in chunks until `seconds` have passed: (fluid, steps, s)."""
    import oracle
    o = oracle.Oracle(case)
    o.init_uniform()
    o.step(1)
    t0 = time.perf_counter()
    steps = 0
    while True:
        o.step(5)
        steps += 5
        dt = time.perf_counter() - t0
        if dt >= seconds:
            return int(o.fluid().sum()), steps, dt


def cpu_baseline(case, steps: int, advection: bool = False):
    """The FP64 CPU oracle as it stands, single thread, on a bounded sample of the workload:
    `steps` steps of the whole slice (2D), or of the block's first 32 z-planes stepped as a
    periodic slab (3D: the whole 256^3 block takes the oracle about a minute per step and 15 GB
    of memory)."""
    n_fluid, steps, dt = _oracle_sample(case, steps, advection)
    if case.nz == 1:
        what = "the same %dx%d slice" % (case.nx, case.ny)
    else:
        what = "the first 32 z-planes of the same %dx%dx%d block as a periodic slab" % (
            case.nx, case.ny, case.nz)
    return {"value": 2.0 * n_fluid * steps / dt / 1e6, "unit": "species-MLUPS", "cores": 1,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": "%d %ssteps of %s (%d fluid nodes), FP64, single thread" % (
                steps, "advective " if advection else "", what, n_fluid)}


def cpu_baseline_batch(cases, seconds: float = 12.0):
    """The oracle on the batch: one worker process per host core (at most 16, the host share of
    one GPU), each stepping its own instance of the batch for `seconds`; the instances are
    independent, so the aggregate is the oracle's batch throughput on this host.  The workers
    are fresh interpreters (spawned, not forked: a forked copy of a process that has loaded the
    GPU runtime must not touch it), started before this process initializes the GPU."""
    import multiprocessing as mp
    P = _host_cores()
    order = sorted(range(len(cases)), key=lambda k: cases[k].nx)
    pick = [cases[order[(i * len(order)) // P]] for i in range(P)]  # spread over the sizes
    ctx = mp.get_context("spawn")
    with ctx.Pool(P) as pool:
        res = pool.starmap(_oracle_timed, [(c, seconds) for c in pick])
    agg = sum(2.0 * nf * st / dt for nf, st, dt in res) / 1e6
    return {"value": agg, "unit": "species-MLUPS", "cores": P, "kind": "oracle",
            "cpu_model": _cpu_model(),
            "per_worker_mean": agg / P,
            "sample": "%d concurrent oracle processes, one per core, each stepping one instance "
                      "of the batch (sides %s) for about %.0f s, FP64" % (
                          P, ",".join(str(c.nx) for c in pick), seconds)}


def storage_label(precision: str, shift: str) -> str:
    """FP64 and FP32 global storage hold f itself; 16-bit global storage holds f - w_a X_in; the
    NODE shift holds f - w_a c(r) with an FP64 reference per node."""
    if shift == "node":
        return precision + "-node-shift"
    if precision in ("fp16", "bf16"):
        return precision + "-global-shift"
    return precision


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--shift", default="global", choices=["global", "node"])
    ap.add_argument("--workload", default="batch_2d",
                    choices=["porous_2d", "porous_3d", "batch_2d", "steady"])
    ap.add_argument("--steady-n", type=int, default=32, help="steady workload: instances")
    ap.add_argument("--steady-side", type=int, default=96, help="steady workload: slice side")
    ap.add_argument("--steady-tol", type=float, default=1e-8, help="steady workload: residual")
    ap.add_argument("--lattice", default="", choices=["", "d2q9", "d2q5", "d3q19", "d3q7"],
                    help="velocity set: d2q9 (default) or d2q5 for porous_2d, d3q19 (default) or "
                         "d3q7 for porous_3d")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--chunk-z", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the single-domain CPU baseline (default 40 in 2D, 6 in 3D)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="seconds each oracle worker steps in the batch CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--advection", action="store_true",
                    help="porous_2d / porous_3d with a net molar flux (nu = -1, 2, 0) and the "
                         "advective coupling of Eq. 26 (FP64 or FP32 storage)")
    args = ap.parse_args(argv)
    if args.advection and args.workload not in ("porous_2d", "porous_3d"):
        ap.error("--advection takes --workload porous_2d or porous_3d")
    if args.advection and (args.precision not in ("fp64", "fp32") or args.shift != "global"):
        ap.error("--advection runs with FP64 or FP32 global storage")
    lattices = WORKLOAD_LATTICES[args.workload]
    if args.lattice and args.lattice.upper() not in lattices:
        ap.error("--workload %s takes --lattice %s" % (args.workload, " or ".join(l.lower() for l in lattices)))
    args.lattice = args.lattice.upper() or lattices[0]

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver shards nothing across GPUs "
              "(use --gpus 1)", file=sys.stderr)
        return 2

    from paper_1809_01600_amd import inputs, lbm_ms

    if args.workload == "steady":
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        return run_steady(args)
    if args.workload == "batch_2d":
        cases = inputs.batch_2d(tau_ref=3.0,
                                accept=lambda solid: lbm_ms.clean_geometry("D2Q9", solid)[1] > 0)
        # the oracle leg first: its worker processes start before the GPU is initialized
        cpu = None if args.no_cpu else cpu_baseline_batch(cases, args.cpu_seconds)
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        return run_batch(args, cases, cpu)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "porous_2d":
        case = inputs.porous_2d()
        case.lattice = args.lattice
        desc = ("porous anode slice %s 1024x1024, overlapping disks r~U[4,12], void fraction "
                "0.40, seed 2, X_in~Dirichlet(6,3,1), j=1.0 A/cm^2" % case.lattice)
    else:
        case = inputs.porous_3d()
        case.lattice = args.lattice
        desc = ("porous anode block %s 256^3, overlapping spheres r~U[3,8], void fraction "
                "~U[0.35,0.50], seed 3, X_in=(0.6,0.3,0.1), j=1.0 A/cm^2" % case.lattice)
    shift = lbm_ms.SHIFT_NODE if args.shift == "node" else lbm_ms.SHIFT_GLOBAL
    if args.advection:
        import dataclasses
        case = dataclasses.replace(case, nu=ADV_NU)
        desc += ", nu=(-1,2,0) with the advective coupling (Eq. 26, velocity model tau %.1f)" % ADV_TAU_FLOW
        s = lbm_ms.Solver(case, precision=args.precision, advection=True, tau_flow=ADV_TAU_FLOW)
    else:
        s = lbm_ms.Solver(case, precision=args.precision, shift_mode=shift, tile_y=args.tile_y,
                          chunk_z=args.chunk_z)
    info = s.get_info()
    n_fluid = int(info.n_fluid)
    s.init()
    s.step(args.warmup)
    check = lambda: lbm_ms.lib().lbm_ms_residual(s.h, ctypes.byref(res))  # noqa: E731
    res = ctypes.c_double(0.0)
    check()
    torch.cuda.synchronize()

    # timed region: K steps with the residual check every check_every steps, then eta.  A check
    # that finds a negative fraction (the limiting current reached in a dead-end pore) or a
    # clamp is recorded, not fatal: this measures the step's throughput.
    K = args.steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    statuses = set()
    while done < K:
        n = min(args.check_every, K - done)
        s.step(n)
        done += n
        statuses.add(int(check()))
    r = res.value
    eta_rc = lbm_ms.lib().lbm_ms_overpotential(s.h, ctypes.byref(res))
    eta = res.value if eta_rc == 0 else None
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # step kernel alone: HIP events on the launch stream around K back-to-back launches
    kernel_ms = s.time_steps(K) / K
    bytes_per_launch = BYTES_PER_NODE[(case.lattice, args.precision)] * n_fluid
    if shift == lbm_ms.SHIFT_NODE:  # FP64 node reference per evolved species, read and written
        bytes_per_launch += NODE_SHIFT_BYTES * n_fluid
    if args.advection:  # the step's two kernels together, timed as one
        bytes_per_launch = adv_bytes_per_node(case.lattice, args.precision) * n_fluid
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    alt = "" if case.lattice == lattices[0] else "_" + case.lattice.lower()
    wl_key = "%s%s_%s_%s%s" % (args.workload, alt, args.precision, args.shift,
                               "_advection" if args.advection else "")
    traffic = measured_traffic(wl_key, kernel_hash())

    ms_per_step = elapsed * 1e3 / K
    value = 2.0 * n_fluid * K / elapsed / 1e6
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "species-MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision.replace("fp", "f"),
        "data": "synthetic",
        "config": {
            "workload": desc,
            "lattice": case.lattice,
            "nx": case.nx, "ny": case.ny, "nz": case.nz,
            "fluid_nodes": n_fluid,
            "storage": storage_label(args.precision, args.shift),
            "ms_solve": "fp64",
            "tau_ref": case.tau_ref,
            "check_every": args.check_every,
            "tile": [64, int(info.tile_y), int(info.chunk_z)],
            "node_mlups": round(n_fluid * K / elapsed / 1e6, 1),
            "residual_at_end": r,
            "eta_V": eta,
            "check_status": sorted(statuses),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_adv_moments+k_adv_step" if args.advection else
                      (("k_step3dc" if int(info.tile_y) in (12, 16) else "k_step3d") if case.nz > 1
                       else "k_step2d"),
            "kernel_us": round(kernel_ms * 1e3, 3),
            "bytes_per_launch": bytes_per_launch,
        },
    }
    if not args.no_cpu:
        default_steps = (20 if case.nz == 1 else 3) if args.advection else (40 if case.nz == 1 else 6)
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_steps or default_steps, args.advection)
    print(json.dumps(line), flush=True)
    s.close()
    return 0


def run_batch(args, cases, cpu):
    """64 ragged porous slices (sides 256..1024, one inlet composition, j ~ U[0, 2] A/cm^2) in one
    launch per step, hipGraph chunks of --check-every steps with the per-instance residual check
    between them, autotuned tile height."""
    import torch
    from paper_1809_01600_amd import autotune, lbm_ms
    shift = lbm_ms.SHIFT_NODE if args.shift == "node" else lbm_ms.SHIFT_GLOBAL
    b = lbm_ms.Batch(cases, precision=args.precision, shift_mode=shift)
    tile = autotune.tune_batch(b)
    b.use_graphs(True)
    b.init()
    _, n_fluid, n_tiles = b.stats()
    b.converge(0.0, args.warmup, check_every=args.check_every, raise_on_fail=False)
    torch.cuda.synchronize()
    K = args.steps
    t0 = time.perf_counter()
    steps, r, rc = b.converge(0.0, K, check_every=args.check_every, raise_on_fail=False)
    eta = b.overpotential()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    active, n_fluid_end, _ = b.stats()
    failed = int(sum(1 for v in b.status if v not in (lbm_ms.OK, lbm_ms.E_NOT_CONVERGED)))
    # node updates actually done (an instance that failed its check left the work list)
    updates = float(sum(int(st) * int(b.instance(k).get_info().n_fluid) for k, st in enumerate(steps)))
    kernel_ms = b.time_steps(min(K, 200)) / min(K, 200)
    bytes_per_launch = BYTES_PER_NODE[("D2Q9", args.precision)] * n_fluid_end
    if shift == lbm_ms.SHIFT_NODE:
        bytes_per_launch += NODE_SHIFT_BYTES * n_fluid_end
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    value = 2.0 * updates / elapsed / 1e6
    order = sorted(range(len(cases)), key=lambda k: cases[k].j_A_cm2)
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "species-MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision.replace("fp", "f"),
        "data": "synthetic",
        "config": {
            "workload": "batch of 64 porous slices D2Q9, sides ~U{256..1024}, void fraction "
                        "~U[0.3,0.5], disks r~U[3,12], seeds 4000+k, X_in=(0.6,0.3,0.1), "
                        "j~U[0,2] A/cm^2, tau_ref 3, one launch per step",
            "instances": len(cases),
            "fluid_nodes": int(n_fluid),
            "tiles": int(n_tiles),
            "storage": storage_label(args.precision, args.shift),
            "ms_solve": "fp64",
            "check_every": args.check_every,
            "graphs": True,
            "tile": [64, int(tile[0]), int(tile[1])],
            "active_at_end": int(active),
            "failed_checks": failed,
            "node_mlups": round(updates / elapsed / 1e6, 1),
            "eta_V_by_j": [[round(cases[k].j_A_cm2, 4), float(eta[k])] for k in order],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("batch_2d_%s_%s" % (args.precision, args.shift), kernel_hash()),
            "kernel": "k_step2d",
            "kernel_us": round(kernel_ms * 1e3, 3),
            "bytes_per_launch": bytes_per_launch,
        },
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    b.close()
    return 0


def run_steady(args):
    """Steady solves per second at a residual tolerance: the batched, warm-started, reduced-
    precision form (one batched job, the network's BF16 prediction as the start, FP16 storage
    with the NODE shift) against the plain FP32 form (one instance at a time from the channel
    composition), on porous slices drawn like the warm-start evaluation (X_in ~ Dirichlet(6,3,1),
    j ~ U[0, 2] A/cm^2, tau_ref 3), each overpotential compared with an FP64 reference converged to
    r = 1e-11.  The network is first trained by the library's kernels on 256 steady 64^2 slices
    the method generates (its time is reported, not counted in the solves)."""
    import numpy as np
    import torch
    from paper_1809_01600_amd import cnn, lbm_ms, warmstart
    quiet = lambda m: None  # noqa: E731

    def phase(m):  # progress on stderr; the JSON line stays alone on stdout
        print("steady: %s (%.1f s)" % (m, time.perf_counter() - t0), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    phase("generating 256 steady 64^2 training slices")
    feat, tgt, fluid = warmstart.generate(256, 64, 50000, chunk=128, tol=1e-9, log=quiet)
    phase("training the network")
    net = cnn.WarmStartNet(seed=0)
    warmstart.train(net, feat, tgt, fluid, epochs=12, batch=16, lr=2e-3, log=quiet)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del feat, tgt, fluid
    cases = warmstart.make_cases(args.steady_n, args.steady_side, 60000)
    phase("FP64 references to r = 1e-11")
    ref, _, _ = warmstart.solve(cases, tol=1e-11, precision="fp64", max_steps=8_000_000)
    keep = [k for k in range(len(cases)) if ref.status[k] == 0]
    eta_ref = ref.overpotential()[keep]
    ref.close()
    cases = [cases[k] for k in keep]
    tol = args.steady_tol
    phase("plain form")
    st_p, stat_p, eta_p, sec_p = warmstart.solve_plain(cases, tol=tol, precision="fp32")
    phase("batched, warm-started form")
    fast, st_f, sec_f = warmstart.solve(cases, X0=warmstart.cnn_start(net, cases), tol=tol,
                                        precision="fp16", shift_mode=lbm_ms.SHIFT_NODE)
    eta_f = fast.overpotential()
    ok_f = int(np.sum(fast.status == 0))
    fast.close()
    n = len(cases)
    line = {
        "metric": METRIC,
        "value": round(n / sec_f, 3),
        "unit": "steady solves/s",
        "n_gpus": 1,
        "steps": int(st_f.sum()),
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {
            "workload": "%d porous slices D2Q9 %dx%d, void fraction ~U[0.3,0.5], disks r~U[3,12], "
                        "X_in~Dirichlet(6,3,1), j~U[0,2] A/cm^2, tau_ref 3, seeds 60000+, steady "
                        "solves to r=%g" % (n, args.steady_side, args.steady_side, tol),
            "fast_form": "one batched job, CNN warm start (BF16 inference), FP16 NODE-shift storage",
            "plain_form": "one instance at a time, uniform start, FP32 storage",
            "plain_solves_per_s": round(n / sec_p, 3),
            "speedup_vs_plain": round(sec_p / sec_f, 2),
            "fast_seconds": round(sec_f, 3),
            "plain_seconds": round(sec_p, 3),
            "fast_converged": ok_f,
            "plain_converged": int(np.sum(stat_p == 0)),
            "fast_mean_steps": float(st_f.mean()),
            "plain_mean_steps": float(st_p.mean()),
            "fast_max_abs_eta_err_V": float(np.nanmax(np.abs(eta_f - eta_ref))),
            "plain_max_abs_eta_err_V": float(np.nanmax(np.abs(eta_p - eta_ref))),
            "reference": "FP64 batched, r=1e-11",
            "network_training_s": round(train_s, 1),
            "parallelism": "single GPU",
        },
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
