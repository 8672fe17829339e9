"""Launch-shape autotuner: times every compiled tile shape on the problem at hand and keeps the
fastest, cached in a JSON file per (lattice, precision, shift, problem size), keyed also on the
built library's contents and the device name, so a rebuilt kernel or another GPU re-tunes.

    from paper_1809_01600_amd import autotune
    best = autotune.tune(solver)          # lbm_ms.Solver
    best = autotune.tune_batch(batch)     # lbm_ms.Batch

The cache lives at $LBM_MS_TUNE_CACHE (default ~/.cache/lbm_ms_tune.json).  Tuning changes only
the launch shape.  In FP64 and in 2D the results do not depend on it; 3D instantiations of
different shapes may contract FP32 multiply-adds differently, so FP32 and 16-bit 3D results can
differ between shapes in the last bits (within the FP32 parity tolerance).
"""

from __future__ import annotations

import hashlib
import json
import os
import time

from . import lbm_ms


def cache_path() -> str:
    return os.environ.get("LBM_MS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lbm_ms_tune.json"))


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def _store(data):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _lattice_name(code):
    return next(name for name, c in lbm_ms.LATTICES.items() if c == code)


_BUILD_ID = None


def _build_id() -> str:
    """Hash of the loaded library file plus the device name."""
    global _BUILD_ID
    if _BUILD_ID is None:
        h = hashlib.sha256()
        with open(lbm_ms.LIB_PATH, "rb") as f:
            h.update(f.read())
        try:
            import torch
            dev = torch.cuda.get_device_properties(torch.cuda.current_device())
            name = "%s/%s" % (dev.name, getattr(dev, "gcnArchName", ""))
        except Exception:
            name = "unknown-device"
        _BUILD_ID = h.hexdigest()[:16] + "|" + name
    return _BUILD_ID


def _key(kind, lattice, precision, shift, dims):
    return "%s|%s|p%d|s%d|%s|%s" % (kind, lattice, precision, shift,
                                    "x".join(str(d) for d in dims), _build_id())


def tune(solver, steps: int = 100, warmup: int = 10, use_cache: bool = True):
    """Pick the fastest tile shape for a single-problem solver (state is restored after)."""
    p = solver.params
    key = _key("single", _lattice_name(p.lattice), p.precision, p.shift_mode, (p.nx, p.ny, p.nz))
    data = _load() if use_cache else {}
    if key in data:
        ty, cz = data[key]["tile"]
        solver.set_tile(ty, cz)
        return tuple(data[key]["tile"])
    blob = solver.save_state()
    timings = {}
    for ty, cz in lbm_ms.tile_options(p.lattice, p.precision, p.shift_mode):
        solver.set_tile(ty, cz)
        solver.step(warmup)
        timings[(ty, cz)] = solver.time_steps(steps) / steps
    best = min(timings, key=timings.get)
    solver.set_tile(*best)
    solver.load_state(blob)
    data = _load()
    data[key] = {"tile": list(best), "us_per_step": {"%d,%d" % k: v * 1e3 for k, v in timings.items()},
                 "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    if use_cache:
        _store(data)
    return best


def tune_batch(batch, steps: int = 20, warmup: int = 3, use_cache: bool = True):
    """Pick the fastest tile height for a batch.  Tuning (re)initializes the batch to the uniform
    inlet composition and advances it; initialize again before a solve."""
    p = batch.params
    sizes = sorted((c.nx, c.ny) for c in batch.cases)
    size_list = hashlib.sha256(repr(sizes).encode()).hexdigest()[:12]
    key = _key("batch", _lattice_name(p.lattice), p.precision, p.shift_mode,
               (len(sizes), sum(a * b for a, b in sizes), size_list))
    data = _load() if use_cache else {}
    if key in data:
        batch.set_tile(*data[key]["tile"])
        return tuple(data[key]["tile"])
    timings = {}
    batch.init()
    for ty, rows in lbm_ms.tile_options(p.lattice, p.precision, p.shift_mode):
        batch.set_tile(ty, rows)
        batch.step(warmup)
        timings[(ty, rows)] = batch.time_steps(steps) / steps
    best = min(timings, key=timings.get)
    batch.set_tile(*best)
    data = _load()
    data[key] = {"tile": list(best), "ms_per_step": {"%d,%d" % k: v for k, v in timings.items()},
                 "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    if use_cache:
        _store(data)
    return best
