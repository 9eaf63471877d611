"""Autotuner for the launch shape of the stage kernels.

The only tunable of the Cartesian kernels is how many rows (2D) or z-planes (3D)
one wave marches through: more rows amortise the halo rows and the pipeline
fill, fewer rows give more waves to fill the 256 CUs.  The tuner times one
SSP-RK2 step (stage 1 + stage 2, HIP events on the current stream) for each
candidate on the caller's own state and keeps the fastest.  Results are cached
in a JSON file keyed by GPU architecture, mesh shape, physics and precision
(default ``~/.cache/dgmi/autotune.json``; override with ``DG_AUTOTUNE_CACHE``).
Results of the solver do not depend on the choice, only its speed.
"""
from __future__ import annotations

import json
import os

import torch

DEFAULT_CANDIDATES = (2, 4, 6, 8, 12, 16, 24, 32, 48, 64)


def cache_path() -> str:
    return os.environ.get("DG_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "dgmi", "autotune.json"))


def _key(solver, shape) -> str:
    arch = torch.cuda.get_device_properties(solver.device).gcnArchName.split(":")[0]
    return "|".join([arch, solver.physics, solver.precision, f"lim{int(solver.limiter)}",
                     "x".join(str(int(v)) for v in shape)])


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def time_step(solver, U, V1, Un, dt, reps: int = 10) -> float:
    """Average seconds of one stage1+stage2 pair on the current stream."""
    st = torch.cuda.current_stream()
    for _ in range(2):
        solver.stage1(U, dt, V1)
        solver.stage2(U, V1, dt, Un)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        solver.stage1(U, dt, V1)
        solver.stage2(U, V1, dt, Un)
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def autotune(solver, U, shape, candidates=DEFAULT_CANDIDATES, reps: int = 10,
             use_cache: bool = True) -> dict:
    """Pick the fastest rows-per-wave for ``solver`` on state ``U``; returns
    ``{"rows": r, "times": {r: seconds}}`` and leaves the solver set to r."""
    key = _key(solver, shape)
    db = _load() if use_cache else {}
    if key in db:
        solver.tiling = int(db[key]["rows"])
        return db[key]
    V1 = solver.empty()
    Un = solver.empty()
    dt = solver.cfl_dt(U, 0.3).item() * 0.5
    times = {}
    limit = max(shape[-1], 1)
    for r in candidates:
        if r > limit:
            continue
        solver.tiling = r
        times[r] = time_step(solver, U, V1, Un, dt, reps)
    best = min(times, key=times.get)
    solver.tiling = best
    entry = {"rows": int(best), "times": {str(k): v for k, v in times.items()}}
    if use_cache:
        db[key] = entry
        _store(db)
    return entry
