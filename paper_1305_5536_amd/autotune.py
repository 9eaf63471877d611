"""Autotuner for the launch shape of the stage kernels.

The tunable of the single-mesh Cartesian kernels is how many rows (2D) or
z-planes (3D) one wave marches through: more rows amortise the halo rows and
the pipeline fill, fewer rows give more waves to fill the 256 CUs.  Batches
add the workgroup size (waves per workgroup) and the grid: one wave per tile,
or a persistent grid of fewer waves that walk the tile list (tuned by
coordinate descent: rows, then workgroup size, then grid).  The tuner times one
SSP-RK2 step (stage 1 + stage 2, HIP events on the current stream) for each
candidate on the caller's own state and keeps the fastest.  Results are cached
in a JSON file keyed by GPU architecture, mesh shape, physics and precision
(default ``~/.cache/dgmi/autotune.json``; override with ``DG_AUTOTUNE_CACHE``).
Results of the solver do not depend on the choice, only its speed.
"""
from __future__ import annotations

import hashlib
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


BATCH_ROWS = (4, 8, 16, 32)
BATCH_WPB = (1, 2, 4)
BATCH_GRID = (0, 2048, 4096, 8192, 16384)


def autotune_batch(solver, U, sizes, reps: int = 5, use_cache: bool = True) -> dict:
    """Pick rows per tile, waves per workgroup and grid size for a batch solver
    on state ``U`` (sizes: the instances' (nx, ny)); returns ``{"rows", "wpb",
    "grid", "times"}`` and leaves the solver set to the choice."""
    h = hashlib.sha1(repr([tuple(int(v) for v in n) for n in sizes]).encode()).hexdigest()[:16]
    key = _key(solver, (len(sizes),)) + "|batch|" + h
    db = _load() if use_cache else {}
    if key in db:
        e = db[key]
        solver.tiling = int(e["rows"])
        solver.launch = (int(e["wpb"]), int(e["grid"]))
        return e
    V1 = solver.empty()
    Un = solver.empty()
    dt = solver.cfl_dt(U, 0.3)
    times = {}

    def t(rows, wpb, grid):
        solver.tiling = rows
        solver.launch = (wpb, grid)
        k = f"{rows},{wpb},{grid}"
        if k not in times:
            times[k] = time_step(solver, U, V1, Un, dt, reps)
        return times[k]

    best = (16, 4, 0)
    best = min(((r, best[1], best[2]) for r in BATCH_ROWS), key=lambda c: t(*c))
    best = min(((best[0], w, best[2]) for w in BATCH_WPB), key=lambda c: t(*c))
    best = min(((best[0], best[1], g) for g in BATCH_GRID), key=lambda c: t(*c))
    solver.tiling = best[0]
    solver.launch = (best[1], best[2])
    entry = {"rows": best[0], "wpb": best[1], "grid": best[2], "times": times}
    if use_cache:
        db[key] = entry
        _store(db)
    return entry


def write_launch_file(path: str, entry: dict) -> str:
    """Write a batch launch shape (``autotune_batch``'s result) as the text file
    ``dg_batch_create`` reads: "rows waves_per_group grid_waves"."""
    with open(path, "w") as f:
        f.write(f"{int(entry['rows'])} {int(entry['wpb'])} {int(entry['grid'])}\n")
    return path
