"""Launch-shape autotuning with a persistent cache.

The C ABI's mrhweno_autotune times candidate 2D launch shapes on the
instances' current states (without advancing them) and applies the fastest.
This module remembers the choice per (GPU architecture, dimension, number of
components, problem-size bucket) in a JSON file, so later contexts of the
same kind apply it without re-timing."""
from __future__ import annotations

import json
import math
import os
from typing import Optional, Tuple

CACHE = os.path.join(os.path.expanduser(os.environ.get("MRHWENO_CACHE_DIR", "~/.cache/mrhweno")),
                     "autotune.json")
ROWS = (16, 24, 32, 40, 48, 64, 96)


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def key(solver) -> str:
    """arch / dim / ncomp / log2 bucket of the total 2D cell count"""
    two = [p for p in solver.problems if p.dim == 2]
    cells = sum(p.ncell for p in two)
    ncomp = max((p.ncomp for p in two), default=0)
    bucket = int(math.log2(max(cells, 1)))
    return f"{_arch()}/dim2/nc{ncomp}/cells2^{bucket}"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def resident_grid() -> int:
    """Work groups of the 2D stage kernel that fit the GPU at once (two per
    compute unit)."""
    import torch
    return 2 * torch.cuda.get_device_properties(0).multi_processor_count


def tune(solver, use_cache: bool = True, grids=None, reps: int = 3) -> Tuple[int, int, Optional[float]]:
    """Apply the cached launch shape for this kind of problem, or time the
    candidates (strip heights ROWS; grids: one work group per work item and
    a persistent grid of resident size, unless given), apply the fastest and
    cache it.  Returns (rows, grid, ms) (ms is None for a cache hit)."""
    if grids is None:
        grids = (0, resident_grid())
    k = key(solver)
    db = _load()
    if use_cache and k in db:
        rows, grid = db[k]["rows"], db[k]["grid"]
        solver.set_launch(rows, grid)
        return rows, grid, None
    rows, grid, ms = solver.autotune(rows=ROWS, grids=grids, reps=reps)
    db[k] = {"rows": rows, "grid": grid, "ms": ms}
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass
    return rows, grid, ms
