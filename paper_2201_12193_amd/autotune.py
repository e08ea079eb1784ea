"""Launch-shape autotuning with a persistent cache.

The C ABI's mrhweno_autotune times candidate 2D launch shapes of the stage
kernel on the instances' current states (without advancing them) and applies
the fastest; mrhweno_autotune_indicator does the same for the strip height of
the 2D KXRCF pass.  This module remembers the choices per (GPU architecture,
dimension, number of components, problem-size bucket) in a JSON file, so
later contexts of the same kind apply them without re-timing."""
from __future__ import annotations

import json
import math
import os
from typing import NamedTuple, Optional

CACHE = os.path.join(os.path.expanduser(os.environ.get("MRHWENO_CACHE_DIR", "~/.cache/mrhweno")),
                     "autotune.json")
ROWS = (8, 16, 24, 32, 40, 48, 56, 64, 72, 96)
KX_ROWS = (0, 8, 16, 24, 32, 46, 64, 96, 140)   # 0: the height chosen per problem


class Launch(NamedTuple):
    rows: int          # rows per work item of the 2D stage kernel
    grid: int          # its grid (0: one work group per work item)
    ms: Optional[float]
    kx_rows: int       # flag rows per work item of the 2D KXRCF pass (0: per problem)


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


def tune(solver, use_cache: bool = True, grids=None, reps: int = 3) -> Launch:
    """Apply the cached launch shapes for this kind of problem, or time the
    candidates (stage kernel: strip heights ROWS and grids, one work group
    per work item and a persistent grid of resident size unless given;
    KXRCF pass: strip heights KX_ROWS), apply the fastest and cache them.
    ms is the stage kernel's mean launch time (None for a cache hit)."""
    if grids is None:
        grids = (0, resident_grid())
    k = key(solver)
    db = _load()
    if use_cache and k in db and "kx_rows" in db[k]:
        e = db[k]
        solver.set_launch(e["rows"], e["grid"])
        solver.set_indicator_launch(e["kx_rows"])
        return Launch(e["rows"], e["grid"], None, e["kx_rows"])
    rows, grid, ms = solver.autotune(rows=ROWS, grids=grids, reps=reps)
    kx_rows, kx_ms = solver.autotune_indicator(rows=KX_ROWS, reps=reps)
    db[k] = {"rows": rows, "grid": grid, "ms": ms, "kx_rows": kx_rows, "kx_ms": kx_ms}
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass
    return Launch(rows, grid, ms, kx_rows)
