"""Launch-shape autotuner for the fused step.

Times every launch variant of the library (columns per wavefront strip x
rows per lane segment) on the caller's solver with HIP events on its
stream and keeps the fastest.  Every variant computes bit-identical
results (tested), so the choice only affects speed.  Results can be cached
in a JSON file keyed by GPU architecture, lattice, dtype and grid size.
"""
from __future__ import annotations

import json
import os

from .tvlbm import tvlbm_num_variants


def _key(solver) -> str:
    import torch

    arch = getattr(torch.cuda.get_device_properties(solver.device), "gcnArchName", "gpu")
    return f"{arch}|q{solver.q}|{solver.tdtype}|{solver.nx}x{solver.ny}|walls{solver.desc.y_bc}"


def autotune(solver, steps: int = 20, reps: int = 2, cache_path: str | None = None):
    """Pick the fastest variant for `solver` (advances its state).
    Returns (variant, {variant: ms_per_step})."""
    import torch

    key = _key(solver)
    if cache_path and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached is not None:
            solver.set_variant(int(cached["variant"]))
            return int(cached["variant"]), cached["ms"]
    times = {}
    for v in range(tvlbm_num_variants()):
        solver.set_variant(v)
        solver.step(2)
        best = float("inf")
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(solver.stream)
            solver.step(steps)
            b.record(solver.stream)
            b.synchronize()
            best = min(best, a.elapsed_time(b) / steps)
        times[v] = best
    v = min(times, key=times.get)
    solver.set_variant(v)
    if cache_path:
        data = {}
        if os.path.exists(cache_path):
            try:
                data = json.load(open(cache_path))
            except (OSError, ValueError):
                data = {}
        data[key] = {"variant": v, "ms": times}
        with open(cache_path, "w") as fh:
            json.dump(data, fh, indent=1)
    return v, times
