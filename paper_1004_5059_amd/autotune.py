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


BATCH_SHAPES = [(16, 8), (16, 16), (32, 8), (32, 16), (64, 4), (64, 8)]
SIZE_CLASSES = [16, 32, 64, 1 << 30]  # max nx of each class


def autotune_batch(instances, steps: int = 200, k_interval: int = 100, dtype: str = "f32"):
    """Per size class (max N_x), pick the (strip width, rows per segment)
    of the batched kernel by coordinate descent over the classes, timing a
    fixed number of steps of the whole batch.  Returns {max_nx: (w, rows)}."""
    import time

    import torch

    from . import inputs
    from .tvlbm import BatchSolver

    b = BatchSolver(instances, dtype=dtype)
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in instances])
    max_nx = max(d["nx"] for d in instances)
    classes = [c for c in SIZE_CLASSES if c < (1 << 30)] + [1 << 30]
    choice = {c: (16 if c <= 16 else 32 if c <= 32 else 64, 8) for c in classes}

    def timed():
        for c, (w, r) in choice.items():
            b.set_shape(c, w, r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(steps, tol=0.0, k_interval=k_interval)
        return time.perf_counter() - t0

    timed()  # warm-up (graph capture)
    for c in classes:
        lo = 0 if c == classes[0] else classes[classes.index(c) - 1]
        if lo >= max_nx:
            continue
        best, best_t = choice[c], float("inf")
        for w, r in BATCH_SHAPES:
            if w > max(16, c) and c < (1 << 30):
                continue
            choice[c] = (w, r)
            t = timed()
            if t < best_t:
                best, best_t = (w, r), t
        choice[c] = best
    b.close()
    return choice
