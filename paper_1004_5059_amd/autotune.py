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


def autotune(solver, steps: int = 20, reps: int = 2, cache_path: str | None = None,
             confirm: int = 3, confirm_steps: int = 200):
    """Pick the fastest variant for `solver` (advances its state): every
    variant over `steps` steps (best of `reps`), then the `confirm` fastest
    of them again over `confirm_steps` steps, where a few launches' timing
    noise no longer decides (the close two-step shapes differ by ~2 %).
    Returns (variant, {variant: ms_per_step of the first pass})."""
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
    def timed(v, n):
        solver.set_variant(v)
        solver.step(2)
        best = float("inf")
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(solver.stream)
            solver.step(n)
            b.record(solver.stream)
            b.synchronize()
            best = min(best, a.elapsed_time(b) / n)
        return best

    times = {v: timed(v, steps) for v in range(tvlbm_num_variants())}
    top = sorted(times, key=times.get)[:max(1, confirm)]
    second = {v: timed(v, confirm_steps) for v in top} if confirm_steps > 0 else times
    v = min(second, key=second.get)
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
TAIL_SHAPES = [(64, 1), (64, 2), (64, 4), (32, 2)]
SIZE_CLASSES = [16, 32, 64, 1 << 30]  # max nx of each class


def apply_batch_tuning(b, tune):
    """Apply a result of autotune_batch to a BatchSolver."""
    for c, (w, r) in tune["shapes"].items():
        b.set_shape(int(c), w, r)
    b.set_tuning(**tune["tuning"])


def _time_steps(b, steps, k_interval):
    import time

    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps, tol=0.0, k_interval=k_interval)
    return time.perf_counter() - t0


TWO_ROWS = [4, 6, 8, 12, 16]
TWO_TAIL_ROWS = [1, 2, 3, 4, 6]


def _autotune_batch_two(instances, fresh, steps, k_interval, tail_fraction):
    """Two steps per launch: rows per segment of the bulk work list, then of
    the tail list (timed on the largest instances, with the tail list in use
    from the start)."""
    b = fresh(instances)
    times = {}
    _time_steps(b, steps, k_interval)  # warm-up (graph capture)
    for r in TWO_ROWS:
        b.set_tuning(two_step=1, two_rows=r)
        times[r] = _time_steps(b, steps, k_interval)
    rows = min(times, key=times.get)
    b.close()
    ny_max = max(d["ny"] for d in instances)
    big = [d for d in instances if d["ny"] == ny_max][:16]
    tb = fresh(big)
    tt = {}
    for r in TWO_TAIL_ROWS:
        tb.set_tuning(two_step=1, two_rows=rows, tail_active=len(big), tail_rows=r)
        _time_steps(tb, k_interval, k_interval)
        tt[r] = _time_steps(tb, 4 * steps, k_interval)
    tail_rows = min(tt, key=tt.get)
    tb.close()
    tail_active = max(1, int(len(instances) * tail_fraction))
    return {"shapes": {}, "tuning": {"prefetch": 0, "tail_active": tail_active, "tail_width": 64,
                                     "tail_rows": tail_rows, "two_step": 1, "two_rows": rows},
            "two_rows_s": {str(k): round(v, 4) for k, v in times.items()},
            "tail_rows_s": {str(k): round(v, 4) for k, v in tt.items()}}


def autotune_batch(instances, steps: int = 200, k_interval: int = 100, dtype: str = "f32",
                   tail_fraction: float = 0.25, n_gh: int = 4):
    """Launch tuning of the batched solve, timed on the instances themselves.

    Two steps per launch where the lattice has that kernel: rows per segment
    of the bulk and of the tail work list.  Otherwise, bulk phase (every
    instance active): the (strip width, rows per segment)
    of each size class (max N_x) by coordinate descent over the classes,
    then the prefetch switch.  Tail phase: the single shape used once at
    most tail_fraction of the instances remain, timed on the instances of
    the largest N_y (up to 16 of them), which are the last to converge.
    Returns {"shapes": {max_nx: (w, rows)}, "tuning": {...}}."""
    from . import inputs
    from .tvlbm import BatchSolver

    def fresh(insts):
        b = BatchSolver(insts, dtype=dtype)
        b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in insts])
        return b

    if dtype == "f32" or n_gh in (3, 4):
        return _autotune_batch_two(instances, fresh, steps, k_interval, tail_fraction)
    b = fresh(instances)
    max_nx = max(d["nx"] for d in instances)
    classes = list(SIZE_CLASSES)
    choice = {c: (16 if c <= 16 else 32 if c <= 32 else 64, 8) for c in classes}
    pf = 1

    def timed():
        for c, (w, r) in choice.items():
            b.set_shape(c, w, r)
        b.set_tuning(prefetch=pf)
        return _time_steps(b, steps, k_interval)

    timed()  # warm-up (graph capture)
    for ci, c in enumerate(classes):
        lo = 0 if ci == 0 else classes[ci - 1]
        if lo >= max_nx:
            continue
        best, best_t = choice[c], float("inf")
        for w, r in BATCH_SHAPES:
            if c < (1 << 30) and w > max(16, c):
                continue
            choice[c] = (w, r)
            t = timed()
            if t < best_t:
                best, best_t = (w, r), t
        choice[c] = best
    times = {}
    for pf in (1, 0):
        times[pf] = timed()
    pf = min(times, key=times.get)
    b.close()

    ny_max = max(d["ny"] for d in instances)
    big = [d for d in instances if d["ny"] == ny_max][:16]
    tb = fresh(big)
    tb.set_tuning(prefetch=pf)
    best, best_t = TAIL_SHAPES[0], float("inf")
    _time_steps(tb, 2 * k_interval, k_interval)
    for w, r in TAIL_SHAPES:
        tb.set_shape(1 << 30, w, r)
        t = _time_steps(tb, 4 * steps, k_interval)
        if t < best_t:
            best, best_t = (w, r), t
    tb.close()
    tail_active = max(1, int(len(instances) * tail_fraction))
    return {"shapes": dict(choice),
            "tuning": {"prefetch": pf, "tail_active": tail_active, "tail_width": best[0],
                       "tail_rows": best[1], "two_step": 0, "two_rows": 8}}


FV_SEG_ROWS = [4, 5, 6, 7, 8, 10, 12, 16]
FV_BAND_ROWS = [8, 12, 16, 24, 32, 48, 64]


def autotune_fv(solver, steps: int = 20, reps: int = 2):
    """Fastest schedule of the fused finite-volume step for `solver` (an
    FVSolver; advances its state): the march (rows per wavefront segment x
    row prefetch) and, for FP32 with q <= 16, the band schedule (rows per
    workgroup segment).  Every schedule computes the same update up to
    rounding order, so the choice only affects speed.  Returns (schedule
    dict, {label: ms/step})."""
    import torch

    cands = [(1, sr, pf) for pf in (False, True) for sr in FV_SEG_ROWS]
    if solver.tdtype == torch.float32 and solver.q <= 16:
        cands += [(2, sr, False) for sr in FV_BAND_ROWS]
    times = {}
    for fused, sr, pf in cands:
        solver.set_schedule(fused, sr, pf)
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
        times[(fused, sr, pf)] = best
    fused, sr, pf = min(times, key=times.get)
    solver.set_schedule(fused, sr, pf)
    labels = {f"{'band' if f == 2 else 'seg'}{r}{'_pf' if p else ''}": t
              for (f, r, p), t in times.items()}
    return solver.schedule(), labels
