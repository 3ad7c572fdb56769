"""Throughput benchmark of the fused TVLBM step on one MI355X.

Workload (the throughput configuration): 1024 x 1024 periodic grid, D2Q16
(4-point Gauss-Hermite tensor set, 3rd-order equilibrium), FP32 populations
in structure-of-arrays with compensated moment sums, tau = 0.6, initial
rho = 1 + 0.01 * smoothed N(0,1), T = 1 + 0.05 sin(2 pi x / 1024), u = 0.
One step = one pass of the fused collide + overlap-stream kernel over the
whole grid.  D2Q36 (6-point set, 4th-order equilibrium) is run as a second
line item.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline (D2Q16, 1024²); batched steady solves/s vs plain"
HBM_PEAK_GBS = 8000.0
SCLK_HZ = 2.4e9  # MI355X peak engine clock


def _kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("tvlbm_kernels.hip", "tvlbm_core.h"):
        h.update(open(os.path.join(ROOT, "paper_1004_5059_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def run_lattice(n: int, size: int, steps: int, warmup: int, variant: int, dtype: str = "f32"):
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.autotune import autotune
    from paper_1004_5059_amd.tvlbm import Solver

    s = Solver(size, size, n_gh=n, dtype=dtype, tau=0.6, device="cuda:0")
    s.set_fields(*inputs.smoothed_density_fields(size, size, std=0.01, t_amp=0.05, seed=1))
    if variant < 0:
        variant, tune = autotune(s, steps=20)
    else:
        s.set_variant(variant)
        tune = {}
    k = s.steps_per_launch()  # 2: the variant sweeps the grid once per two steps
    s.step(warmup)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(s.stream)
    s.step(steps)
    ev[1].record(s.stream)
    # With two steps per launch, tvlbm_step makes steps//2 two-step launches
    # and, for an odd count, one single step; time single-step launches on
    # their own on the same stream, so that the two-step kernel's average
    # launch duration can be separated.
    n2 = steps // 2 if k == 2 else 0
    n1 = steps - 2 * n2
    reps1 = 20
    ev[2].record(s.stream)
    for _ in range(reps1):
        s.step(1)
    ev[3].record(s.stream)
    ev[3].synchronize()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1])
    ms1 = ev[2].elapsed_time(ev[3]) / reps1
    launch_ms = (ms - n1 * ms1) / n2 if n2 > 0 else ms / steps
    _, tot = s.moments()
    s.close()
    q = n * n
    cells = size * size
    esz = 4 if dtype == "f32" else 8
    # algorithmic bytes: one read and one write per population per cell-update
    bytes_per_launch = 2 * esz * q * cells * k
    return {
        "mlups": cells * steps / (ms / 1e3) / 1e6,
        "ms_per_step": ms / steps,
        "steps": steps,
        "warmup": warmup,
        "variant": variant,
        "steps_per_launch": k,
        "launches": {"two_step": n2, "one_step": n1},
        "launch_ms": launch_ms,
        "one_step_launch_ms": ms1,
        "kernel": "k_march2 (two steps per launch)" if k == 2 else "k_march (one step per launch)",
        "tune_ms": {str(k): round(v, 5) for k, v in tune.items()},
        "achieved_gbs": bytes_per_launch / (launch_ms / 1e3) / 1e9,
        "bytes_per_launch": bytes_per_launch,
        "mass": float(tot[0]),
    }


def run_fv(n: int, size: int, steps: int, warmup: int, dtype: str = "f32", walls: bool = True,
           sched="auto", tau_g: float = 0.0, pscale: bool = False):
    """The finite-volume update, eq.(FVLB), on a size x size mesh: walls at the
    first and last rows on the hyperbolic-tangent mesh of Sec. X scaled to
    spacings 0.5 .. ~2.3 (or periodic and uniform), dt = 0.05, tau = 0.2."""
    import numpy as np
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.tvlbm import FVSolver

    dy = None
    if walls:
        y = inputs.tanh_mesh(10.0, size - 1, 2.3)
        dy = np.diff(y)
        dy = dy * (0.5 / dy.min())
    s = FVSolver(size, size, n_gh=n, dtype=dtype, dx=1.0, dt=0.05, tau=0.2, dy=dy, walls=walls,
                 wall_lo=(0.0, 1.0), wall_hi=(0.04, 1.1), device="cuda:0")
    s.set_prandtl(tau_g, pscale)
    s.set_fields(*inputs.smoothed_density_fields(size, size, std=0.01, t_amp=0.05, seed=1))
    if sched == "auto":
        from paper_1004_5059_amd.autotune import autotune_fv

        autotune_fv(s)
        s.set_fields(*inputs.smoothed_density_fields(size, size, std=0.01, t_amp=0.05, seed=1))
    elif sched:
        s.set_schedule(**sched)
    schedule = s.schedule()
    s.step(warmup)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(steps)
    b.record(s.stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    _, tot = s.moments()
    s.close()
    q, cells = n * n, size * size
    esz = 4 if dtype == "f32" else 8
    bytes_per_step = 2 * esz * q * cells  # algorithmic: read f, write f' once per step
    return {"mlups": round(cells * steps / (ms / 1e3) / 1e6, 1),
            "ms_per_step": round(ms / steps, 5),
            "achieved_gbs": round(bytes_per_step / (ms / 1e3 / steps) / 1e9, 1),
            "frac": round(bytes_per_step / (ms / 1e3 / steps) / 1e9 / HBM_PEAK_GBS, 4),
            "finite": bool(np.isfinite(tot).all()), "walls": walls, "dtype": dtype,
            "lattice": f"D2Q{q}", "schedule": schedule,
            **({"tau_g": tau_g, "pressure_scaled": pscale} if tau_g > 0 or pscale else {})}


def run_batched(n_inst: int = 256, plain_per_size: int = 2, tol: float = 1e-8, k: int = 100,
                solve: bool = True, load_steps: int = 500, two_rows: int = 0):
    """Batched steady solves of the thermal-Couette sampler (seed 2026) in one
    persistent, graph-captured run, against plain single-instance solves.

    The plain leg solves a stratified sample (plain_per_size instances of
    every N_y) one after another with the single-instance path; every
    instance of the batch takes exactly as many steps plain as batched (the
    arithmetic is identical, tested bitwise), so the plain wall time of the
    whole batch is the sum over instances of steps x the measured plain time
    per step of its size (residual checks included).

    Before the solve, load_steps steps with every instance active give the
    batched kernel's full-load throughput; solve=False stops there.
    two_rows > 0: a fixed tuning (two-step segments of two_rows rows)
    instead of the autotuner's, for counter runs that must repeat exactly."""
    import numpy as np
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.autotune import apply_batch_tuning, autotune, autotune_batch
    from paper_1004_5059_amd.tvlbm import BatchSolver, Solver

    insts = inputs.couette_instances(n_inst, seed=2026)
    t0 = time.perf_counter()
    if two_rows > 0:
        tune = {"tuning": dict(prefetch=0, tail_active=64, tail_width=64, tail_rows=6, two_step=1,
                               two_rows=two_rows), "shapes": {}}
    else:
        tune = autotune_batch(insts)
    t_tune = time.perf_counter() - t0
    b = BatchSolver(insts, dtype="f32")
    apply_batch_tuning(b, tune)
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in insts])
    b.run(2 * k, tol=0.0, k_interval=k)  # warm-up, graph capture
    cells = np.array([d["nx"] * d["ny"] for d in insts])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(load_steps, tol=0.0, k_interval=k)
    t_load = (time.perf_counter() - t0) / load_steps
    load = {"steps": load_steps, "us_per_step": round(t_load * 1e6, 2),
            "mlups": round(float(cells.sum()) / t_load / 1e6, 1),
            "achieved_gbs": round(128.0 * float(cells.sum()) / t_load / 1e9, 1)}  # 8Q B/cell
    if not solve:
        b.close()
        return {"instances": n_inst, "full_load": load, "tuning": tune["tuning"],
                "shapes": {str(c): list(v) for c, v in tune["shapes"].items()}}
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in insts])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok, steps, r = b.run(5_000_000, tol, k)
    t_batch = time.perf_counter() - t0
    b.close()
    # plain: per-size time per step from a stratified sample
    rng = np.random.default_rng(0)
    per_step = {}
    sample = []
    for ny in sorted(set(d["ny"] for d in insts)):
        idx = [i for i, d in enumerate(insts) if d["ny"] == ny]
        pick = rng.choice(idx, min(plain_per_size, len(idx)), replace=False)
        # the plain path gets its own best launch variant for this size
        d = insts[idx[0]]
        probe = Solver(d["nx"], d["ny"], n_gh=4, dtype="f32", tau=d["tau"], walls=True,
                       wall_lo=(0.0, d["T_bot"]), wall_hi=(d["u_top"], d["T_top"]))
        probe.set_fields(*inputs.uniform_fields(d["nx"], d["ny"]))
        variant, _ = autotune(probe, steps=200)
        probe.close()
        ts, ns = 0.0, 0
        for i in pick:
            d = insts[i]
            s = Solver(d["nx"], d["ny"], n_gh=4, dtype="f32", tau=d["tau"], walls=True,
                       wall_lo=(0.0, d["T_bot"]), wall_hi=(d["u_top"], d["T_top"]))
            s.set_variant(variant)
            s.set_fields(*inputs.uniform_fields(d["nx"], d["ny"]))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            conv, n, rr = s.solve(5_000_000, tol, k)
            ts += time.perf_counter() - t1
            ns += n
            sample.append(int(i))
            s.close()
        per_step[ny] = ts / max(ns, 1)
    t_plain = float(sum(steps[i] * per_step[d["ny"]] for i, d in enumerate(insts)))
    return {
        "instances": n_inst, "converged": bool(ok), "tol": tol, "k_interval": k,
        "batched_wall_s": round(t_batch, 3), "batched_solves_per_s": round(n_inst / t_batch, 3),
        "plain_wall_s_est": round(t_plain, 3), "plain_solves_per_s": round(n_inst / t_plain, 3),
        "speedup": round(t_plain / t_batch, 2),
        "aggregate_mlups": round(float(np.sum(cells * steps)) / t_batch / 1e6, 1),
        "cell_updates": float(np.sum(cells * steps)),
        "steps_max": int(np.max(steps)), "steps_mean": float(np.mean(steps)),
        "plain_sample": f"{len(sample)} instances ({plain_per_size} per N_y) solved one by one; "
                        "whole-batch plain time = sum of steps x per-size time per step",
        "full_load": load,
        "shapes": {str(c): list(v) for c, v in tune["shapes"].items()},
        "tuning": tune["tuning"], "autotune_s": round(t_tune, 2),
    }


def run_c0(steps: int = 200):
    """The small latency-bound case: 64 x 64 periodic D2Q16 in FP64, tau 0.8,
    shear wave u_x = 0.01 sin(2 pi y / 64) plus uniform population noise
    +-1e-4 (seed 0), 200 steps."""
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.tvlbm import Solver

    from paper_1004_5059_amd.autotune import autotune

    s = Solver(64, 64, n_gh=4, dtype="f64", tau=0.8, device="cuda:0")
    s.set_fields(*inputs.shear_wave_fields(64, 64, eps=0.01),
                 inputs.population_noise(16, 64, 64, amp=1e-4, seed=0))
    variant, _ = autotune(s, steps=20)
    s.set_fields(*inputs.shear_wave_fields(64, 64, eps=0.01),
                 inputs.population_noise(16, 64, 64, amp=1e-4, seed=0))
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(steps)
    b.record(s.stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    k = s.steps_per_launch()
    s.close()
    return {"steps": steps, "ms": round(ms, 3), "us_per_step": round(ms * 1e3 / steps, 2),
            "mlups": round(64 * 64 * steps / (ms / 1e3) / 1e6, 1), "variant": variant,
            "steps_per_launch": k}


def copy_ceiling(mib: int = 1024, reps: int = 10):
    """The library's 16-byte streaming copy kernel on two buffers of `mib`
    MiB each (four times the 256 MB Infinity Cache): the HBM read + write
    rate a streaming kernel reaches on this GPU."""
    import torch

    from paper_1004_5059_amd.tvlbm import tvlbm_stream_copy

    nbytes = mib * (1 << 20)
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    tvlbm_stream_copy(a, b, nbytes, st)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        tvlbm_stream_copy(a, b, nbytes, st)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a[:: 1 << 16], b[:: 1 << 16]))
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms / 1e3) / 1e9,
            "kernel": "k_stream_copy (16-byte grid-stride, library)", "copied": ok}


def run_c2(tol: float = 1e-8, k: int = 100):
    """The bounded thermal flow: 512 x 256 channel, rows refined 2:1 in
    16-cell bands at both walls (288 rows), D2Q16, FP32, tau 0.7, walls
    (u, T) = (0, 1) and (0.05, 1.1), from the uniform state to residual 1e-8
    (K = 100); wall time, steps, per-step kernel time, mass drift and the
    profile's distance from the closed-form thermal Couette solution."""
    import numpy as np
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.tvlbm import Solver

    dy = inputs.refined_wall_rows(h=256, band=16, ratio=2)
    ny = len(dy)
    s = Solver(512, ny, n_gh=4, dtype="f32", tau=0.7, dy=dy, walls=True, wall_lo=(0.0, 1.0),
               wall_hi=(0.05, 1.1), device="cuda:0")
    s.set_fields(*inputs.uniform_fields(512, ny))
    m0 = s.moments()[1][0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv, steps, r = s.solve(3_000_000, tol, k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fld, tot = s.moments()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(200)
    b.record(s.stream)
    b.synchronize()
    us_step = a.elapsed_time(b) * 1e3 / 200
    s.close()
    q = fld.double().cpu().numpy().mean(axis=2)
    yb = np.concatenate([[0.0], np.cumsum(dy)])
    yc = 0.5 * (yb[1:] + yb[:-1]) / yb[-1]
    ucf = 0.05 * yc
    tcf = 1.0 + 0.1 * yc + 0.05 ** 2 / 4.0 * yc * (1 - yc)
    cells = 512 * ny
    return {"converged": bool(conv), "steps": int(steps), "residual": r, "wall_s": round(wall, 3),
            "us_per_step": round(us_step, 2), "mlups": round(cells / us_step, 1),
            "achieved_gbs": round(128.0 * cells / (us_step * 1e-6) / 1e9, 1),
            "mass_drift": float(abs(tot[0] - m0) / m0),
            "couette_u_err": round(float(np.max(np.abs(q[1] - ucf)) / 0.05), 5),
            "couette_T_err": round(float(np.max(np.abs(q[3] - tcf)) / 0.1), 5),
            "kernel": "k_rows (non-uniform rows, diffuse walls)"}


def run_c2_steps(steps: int, warmup: int = 200):
    """The bounded-flow channel's step alone (512 x 288 refined rows, D2Q16
    FP32, walls as in run_c2) from the uniform state: `warmup` steps, then
    `steps` timed ones -- the row-table kernel under rocprofv3 counters
    without the 256k-step solve."""
    import torch

    from paper_1004_5059_amd import inputs
    from paper_1004_5059_amd.tvlbm import Solver

    dy = inputs.refined_wall_rows(h=256, band=16, ratio=2)
    ny = len(dy)
    s = Solver(512, ny, n_gh=4, dtype="f32", tau=0.7, dy=dy, walls=True, wall_lo=(0.0, 1.0),
               wall_hi=(0.05, 1.1), device="cuda:0")
    s.set_fields(*inputs.uniform_fields(512, ny))
    s.step(warmup)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    s.step(steps)
    b.record(s.stream)
    b.synchronize()
    us = a.elapsed_time(b) * 1e3 / steps
    s.close()
    return {"grid": [512, ny], "steps": steps, "warmup": warmup, "us_per_step": round(us, 3),
            "mlups": round(512 * ny / us, 1), "kernel": "k_rows (non-uniform rows, diffuse walls)"}


def run_c4(n_train: int = 4096, n_test: int = 256, epochs: int = 40, batch: int = 32,
           lr: float = 2e-3, gen_start: str = "closed_form", tol: float = 1e-8):
    """Learned warm start: training states from batched steady solves of the
    thermal-Couette sampler (seed 2026), the bf16-MFMA network trained on
    them (residual from the closed-form profile), then the held-out
    instances (seed 2027) solved from the uniform start, from the
    closed-form profile and from the network's prediction (inference
    included, fallback re-solves counted).  The training solves start from
    the closed-form profile by default (about 4x fewer steps than from
    uniform; the states agree to what the stopping rule leaves)."""
    import numpy as np
    import torch

    from paper_1004_5059_amd import inputs, warmstart as ws
    from paper_1004_5059_amd.autotune import autotune_batch
    from paper_1004_5059_amd.tvlbm import TvNet

    H, W = 256, 128
    tune = autotune_batch(inputs.couette_instances(256, seed=2026))
    quiet = lambda msg: None  # noqa: E731
    t0 = time.perf_counter()
    tr, prof, steps = ws.generate(n_train, seed=2026, log=quiet, tune=tune, start=gen_start,
                                  tol=tol)
    t_gen = time.perf_counter() - t0
    param = ws.make_param(tr, prof, residual=True)
    net = TvNet(ws.C_IN, H, W, max_batch=batch)
    net.set_params(ws.init_params(ws.C_IN, seed=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ws.train(net, tr, prof, H, W, epochs=epochs, batch=batch, lr=lr, log=quiet, param=param)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    te = inputs.couette_instances(n_test, seed=2027)
    res = ws.warm_vs_uniform(net, te, H, W, tol=tol, log=quiet, tune=tune, param=param)
    net.close()
    res.pop("fallback_instances")
    out = {"n_train": n_train, "n_test": n_test, "train_seed": 2026, "test_seed": 2027,
           "epochs": epochs, "data_generation_start": gen_start,
           "data_generation_s": round(t_gen, 2), "train_steps_mean": float(np.mean(steps)),
           "training_s": round(t_train, 2), "final_loss": hist[-1]}
    out.update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items()})
    return out


def cpu_baseline(size: int, target_s: float = 15.0, c3_cell_updates: float = 0.0):
    """The FP64 oracle, as it stands, on this host's cores: a bounded sample
    (a few steps of the same 1024^2 D2Q16 workload), the same on one core,
    and the walled channels of the batched solve: one instance per N_y of
    the sampler, 50 steps each, whose cell-update rate gives an estimate of
    the oracle's time for the whole batch (c3_cell_updates: the batch's
    total cell-updates to convergence, from the batched leg)."""
    import numpy as np

    from oracle import oracle as orc
    from paper_1004_5059_amd import inputs

    lat = orc.OracleLattice(4, 3)
    g = orc.OracleGrid(lat, size, size, tau=0.6)
    f = g.set_fields(*inputs.smoothed_density_fields(size, size, std=0.01, t_amp=0.05, seed=1))
    f = g.run(f, 1)  # first touch of the arrays
    t = time.perf_counter()
    f = g.run(f, 4)  # per-step time without the start-up of a single call
    one = (time.perf_counter() - t) / 4
    steps = max(1, min(2000, int(target_s / max(one, 1e-3))))
    t = time.perf_counter()
    f = g.run(f, steps)
    dt = time.perf_counter() - t
    cores = orc.threads()
    out = {"value": size * size * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
           "kind": "oracle",
           "sample": f"{steps} FP64 oracle steps of the {size}x{size} D2Q16 workload"}
    orc.set_threads(1)
    try:
        t = time.perf_counter()
        g.run(f, 3)
        out["one_core_mlups"] = round(size * size * 3 / (time.perf_counter() - t) / 1e6, 3)
    finally:
        orc.set_threads(cores)
    # walled channels of the batched solve, one per N_y
    insts = inputs.couette_instances(256, seed=2026)
    pick = {}
    for d in insts:
        pick.setdefault(d["ny"], d)
    cells, secs = 0, 0.0
    for ny in sorted(pick):
        d = pick[ny]
        gw = orc.OracleGrid(lat, d["nx"], d["ny"], tau=d["tau"], walls=True,
                            wall_lo=(0.0, d["T_bot"]), wall_hi=(d["u_top"], d["T_top"]))
        fw = gw.run(gw.set_fields(*inputs.uniform_fields(d["nx"], d["ny"])), 1)
        t = time.perf_counter()
        gw.run(fw, 50)
        secs += time.perf_counter() - t
        cells += d["nx"] * d["ny"] * 50
    rate = cells / secs
    out["c3_subset"] = {"instances": len(pick), "steps_each": 50, "mlups": round(rate / 1e6, 2),
                        "cores": cores}
    if c3_cell_updates > 0:
        out["c3_subset"]["oracle_batch_s_est"] = round(c3_cell_updates / rate, 1)
    return out


def counters_from_profile(steps_per_launch: int, variant: int):
    """Counted HBM bytes and VALU wave-instructions per launch of the step
    kernel, from committed rocprofv3 counter runs, if they were taken on the
    current kernel source and on the same launch variant; else None."""
    p = os.path.join(ROOT, "profiles", "fused_step_d2q16_1024_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_hash") != _kernel_hash():
        return None
    v = d.get("variants", {}).get(str(variant))
    if v is None or v.get("steps_per_launch") != steps_per_launch:
        return None
    return v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    # the first ~300 steps of a fresh solver run 5-8 % slower than the steady
    # state (26 us against 24.4 us at 1024^2 D2Q16): warm up past them
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--variant", type=int, default=-1,
                    help="launch variant of the D2Q16 fused step (1024^2, 4096^2, FP64); "
                         "-1 (default): the autotuner's choice on this GPU")
    ap.add_argument("--variant36", type=int, default=-1,
                    help="launch variant of the D2Q36 step; -1 (default): autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-d2q36", action="store_true")
    ap.add_argument("--no-4096", action="store_true", help="skip the 4096^2 run")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-ceiling measurement")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 lines (1024^2 and 64^2)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched steady-solve leg")
    ap.add_argument("--no-fv", action="store_true", help="skip the finite-volume legs")
    ap.add_argument("--no-c2", action="store_true", help="skip the bounded-flow steady solve")
    ap.add_argument("--no-c4", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--fv-only", action="store_true", help="run only the finite-volume legs")
    ap.add_argument("--fv-size", type=int, default=1024, help="mesh size of the finite-volume legs")
    ap.add_argument("--profile-variants", default="",
                    help="comma-separated D2Q16 launch variants: run only the D2Q16 leg once per "
                         "variant (steps/warmup as given) and one 256 MiB stream copy, for counter "
                         "runs under rocprofv3, then exit")
    ap.add_argument("--profile-variants36", default="",
                    help="with --profile-variants: D2Q36 launch variants to run the same way")
    ap.add_argument("--batched-two-rows", type=int, default=0,
                    help="batched leg: fixed two-step segment rows instead of autotuning "
                         "(for counter runs)")
    ap.add_argument("--batched-load-only", action="store_true",
                    help="batched leg: full-load steps only, no steady solves")
    ap.add_argument("--profile-rows", type=int, default=0,
                    help="run only K steps of the bounded-flow channel (refined rows, after 200 "
                         "warm-up steps), for counter runs under rocprofv3, then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the TVLBM path here is single-GPU "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    def leg(name, fn, *a):
        t0 = time.perf_counter()
        r = fn(*a)
        print(f"[bench] {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        return r

    v16, v36 = args.variant, args.variant36

    def fv_legs():
        fv_steps, fv_warm = max(20, args.steps // 4), max(10, args.warmup // 2)
        return {"d2q16_f32_walls": leg("FV D2Q16", run_fv, 4, args.fv_size, fv_steps, fv_warm),
                "d2q16_f32_walls_two_pass": leg("FV D2Q16 two-pass", run_fv, 4, args.fv_size,
                                                fv_steps, fv_warm, "f32", True, {"fused": False}),
                "d2q16_f32_periodic": leg("FV D2Q16 periodic", run_fv, 4, args.fv_size, fv_steps,
                                          fv_warm, "f32", False),
                "d2q16_f32_walls_prandtl": leg("FV D2Q16 Pr 1/5", run_fv, 4, args.fv_size,
                                               fv_steps, fv_warm, "f32", True, "auto", 0.1, True),
                "d2q36_f32_walls": leg("FV D2Q36", run_fv, 6, args.fv_size, fv_steps // 2,
                                       fv_warm // 2),
                "d2q16_f64_walls": leg("FV D2Q16 FP64", run_fv, 4, args.fv_size, fv_steps // 2,
                                       fv_warm // 2, "f64")}

    if args.fv_only:
        print(json.dumps({"fv": fv_legs()}), flush=True)
        return
    if args.profile_rows > 0:
        print(json.dumps({"profile_rows": leg("C2 steps", run_c2_steps, args.profile_rows)}),
              flush=True)
        return
    if args.profile_variants:
        # each variant's k_march2 launches have their own grid size, which
        # tells them apart in a counter run; the copy calibrates the counters
        res = {}
        for v in (int(x) for x in args.profile_variants.split(",")):
            r = leg(f"D2Q16 variant {v}", run_lattice, 4, args.size, args.steps, args.warmup, v)
            res[str(v)] = {"mlups": round(r["mlups"], 1), "launch_us": round(r["launch_ms"] * 1e3, 3),
                           "steps_per_launch": r["steps_per_launch"]}
        for v in (int(x) for x in args.profile_variants36.split(",") if x):
            r = leg(f"D2Q36 variant {v}", run_lattice, 6, args.size, args.steps, args.warmup, v)
            res[f"d2q36_{v}"] = {"mlups": round(r["mlups"], 1),
                                 "launch_us": round(r["launch_ms"] * 1e3, 3),
                                 "steps_per_launch": r["steps_per_launch"]}
        res["copy"] = leg("stream copy", copy_ceiling, 256, 3)
        print(json.dumps({"profile_variants": res}), flush=True)
        return
    # The headline leg runs first: once other solvers have allocated and freed
    # device memory, the same step on new buffers runs 3-5 % slower (measured
    # 25.3-25.6 us against 24.5 us at 1024^2 D2Q16, even after emptying
    # torch's cache, at the same addresses), most likely because memory mapped
    # again comes back in smaller physical fragments.
    r16 = leg("D2Q16", run_lattice, 4, args.size, args.steps, args.warmup, v16)
    # The other lattice lines are figures of their own, not the headline's
    # K steps: each times at least 200 steps after at least 100 warm-up steps,
    # so that the single steps closing every run (the state semantics) and
    # the first slower steps of a fresh solver do not set their rate.
    k2, w2 = max(args.steps, 200), max(args.warmup, 100)
    r36 = None if args.no_d2q36 else leg("D2Q36", run_lattice, 6, args.size, k2, w2, v36)
    big = None if args.no_4096 else leg("D2Q16 4096", run_lattice, 4, 4096, max(200, args.steps // 10),
                                        max(100, args.warmup // 20), v16)
    r64 = None if args.no_f64 else leg("D2Q16 FP64", run_lattice, 4, args.size, k2, w2, v16, "f64")
    fv = None if args.no_fv else fv_legs()
    c0 = None if args.no_f64 else leg("C0 64x64 FP64", run_c0)
    cp = None if args.no_copy else leg("copy ceiling", copy_ceiling)
    bat = None if args.no_batched else leg("batched", run_batched, 256, 2, 1e-8, 100,
                                           not args.batched_load_only, 500, args.batched_two_rows)
    c2 = None if args.no_c2 else leg("C2 bounded flow", run_c2)
    c4 = None if args.no_c4 else leg("C4 warm start", run_c4)
    cpu = None if args.no_cpu_baseline else leg("cpu baseline", cpu_baseline, args.size, 15.0,
                                                (bat or {}).get("cell_updates", 0.0))
    achieved = r16["achieved_gbs"]
    prof = counters_from_profile(r16["steps_per_launch"], r16["variant"])
    traffic = None if prof is None else prof.get("hbm_bytes_per_launch")
    launch_s = r16["launch_ms"] / 1e3
    # HBM bytes actually moved per second: counted traffic per launch over
    # the live average launch duration (below the algorithmic rate when a
    # launch advances two steps on one read and one write)
    measured = None if traffic is None else traffic / launch_s / 1e9
    # vector-issue share: a wave64 VALU instruction holds a 16-lane SIMD for
    # 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz
    valu = None if prof is None else prof.get("sq_insts_valu_per_dispatch")
    valu_frac = None if valu is None else valu * 4 / (1024 * SCLK_HZ * launch_s)
    out = {
        "metric": METRIC,
        "value": round(r16["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r16["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D2Q16 {args.size}x{args.size} periodic, FP32 SoA, tau=0.6, "
                               "smoothed-density init", "grid": [args.size, args.size],
                   "lattice": "D2Q16", "eq_order": 3, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": r16["kernel"], "steps_per_launch": r16["steps_per_launch"],
                     "algorithmic_bytes_per_launch": r16["bytes_per_launch"],
                     "launch_us": round(r16["launch_ms"] * 1e3, 3),
                     "launches_timed": r16["launches"],
                     "one_step_launch_us": round(r16["one_step_launch_ms"] * 1e3, 3),
                     "hbm_counted_gbs": None if measured is None else round(measured, 1),
                     "hbm_counted_frac": None if measured is None else round(measured / HBM_PEAK_GBS, 4),
                     "valu_issue_frac": None if valu_frac is None else round(valu_frac, 4),
                     "note": "frac: algorithmic bytes (one read + one write of every population per "
                             "cell-update) over the live launch time; a two-step launch reads and "
                             "writes each population once per two steps, so frac can exceed 1. "
                             "hbm_counted_frac: HBM bytes counted by rocprofv3 per launch over the "
                             "same time; valu_issue_frac: VALU issue cycles over SIMD cycles"},
        "cpu_baseline": cpu,
        "variant": r16["variant"],
        "d2q36": None if r36 is None else {
            "mlups": round(r36["mlups"], 1), "ms_per_step": round(r36["ms_per_step"], 5),
            "steps": r36["steps"], "warmup": r36["warmup"],
            "achieved_gbs": round(r36["achieved_gbs"], 1),
            "frac": round(r36["achieved_gbs"] / HBM_PEAK_GBS, 4), "variant": r36["variant"]},
        "autotune_ms_per_step": r16["tune_ms"],
        "d2q16_4096": None if big is None else {
            "mlups": round(big["mlups"], 1), "achieved_gbs": round(big["achieved_gbs"], 1),
            "frac": round(big["achieved_gbs"] / HBM_PEAK_GBS, 4), "variant": big["variant"],
            "steps_per_launch": big["steps_per_launch"], "steps": big["steps"],
            "warmup": big["warmup"]},
        "d2q16_f64": None if r64 is None else {
            "mlups": round(r64["mlups"], 1), "achieved_gbs": round(r64["achieved_gbs"], 1),
            "frac": round(r64["achieved_gbs"] / HBM_PEAK_GBS, 4), "variant": r64["variant"],
            "steps_per_launch": r64["steps_per_launch"], "steps": r64["steps"],
            "warmup": r64["warmup"]},
        "c0_64x64_f64": c0,
        "copy_ceiling_gbs": None if cp is None else round(cp["gbs"], 1),
        "c2_bounded_flow": c2,
        "c4_warm_start": c4,
        "batched": bat,
        "finite_volume": fv,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
