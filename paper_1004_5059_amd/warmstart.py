"""Learned warm start for batched thermal-Couette solves.

Pipeline (all GPU work in the library's kernels; numpy only arranges
canvases):
  1. generate: batched TVLBM solves of sampled channels from a uniform start
     (rho = 1, u = 0, T = 1) to residual tol; the steady fields are stored
     as column profiles (the channels are invariant along x).
  2. train: the four-layer 3x3 bf16-MFMA network (TvNet) maps an input
     canvas -- geometry mask, broadcast maps of (tau, top-wall u, wall dT,
     N_y) and the normalised wall-normal coordinate y/H -- to normalised
     (rho, ux, uy, T) fields; masked MSE, Adam.
  3. warm start: predict, rescale rho to unit mean (walls conserve mass, so
     the steady state is the one with the uniform start's mass), seed the
     batched solve with f = feq(prediction), run to tol; instances whose
     warm-started solve fails to converge (or goes non-finite) are re-solved
     from the uniform start.

Output parametrisation: with residual=True the network predicts the
difference between the steady fields and the closed-form thermal Couette
profile of the instance's parameters (u = U y/H, T = T_b + dT y/H +
U^2/(2 c_P) (y/H)(1 - y/H), uniform pressure rho T, c_P = 2), scaled by the
per-channel spread of that difference over the training set; the profile is
added back to the prediction.  The profile alone, used as a start, is
reported as a second baseline.

The canvas is H x W = (max N_y) x (max N_x); instance k occupies rows
0..ny-1 and columns 0..nx-1.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import inputs
from .tvlbm import BatchSolver, TvNet

# output normalisation: t = (field - offset) / scale
OUT_OFFSET = np.array([1.0, 0.0, 0.0, 1.0])
OUT_SCALE = np.array([0.05, 0.08, 0.01, 0.2])
C_IN = 6


def canvas_inputs(insts, H: int, W: int):
    """x [B][H][W][6] float32 and mask [B][H][W] float32."""
    B = len(insts)
    x = np.zeros((B, H, W, C_IN), dtype=np.float32)
    mask = np.zeros((B, H, W), dtype=np.float32)
    for k, d in enumerate(insts):
        ny, nx = d["ny"], d["nx"]
        yc = (np.arange(ny) + 0.5) / ny
        x[k, :ny, :nx, 0] = 1.0
        x[k, :ny, :nx, 1] = (d["tau"] - 0.875) / 0.325
        x[k, :ny, :nx, 2] = d.get("u_top", 0.0) / 0.08
        x[k, :ny, :nx, 3] = (d.get("T_top", 1.0) - d.get("T_bot", 1.0)) / 0.2
        x[k, :ny, :nx, 4] = ny / 256.0
        x[k, :ny, :nx, 5] = yc[:, None]
        mask[k, :ny, :nx] = 1.0
    return x, mask


def closed_form_profile(d):
    """[4][ny] closed-form steady thermal Couette profile (rho, ux, uy, T) at
    the row centres, rho from uniform pressure with unit mean."""
    ny = d["ny"]
    y = (np.arange(ny) + 0.5) / ny
    U = d.get("u_top", 0.0)
    Tb, Tt = d.get("T_bot", 1.0), d.get("T_top", 1.0)
    T = Tb + (Tt - Tb) * y + U * U / 4.0 * y * (1.0 - y)
    rho = (1.0 / T) / np.mean(1.0 / T)
    return np.stack([rho, U * y, np.zeros(ny), T])


def make_param(insts=None, profiles=None, residual=True):
    """Output parametrisation: offsets and scales of the network's channels
    (fixed constants, or the closed-form profile and the spread of the
    residual over the training set)."""
    if not residual:
        return {"residual": False, "scale": OUT_SCALE.copy()}
    res = np.concatenate([(p - closed_form_profile(d)).T for d, p in zip(insts, profiles)])
    scale = np.maximum(res.std(axis=0), 1e-6)
    return {"residual": True, "scale": scale}


def _offset(d, param):
    if param["residual"]:
        return closed_form_profile(d).T  # [ny][4]
    return np.broadcast_to(OUT_OFFSET, (d["ny"], 4))


def canvas_targets(insts, profiles, H: int, W: int, param=None):
    """Normalised steady fields on the canvas from column profiles [4][ny]."""
    param = param or make_param(residual=False)
    t = np.zeros((len(insts), H, W, 4), dtype=np.float32)
    for k, (d, p) in enumerate(zip(insts, profiles)):
        ny, nx = d["ny"], d["nx"]
        t[k, :ny, :nx, :] = ((p.T - _offset(d, param)) / param["scale"])[:, None, :]
    return t


def predicted_fields(insts, y, param=None):
    """Network output [B][H][W][4] -> per-instance (rho, ux, uy, T) arrays,
    with rho rescaled to unit mean."""
    param = param or make_param(residual=False)
    out = []
    for k, d in enumerate(insts):
        ny, nx = d["ny"], d["nx"]
        f = y[k, :ny, :nx, :].astype(np.float64) * param["scale"] + _offset(d, param)[:, None, :]
        rho = f[..., 0] / f[..., 0].mean()
        T = np.clip(f[..., 3], 0.5, 2.0)
        out.append((rho, f[..., 1], f[..., 2], T))
    return out


def closed_form_fields(insts):
    """The closed-form profiles as (rho, ux, uy, T) fields, a start without
    learning."""
    out = []
    for d in insts:
        p = closed_form_profile(d)
        out.append(tuple(np.repeat(p[c][:, None], d["nx"], axis=1) for c in range(4)))
    return out


def solve_batch(insts, fields=None, max_steps=2_000_000, tol=1e-8, k=100, dtype="f32", tune=None):
    """Batched solve; returns (steps, residuals, profiles, seconds).  tune: a
    result of autotune.autotune_batch (launch shapes only; results do not
    depend on it)."""
    import torch

    b = BatchSolver(insts, dtype=dtype)
    if tune is not None:
        from .autotune import apply_batch_tuning

        apply_batch_tuning(b, tune)
    if fields is None:
        fields = [inputs.uniform_fields(d["nx"], d["ny"]) for d in insts]
    b.set_fields(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok, steps, r = b.run(max_steps, tol, k)
    dt = time.perf_counter() - t0
    # an instance that went non-finite has r = nan and nan fields; the
    # others are unaffected (the caller decides what to do with it)
    prof = [f[:, :, 0] for f in b.fields(allow_nonfinite=True)]
    b.close()
    return steps, r, prof, dt


def generate(n: int, seed: int, batch: int = 256, log=print, start: str = "uniform", **kw):
    """Steady states of n sampled channels, solved in batches of `batch`.

    start: "uniform" (rho = 1, u = 0, T = 1) or "closed_form" (the
    closed-form thermal-Couette profile, about 4x fewer steps to the same
    tolerance; the converged states then differ from the uniform start's
    by what the stopping rule leaves, ~1e-3)."""
    if start not in ("uniform", "closed_form"):
        raise ValueError(f"start must be 'uniform' or 'closed_form', not {start!r}")
    insts = inputs.couette_instances(n, seed=seed)
    profiles, steps = [], []
    for s in range(0, n, batch):
        chunk = insts[s:s + batch]
        fields = closed_form_fields(chunk) if start == "closed_form" else None
        st, r, prof, dt = solve_batch(chunk, fields=fields, **kw)
        if not np.all(r < kw.get("tol", 1e-8)):
            raise RuntimeError(f"data generation: {int(np.sum(~(r < kw.get('tol', 1e-8))))} "
                               "instances did not converge")
        profiles += prof
        steps += list(st)
        log(f"generated {s + len(chunk)}/{n} steady states ({dt:.1f} s, max steps {int(np.max(st))})")
    return insts, profiles, np.array(steps)


def train(net, insts, profiles, H, W, epochs=30, batch=32, lr=2e-3, seed=0, log=print, param=None):
    import torch

    x, mask = canvas_inputs(insts, H, W)
    t = canvas_targets(insts, profiles, H, W, param)
    rng = np.random.default_rng(seed)
    n = len(insts)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = order[s:s + batch]
            xb = torch.as_tensor(x[idx]).cuda()
            tb = torch.as_tensor(t[idx]).cuda()
            mb = torch.as_tensor(mask[idx]).cuda()
            net.forward(xb)
            losses.append(net.backward(tb, mb))
            net.adam_step(lr * (0.5 * (1 + np.cos(np.pi * ep / epochs))))
        hist.append(float(np.mean(losses)))
        log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.3e}")
    return hist


def predict(net, insts, H, W, batch=32):
    import torch

    x, _ = canvas_inputs(insts, H, W)
    ys = []
    for s in range(0, len(insts), batch):
        xb = torch.as_tensor(x[s:s + batch]).cuda()
        ys.append(net.forward(xb).cpu().numpy())
    return np.concatenate(ys)


def init_params(c_in: int, seed: int = 0):
    """He-uniform initial weights, zero biases (flat layout of the C ABI)."""
    rng = np.random.default_rng(seed)
    chans = [c_in, 32, 32, 32, 4]
    parts = []
    for i in range(4):
        lim = np.sqrt(6.0 / (9 * chans[i]))
        parts.append(rng.uniform(-lim, lim, chans[i + 1] * chans[i] * 9))
        parts.append(np.zeros(chans[i + 1]))
    return np.concatenate(parts).astype(np.float32)


def warm_vs_uniform(net, insts, H, W, max_steps=2_000_000, tol=1e-8, log=print, tune=None,
                    param=None, warm_max_steps=None):
    """Solve the same instances from the uniform start, from the closed-form
    profile and from the network's prediction (inference time included);
    returns a summary dict.

    Fallback: a warm-started instance that does not reach tol within
    warm_max_steps (default max_steps) or goes non-finite is solved again
    from the uniform start (its steps and time are added to the warm
    totals), so every instance ends at the steady state the uniform start
    reaches."""
    import torch

    st_u, r_u, prof_u, t_u = solve_batch(insts, max_steps=max_steps, tol=tol, tune=tune)
    st_c, r_c, _, t_c = solve_batch(insts, fields=closed_form_fields(insts), max_steps=max_steps,
                                    tol=tol, tune=tune)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = predict(net, insts, H, W)
    fields = predicted_fields(insts, y, param)
    t_inf = time.perf_counter() - t0
    wmax = max_steps if warm_max_steps is None else warm_max_steps
    st_w, r_w, prof_w, t_w = solve_batch(insts, fields=fields, max_steps=wmax, tol=tol, tune=tune)
    bad = [k for k in range(len(insts)) if not (r_w[k] < tol) or not np.all(np.isfinite(prof_w[k]))]
    t_fb = 0.0
    if bad:
        sub = [insts[k] for k in bad]
        st_f, r_f, prof_f, t_fb = solve_batch(sub, max_steps=max_steps, tol=tol, tune=tune)
        for j, k in enumerate(bad):
            st_w[k] += st_f[j]
            prof_w[k] = prof_f[j]
    err = [float(np.max(np.abs(pw - pu))) for pw, pu in zip(prof_w, prof_u)]
    pred_err, pred_err_T, cf_err = [], [], []
    for k, d in enumerate(insts):
        pf = np.stack([a[:, 0] for a in fields[k]])
        pred_err.append(float(np.max(np.abs(pf[1] - prof_u[k][1])) / max(d["u_top"], 1e-3)))
        dT = max(d.get("T_top", 1.0) - d.get("T_bot", 1.0), 1e-3)
        pred_err_T.append(float(np.max(np.abs(pf[3] - prof_u[k][3])) / dT))
        cf = closed_form_profile(d)
        cf_err.append(float(np.max(np.abs(cf[1] - prof_u[k][1])) / max(d["u_top"], 1e-3)))
    out = {
        "n": len(insts), "fallback_instances": bad,
        "uniform_steps_mean": float(np.mean(st_u)), "warm_steps_mean": float(np.mean(st_w)),
        "uniform_steps_max": int(np.max(st_u)), "warm_steps_max": int(np.max(st_w)),
        "uniform_wall_s": t_u, "warm_wall_s": t_w + t_inf + t_fb, "inference_s": t_inf,
        "fallbacks": len(bad), "steady_field_maxdiff": float(np.max(err)),
        # (nanmedian: a prediction that is not finite is a fallback case)
        "pred_u_err_rel_median": float(np.nanmedian(pred_err)),
        "pred_T_err_rel_median": float(np.nanmedian(pred_err_T)),
        "closed_form_u_err_rel_median": float(np.median(cf_err)),
        "closed_form_steps_mean": float(np.mean(st_c)), "closed_form_steps_max": int(np.max(st_c)),
        "closed_form_wall_s": t_c, "closed_form_converged": bool(np.all(r_c < tol)),
        "speedup_steps_vs_closed_form": float(np.mean(st_c) / np.mean(st_w)),
        "speedup_steps": float(np.mean(st_u) / np.mean(st_w)),
        "speedup_wall": float(t_u / (t_w + t_inf + t_fb)),
    }
    log(json.dumps(out))
    return out


def main(argv=None):
    import argparse

    import torch

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--n-test", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default="warmstart_result.json")
    ap.add_argument("--gen-start", choices=["uniform", "closed_form"], default="uniform",
                    help="start of the training-data solves")
    ap.add_argument("--absolute", action="store_true",
                    help="predict the fields themselves instead of the residual from the "
                         "closed-form profile")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    H, W = 256, 128
    from .autotune import autotune_batch

    tune = autotune_batch(inputs.couette_instances(256, seed=2026))
    log(f"batch tuning: {tune}")
    t0 = time.perf_counter()
    tr, prof, steps = generate(a.n_train, seed=2026, log=log, tune=tune, start=a.gen_start)
    t_gen = time.perf_counter() - t0
    param = make_param(tr, prof, residual=not a.absolute)
    log(f"output parametrisation: residual={param['residual']} scale={param['scale'].tolist()}")
    net = TvNet(C_IN, H, W, max_batch=a.batch)
    net.set_params(init_params(C_IN, seed=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, tr, prof, H, W, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log, param=param)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    te = inputs.couette_instances(a.n_test, seed=2027)
    res = warm_vs_uniform(net, te, H, W, log=log, tune=tune, param=param)
    res.update({"data_generation_s": t_gen, "training_s": t_train, "n_train": a.n_train,
                "epochs": a.epochs, "final_loss": hist[-1], "train_steps_mean": float(np.mean(steps)),
                "residual": param["residual"], "out_scale": param["scale"].tolist(),
                "data_generation_start": a.gen_start})
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    log(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
