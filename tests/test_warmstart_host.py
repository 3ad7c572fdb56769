"""Host-side pieces of the warm-start pipeline: the closed-form thermal
Couette profile (Sec. IV transport with Pr = 1, c_P = 2) and the output
parametrisation's round trip (no GPU)."""
import numpy as np
import pytest

from paper_1004_5059_amd import inputs, warmstart as ws


def test_closed_form_profile_properties():
    d = dict(nx=8, ny=64, tau=0.7, u_top=0.06, T_bot=1.0, T_top=1.15)
    rho, ux, uy, T = ws.closed_form_profile(d)
    y = (np.arange(64) + 0.5) / 64
    assert np.allclose(ux, 0.06 * y, rtol=0, atol=1e-15)
    assert np.all(uy == 0)
    # energy balance with viscous heating: T'' = -U^2/(2 H^2) in units of y/H
    d2 = np.diff(T, 2) * 64 * 64
    assert np.allclose(d2, -0.06 ** 2 / 2, rtol=1e-9)
    assert abs(T[0] - (1.0 + 0.15 * y[0] + 0.06 ** 2 / 4 * y[0] * (1 - y[0]))) < 1e-15
    # uniform pressure and unit mean density
    P = rho * T
    assert np.ptp(P) < 1e-14 and abs(rho.mean() - 1.0) < 1e-14


@pytest.mark.parametrize("residual", [False, True])
def test_output_parametrisation_round_trip(residual):
    insts = inputs.couette_instances(6, seed=5, sizes=[32, 48])
    rng = np.random.default_rng(0)
    prof = []
    for d in insts:
        p = ws.closed_form_profile(d) + 1e-3 * rng.standard_normal((4, d["ny"]))
        p[0] /= p[0].mean()
        p[3] = np.clip(p[3], 0.6, 1.9)
        prof.append(p)
    param = ws.make_param(insts, prof, residual=residual)
    H, W = 48, 24
    t = ws.canvas_targets(insts, prof, H, W, param)
    f = ws.predicted_fields(insts, t, param)
    for d, p, q in zip(insts, prof, f):
        for c in range(4):
            assert np.allclose(q[c], p[c][:, None], rtol=0, atol=1e-6), c
    # outside each instance the canvas is zero
    for k, d in enumerate(insts):
        assert np.all(t[k, d["ny"]:, :, :] == 0) and np.all(t[k, :, d["nx"]:, :] == 0)
