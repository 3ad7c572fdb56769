"""Parity at the throughput configuration's horizon: the C1 recipe (periodic,
FP32 populations, tau 0.6, rho = 1 + 0.01 smoothed N(0,1), T = 1 + 0.05
sin(2 pi x / N), u = 0) on 256 x 256 for 1000 steps, D2Q16 (order 3) and
D2Q36 (order 4), for the one-step launch shape (variant 0), the column-pair
step (14) and the two-step sweep (22): every population within 1e-5 of the
FP64 oracle (relative infinity norm), density and temperature likewise, the
velocity within the bound the population bar implies (|du| <= sum_l |xi_l|
times the population error bar, 1e-5 max|f|: u is a small difference of
O(1) populations, so its FP32 error is that of the populations, not 1e-5 of
u), and the FP64 totals of the GPU state conserved to 1e-6 over the 1000
steps."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_common import rel_inf, to_np  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_1004_5059_amd import inputs  # noqa: E402
from paper_1004_5059_amd.tvlbm import LATTICE_ORDER, Solver  # noqa: E402

N, STEPS, TAU = 256, 1000, 0.6
_ref = {}


def _oracle(n):
    if n not in _ref:
        lat = orc.OracleLattice(n, LATTICE_ORDER[n])
        g = orc.OracleGrid(lat, N, N, tau=TAU)
        f0 = g.set_fields(*inputs.smoothed_density_fields(N, N, std=0.01, t_amp=0.05, seed=1))
        f = g.run(f0, STEPS)
        _ref[n] = (g, f)
    return _ref[n]


@pytest.mark.parametrize("n", [4, 6])
@pytest.mark.parametrize("variant", [0, 14, 22])
def test_c1_recipe_1000_steps(n, variant):
    g, f_ref = _oracle(n)
    s = Solver(N, N, n_gh=n, dtype="f32", tau=TAU)
    s.set_variant(variant)
    s.set_fields(*inputs.smoothed_density_fields(N, N, std=0.01, t_amp=0.05, seed=1))
    t0 = s.moments()[1]
    s.step(STEPS)
    f = to_np(s.populations())
    err = rel_inf(f, f_ref)
    fld, t1 = s.moments()
    fld = to_np(fld)
    ref = g.fields(f_ref)
    print(f"D2Q{n * n} variant {variant} ({s.steps_per_launch()} step(s)/launch): "
          f"populations {err:.2e}, mass {abs(t1[0] - t0[0]) / t0[0]:.2e}, "
          f"energy {abs(t1[3] - t0[3]) / t0[3]:.2e}")
    assert err <= 1e-5
    assert rel_inf(fld[0], ref[0]) <= 1e-5 and rel_inf(fld[3], ref[3]) <= 1e-5
    du_bar = np.sum(np.hypot(g.lat.xi[:, 0], g.lat.xi[:, 1])) * 1e-5 * np.max(np.abs(f_ref))
    for c in (1, 2):
        du = np.max(np.abs(fld[c] - ref[c]))
        print(f"  u{'xy'[c - 1]}: max |du| {du:.2e} (bar {du_bar:.2e})")
        assert du <= du_bar
    assert abs(t1[0] - t0[0]) / t0[0] <= 1e-6
    assert abs(t1[3] - t0[3]) / t0[3] <= 1e-6
    scale = np.sum(np.abs(f_ref)) * np.max(np.abs(g.lat.xi))
    assert abs(t1[1] - t0[1]) / scale <= 1e-6 and abs(t1[2] - t0[2]) / scale <= 1e-6
    s.close()
