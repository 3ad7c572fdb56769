"""tvlbm_moments_static, the allocation-free variant of tvlbm_moments,
through the C ABI: its fields, totals and flag agree with tvlbm_moments on
two calls in a row, the second on a smaller grid (the static scratch keeps
the first call's contents), for uniform and non-uniform rows, FP32 and
FP64; oversized grids are refused before anything is enqueued; and it
enqueues nothing but kernels (it is captured into a HIP graph and replayed,
with the program's own work and synchronisations between replays)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1004_5059_amd import inputs  # noqa: E402
from paper_1004_5059_amd import tvlbm  # noqa: E402
from paper_1004_5059_amd.tvlbm import Solver  # noqa: E402


def _static(s):
    fld = torch.full((4, s.ny, s.nx), float("nan"), dtype=s.tdtype, device=s.device)
    tot = torch.full((4,), float("nan"), dtype=torch.float64, device=s.device)
    flag = torch.full((1,), 7, dtype=torch.int32, device=s.device)
    tvlbm.tvlbm_moments_static(s.ctx, fld, tot, flag)
    s.stream.synchronize()
    return fld, tot.cpu().numpy(), int(flag.item())


def _case(nx, ny, dtype, dy=None, walls=False, steps=7, stream=None):
    s = Solver(nx, ny, n_gh=4, dtype=dtype, tau=0.7, dy=dy, walls=walls,
               wall_hi=(0.03, 1.05) if walls else (0.0, 1.0), stream=stream)
    s.set_fields(*inputs.shear_wave_fields(nx, ny, eps=0.02),
                 inputs.population_noise(16, ny, nx, amp=1e-4, seed=3))
    s.step(steps)
    return s


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_static_moments_match_moments_twice(dtype):
    dy = inputs.refined_wall_rows(h=40, band=4)
    cases = [(300, 220, None, False), (70, 33, None, False),
             (96, len(dy), dy, True), (40, len(dy), dy, True)]
    for nx, ny, d, w in cases:  # each pair: a larger grid, then a smaller one
        s = _case(nx, ny, dtype, d, w)
        fld, tot, flag = _static(s)
        ref, ref_tot = s.moments()
        assert flag == 0
        assert torch.equal(fld, ref), (nx, ny)
        np.testing.assert_array_equal(tot, ref_tot)
        s.close()


def test_static_moments_flag_and_nulls():
    s = _case(64, 48, "f32")
    tvlbm.tvlbm_moments_static(s.ctx, None, None, None)  # all outputs optional
    s.stream.synchronize()
    fld, tot, flag = _static(s)
    assert flag == 0 and np.isfinite(tot).all()
    # a non-positive density sets the flag, as tvlbm_moments reports ENONFINITE
    rho, ux, uy, T = inputs.uniform_fields(64, 48)
    rho = rho.copy()
    rho[5, 7] = -0.5
    s.set_fields(rho, ux, uy, T)
    fld, tot, flag = _static(s)
    assert flag == 1
    _, rc = tvlbm.tvlbm_moments(s.ctx, check=False)
    assert rc == tvlbm.TVLBM_ENONFINITE
    s.close()


def test_static_moments_refuses_oversized_grid():
    # 4100 x 4112 with non-uniform rows needs ceil(4100 / 64) x (4112 / 4)
    # = 65 x 1028 = 66,820 blocks of 64 columns x 4 rows, > 65,536
    nx, ny = 4100, 4112
    dy = np.full(ny, 1.0)
    dy[0] = 0.5
    s = Solver(nx, ny, n_gh=4, dtype="f32", tau=0.7, dy=dy)
    s.set_fields(*inputs.uniform_fields(nx, ny))
    with pytest.raises(tvlbm.TvlbmError) as e:
        tvlbm.tvlbm_moments_static(s.ctx, None, None, None)
    assert e.value.code == tvlbm.TVLBM_EINVAL
    assert "static scratch" in tvlbm.tvlbm_last_error(s.ctx)
    s.close()


def test_static_moments_in_a_captured_graph():
    st = torch.cuda.Stream()  # capture needs a stream other than the null stream
    s = _case(128, 96, "f32", stream=st)
    fld = torch.zeros((4, s.ny, s.nx), dtype=torch.float32, device=s.device)
    tot = torch.zeros(4, dtype=torch.float64, device=s.device)
    flag = torch.zeros(1, dtype=torch.int32, device=s.device)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        g.capture_begin()
        tvlbm.tvlbm_moments_static(s.ctx, fld, tot, flag)
        g.capture_end()
    torch.cuda.synchronize()
    for rep in range(3):
        # the program's own work between replays; an even number of steps,
        # so that the state is in the buffer it was in at capture
        s.step(2)
        torch.cuda.synchronize()
        fld.fill_(float("nan"))
        tot.fill_(float("nan"))
        flag.fill_(5)
        g.replay()
        torch.cuda.synchronize()
        ref, ref_tot = s.moments()
        assert torch.equal(fld, ref), rep
        np.testing.assert_array_equal(tot.cpu().numpy(), ref_tot)
        assert int(flag.item()) == 0
    s.close()
