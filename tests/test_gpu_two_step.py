"""The two-steps-per-launch variants (g^{k+2} from g^k in one sweep) against
the one-step march: bitwise equal populations, fields and totals after odd
and even step counts, on widths around the 62-column strips and on heights
down to two rows, D2Q9, D2Q16 and D2Q36, compensated and plain sums; the
grids the variant does not apply to (non-uniform rows, FP64 D2Q36) run the
one-step march; FP64 D2Q9/D2Q16 bitwise as well; and the oracle on a ragged
grid.  With diffuse walls (strips of 60 columns, the walls' ghosts of the
intermediate step formed in the sweep) the same bitwise equality on widths
around the strip and heights down to two rows, and the oracle.""" 
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_common import c0_inputs, make_pair, rel_inf  # noqa: E402
from paper_1004_5059_amd import inputs, tvlbm  # noqa: E402
from paper_1004_5059_amd.tvlbm import Solver  # noqa: E402

# the variant table's two-step entries (output rows per segment 3, 4, 5, 6,
# 8, 7, 9, 10, 12)
TWO = [19, 20, 21, 22, 23, 24, 25, 26, 27]


def _solver(nx, ny, n, variant, dtype="f32", compensated=True, walls=False, tau=0.7):
    s = Solver(nx, ny, n_gh=n, dtype=dtype, tau=tau, compensated=compensated, walls=walls,
               wall_hi=(0.03, 1.05))
    s.set_variant(variant)
    return s


def _state(s):
    F, tot = s.moments()
    return s.populations().cpu().numpy(), F.cpu().numpy(), np.asarray(tot)


def test_variant_table_has_the_two_step_entries():
    assert tvlbm.tvlbm_num_variants() == 28
    s = _solver(64, 16, 4, TWO[0])
    assert s.steps_per_launch() == 2
    s.set_variant(0)
    assert s.steps_per_launch() == 1
    s.close()
    s = _solver(64, 16, 4, TWO[0], walls=True)
    assert s.steps_per_launch() == 2
    s.close()
    s = Solver(64, 16, n_gh=4, dtype="f32", tau=0.7, walls=True, dy=np.r_[np.full(4, 0.5), np.ones(14)][:16])
    s.set_variant(TWO[0])
    assert s.steps_per_launch() == 1  # non-uniform rows
    s.close()
    s = _solver(64, 16, 4, TWO[0], dtype="f64")
    assert s.steps_per_launch() == 2
    s.close()
    s = _solver(64, 16, 6, TWO[0], dtype="f64")
    assert s.steps_per_launch() == 1
    s.close()
    s = _solver(64, 16, 6, TWO[0])
    assert s.steps_per_launch() == 2
    s.close()


@pytest.mark.parametrize("n", [3, 4, 6])
@pytest.mark.parametrize("nx,ny", [(2, 2), (5, 3), (61, 9), (62, 17), (63, 2), (124, 33),
                                   (125, 40), (190, 5)])
def test_two_step_matches_one_step_bitwise(n, nx, ny):
    fields, noise = c0_inputs(nx, ny, q=n * n, seed=nx + ny)
    ref = _solver(nx, ny, n, 0)
    ref.set_fields(*fields, noise)
    runs = []
    for v in TWO:
        s = _solver(nx, ny, n, v)
        s.set_fields(*fields, noise)
        runs.append(s)
    for k in (1, 2, 3, 5, 8):  # cumulative 1, 3, 6, 11, 19 steps
        ref.step(k)
        want = _state(ref)
        for v, s in zip(TWO, runs):
            s.step(k)
            got = _state(s)
            for a, b in zip(got, want):
                assert np.array_equal(a, b), (v, k)
    for s in runs + [ref]:
        s.close()


@pytest.mark.parametrize("compensated", [True, False])
def test_two_step_plain_and_compensated_sums(compensated):
    nx, ny = 130, 37
    fields, noise = c0_inputs(nx, ny, q=16, seed=5)
    a, b = _solver(nx, ny, 4, 0, compensated=compensated), _solver(nx, ny, 4, 22, compensated=compensated)
    for s in (a, b):
        s.set_fields(*fields, noise)
        s.step(14)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.close(), b.close()


@pytest.mark.parametrize("kw", [dict(n=6, dtype="f64"), dict(n=6, dtype="f64", walls=True),
                                dict(refined=True), dict(refined=True, walls=True)])
def test_grids_outside_the_two_step_kernel_run_the_one_step_march(kw):
    n = kw.pop("n", 4)
    nx, ny = 70, 29
    fields, noise = c0_inputs(nx, ny, q=n * n, seed=9)
    if kw.pop("refined", False):
        dy = np.r_[np.full(6, 0.5), np.ones(ny - 6)]
        a = Solver(nx, ny, n_gh=n, tau=0.7, dy=dy, **kw)
        b = Solver(nx, ny, n_gh=n, tau=0.7, dy=dy, **kw)
        b.set_variant(22)
    else:
        a, b = _solver(nx, ny, n, 0, **kw), _solver(nx, ny, n, 22, **kw)
    assert b.steps_per_launch() == 1
    for s in (a, b):
        s.set_fields(*fields, noise)
        s.step(9)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.close(), b.close()


@pytest.mark.parametrize("variant", TWO)
def test_two_step_against_the_oracle(variant):
    """D2Q16 FP32 on a ragged 131 x 45 grid, 13 steps (6 two-step launches
    and a single step), every population within 1e-5 of the FP64 oracle,
    mass and energy conserved."""
    nx, ny, K = 131, 45, 13
    s, g = make_pair(nx, ny, n=4, dtype="f32", tau=0.6, variant=variant)
    fields = inputs.smoothed_density_fields(nx, ny, std=0.01, t_amp=0.05, seed=3)
    noise = inputs.population_noise(16, ny, nx, amp=1e-4, seed=4)
    s.set_fields(*fields, noise)
    _, t0 = s.moments()
    s.step(K)
    _, t1 = s.moments()
    fr = g.run(g.set_fields(*fields, noise), K)
    assert rel_inf(s.populations().cpu().numpy(), fr) <= 1e-5
    assert abs(t1[0] - t0[0]) / t0[0] <= 1e-6 and abs(t1[3] - t0[3]) / t0[3] <= 1e-6
    s.close()


def test_two_step_full_size_bitwise():
    """1024 x 1024 D2Q16, the benchmark's initial state, 11 steps: every
    population equal to the one-step march's."""
    N = 1024
    fields = inputs.smoothed_density_fields(N, N, std=0.01, t_amp=0.05, seed=1)
    out = []
    for v in (0, 22):
        s = _solver(N, N, 4, v, tau=0.6)
        s.set_fields(*fields)
        s.step(11)
        out.append(s.populations().cpu().numpy())
        s.close()
    assert np.array_equal(out[0], out[1])


def test_two_step_d2q36_against_the_oracle():
    """D2Q36 (order 4) FP32, 77 x 40, 9 steps (4 two-step launches and a
    single step), within 1e-5 of the FP64 oracle."""
    nx, ny, K = 77, 40, 9
    s, g = make_pair(nx, ny, n=6, dtype="f32", tau=0.6, variant=22)
    assert s.steps_per_launch() == 2
    fields = inputs.smoothed_density_fields(nx, ny, std=0.01, t_amp=0.05, seed=5)
    noise = inputs.population_noise(36, ny, nx, amp=1e-4, seed=6)
    s.set_fields(*fields, noise)
    s.step(K)
    fr = g.run(g.set_fields(*fields, noise), K)
    assert rel_inf(s.populations().cpu().numpy(), fr) <= 1e-5
    s.close()


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("nx,ny", [(5, 3), (62, 17), (125, 40)])
def test_two_step_fp64_matches_one_step_bitwise(n, nx, ny):
    fields, noise = c0_inputs(nx, ny, q=n * n, seed=nx)
    a, b = _solver(nx, ny, n, 0, dtype="f64"), _solver(nx, ny, n, 22, dtype="f64")
    assert b.steps_per_launch() == 2
    for s in (a, b):
        s.set_fields(*fields, noise)
    for k in (1, 4, 7):
        a.step(k), b.step(k)
        for x, y in zip(_state(a), _state(b)):
            assert np.array_equal(x, y), k
    a.close(), b.close()


def test_two_step_fp64_against_the_oracle():
    """D2Q16 FP64, 131 x 45, 13 steps, within 1e-12 of the oracle."""
    nx, ny, K = 131, 45, 13
    s, g = make_pair(nx, ny, n=4, dtype="f64", tau=0.6, variant=22)
    fields = inputs.smoothed_density_fields(nx, ny, std=0.01, t_amp=0.05, seed=3)
    noise = inputs.population_noise(16, ny, nx, amp=1e-4, seed=4)
    s.set_fields(*fields, noise)
    s.step(K)
    fr = g.run(g.set_fields(*fields, noise), K)
    assert rel_inf(s.populations().cpu().numpy(), fr) <= 1e-12
    s.close()


def test_checkpoint_across_one_and_two_step_variants(tmp_path):
    """Saved after 9 steps with a two-step variant (4 two-step launches and a
    single step), loaded into a solver on the one-step variant, continued 6
    steps: the same populations, fields and totals as 15 one-step steps."""
    from paper_1004_5059_amd import tvlbm as T

    nx, ny = 130, 37
    fields, noise = c0_inputs(nx, ny, q=16, seed=8)
    ref = _solver(nx, ny, 4, 0)
    ref.set_fields(*fields, noise)
    ref.step(15)
    s = _solver(nx, ny, 4, 22)
    s.set_fields(*fields, noise)
    s.step(9)
    p = str(tmp_path / "ck.bin")
    T.tvlbm_save(s.ctx, p)
    s.close()
    t = _solver(nx, ny, 4, 0)
    T.tvlbm_load(t.ctx, p)
    assert t.step_count == 9
    t.step(6)
    for x, y in zip(_state(t), _state(ref)):
        assert np.array_equal(x, y)
    t.close(), ref.close()


@pytest.mark.parametrize("variant", TWO)
def test_c0_shear_wave_two_step_fp64(variant):
    """The 64 x 64 FP64 case (tau 0.8, shear wave plus noise, 200 steps) on
    the two-step variants: within 1e-12 of the oracle."""
    s, g = make_pair(64, 64, n=4, dtype="f64", tau=0.8, variant=variant)
    assert s.steps_per_launch() == 2
    fields, noise = c0_inputs()
    s.set_fields(*fields, noise)
    s.step(200)
    fr = g.run(g.set_fields(*fields, noise), 200)
    assert rel_inf(s.populations().cpu().numpy(), fr) <= 1e-12
    s.close()


WALLS = dict(walls=True, wall_lo=(-0.01, 0.97), wall_hi=(0.04, 1.12))


def _wsolver(nx, ny, n, variant, dtype="f32", tau=0.7):
    s = Solver(nx, ny, n_gh=n, dtype=dtype, tau=tau, **WALLS)
    s.set_variant(variant)
    return s


@pytest.mark.parametrize("n", [3, 4, 6])
@pytest.mark.parametrize("nx,ny", [(2, 2), (5, 3), (59, 9), (60, 17), (61, 2), (121, 33),
                                   (130, 40), (190, 5)])
def test_walled_two_step_matches_one_step_bitwise(n, nx, ny):
    fields, noise = c0_inputs(nx, ny, q=n * n, seed=3 * nx + ny)
    ref = _wsolver(nx, ny, n, 0)
    ref.set_fields(*fields, noise)
    runs = []
    for v in TWO:
        s = _wsolver(nx, ny, n, v)
        assert s.steps_per_launch() == 2
        s.set_fields(*fields, noise)
        runs.append(s)
    for k in (1, 2, 3, 5, 8):  # cumulative 1, 3, 6, 11, 19 steps
        ref.step(k)
        want = _state(ref)
        for v, s in zip(TWO, runs):
            s.step(k)
            got = _state(s)
            for a, b in zip(got, want):
                assert np.array_equal(a, b), (v, k)
    for s in runs + [ref]:
        s.close()


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("nx,ny", [(5, 3), (60, 17), (125, 40)])
def test_walled_two_step_fp64_matches_one_step_bitwise(n, nx, ny):
    fields, noise = c0_inputs(nx, ny, q=n * n, seed=nx + 7)
    a, b = _wsolver(nx, ny, n, 0, "f64"), _wsolver(nx, ny, n, 22, "f64")
    assert b.steps_per_launch() == 2
    for s in (a, b):
        s.set_fields(*fields, noise)
    for k in (1, 4, 7):
        a.step(k), b.step(k)
        for x, y in zip(_state(a), _state(b)):
            assert np.array_equal(x, y), k
    a.close(), b.close()


@pytest.mark.parametrize("n,dtype,tol", [(4, "f32", 1e-5), (4, "f64", 1e-12), (6, "f32", 1e-5)])
def test_walled_two_step_against_the_oracle(n, dtype, tol):
    """Walled 131 x 45 grid, 21 steps (10 two-step launches and a single
    step), against the FP64 oracle; mass conserved by the walls."""
    nx, ny, K = 131, 45, 21
    s, g = make_pair(nx, ny, n=n, dtype=dtype, tau=0.6, variant=22, **WALLS)
    assert s.steps_per_launch() == 2
    fields = inputs.shear_wave_fields(nx, ny, eps=0.02)
    noise = inputs.population_noise(n * n, ny, nx, amp=1e-4, seed=12)
    s.set_fields(*fields, noise)
    _, t0 = s.moments()
    s.step(K)
    _, t1 = s.moments()
    fr = g.run(g.set_fields(*fields, noise), K)
    assert rel_inf(s.populations().cpu().numpy(), fr) <= tol
    assert abs(t1[0] - t0[0]) / t0[0] <= (1e-13 if dtype == "f64" else 1e-6)
    s.close()


@pytest.mark.parametrize("walls", [False, True])
def test_state_after_even_two_step_runs(tmp_path, walls):
    """An even step count on a two-step variant ends with a two-step launch,
    and g^{k-1} (from which f^k, the fields and the totals come) is formed
    when first asked for.  Every way of observing the state right after such
    runs -- moments, the allocation-free moments, populations, the residual,
    a checkpoint -- and stepping on afterwards must match single steps
    bitwise."""
    from paper_1004_5059_amd import tvlbm as T

    nx, ny = 70, 23
    kw = WALLS if walls else {}
    fields, noise = c0_inputs(nx, ny, q=16, seed=31)
    ref = Solver(nx, ny, n_gh=4, dtype="f32", tau=0.7, **kw)
    ref.set_fields(*fields, noise)
    s = Solver(nx, ny, n_gh=4, dtype="f32", tau=0.7, **kw)
    s.set_variant(22)
    assert s.steps_per_launch() == 2
    s.set_fields(*fields, noise)
    for k in (2, 4, 6):  # cumulative 2, 6, 12: all two-step launches
        ref.step(k)
        s.step(k)
        fld = torch.empty((4, ny, nx), dtype=torch.float32, device="cuda:0")
        tot = torch.empty(4, dtype=torch.float64, device="cuda:0")
        T.tvlbm_moments_static(s.ctx, fld, tot, None)  # the first observer forms g^{k-1}
        torch.cuda.synchronize()
        F, t_ref = ref.moments()
        assert np.array_equal(fld.cpu().numpy(), F.cpu().numpy()), k
        assert np.array_equal(tot.cpu().numpy(), np.asarray(t_ref)), k
        for x, y in zip(_state(s), _state(ref)):
            assert np.array_equal(x, y), k
    # the residual of a solve over even chunks, and a checkpoint taken right
    # after a two-step launch, continued on the one-step variant
    s.residual(), ref.residual()  # snapshots
    ref.step(8)
    s.step(8)
    r_s, r_ref = s.residual(), ref.residual()
    assert np.isfinite(r_s) and r_s == r_ref
    ref.step(4)
    s.step(4)
    p = str(tmp_path / "ck.bin")
    T.tvlbm_save(s.ctx, p)
    t = Solver(nx, ny, n_gh=4, dtype="f32", tau=0.7, **kw)
    T.tvlbm_load(t.ctx, p)
    assert t.step_count == ref.step_count
    for x, y in zip(_state(t), _state(ref)):
        assert np.array_equal(x, y)
    t.step(5)
    ref.step(5)
    for x, y in zip(_state(t), _state(ref)):
        assert np.array_equal(x, y)
    for x in (s, t, ref):
        x.close()
