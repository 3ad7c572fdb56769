"""Batched steady solves: every instance of a batch must equal the same
instance solved alone through the single-instance path (bitwise: the same
per-cell arithmetic runs in both), and match the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_common import rel_inf, to_np  # noqa: E402
from oracle import oracle as orc  # noqa: E402
from paper_1004_5059_amd import inputs  # noqa: E402
from paper_1004_5059_amd.tvlbm import BatchSolver, Solver  # noqa: E402

INST = [
    dict(nx=16, ny=32, tau=0.6, u_top=0.03, T_top=1.05),
    dict(nx=24, ny=48, tau=1.1, u_top=0.07, T_top=1.18),
    dict(nx=40, ny=80, tau=0.8, u_top=0.0, T_top=1.1),
    dict(nx=64, ny=128, tau=0.7, u_top=0.05, T_top=1.0),
    dict(nx=100, ny=20, tau=0.9, u_top=0.02, T_top=1.02),
]


def _single(d, dtype, steps, k):
    """The same instance alone, through the single-grid solve (residual
    checks, and in FP32 the mass put back, every k steps, as a batched run
    does)."""
    s = Solver(d["nx"], d["ny"], n_gh=4, dtype=dtype, tau=d["tau"], walls=True,
               wall_lo=(0.0, 1.0), wall_hi=(d["u_top"], d["T_top"]))
    s.set_fields(*inputs.uniform_fields(d["nx"], d["ny"]))
    conv, n, r = s.solve(steps, 0.0, k)
    assert not conv and n == steps
    f = to_np(s.moments()[0])
    s.close()
    return f


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_equals_single_instance_runs(dtype):
    b = BatchSolver(INST, dtype=dtype)
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in INST])
    ok, steps, r = b.run(max_steps=300, tol=0.0, k_interval=100)
    assert not ok and np.all(steps == 300)
    out = b.fields()
    for d, f in zip(INST, out):
        assert np.array_equal(f, _single(d, dtype, 300, 100)), d
    b.close()


def test_batch_shapes_do_not_change_results():
    res = []
    for shape in [None, (128, 16, 4), (128, 32, 16), (128, 64, 1)]:
        b = BatchSolver(INST, dtype="f32")
        if shape:
            b.set_shape(*shape)
        b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in INST])
        b.run(max_steps=100, tol=0.0, k_interval=50)
        res.append(b.fields())
        b.close()
    for r in res[1:]:
        for a, c in zip(r, res[0]):
            assert np.array_equal(a, c)


def test_batch_against_oracle_fp64():
    inst = INST[:3]
    b = BatchSolver(inst, dtype="f64")
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in inst])
    b.run(max_steps=60, tol=0.0, k_interval=20)
    out = b.fields()
    lat = orc.OracleLattice(4, 3)
    for d, f in zip(inst, out):
        g = orc.OracleGrid(lat, d["nx"], d["ny"], tau=d["tau"], walls=True, wall_lo=(0.0, 1.0),
                           wall_hi=(d["u_top"], d["T_top"]))
        ref = g.fields(g.run(g.set_fields(*inputs.uniform_fields(d["nx"], d["ny"])), 60))
        assert rel_inf(f[0], ref[0]) <= 1e-12 and rel_inf(f[3], ref[3]) <= 1e-12
        assert np.max(np.abs(f[1] - ref[1])) <= 1e-12 * max(1.0, np.max(np.abs(ref[1])))


def test_batch_retires_converged_instances_like_single_solves():
    inst = [dict(nx=16, ny=32, tau=0.9, u_top=0.04, T_top=1.1),
            dict(nx=24, ny=48, tau=0.6, u_top=0.02, T_top=1.05)]
    b = BatchSolver(inst, dtype="f32")
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in inst])
    ok, steps, r = b.run(max_steps=400000, tol=1e-8, k_interval=100)
    assert ok and np.all(r < 1e-8)
    out = b.fields()
    for d, f, st in zip(inst, out, steps):
        s = Solver(d["nx"], d["ny"], n_gh=4, dtype="f32", tau=d["tau"], walls=True,
                   wall_lo=(0.0, 1.0), wall_hi=(d["u_top"], d["T_top"]))
        s.set_fields(*inputs.uniform_fields(d["nx"], d["ny"]))
        conv, n, rr = s.solve(400000, 1e-8, 100)
        assert conv and n == st
        assert np.array_equal(to_np(s.moments()[0]), f)
        s.close()
    assert steps[0] != steps[1]
    b.close()


@pytest.mark.parametrize("tuning", [dict(prefetch=0), dict(prefetch=1, tail_active=1, tail_rows=1),
                                    dict(prefetch=0, tail_active=2, tail_width=32, tail_rows=2),
                                    dict(prefetch=0, tail_active=3, tail_width=16, tail_rows=5),
                                    dict(two_step=0),
                                    dict(two_step=0, tail_active=2, tail_width=32, tail_rows=2),
                                    dict(two_step=1, two_rows=3),
                                    dict(two_step=1, two_rows=16, tail_active=1, tail_rows=1),
                                    dict(two_step=1, two_rows=5, tail_active=3, tail_rows=7)])
def test_batch_tuning_does_not_change_results(tuning):
    """Prefetch on/off, one or two steps per launch (rows per segment), and
    the switch to the tail work list (taken when the first instance retires,
    or from the start when tail_active >= n) keep the steps and the fields
    bitwise."""
    inst = [dict(nx=16, ny=32, tau=0.9, u_top=0.04, T_top=1.1),
            dict(nx=40, ny=48, tau=0.6, u_top=0.02, T_top=1.05),
            dict(nx=70, ny=36, tau=0.75, u_top=0.05, T_top=1.15)]
    res = []
    for t in (None, tuning):
        b = BatchSolver(inst, dtype="f32")
        if t:
            b.set_tuning(**t)
            got = b.tuning()
            assert all(got[k] == v for k, v in t.items())
        b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in inst])
        ok, steps, r = b.run(max_steps=400000, tol=1e-8, k_interval=100)
        assert ok
        res.append((steps, b.fields()))
        b.close()
    assert np.array_equal(res[0][0], res[1][0])
    for a, c in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, c)


def test_batch_tuning_rejects_bad_values():
    b = BatchSolver(INST[:1], dtype="f32")
    for bad in [dict(prefetch=2), dict(tail_active=-1), dict(tail_width=48), dict(tail_rows=0),
                dict(tail_rows=256), dict(two_step=2), dict(two_rows=0), dict(two_rows=256)]:
        with pytest.raises(Exception):
            b.set_tuning(**bad)
    b.close()


def test_fp32_steady_solves_keep_their_mass():
    """FP32 batched and single solves to r < 1e-8 of channels with large wall
    temperature differences (the collision's FP32 rounding drifts the mass
    by ~1e-9 per step there): the starting mass is put back at every
    residual check, so the drift over the solve stays below 1e-6, and the
    batched solve equals the single solves bitwise."""
    inst = [dict(nx=48, ny=96, tau=0.7, u_top=0.06, T_top=1.19),
            dict(nx=32, ny=64, tau=1.1, u_top=0.02, T_top=1.2)]
    b = BatchSolver(inst, dtype="f32")
    b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in inst])
    ok, steps, r = b.run(max_steps=2_000_000, tol=1e-8, k_interval=100)
    assert ok
    out = b.fields()
    b.close()
    for d, f, st in zip(inst, out, steps):
        mass = float(np.sum(f[0].astype(np.float64)))
        drift = abs(mass - d["nx"] * d["ny"]) / (d["nx"] * d["ny"])
        print(f"{d}: {st} steps, mass drift {drift:.2e}")
        assert drift <= 1e-6
        s = Solver(d["nx"], d["ny"], n_gh=4, dtype="f32", tau=d["tau"], walls=True,
                   wall_lo=(0.0, 1.0), wall_hi=(d["u_top"], d["T_top"]))
        s.set_fields(*inputs.uniform_fields(d["nx"], d["ny"]))
        m0 = s.moments()[1][0]
        conv, n, rr = s.solve(2_000_000, 1e-8, 100)
        fld, tot = s.moments()
        assert conv and n == st
        assert abs(tot[0] - m0) / m0 <= 1e-6
        assert np.array_equal(to_np(fld), f)
        s.close()


def test_batch_two_step_k_not_multiple_of_four():
    """K = 50 (chunks of 24 two-step launches and two single steps): the same
    result as one step per launch."""
    inst = INST[:3]
    res = []
    for t in (dict(two_step=0), dict(two_step=1)):
        b = BatchSolver(inst, dtype="f32")
        b.set_tuning(**t)
        b.set_fields([inputs.uniform_fields(d["nx"], d["ny"]) for d in inst])
        b.run(max_steps=150, tol=0.0, k_interval=50)
        res.append(b.fields())
        b.close()
    for a, c in zip(*res):
        assert np.array_equal(a, c)
