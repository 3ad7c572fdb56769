"""The learned warm start end to end at reduced size: steady states from
batched solves, training of the bf16-MFMA network, and the steps a
warm-started batched solve saves over the uniform start on held-out
instances (the fallback re-solve from uniform must not be needed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1004_5059_amd import inputs, warmstart as ws  # noqa: E402
from paper_1004_5059_amd.tvlbm import TvNet  # noqa: E402


@pytest.mark.parametrize("residual", [False, True])
def test_warm_start_saves_steps_on_held_out_instances(residual):
    H, W = 64, 32
    sizes = [32, 48, 64]
    train = inputs.couette_instances(96, seed=11, sizes=sizes)
    _, _, prof, _ = ws.solve_batch(train)
    param = ws.make_param(train, prof, residual=residual)
    net = TvNet(ws.C_IN, H, W, max_batch=16)
    net.set_params(ws.init_params(ws.C_IN, seed=0))
    hist = ws.train(net, train, prof, H, W, epochs=60, batch=16, lr=3e-3, log=lambda s: None,
                    param=param)
    assert hist[-1] < 0.2 * hist[0]
    test = inputs.couette_instances(16, seed=12, sizes=sizes)
    res = ws.warm_vs_uniform(net, test, H, W, log=print, param=param)
    assert res["fallbacks"] == 0
    assert res["warm_steps_mean"] < res["uniform_steps_mean"]
    assert res["steady_field_maxdiff"] < 1e-3
    net.close()


# --- fallback: a warm-started instance that does not converge, or goes
# non-finite, is solved again from the uniform start.  Per-instance results
# of the batched solve do not depend on the other instances in the batch
# (tested bitwise elsewhere), so the re-solved instances must end exactly
# where the uniform start's solve ends, after exactly its steps.
FB_SIZES = [32, 48]
FB_H, FB_W = 64, 32


def test_fallback_when_the_warm_solve_runs_out_of_steps():
    test = inputs.couette_instances(6, seed=21, sizes=FB_SIZES)
    net = TvNet(ws.C_IN, FB_H, FB_W, max_batch=16)
    net.set_params(ws.init_params(ws.C_IN, seed=0))  # untrained
    budget = 200
    res = ws.warm_vs_uniform(net, test, FB_H, FB_W, log=print, param=ws.make_param(residual=False),
                             warm_max_steps=budget)
    net.close()
    assert res["fallbacks"] == len(test)
    assert res["fallback_instances"] == list(range(len(test)))
    assert res["steady_field_maxdiff"] == 0.0
    n = len(test)
    assert round(res["warm_steps_mean"] * n) == round(res["uniform_steps_mean"] * n) + budget * n
    assert res["warm_steps_max"] == res["uniform_steps_max"] + budget


def test_fallback_on_a_non_finite_prediction(monkeypatch):
    test = inputs.couette_instances(6, seed=22, sizes=FB_SIZES)

    def bad_predict(net, insts, H, W, batch=32):
        # zeros are the uniform start in the fixed output parametrisation;
        # instance 2's prediction is not finite
        y = np.zeros((len(insts), H, W, 4), dtype=np.float32)
        y[2, :, :, 0] = np.nan
        return y

    monkeypatch.setattr(ws, "predict", bad_predict)
    res = ws.warm_vs_uniform(None, test, FB_H, FB_W, log=print, param=ws.make_param(residual=False))
    assert res["fallback_instances"] == [2]
    assert res["fallbacks"] == 1
    assert res["steady_field_maxdiff"] == 0.0
    # instance 2 spent one residual interval (100 steps) before its NaN
    # residual stopped it
    n = len(test)
    assert round(res["warm_steps_mean"] * n) == round(res["uniform_steps_mean"] * n) + 100
