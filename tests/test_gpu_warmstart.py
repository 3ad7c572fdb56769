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
