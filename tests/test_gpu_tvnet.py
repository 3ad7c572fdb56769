"""The warm-start network's bf16 MFMA kernels against the FP64 oracle:
forward output to 2e-2 relative, gradients with cosine >= 0.999 per layer,
one Adam step against the oracle's update."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import convnet as cn  # noqa: E402
from paper_1004_5059_amd.tvlbm import TvNet  # noqa: E402


def _bf16(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).float().numpy() \
        .astype(np.float64)


def _setup(B=2, H=13, W=70, c_in=6, seed=0):
    rng = np.random.default_rng(seed)
    params = cn.init_params(c_in, 32, 4, seed=seed)
    params = [(w, 0.1 * rng.standard_normal(b.shape)) for w, b in params]
    x = rng.uniform(-1, 1, (B, H, W, c_in))
    t = 0.5 * rng.standard_normal((B, H, W, 4))
    mask = (rng.random((B, H, W)) > 0.2).astype(np.float64)
    return params, x, t, mask


@pytest.mark.parametrize("shape", [(2, 13, 70), (1, 8, 128), (3, 5, 17)])
def test_forward_and_gradients_match_oracle(shape):
    B, H, W = shape
    params, x, t, mask = _setup(B, H, W)
    net = TvNet(6, H, W, max_batch=B)
    flat = cn.flatten(params)
    net.set_params(flat.astype(np.float32))
    dev = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda()
    y = net.forward(dev(x)).cpu().numpy().astype(np.float64)
    # oracle on the bf16-rounded inputs and weights the kernels consume
    pb = [(_bf16(w), b) for w, b in params]
    y_ref, cache = cn.forward(pb, _bf16(x))
    err = np.max(np.abs(y - y_ref)) / np.max(np.abs(y_ref))
    assert err <= 2e-2, err
    loss = net.backward(dev(t), dev(mask))
    assert abs(loss - cn.loss(y_ref, t, mask)) <= 2e-2 * cn.loss(y_ref, t, mask)
    g = net.grads().astype(np.float64)
    g_ref = cn.flatten(cn.backward(pb, cache, cn.loss_grad(y_ref, t, mask)))
    o = 0
    for w, b in params:
        for arr in (w, b):
            n = arr.size
            a, r = g[o:o + n], g_ref[o:o + n]
            cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r) + 1e-300))
            assert cos >= 0.999, (o, cos)
            assert abs(np.linalg.norm(a) / np.linalg.norm(r) - 1) <= 0.05
            o += n
    net.close()


def test_adam_step_matches_oracle():
    params, x, t, mask = _setup()
    net = TvNet(6, 13, 70, max_batch=2)
    flat = cn.flatten(params).astype(np.float32)
    net.set_params(flat)
    dev = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float32)).cuda()
    net.forward(dev(x))
    net.backward(dev(t), dev(mask))
    g = net.grads().astype(np.float64)
    net.adam_step(1e-3)
    p = flat.astype(np.float64).copy()
    m, v = np.zeros_like(p), np.zeros_like(p)
    cn.adam_step(p, g, m, v, 1, 1e-3)
    np.testing.assert_allclose(net.params(), p, rtol=0, atol=2e-6)
    net.close()
