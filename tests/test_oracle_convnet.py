"""Pins of the FP64 warm-start-network oracle: convolution against scipy's
correlate, gradients against central finite differences, Adam's first step
against its closed form (|update| = lr for every coordinate with g != 0)."""
import numpy as np
from scipy.signal import correlate

from oracle import convnet as cn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cn.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate(x[bi, :, :, c], w[o, c], mode="same") for c in range(3))
            np.testing.assert_allclose(out[bi, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    c_in = 3
    params = cn.init_params(c_in, width=5, c_out=4, seed=2)
    x = rng.standard_normal((2, 6, 5, c_in))
    t = rng.standard_normal((2, 6, 5, 4))
    mask = (rng.random((2, 6, 5)) > 0.3).astype(float)
    y, cache = cn.forward(params, x)
    grads = cn.backward(params, cache, cn.loss_grad(y, t, mask))
    flat = cn.flatten(params)
    gflat = cn.flatten(grads)
    h = 1e-6
    idx = rng.choice(flat.size, 40, replace=False)
    for k in idx:
        fp = flat.copy(); fp[k] += h
        fm = flat.copy(); fm[k] -= h
        lp = cn.loss(cn.forward(cn.unflatten(fp, c_in, 5), x)[0], t, mask)
        lm = cn.loss(cn.forward(cn.unflatten(fm, c_in, 5), x)[0], t, mask)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, fd, gflat[k])


def test_gelu_grad_matches_finite_difference():
    z = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (cn.gelu(z + h) - cn.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(cn.gelu_grad(z), fd, atol=1e-8)


def test_adam_first_step_closed_form():
    p = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    m, v = np.zeros(5), np.zeros(5)
    cn.adam_step(p, g, m, v, 1, lr=1e-3, eps=1e-14)
    np.testing.assert_allclose(np.abs(p[g != 0]), 1e-3, rtol=1e-12)
    assert np.all(np.sign(p[g != 0]) == -np.sign(g[g != 0]))
    assert p[3] == 0.0


def test_gelu_matches_tabulated_normal_cdf():
    """GELU(z) = z Phi(z) with Phi the standard normal CDF, here from its
    table (Phi(-z) = 1 - Phi(z)); the tanh approximation of GELU is off by
    ~1e-4 at z = 1 and fails this."""
    phi = {0.5: 0.6914624612740131, 1.0: 0.8413447460685429, 1.5: 0.9331927987311419,
           2.0: 0.9772498680518208, 2.5: 0.9937903346742238, 3.0: 0.9986501019683699}
    z = np.array([0.0] + [s * v for v in phi for s in (1.0, -1.0)])
    want = np.array([0.0] + [s * v * (phi[v] if s > 0 else 1.0 - phi[v])
                             for v in phi for s in (1.0, -1.0)])
    np.testing.assert_allclose(cn.gelu(z), want, rtol=1e-14, atol=1e-16)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so
    each update is lr g / (|g| + eps): after t steps p = -t lr sign(g) for
    eps << |g|.  A bias correction with the wrong power of t fails at t >= 2."""
    g = np.array([1.0, -2.0, 0.5, 3.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 7):
        cn.adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-14)
        np.testing.assert_allclose(p, -t * 1e-3 * np.sign(g), rtol=1e-11)
