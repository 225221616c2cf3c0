"""Pins of the oracle's 3-D conv net (learned PCG initial guess)."""
import numpy as np
from scipy import ndimage

from oracle import convnet


def test_single_channel_conv_is_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 5, 6, 7))
    w = rng.standard_normal((1, 1, 27))
    z = convnet.conv(x, w, np.array([0.3]))
    ref = ndimage.correlate(x[0], w[0, 0].reshape(3, 3, 3), mode="constant", cval=0.0) + 0.3
    assert np.allclose(z[0], ref, rtol=1e-13, atol=1e-13)


def test_multichannel_conv_is_sum_of_correlations():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 5, 6))
    w = rng.standard_normal((2, 3, 27))
    z = convnet.conv(x, w, np.zeros(2))
    for o in range(2):
        ref = sum(ndimage.correlate(x[i], w[o, i].reshape(3, 3, 3), mode="constant") for i in range(3))
        assert np.allclose(z[o], ref, rtol=1e-12, atol=1e-12)


def test_gradients_by_central_differences():
    rng = np.random.default_rng(2)
    shape = (4, 5, 6)
    x = rng.standard_normal((3,) + shape)
    target = rng.standard_normal(shape)
    params = convnet.init_params(rng)
    for w, b in params:
        b += 0.1 * rng.standard_normal(b.shape)
    L, grads = convnet.loss_and_grads(params, x, target)
    eps = 1e-6
    for li, (w, b) in enumerate(params):
        for idx in [(0, 0, 13), (w.shape[0] - 1, w.shape[1] - 1, 26), (0, w.shape[1] // 2, 4)]:
            old = w[idx]
            w[idx] = old + eps
            Lp, _ = convnet.loss_and_grads(params, x, target)
            w[idx] = old - eps
            Lm, _ = convnet.loss_and_grads(params, x, target)
            w[idx] = old
            fd = (Lp - Lm) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) <= 1e-7 * max(1.0, abs(fd)), (li, idx)
        old = b[0]
        b[0] = old + eps
        Lp, _ = convnet.loss_and_grads(params, x, target)
        b[0] = old - eps
        Lm, _ = convnet.loss_and_grads(params, x, target)
        b[0] = old
        assert abs((Lp - Lm) / (2 * eps) - grads[li][1][0]) <= 1e-7 * max(1.0, abs(grads[li][1][0]))


def test_parameter_count():
    params = convnet.init_params(np.random.default_rng(0))
    assert sum(w.size + b.size for w, b in params) == 15601
