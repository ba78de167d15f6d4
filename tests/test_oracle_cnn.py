"""Pins of the oracle's warm-start network: convolution against SciPy's 2-D
correlation, backward pass against central finite differences, Adam's first
step against its closed form, and bfloat16 rounding against torch."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_conv_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    y = cnn.conv(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(x[n, :, :, ci], W[:, :, ci, co], mode="same")
                              for ci in range(3))
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    theta = cnn.init_params(2) + 0.01 * rng.standard_normal(cnn.n_params())
    x = rng.standard_normal((1, 6, 6, 3))
    t = rng.standard_normal((1, 6, 6))
    m = (rng.uniform(size=(1, 6, 6)) > 0.2).astype(float)
    loss, g = cnn.loss_and_grad(theta, x, t, m)
    idx = rng.choice(cnn.n_params(), 60, replace=False)
    # always include biases of every layer
    starts = np.cumsum([0] + [int(np.prod(s)) for s in cnn.SHAPES])
    idx = np.unique(np.concatenate([idx, starts[1:-1:2] - 1, [starts[-1] - 1]]))
    eps = 1e-6
    for k in idx:
        tp = theta.copy(); tp[k] += eps
        tm = theta.copy(); tm[k] -= eps
        fd = (cnn.loss_and_grad(tp, x, t, m)[0] - cnn.loss_and_grad(tm, x, t, m)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adam_first_step_is_signed_learning_rate():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -7.0, 1e-3])
    new, m, v = cnn.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(new, theta - 0.01 * np.sign(g), atol=1e-15)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, 1000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.005859375]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(a), ref)
