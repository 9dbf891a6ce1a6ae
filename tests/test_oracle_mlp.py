"""Pins of the FP64 network reference (oracle/mlp.py) against facts that do not come
from it: the normal CDF's tabulated value, the odd part of GELU, central finite
differences of the loss, the closed form of Adam's first steps, and the exact kernel
it trains on (a unit delta at w = 0, the side rule)."""
import math

import numpy as np

from oracle import mlp
from oracle.wkernel import nk_rule

TINY = [5, 7, 6, 9]          # two hidden layers, 8 kernel outputs + 1 error output


def test_gelu_closed_forms():
    # Phi(1) = 0.8413447460685429 (standard normal table)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    z = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)   # z Phi(z) + z Phi(-z) = z
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_param_count_and_layout():
    assert mlp.n_params() == 5 * 256 + 256 + 3 * (256 * 256 + 256) + 256 * 451 + 451
    th = np.arange(mlp.n_params(TINY), dtype=np.float64)
    (W0, b0), (W1, b1), (W2, b2) = mlp.unpack(th, TINY)
    assert W0.shape == (5, 7) and W0[1, 0] == 7 and b0[0] == 35
    assert W2.shape == (6, 9) and b2[-1] == th[-1]


def test_gradient_matches_central_differences():
    """Kernel-loss gradient for every parameter except the error output's own weights,
    error-loss gradient for those (its target held constant)."""
    rng = np.random.default_rng(0)
    th = mlp.init(1, TINY) + rng.normal(0, 0.05, mlp.n_params(TINY))
    X = rng.normal(0, 1, (11, 5))
    T = rng.normal(0, 0.5, (11, 8))
    lk, le, g = mlp.loss_grad(th, X, T, TINY)
    P, _ = mlp.forward(th, X, TINY)
    et = mlp.error_target(P, T)
    # indices of the error output's weights (last column of W2) and bias
    n = mlp.n_params(TINY)
    o2 = n - (6 * 9 + 9)
    err_idx = set(o2 + 9 * r + 8 for r in range(6)) | {n - 1}
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        k = 1 if i in err_idx else 0
        fd[i] = (mlp.loss(th + e, X, T, TINY, et)[k] - mlp.loss(th - e, X, T, TINY, et)[k]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-7 * np.linalg.norm(fd)
    assert abs(lk + le - sum(mlp.loss(th, X, T, TINY))) < 1e-12


def test_error_output_does_not_train_hidden_layers():
    rng = np.random.default_rng(2)
    th = mlp.init(3, TINY)
    X = rng.normal(0, 1, (6, 5))
    P, _ = mlp.forward(th, X, TINY)
    T = P[:, :8].copy()                              # kernel outputs already exact
    _, le, g = mlp.loss_grad(th, X, T, TINY)
    assert le > 0
    (gW0, gb0), (gW1, gb1), (gW2, gb2) = mlp.unpack(g, TINY)
    assert np.all(gW0 == 0) and np.all(gW1 == 0) and np.all(gb1 == 0)
    assert np.all(gW2[:, :8] == 0) and np.any(gW2[:, 8] != 0)


def test_adam_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    t1, m, v = mlp.adam(th, g, m, v, 1, 1e-2)
    assert np.allclose(t1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # second step with the same gradient: bias-corrected moments are g and g^2 again
    t2, _, _ = mlp.adam(t1, g, m, v, 2, 1e-2)
    assert np.allclose(t2, t1 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_features_and_targets():
    L = math.radians(3.0)
    w = np.array([0.0, 5.0, -40.0, 300.0])
    x, nk = mlp.features(w, L, [0.1, -0.5, 0.2, 0.0], [0.0, 0.3, -0.1, 0.4])
    assert np.array_equal(nk, nk_rule(w, L, L, 2, 2.0, None))
    assert np.allclose(x[:, 0], w * (2 * L) ** 2 / 4) and np.allclose(x[:, 1], 0.75)
    assert np.allclose(x[:, 4], nk / 15.0)
    t0 = mlp.kernel_target(0.0, L)                   # w = 0: unit delta at the centre
    assert t0[2 * (7 * 15 + 7)] == 1.0 and np.count_nonzero(t0) == 1
    assert mlp.kernel_target(3000.0, L) is None      # side above 15
    t1 = mlp.kernel_target(5.0, L)
    c = t1[0::2] + 1j * t1[1::2]
    assert abs(np.sum(np.abs(c) ** 2) - 1.0) < 1e-3  # unit-modulus chirp: Parseval
