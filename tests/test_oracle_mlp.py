"""Pins of the controller network's oracle (oracle/mlp.py) against
mathematics: finite differences, closed forms of the loss gradient and of
Adam's first step, and exact bfloat16 rounding cases."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, N=16):
    rng = np.random.default_rng(seed)
    theta = mlp.init(seed)
    X = rng.standard_normal((N, 8))
    T = rng.standard_normal((N, 2))
    return theta, X, T


def test_parameter_count():
    assert mlp.n_params() == 4866
    assert mlp.init(0).size == 4866


def test_gradient_matches_central_differences():
    theta, X, T = _data(3)
    L, g = mlp.grad(theta, X, T)
    assert L == pytest.approx(mlp.loss(theta, X, T), rel=1e-14)
    rng = np.random.default_rng(4)
    idx = rng.choice(theta.size, 200, replace=False)
    idx = np.concatenate([idx, [0, 511, 575, 576, 4159 + 576, theta.size - 1]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_output_bias_gradient_is_mean_residual():
    theta, X, T = _data(5)
    y, _ = mlp.forward(theta, X)
    _, g = mlp.grad(theta, X, T)
    assert np.allclose(g[-2:], (y - T).mean(0), rtol=1e-14, atol=1e-16)


def test_linear_regime_is_a_product_of_matrices():
    # positive weights and inputs keep every ReLU active: y = W3 (W2 (W1 x + b1) + b2) + b3
    rng = np.random.default_rng(6)
    theta = np.abs(rng.standard_normal(mlp.n_params())) * 0.1
    X = np.abs(rng.standard_normal((5, 8)))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    ref = ((X @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    y, _ = mlp.forward(theta, X)
    assert np.allclose(y, ref, rtol=1e-14)


def test_adam_first_step_moves_by_lr_times_sign():
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t1, m, v = mlp.adam(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-16)
    assert np.allclose(t1, theta - 0.01 * np.sign(g), rtol=0, atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_cases():
    one = np.float32(1.0)
    cases = {1.0: 1.0, 1 + 2 ** -7: 1 + 2 ** -7, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6,
             -(1 + 3 * 2 ** -9): -(1 + 2 ** -7), 3.0e-3: None}
    for x, want in cases.items():
        got = float(mlp.to_bf16(np.array([x], np.float32))[0])
        if want is None:  # nearest representable: 8 significant bits
            assert abs(got - x) <= abs(x) * 2 ** -8
        else:
            assert got == want, (x, got)
    assert one == mlp.to_bf16(np.array([1.0], np.float32))[0]


def test_bf16_inference_is_close_to_float64():
    theta, X, _ = _data(7, N=64)
    y64, _ = mlp.forward(theta, X)
    y16 = mlp.forward_bf16(theta, X)
    assert np.max(np.abs(y16 - y64)) <= 0.05 * max(1.0, np.max(np.abs(y64)))


def test_standardize_stats_hand_values():
    # population statistics: column [1, 2, 3, 4] has mean 2.5 and standard
    # deviation sqrt(1.25); a constant column keeps its mean and gets 1
    X = np.zeros((4, 8))
    X[:, 0] = [1.0, 2.0, 3.0, 4.0]
    X[:, 1] = 5.0
    X[:, 2] = [-2.0, 2.0, -2.0, 2.0]
    T = np.array([[0.0, 7.0], [2.0, 7.0], [4.0, 7.0], [6.0, 7.0]])
    xm, xs, tm, ts = mlp.standardize_stats(X, T)
    assert xm[0] == 2.5 and xs[0] == pytest.approx(np.sqrt(1.25), rel=1e-15)
    assert xm[1] == 5.0 and xs[1] == 1.0
    assert xm[2] == 0.0 and xs[2] == 2.0
    assert np.all(xm[3:] == 0.0) and np.all(xs[3:] == 1.0)
    assert tm.tolist() == [3.0, 7.0] and ts[0] == pytest.approx(np.sqrt(5.0), rel=1e-15) and ts[1] == 1.0


def test_bf16_inference_hand_rounded_network():
    # A network whose every number is worked out by hand.  Each path checks one
    # rounding: inputs, layer-1 weights, layer-1 activations, layer-2
    # activations; dropping any of them changes an output.
    theta = np.zeros(mlp.n_params())
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    X = np.zeros((1, 8))
    X[0, 0] = 1.0
    X[0, 1] = 1.0
    X[0, 2] = 1 + 2.0 ** -8 + 2.0 ** -12          # input: bfloat16 gives 1 + 2^-7
    W1[0, 0], b1[0] = 1.0, 3 * 2.0 ** -8          # z = 1 + 3 2^-8, a tie: rounds to 1 + 2^-6
    W1[1, 1], b1[1] = 1 + 2.0 ** -9, -1.0         # weight: bfloat16 gives 1, so a = 0
    W1[2, 2], b1[2] = 1.0, -1.0                    # a = 2^-7
    W2[0, 0], b2[0] = 1.0, -1.0                    # (1 + 2^-6) - 1 = 2^-6
    W2[1, 0], b2[1] = 1 + 2.0 ** -7, 0.0           # 1 + 3 2^-7 + 2^-13 rounds to 1 + 3 2^-7
    W2[2, 1] = 1.0                                  # passes the weight-rounding path (0)
    W2[3, 2] = 1.0                                  # passes the input-rounding path (2^-7)
    W3[0, 0], W3[0, 2], W3[0, 3] = 1.0, 1.0, 1.0   # y0 = 2^-6 + 0 + 2^-7
    W3[1, 1], b3[1] = 1.0, -1.0                    # y1 = 3 2^-7
    y = mlp.forward_bf16(theta, X)
    assert y.dtype == np.float32
    assert y[0, 0] == np.float32(2.0 ** -6 + 2.0 ** -7)
    assert y[0, 1] == np.float32(3 * 2.0 ** -7)
