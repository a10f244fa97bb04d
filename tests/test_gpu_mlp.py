"""GPU parity of the learned controller's training and inference kernels
against oracle/mlp.py (run on an MI355X; every call goes through the C ABI).

Tolerances: the GPU computes in float32 where the oracle uses float64, so the
loss and gradient are compared to 1e-4 of the largest gradient entry (sums of
up to thousands of float32 products); Adam steps to 1e-3 of the learning rate
wherever the gradient is not negligible; float32 inference to 1e-5 relative;
bfloat16 inference against the oracle's bfloat16 emulation to 2e-2 in
standardised units (a float32-vs-float64 sum can round a hidden activation to
the neighbouring bfloat16 value)."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 8)) * np.array([3.0, 0.2, 1.0, 5.0, 0.5, 2.0, 1.0, 0.7]) + np.arange(8)
    T = np.stack([np.sin(X[:, 0]) + 0.1 * X[:, 3], np.tanh(X[:, 1] * X[:, 2])], 1) * np.array([7.0, 0.3]) + 1.5
    return X.astype(np.float32), T.astype(np.float32)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _std(X, T, stats):
    xm, xs, tm, ts = stats
    return (X.astype(np.float64) - xm) / xs, (T.astype(np.float64) - tm) / ts


def _net(seed=11):
    import paper_1511_04515_amd as E
    theta = mlp.init(seed)
    return E.Mlp(theta.astype(np.float32)), theta.astype(np.float32).astype(np.float64)


def test_standardisation_matches_oracle():
    X, T = _data(5000, 1)
    net, _ = _net()
    net.fit_norm(_dev(X), _dev(T))
    got = net.norm()
    xm, xs, tm, ts = mlp.standardize_stats(X, T)
    ref = np.concatenate([xm, xs, tm, ts])
    assert np.allclose(got, ref, rtol=1e-6, atol=1e-6)
    net.close()


@pytest.mark.parametrize("n", [1, 64, 1000, 4096])
def test_gradient_matches_oracle(n):
    X, T = _data(n, 2)
    stats = mlp.standardize_stats(*_data(4096, 3))
    net, theta = _net()
    net.set_norm(np.concatenate(stats).astype(np.float32))
    loss, g = net.grad(_dev(X), _dev(T))
    Xs, Ts = _std(X, T, [s.astype(np.float32).astype(np.float64) for s in stats])
    L_ref, g_ref = mlp.grad(theta, Xs, Ts)
    assert loss == pytest.approx(L_ref, rel=1e-4)
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref)) + 1e-9
    net.close()


def test_adam_steps_match_oracle():
    X, T = _data(2048, 4)
    stats = [s.astype(np.float32).astype(np.float64) for s in mlp.standardize_stats(X, T)]
    net, theta = _net(5)
    net.set_norm(np.concatenate(stats).astype(np.float32))
    Xd, Td = _dev(X), _dev(T)
    Xs, Ts = _std(X, T, stats)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    lr = 1e-3
    for step in range(1, 4):
        _, g_ref = mlp.grad(theta, Xs, Ts)
        theta_next, m, v = mlp.adam(theta, g_ref, m, v, step, lr=lr)
        net.adam_step(Xd, Td, lr=lr)
        got = net.params().astype(np.float64)
        big = np.abs(g_ref) > 1e-4 * np.max(np.abs(g_ref))
        assert np.max(np.abs(got - theta_next)[big]) <= 1e-3 * lr * step + 1e-6
        assert np.max(np.abs(got - theta_next)) <= 2 * lr * step + 1e-6
        theta = got  # follow the GPU's parameters so errors do not accumulate
    net.close()


def test_inference_float32_and_bfloat16_match_oracle():
    X, T = _data(777, 6)
    stats = [s.astype(np.float32).astype(np.float64) for s in mlp.standardize_stats(X, T)]
    net, theta = _net(7)
    net.set_norm(np.concatenate(stats).astype(np.float32))
    xm, xs, tm, ts = stats
    Xs = (X.astype(np.float64) - xm) / xs
    y32 = net.forward(_dev(X), bf16=False).cpu().numpy()
    ref, _ = mlp.forward(theta, Xs)
    assert np.allclose((y32 - tm) / ts, ref, rtol=1e-5, atol=1e-5)
    y16 = net.forward(_dev(X), bf16=True).cpu().numpy()
    ref16 = mlp.forward_bf16(theta, Xs)
    assert np.max(np.abs((y16 - tm) / ts - ref16)) <= 2e-2
    net.close()


def test_training_reduces_the_loss():
    X, T = _data(8192, 8)
    net, _ = _net(9)
    Xd, Td = _dev(X), _dev(T)
    net.fit_norm(Xd, Td)
    l0, _ = net.grad(Xd, Td)
    for i in range(400):
        lo = (i * 1024) % 8192
        net.adam_step(Xd[lo:lo + 1024], Td[lo:lo + 1024], lr=3e-3)
    l1, _ = net.grad(Xd, Td)
    assert l1 < 0.1 * l0, (l0, l1)
    net.close()
