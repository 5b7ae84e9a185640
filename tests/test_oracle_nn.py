"""Pins of the learned-projection oracle (oracle/nn.py).

The network is the project's own addition, so the pins are mathematical:
central finite differences for every gradient, the adjoint (dot-product)
identity of the convolution, a library correlation for the single-channel
case, shift equivariance of circular padding, closed forms of Adam's first
step, and torch's bfloat16 conversion for the rounding.
"""
import numpy as np
import pytest
import torch

from oracle import nn


def _sample(seed, s=2, L=8):
    g = np.random.default_rng(seed)
    return g.standard_normal((s, nn.C_IN, L))


def test_parameter_count():
    assert nn.n_params() == 64 * 6 * 3 + 64 + 2 * (64 * 64 * 3 + 64) + 2 * 64 * 3 + 2 == 26306


@pytest.mark.parametrize("periodic", [True, False])
def test_single_channel_conv_is_correlation(periodic):
    g = np.random.default_rng(1)
    x = g.standard_normal(11)
    w = g.standard_normal(3)
    out = nn.conv1d(x[None, None, :], w[None, None, :], np.array([0.5]), periodic)[0, 0]
    xp = np.concatenate([[x[-1] if periodic else 0.0], x, [x[0] if periodic else 0.0]])
    ref = np.correlate(xp, w, mode="valid") + 0.5
    assert np.allclose(out, ref, rtol=0, atol=1e-14)


def test_circular_padding_is_shift_equivariant():
    theta = nn.init_params(3)
    x = _sample(4, L=16)
    y, _ = nn.forward(theta, x, True)
    y2, _ = nn.forward(theta, np.roll(x, 5, axis=-1), True)
    assert np.allclose(np.roll(y, 5, axis=-1), y2, rtol=0, atol=1e-12)


@pytest.mark.parametrize("periodic", [True, False])
def test_adjoint_identity(periodic):
    g = np.random.default_rng(5)
    x = g.standard_normal((3, 7, 10))
    W = g.standard_normal((4, 7, 3))
    dz = g.standard_normal((3, 4, 10))
    lhs = np.sum(nn.conv1d(x, W, None, periodic) * dz)
    rhs = np.sum(x * nn.conv1d_adjoint(dz, W, periodic))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("periodic", [True, False])
def test_backward_matches_central_differences(periodic):
    theta = nn.init_params(7)
    x = _sample(8)
    g = np.random.default_rng(9)
    dy = g.standard_normal((2, nn.C_OUT, 8))

    def f(th, xx):
        y, _ = nn.forward(th, xx, periodic)
        return float(np.sum(y * dy))

    y, cache = nn.forward(theta, x, periodic)
    grad, dx = nn.backward(theta, cache, dy, periodic)
    h = 1e-6
    # every bias and a random sample of weights in every layer
    idx = list(g.choice(nn.n_params(), 240, replace=False))
    o = 0
    for co, ci in nn.layer_shapes():
        o += co * ci * 3
        idx += list(range(o, o + co))
        o += co
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (f(tp, x) - f(tm, x)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(fd)), i
    for j in range(0, x.size, 7):
        xp, xm = x.copy().ravel(), x.copy().ravel()
        xp[j] += h
        xm[j] -= h
        fd = (f(theta, xp.reshape(x.shape)) - f(theta, xm.reshape(x.shape))) / (2 * h)
        assert abs(fd - dx.ravel()[j]) <= 1e-7 * max(1.0, abs(fd))


def test_silu_grad_and_mse_grad():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (nn.silu(z + h) - nn.silu(z - h)) / (2 * h)
    assert np.allclose(nn.silu_grad(z), fd, rtol=0, atol=1e-8)
    g = np.random.default_rng(2)
    y, t = g.standard_normal(20), g.standard_normal(20)
    loss, dy = nn.mse(y, t)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-15
    yp = y.copy()
    yp[3] += h
    ym = y.copy()
    ym[3] -= h
    assert abs((nn.mse(yp, t)[0] - nn.mse(ym, t)[0]) / (2 * h) - dy[3]) < 1e-8


def test_zero_last_layer_gives_zero_increment():
    theta = nn.init_params(11, zero_last=True)
    x = _sample(12, L=16)
    y, _ = nn.forward(theta, x, False)
    assert np.all(y == 0.0)
    g = np.random.default_rng(13)
    c = [g.standard_normal((1, 2, 16)) for _ in range(3)]
    norm = ([1.0, 0.1], [0.2, 0.1], [1e-3, 2e-3])
    out = nn.learned_step(theta, c[0], c[1], c[2], norm, False)
    assert np.array_equal(out, c[2])


def test_support_rule_hand_worked():
    """Blocks whose density is zero within two blocks keep c_n; the mask by hand
    for a plasma on blocks 5..6 of 12, with walls and periodic."""
    c = np.zeros((1, 2, 12))
    c[0, 0, 5:7] = 1.0
    c[0, 1, :] = 0.25           # momentum does not enter the mask
    walls = nn.outside_support(c, periodic=False)[0]
    assert walls.tolist() == [True, True, True, False, False, False, False, False, False,
                              True, True, True]
    c2 = np.zeros((1, 2, 12))
    c2[0, 0, 0] = 1.0            # plasma at block 0: the wrap reaches 10 and 11
    per = nn.outside_support(c2, periodic=True)[0]
    assert per.tolist() == [False, False, False, True, True, True, True, True, True, True,
                            False, False]
    wal2 = nn.outside_support(c2, periodic=False)[0]
    assert wal2.tolist() == [False, False, False] + [True] * 9
    # the step: unchanged outside, c_n + delta y inside (nonzero last layer)
    theta = nn.init_params(3)
    g = np.random.default_rng(4)
    prev = [c + 1e-3 * g.standard_normal(c.shape) * (c != 0) for _ in range(2)]
    norm = ([0.5, 0.1], [0.4, 0.2], [1e-2, 2e-2])
    out = nn.learned_step(theta, prev[0], prev[1], c, norm, False)
    assert np.array_equal(out[0][:, walls], c[0][:, walls])
    assert np.all(out[0][:, ~walls] != c[0][:, ~walls])


def test_adam_first_step_closed_form():
    g = np.random.default_rng(14)
    theta = g.standard_normal(50)
    grad = g.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    t1, m, v = nn.adam_step(theta, grad, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    # bias-corrected first and second moments equal g and g^2 after one step
    assert np.allclose(t1, theta - lr * grad / (np.abs(grad) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)


def test_bf16_rounding_matches_torch():
    g = np.random.default_rng(15)
    x = np.concatenate([g.standard_normal(2000) * 10.0 ** g.integers(-6, 6, 2000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.5, 0.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16_round(x), ref)
    assert nn.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie to even
    assert nn.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_bf16_operands_stay_within_bf16_tolerance():
    theta = nn.init_params(16)
    x = _sample(17, L=32)
    y, c = nn.forward(theta, x, True)
    yb, cb = nn.forward(theta, x, True, bf16=True)
    rel = np.sqrt(np.sum((y - yb) ** 2) / np.sum(y ** 2 + yb ** 2))
    assert 1e-5 < rel < 1e-2
    dy = np.random.default_rng(18).standard_normal(y.shape)
    g, _ = nn.backward(theta, c, dy, True)
    gb, _ = nn.backward(theta, cb, dy, True, bf16=True)
    rel = np.sqrt(np.sum((g - gb) ** 2) / np.sum(g ** 2 + gb ** 2))
    assert rel < 1e-2


def test_features_and_targets():
    c0 = np.full((1, 2, 4), 2.0)
    c1 = c0 + 1.0
    c2 = c1 + 2.0
    norm = ([1.0, 0.5], [2.0, 4.0], [0.5, 0.25])
    x = nn.features(c0, c1, c2, norm)
    assert np.allclose(x[0, 0], (5.0 - 1.0) / 2.0) and np.allclose(x[0, 1], (5.0 - 0.5) / 4.0)
    assert np.allclose(x[0, 2], 2.0 / 0.5) and np.allclose(x[0, 3], 2.0 / 0.25)
    assert np.allclose(x[0, 4], 1.0 / 0.5) and np.allclose(x[0, 5], 1.0 / 0.25)
    t = nn.targets(c1, c2, norm)
    assert np.allclose(t[0, 0], 4.0) and np.allclose(t[0, 1], 8.0)
