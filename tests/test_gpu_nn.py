"""Learned-projection kernels (matrix-core convolutions, backward, Adam) against
the FP64 oracle of oracle/nn.py, through the C ABI.

Bars:
* forward output and parameter gradient within eps = 3e-4 (eq. 4.2 form) of
  the oracle run with the same bfloat16 operand rounding. What remains is the
  FP32 accumulation order, FP32 SiLU, and the rare element whose FP32 and FP64
  activations round to different bfloat16 neighbours;
* within eps = 1e-2 of the plain FP64 oracle (bfloat16 has 8 significant bits;
  a 192-term dot product of values rounded to 2^-9 relative error);
* Adam, MSE, features and the learned step within FP32 rounding (1e-6);
* backward bit-reproducible run to run.
"""
import numpy as np
import pytest
import torch

from oracle import nn as onn
from helpers import lib, to_dev

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(a * a + b * b), 1e-300)))


class Net:
    def __init__(self, theta, batch, n_c):
        E = lib()
        self.E = E
        self.params = to_dev(theta, torch.float32)
        self.pack = torch.zeros(E.NN_PACK_BYTES, dtype=torch.uint8, device="cuda")
        E.efpi_nn_pack(self.params, self.pack)
        self.ws = torch.empty(E.efpi_nn_workspace_size(batch, n_c), dtype=torch.uint8,
                              device="cuda")
        self.batch, self.n_c = batch, n_c

    def forward(self, x, periodic):
        y = torch.empty(self.batch, 2, self.n_c, dtype=torch.float32, device="cuda")
        self.E.efpi_nn_forward(self.params, self.pack, x, y, self.batch, self.n_c, periodic,
                               self.ws)
        return y

    def backward(self, x, dy, periodic):
        g = torch.empty(self.E.NN_PARAMS, dtype=torch.float32, device="cuda")
        self.E.efpi_nn_backward(self.pack, x, dy, g, self.batch, self.n_c, periodic, self.ws)
        return g


def theta_f32(seed):
    # the GPU holds FP32 parameters: give the oracle the same values
    return onn.init_params(seed).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("batch,n_c,periodic", [(1, 64, True), (3, 100, False), (2, 256, True),
                                                (5, 37, True), (4, 1024, False)])
def test_forward_backward_match_oracle(batch, n_c, periodic):
    g = np.random.default_rng(batch * 1000 + n_c)
    theta = theta_f32(batch + n_c)
    x = g.standard_normal((batch, 6, n_c)).astype(np.float32)
    dy = g.standard_normal((batch, 2, n_c)).astype(np.float32)
    net = Net(theta, batch, n_c)
    xd, dyd = to_dev(x, torch.float32), to_dev(dy, torch.float32)
    y = net.forward(xd, periodic).cpu().numpy()
    grad = net.backward(xd, dyd, periodic).cpu().numpy()
    yb, cb = onn.forward(theta, x.astype(np.float64), periodic, bf16=True)
    gb, _ = onn.backward(theta, cb, dy.astype(np.float64), periodic, bf16=True)
    assert rel(y, yb) < 3e-4
    assert rel(grad, gb) < 3e-4
    # every layer's gradient separately (a wrong layer could hide in the total)
    for (gw, gbias), (ow, obias) in zip(onn.unpack(grad.astype(np.float64)), onn.unpack(gb)):
        assert rel(gw, ow) < 3e-4 and rel(gbias, obias) < 3e-4
    y64, c64 = onn.forward(theta, x.astype(np.float64), periodic)
    g64, _ = onn.backward(theta, c64, dy.astype(np.float64), periodic)
    assert rel(y, y64) < 1e-2 and rel(grad, g64) < 1e-2


def test_backward_is_deterministic():
    g = np.random.default_rng(3)
    theta = theta_f32(3)
    x = to_dev(g.standard_normal((8, 6, 256)), torch.float32)
    dy = to_dev(g.standard_normal((8, 2, 256)), torch.float32)
    net = Net(theta, 8, 256)
    net.forward(x, True)
    g1 = net.backward(x, dy, True).cpu().numpy()
    net.forward(x, True)
    g2 = net.backward(x, dy, True).cpu().numpy()
    assert np.array_equal(g1, g2)


def test_zero_last_layer_output_is_zero():
    theta = onn.init_params(4, zero_last=True)
    net = Net(theta, 2, 64)
    x = to_dev(np.random.default_rng(4).standard_normal((2, 6, 64)), torch.float32)
    assert torch.count_nonzero(net.forward(x, False)).item() == 0


def test_mse_and_adam_match_oracle():
    E = lib()
    g = np.random.default_rng(5)
    y = g.standard_normal((3, 2, 50)).astype(np.float32)
    t = g.standard_normal((3, 2, 50)).astype(np.float32)
    yd, td = to_dev(y, torch.float32), to_dev(t, torch.float32)
    dy = torch.empty_like(yd)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    E.efpi_nn_mse(yd, td, dy, loss)
    lo, dyo = onn.mse(y.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - lo) <= 1e-6 * lo
    assert rel(dy.cpu().numpy(), dyo) < 1e-6

    theta = theta_f32(6)
    grad = g.standard_normal(E.NN_PARAMS).astype(np.float32)
    params = to_dev(theta, torch.float32)
    gd = to_dev(grad, torch.float32)
    m = torch.zeros(E.NN_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    pack = torch.zeros(E.NN_PACK_BYTES, dtype=torch.uint8, device="cuda")
    th, mo, vo = theta.copy(), np.zeros(E.NN_PARAMS), np.zeros(E.NN_PARAMS)
    for step in (1, 2, 3):
        E.efpi_nn_adam(params, gd, m, v, step, 1e-3, pack)
        th, mo, vo = onn.adam_step(th, grad.astype(np.float64), mo, vo, step, 1e-3)
    assert np.max(np.abs(params.cpu().numpy() - th)) < 1e-6
    # the pack written by Adam equals a fresh pack of the updated parameters
    pack2 = torch.zeros_like(pack)
    E.efpi_nn_pack(params, pack2)
    assert torch.equal(pack, pack2)


def test_features_targets_and_step_match_oracle():
    E = lib()
    g = np.random.default_rng(7)
    n_c, T = 40, 9
    states = 1.0 + 0.1 * g.standard_normal((T, 2, n_c))
    norm_t = ([1.0, 0.05], [0.1, 0.08], [2e-3, 3e-3])
    norm = E.nn_norm(*norm_t)
    idx = np.array([2, 5, 7, 3], np.int32)
    sd = to_dev(states, torch.float64)
    x = torch.empty(4, 6, n_c, dtype=torch.float32, device="cuda")
    t = torch.empty(4, 2, n_c, dtype=torch.float32, device="cuda")
    E.efpi_nn_features(sd, to_dev(idx, torch.int32), n_c, norm, x, t)
    xo = onn.features(states[idx - 2], states[idx - 1], states[idx], norm_t)
    to = onn.targets(states[idx], states[idx + 1], norm_t)
    nf = np.float32
    xo32 = onn.features(states[idx - 2], states[idx - 1], states[idx],
                        tuple(np.array(a, nf).astype(np.float64) for a in norm_t))
    assert np.max(np.abs(x.cpu().numpy() - xo32) / (1.0 + np.abs(xo32))) < 1e-5
    assert rel(t.cpu().numpy(), to) < 1e-5
    y = g.standard_normal((4, 2, n_c)).astype(np.float32)
    out = torch.empty(4, 2, n_c, dtype=torch.float64, device="cuda")
    cn = to_dev(states[idx], torch.float64)
    E.efpi_nn_step(cn, to_dev(y, torch.float32), 4, n_c, norm, out)
    delta = np.array(norm_t[2], np.float32).astype(np.float64).reshape(1, 2, 1)
    assert np.allclose(out.cpu().numpy(), states[idx] + delta * y, rtol=0, atol=1e-15)
    assert rel(xo, xo32) < 1e-6


def test_training_reduces_loss():
    """Adam on the GPU fits a fixed random teacher network (same architecture)."""
    E = lib()
    batch, n_c = 16, 64
    g = np.random.default_rng(8)
    teacher = onn.init_params(100)
    x = g.standard_normal((batch, 6, n_c))
    t, _ = onn.forward(teacher, x, True)
    net = Net(theta_f32(9), batch, n_c)
    xd, td = to_dev(x, torch.float32), to_dev(t, torch.float32)
    m = torch.zeros(E.NN_PARAMS, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    dy = torch.empty(batch, 2, n_c, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(1, 501):
        y = net.forward(xd, True)
        E.efpi_nn_mse(y, td, dy, loss)
        grad = net.backward(xd, dy, True)
        E.efpi_nn_adam(net.params, grad, m, v, step, 3e-3, net.pack)
        if step in (1, 500):
            losses.append(loss.item())
    assert losses[1] < 0.1 * losses[0]


@pytest.mark.parametrize("periodic", [True, False])
def test_predict_step_matches_oracle(periodic):
    """Fused features + forward + step against the oracle's learned step."""
    E = lib()
    g = np.random.default_rng(21)
    n_c = 96
    theta = theta_f32(21)
    states = 1.0 + 0.1 * g.standard_normal((3, 2, n_c))
    norm_t = ([1.0, 0.05], [0.1, 0.08], [2e-3, 3e-3])
    norm32 = tuple(np.array(a, np.float32).astype(np.float64) for a in norm_t)
    net = Net(theta, 1, n_c)
    out = torch.empty(2 * n_c, dtype=torch.float64, device="cuda")
    E.efpi_nn_predict_step(net.params, net.pack, to_dev(states, torch.float64), n_c, periodic,
                           E.nn_norm(*norm_t), out, net.ws)
    got = out.cpu().numpy().reshape(2, n_c)
    ref = onn.learned_step(theta, states[0:1], states[1:2], states[2:3], norm32, periodic,
                           bf16=True)[0]
    # compare the increments (the states themselves agree to ~1e-3 trivially)
    assert rel(got - states[2], ref - states[2]) < 3e-4


@pytest.mark.parametrize("periodic", [True, False])
def test_predict_step_support_rule(periodic):
    """A plasma on blocks 30..59 of 96 with exact vacuum elsewhere: blocks more than
    two blocks from any density keep c_n bit for bit (both moments), the others
    match the oracle's increments."""
    E = lib()
    g = np.random.default_rng(22)
    n_c = 96
    theta = theta_f32(22)
    states = np.zeros((3, 2, n_c))
    states[:, 0, 30:60] = 1.0 + 0.1 * g.standard_normal((3, 30))
    states[:, 1, 30:60] = 0.05 * g.standard_normal((3, 30))
    norm_t = ([0.3, 0.0], [0.45, 0.03], [2e-3, 3e-3])
    norm32 = tuple(np.array(a, np.float32).astype(np.float64) for a in norm_t)
    net = Net(theta, 1, n_c)
    out = torch.empty(2 * n_c, dtype=torch.float64, device="cuda")
    E.efpi_nn_predict_step(net.params, net.pack, to_dev(states, torch.float64), n_c, periodic,
                           E.nn_norm(*norm_t), out, net.ws)
    got = out.cpu().numpy().reshape(2, n_c)
    outside = onn.outside_support(states[2:3], periodic)[0]
    assert outside.sum() == n_c - 34
    assert np.array_equal(got[:, outside], states[2][:, outside])
    ref = onn.learned_step(theta, states[0:1], states[1:2], states[2:3], norm32, periodic,
                           bf16=True)[0]
    assert np.array_equal(ref[:, outside], states[2][:, outside])
    assert rel(got - states[2], ref - states[2]) < 3e-4


def test_training_noise_statistics():
    """Input-state noise of the training features: zero mean, the requested
    scale (noise * delta), independent of the exact features, deterministic."""
    E = lib()
    g = np.random.default_rng(31)
    n_c, T = 512, 6
    states = 1.0 + 0.1 * g.standard_normal((T, 2, n_c))
    norm_t = ([1.0, 0.0], [0.5, 0.25], [2e-3, 4e-3])
    norm = E.nn_norm(*norm_t)
    idx = to_dev(np.full(64, 3, np.int32), torch.int32)
    sd = to_dev(states, torch.float64)
    x0 = torch.empty(64, 6, n_c, dtype=torch.float32, device="cuda")
    t0 = torch.empty(64, 2, n_c, dtype=torch.float32, device="cuda")
    x1, t1, x2 = torch.empty_like(x0), torch.empty_like(t0), torch.empty_like(x0)
    E.efpi_nn_features(sd, idx, n_c, norm, x0, t0)
    E.efpi_nn_features(sd, idx, n_c, norm, x1, t1, noise=0.5, seed=9)
    E.efpi_nn_features(sd, idx, n_c, norm, x2, noise=0.5, seed=9)
    d = (x1 - x0).cpu().numpy().astype(np.float64)
    # channel 0: perturbation of c_n in units of sigma: std = 0.5 * delta / sigma
    for m in range(2):
        s = d[:, m].std()
        expect = 0.5 * norm_t[2][m] / norm_t[1][m]
        assert abs(s - expect) < 0.03 * expect
        assert abs(d[:, m].mean()) < 0.05 * expect
    # target from the perturbed c_n
    assert torch.allclose(t1 + (x1[:, 0:2] - x0[:, 0:2]) * torch.tensor(
        [norm_t[1][0] / norm_t[2][0], norm_t[1][1] / norm_t[2][1]], device="cuda").view(1, 2, 1),
        t0, rtol=0, atol=1e-3)
    assert torch.equal(x1, x2)
