"""Oracle of the learned projection network, FP64 — TEST INFRASTRUCTURE ONLY.

The learned projection replaces the least-squares slope of eq. 3.18 by a small
network that maps the last three coarse states (c_{n-2}, c_{n-1}, c_n) to the
increment c_{n+1} - c_n of a projective step (eq. 3.17).  The paper states the
projective cycle, not this network: everything here is the added surrogate,
defined as follows.

Network: four 1D convolutions with kernel width 3 over the coarse index,
channel widths 6 -> 64 -> 64 -> 64 -> 2, SiLU after the first three, "same"
padding that is circular for periodic domains and zero for walled ones.
Parameters, in one flat vector: for each layer W[c_out][c_in][3] then b[c_out]
(26,306 values).

Input features of sample (c_{n-2}, c_{n-1}, c_n), for moment m in (density,
momentum):  x[m] = (c_n - mu_m) / sigma_m,  x[2 + m] = (c_n - c_{n-1}) / delta_m,
x[4 + m] = (c_{n-1} - c_{n-2}) / delta_m.  Output y[m] approximates
(c_{n+1} - c_n) / delta_m, so the learned step is c_{n+1} = c_n + delta * y,
except outside the plasma's support: a coarse block whose density in c_n is
exactly zero at itself and at every block within SUPPORT_RADIUS (wrapping on
periodic domains, only the existing blocks between walls) keeps c_n (both
moments).  Plasma moves a bounded distance per macro step, and a plain EFPI
step leaves such blocks exactly empty (no ions deposit there); the network's
outputs are never exactly zero, so without the rule a learned step would seed
the whole vacuum with a tiny density that the next lift fills with ions.

The GPU feeds the matrix cores bfloat16 operands with FP32 accumulation.  With
``bf16=True`` this oracle rounds the same operands (weights, layer inputs and
output gradients of each product) to bfloat16 (round to nearest even) and keeps
every sum in FP64, so the two sides then differ only by accumulation order.
"""
from __future__ import annotations

import numpy as np

C_IN = 6
SUPPORT_RADIUS = 2
HIDDEN = 64
C_OUT = 2
WIDTHS = (C_IN, HIDDEN, HIDDEN, HIDDEN, C_OUT)
KW = 3


def layer_shapes():
    return [(WIDTHS[i + 1], WIDTHS[i]) for i in range(len(WIDTHS) - 1)]


def n_params() -> int:
    return sum(co * ci * KW + co for co, ci in layer_shapes())


def unpack(theta):
    """Views (W, b) per layer into the flat parameter vector."""
    out, o = [], 0
    for co, ci in layer_shapes():
        W = theta[o:o + co * ci * KW].reshape(co, ci, KW)
        o += co * ci * KW
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(seed: int, zero_last: bool = False):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (fan_in = 3 c_in)."""
    g = np.random.default_rng(seed)
    theta = np.empty(n_params())
    for (W, b), (co, ci) in zip(unpack(theta), layer_shapes()):
        a = 1.0 / np.sqrt(ci * KW)
        W[...] = g.uniform(-a, a, W.shape)
        b[...] = g.uniform(-a, a, b.shape)
    if zero_last:
        W, b = unpack(theta)[-1]
        W[...] = 0.0
        b[...] = 0.0
    return theta


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), through FP32, returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad(x, periodic: bool):
    """One cell of padding on each side of the last axis."""
    if periodic:
        return np.concatenate([x[..., -1:], x, x[..., :1]], axis=-1)
    z = np.zeros(x.shape[:-1] + (1,))
    return np.concatenate([z, x, z], axis=-1)


def conv1d(x, W, b, periodic: bool):
    """out[s, o, i] = b[o] + sum_{c, k} W[o, c, k] x[s, c, i + k - 1] (padded)."""
    xp = _pad(x, periodic)
    L = x.shape[-1]
    out = np.einsum("ock,sckl->sol", W, np.stack([xp[..., k:k + L] for k in range(KW)], axis=2))
    if b is not None:
        out = out + b[None, :, None]
    return out


def conv1d_adjoint(dz, W, periodic: bool):
    """Adjoint of conv1d in x: dx[s, c, j] = sum_{o, k} W[o, c, k] dz[s, o, j - k + 1]."""
    L = dz.shape[-1]
    dx = np.zeros((dz.shape[0], W.shape[1], L))
    for k in range(KW):
        # term k of conv1d reads x at i + k - 1; scatter dz back there
        contrib = np.einsum("oc,sol->scl", W[:, :, k], dz)
        shift = k - 1
        if periodic:
            dx += np.roll(contrib, shift, axis=-1)
        else:
            if shift == 0:
                dx += contrib
            elif shift > 0:
                dx[..., shift:] += contrib[..., :L - shift]
            else:
                dx[..., :L + shift] += contrib[..., -shift:]
    return dx


def _sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def silu(z):
    return z * _sigmoid(z)


def silu_grad(z):
    s = _sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, periodic: bool, bf16: bool = False):
    """Network output y[s, 2, L] and the cache (layer inputs, pre-activations)."""
    rnd = bf16_round if bf16 else (lambda a: a)
    a = np.asarray(x, dtype=np.float64)
    inputs, pre = [], []
    layers = unpack(np.asarray(theta, dtype=np.float64))
    for i, (W, b) in enumerate(layers):
        inputs.append(a)
        z = conv1d(rnd(a), rnd(W), b, periodic)
        pre.append(z)
        a = silu(z) if i < len(layers) - 1 else z
    return a, (inputs, pre)


def backward(theta, cache, dy, periodic: bool, bf16: bool = False):
    """Gradient of sum(dy * y) with respect to the flat parameters, and dL/dx.

    Hand-derived from forward: for layer l with input a and pre-activation z,
    dW[o, c, k] = sum_{s, i} dz[s, o, i] a[s, c, i + k - 1], db[o] = sum dz[s, o, :],
    da = conv1d_adjoint(dz, W), and the layer below gets dz' = da * SiLU'(z').
    """
    rnd = bf16_round if bf16 else (lambda a: a)
    inputs, pre = cache
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.zeros_like(theta)
    glayers = unpack(grad)
    layers = unpack(theta)
    dz = np.asarray(dy, dtype=np.float64)
    dx = None
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        gW, gb = glayers[i]
        a = inputs[i]
        ap = _pad(rnd(a), periodic)
        L = a.shape[-1]
        dzr = rnd(dz)
        for k in range(KW):
            gW[:, :, k] = np.einsum("sol,scl->oc", dzr, ap[..., k:k + L])
        gb[:] = dz.sum(axis=(0, 2))
        da = conv1d_adjoint(dzr, rnd(W), periodic)
        if i > 0:
            dz = da * silu_grad(pre[i - 1])
        else:
            dx = da
    return grad, dx


def mse(y, t):
    """Mean squared error over every element and its gradient in y."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(theta, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(c_nm2, c_nm1, c_n, norm):
    """Network input x[s, 6, N_c] from three coarse states [s, 2, N_c].

    norm = (mu[2], sigma[2], delta[2]).
    """
    mu, sigma, delta = (np.asarray(a, dtype=np.float64).reshape(1, 2, 1) for a in norm)
    c_nm2, c_nm1, c_n = (np.asarray(a, dtype=np.float64) for a in (c_nm2, c_nm1, c_n))
    return np.concatenate([(c_n - mu) / sigma, (c_n - c_nm1) / delta, (c_nm1 - c_nm2) / delta],
                          axis=1)


def targets(c_n, c_np1, norm):
    """Training target (c_{n+1} - c_n) / delta, shape [s, 2, N_c]."""
    delta = np.asarray(norm[2], dtype=np.float64).reshape(1, 2, 1)
    return (np.asarray(c_np1, dtype=np.float64) - np.asarray(c_n, dtype=np.float64)) / delta


def outside_support(c_n, periodic: bool):
    """[batch][n_c] mask of the blocks whose density is zero in c_n at every block
    within SUPPORT_RADIUS of them (the learned step leaves those unchanged)."""
    dens = np.asarray(c_n, dtype=np.float64)[:, 0, :]
    nc = dens.shape[-1]
    out = np.ones(dens.shape, dtype=bool)
    for k in range(nc):
        for d in range(-SUPPORT_RADIUS, SUPPORT_RADIUS + 1):
            j = k + d
            if periodic:
                j %= nc
            elif not 0 <= j < nc:
                continue
            out[:, k] &= dens[:, j] == 0.0
    return out


def learned_step(theta, c_nm2, c_nm1, c_n, norm, periodic: bool, bf16: bool = False):
    """c_{n+1} = c_n + delta * y(features) inside the support, c_n outside it: the
    learned projective step."""
    x = features(c_nm2, c_nm1, c_n, norm)
    y, _ = forward(theta, x, periodic, bf16)
    delta = np.asarray(norm[2], dtype=np.float64).reshape(1, 2, 1)
    c_n = np.asarray(c_n, dtype=np.float64)
    keep = outside_support(c_n, periodic)[:, None, :]
    return np.where(keep, c_n, c_n + delta * y)
