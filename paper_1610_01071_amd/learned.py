"""Learned projective integration driven through the C ABI.

The network of efpi_nn_* (include/efpi.h) predicts the increment of a
projective step (eq. 3.17) from the last three coarse states.  This module
orchestrates, on the GPU:

* ``plain_run``: coarse trajectories of plain EFPI macro steps (lift, restricted
  fine burst, least-squares slope of eq. 3.18, projection), which are the
  training data and the reference;
* ``Trainer``: Adam on mini-batches of (c_{n-2}, c_{n-1}, c_n) -> c_{n+1} - c_n,
  with the library's forward, backward, loss and optimizer kernels;
* ``run_learned``: macro steps that take the learned step, with a fine burst
  every ``judge_period`` steps that both advances the state and judges the
  network on both moments (the error of eq. 4.2 between the learned candidate
  and the burst step, less plain EFPI's own one-step noise); these one-step
  errors, summed over the learned steps they stand for, bound the run's
  accumulated error, and once that sum passes its threshold for either moment
  the rest of the run is plain EFPI.

Python only chooses indices, loops and branches; all arithmetic runs in the
library's kernels.  The one host computation is the normalisation of the
features and targets (means and standard deviations of the training set).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import efpi as E


def lift_shift(seed: int, n: int) -> int:
    """32-bit Cranley-Patterson rotation of macro step n of a run (SplitMix64 of seed, n)."""
    z = (seed * 0x9E3779B97F4A7C15 + (n + 1) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return (z ^ (z >> 31)) & 0xFFFFFFFF


def plain_run(ctx: E.Context, c0: torch.Tensor, steps: int, seed: int, out=None):
    """`steps` plain EFPI macro steps from c0; returns the states [steps + 1][2 N_c]."""
    nc2 = c0.numel()
    traj = out if out is not None else torch.empty(steps + 1, nc2, dtype=torch.float64,
                                                   device=c0.device)
    traj[0].copy_(c0)
    for n in range(steps):
        E.efpi_macro_step(ctx.ctx, traj[n], traj[n + 1], [lift_shift(seed, n)])
    return traj


def fit_norm(trajs) -> E.NnNorm:
    """Feature and target scales from training trajectories (host statistics)."""
    states = np.concatenate([t.cpu().numpy().reshape(t.shape[0], 2, -1) for t in trajs], axis=0)
    inc = np.concatenate([np.diff(t.cpu().numpy().reshape(t.shape[0], 2, -1), axis=0)
                          for t in trajs], axis=0)
    mu = states.mean(axis=(0, 2))
    sigma = states.std(axis=(0, 2))
    delta = np.sqrt(np.mean(inc * inc, axis=(0, 2)))
    return E.nn_norm(mu, np.maximum(sigma, 1e-12), np.maximum(delta, 1e-12))


@dataclass
class Trainer:
    n_c: int
    periodic: bool
    batch: int = 32
    seed: int = 0
    params: torch.Tensor = field(init=False)

    def __post_init__(self):
        g = np.random.default_rng(self.seed)
        theta = np.empty(E.NN_PARAMS, np.float32)
        o = 0
        for co, ci in ((64, 6), (64, 64), (64, 64), (2, 64)):
            a = 1.0 / np.sqrt(3 * ci)
            theta[o:o + co * ci * 3] = g.uniform(-a, a, co * ci * 3)
            o += co * ci * 3
            theta[o:o + co] = 0.0
            o += co
        # biases and the last layer start at zero: the untrained network predicts no change
        theta[o - 2 - 2 * 64 * 3:o] = 0.0
        dev = "cuda"
        self.params = torch.as_tensor(theta).to(dev)
        self.pack = torch.zeros(E.NN_PACK_BYTES, dtype=torch.uint8, device=dev)
        E.efpi_nn_pack(self.params, self.pack)
        self.m = torch.zeros(E.NN_PARAMS, dtype=torch.float32, device=dev)
        self.v = torch.zeros_like(self.m)
        self.grad = torch.empty_like(self.m)
        self.step_count = 0
        self._ws = {}

    def workspace(self, batch):
        if batch not in self._ws:
            self._ws[batch] = torch.empty(E.efpi_nn_workspace_size(batch, self.n_c),
                                          dtype=torch.uint8, device="cuda")
        return self._ws[batch]

    def train(self, states: torch.Tensor, valid_index: np.ndarray, norm: E.NnNorm, iters: int,
              lr: float = 2e-3, lr_final: float = 2e-4, noise: float = 0.0):
        """Adam over random mini-batches of the samples n in valid_index of `states`.

        noise > 0 perturbs the input states of every batch (in units of the
        increment scale) so that the network learns to correct its own errors
        when its steps are chained."""
        g = np.random.default_rng(self.seed + 1)
        B, nc = self.batch, self.n_c
        idx_all = torch.as_tensor(
            g.choice(valid_index, size=(iters, B)).astype(np.int32)).to("cuda")
        x = torch.empty(B, 6, nc, dtype=torch.float32, device="cuda")
        t = torch.empty(B, 2, nc, dtype=torch.float32, device="cuda")
        y = torch.empty_like(t)
        dy = torch.empty_like(t)
        loss = torch.empty(iters, dtype=torch.float32, device="cuda")
        ws = self.workspace(B)
        for i in range(iters):
            E.efpi_nn_features(states, idx_all[i], nc, norm, x, t, noise=noise,
                               seed=self.seed * 1_000_003 + self.step_count)
            E.efpi_nn_forward(self.params, self.pack, x, y, B, nc, self.periodic, ws)
            E.efpi_nn_mse(y, t, dy, loss[i:i + 1])
            E.efpi_nn_backward(self.pack, x, dy, self.grad, B, nc, self.periodic, ws)
            self.step_count += 1
            rate = lr * (lr_final / lr) ** (i / max(iters - 1, 1))
            E.efpi_nn_adam(self.params, self.grad, self.m, self.v, self.step_count, rate, self.pack)
        return loss

    def evaluate(self, states: torch.Tensor, index: np.ndarray, norm: E.NnNorm) -> float:
        """Mean squared error (normalised units) on the samples n in `index`."""
        nc, B = self.n_c, len(index)
        x = torch.empty(B, 6, nc, dtype=torch.float32, device="cuda")
        t = torch.empty(B, 2, nc, dtype=torch.float32, device="cuda")
        y = torch.empty_like(t)
        dy = torch.empty_like(t)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        E.efpi_nn_features(states, torch.as_tensor(np.asarray(index, np.int32)).to("cuda"), nc,
                           norm, x, t)
        E.efpi_nn_forward(self.params, self.pack, x, y, B, nc, self.periodic, self.workspace(B))
        E.efpi_nn_mse(y, t, dy, loss)
        return loss.item()


@dataclass
class LearnedRun:
    states: torch.Tensor      # [steps + 1][2 N_c]
    judged: int               # burst steps taken to judge the network
    fallback: int             # plain steps taken after the error bound was passed
    learned: int              # learned steps
    eps: list                 # one-step judge errors of the coarse density (eq. 4.2)
    eps_momentum: list        # the same for the momentum coefficients
    wall_ms: float
    acc: list = field(default_factory=list)           # accumulated density bound after each judgement
    acc_momentum: list = field(default_factory=list)  # the same for the momentum
    fell_back_at: int = -1    # macro step from which the run is plain (-1: never)
    noise: tuple = (0.0, 0.0)  # one-step spread of two plain bursts (density, momentum)


def run_learned(ctx: E.Context, trainer: Trainer, norm: E.NnNorm, c0: torch.Tensor, steps: int,
                seed: int, judge_period: int = 4, threshold: float = 2e-3,
                threshold_momentum: float = None, bootstrap: int = 2) -> LearnedRun:
    """Learned-projection EFPI for `steps` macro steps from c0.

    Steps 0..bootstrap-1 are plain EFPI (the network needs three states); step 0
    is also taken a second time with another lift rotation, and the error of
    eq. 4.2 between the two results, nu (per moment), is the one-step noise of
    plain EFPI itself.  From step `bootstrap` on, every judge_period-th step
    (the first one included) is a judgement: a fine burst (the plain EFPI step
    with the lift rotation the plain run uses at that step), which the run
    continues from, compared with the learned candidate from the same state.  The
    one-step error e holds the burst's own noise as well as the network's error,
    so the network's part is taken as b = sqrt(max(e^2 - nu^2 / 2, 0)) (the
    candidate against one noisy burst, where two bursts differ by nu).  Each
    judgement vouches for the judge_period - 1 learned steps after it: b times
    their number is added to the accumulated-error bound of each moment before
    they are taken (errors of successive steps add at most linearly).  When the
    bound passes threshold (density) or threshold_momentum (momentum; default:
    threshold), every later step is plain EFPI, so no learned step is taken on a
    judgement that failed.  This is the paper's remark on reverting to the fine
    solver when an error estimate fails (Sec. 3.1), applied to the learned steps.
    """
    if ctx.moments != 2:
        raise ValueError("the learned projection takes the two-moment coarse state (n, j)")
    thr_m = threshold if threshold_momentum is None else threshold_momentum
    nc = trainer.n_c
    nc2 = c0.numel()
    dev = c0.device
    traj = torch.empty(steps + 1, nc2, dtype=torch.float64, device=dev)
    traj[0].copy_(c0)
    cand = torch.empty(nc2, dtype=torch.float64, device=dev)
    eps_dev = torch.zeros(4, dtype=torch.float64, device=dev)
    ws = trainer.workspace(1)
    judged = fallback = learned = 0
    eps_log, eps_mom, acc_log, accm_log = [], [], [], []
    acc = acc_m = 0.0
    plain_from = -1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # one-step noise of plain EFPI: step 0 with a second rotation
    E.efpi_macro_step(ctx.ctx, traj[0], cand, [lift_shift(seed ^ 0x5BD1E995, 0)])
    for n in range(steps):
        if n < bootstrap or plain_from >= 0:
            E.efpi_macro_step(ctx.ctx, traj[n], traj[n + 1], [lift_shift(seed, n)])
            if n == 0:
                E.efpi_rel_l2(cand[:nc], traj[1][:nc], eps_dev[2:3])
                E.efpi_rel_l2(cand[nc:], traj[1][nc:], eps_dev[3:4])
            if n >= bootstrap:
                fallback += 1
            continue
        # learned step from states n-2, n-1, n
        if (n - bootstrap) % judge_period == 0:
            E.efpi_nn_predict_step(trainer.params, trainer.pack, traj[n - 2:n + 1], nc,
                                   trainer.periodic, norm, cand, ws)
            E.efpi_macro_step(ctx.ctx, traj[n], traj[n + 1], [lift_shift(seed, n)])
            E.efpi_rel_l2(cand[:nc], traj[n + 1][:nc], eps_dev[0:1])
            E.efpi_rel_l2(cand[nc:], traj[n + 1][nc:], eps_dev[1:2])
            e, e_mom, nu, nu_m = (float(a) for a in eps_dev.cpu())
            judged += 1
            span = max(judge_period - 1, 1)
            acc += span * float(np.sqrt(max(e * e - 0.5 * nu * nu, 0.0)))
            acc_m += span * float(np.sqrt(max(e_mom * e_mom - 0.5 * nu_m * nu_m, 0.0)))
            eps_log.append(e)
            eps_mom.append(e_mom)
            acc_log.append(acc)
            accm_log.append(acc_m)
            if acc > threshold or acc_m > thr_m:
                plain_from = n + 1
        else:
            E.efpi_nn_predict_step(trainer.params, trainer.pack, traj[n - 2:n + 1], nc,
                                   trainer.periodic, norm, traj[n + 1], ws)
            learned += 1
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    noise = tuple(float(a) for a in eps_dev[2:4].cpu())
    return LearnedRun(traj, judged, fallback, learned, eps_log, eps_mom, wall, acc_log, accm_log,
                      plain_from, noise)
