"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module draws random numbers and evaluates the analytic initial profiles of
the paper's test problems; it holds none of the method's arithmetic.  Both the
GPU path and the CPU oracle receive the arrays it returns as plain inputs.

Workloads (the paper's test problems at the sizes of the benchmark configs):
* ion-acoustic wave (Sec. 4.1, eq. 4.1): n(x) = 1 + delta cos(2 pi x / L) and
  mean velocity u(x) = delta cos(2 pi x / L) (in ion-sound units), Maxwellian
  ions of thermal speed sqrt(T_i / T_e), periodic domain;
* plasma slab expanding into vacuum (Sec. 4.2, with a uniform slab): n = 1 on
  the central fraction `width` of the domain, 0 outside, u = 0, absorbing walls.
"""
from __future__ import annotations

import numpy as np

SEED = 2016


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def iaw_profile(n_cells: int, length: float, delta: float = 0.2, mode: int = 1,
                with_velocity: bool = True, n_nodes: int | None = None):
    """Node density and mean velocity of the ion-acoustic-wave initial state (eq. 4.1)."""
    n_nodes = n_cells if n_nodes is None else n_nodes
    x = np.arange(n_nodes) * (length / n_cells)
    c = np.cos(2.0 * np.pi * mode * x / length)
    n = 1.0 + delta * c
    u = delta * c if with_velocity else np.zeros_like(c)
    return n, u


def slab_profile(n_cells: int, width: float = 0.25):
    """Node density (N + 1 wall-bounded nodes) of a centred uniform slab, and u = 0."""
    k = np.arange(n_cells + 1)
    lo = n_cells * (1.0 - width) / 2.0
    hi = n_cells * (1.0 + width) / 2.0
    n = ((k >= lo) & (k < hi)).astype(np.float64)
    return n, np.zeros_like(n)


def lift_shift(seed: int) -> int:
    """32-bit Cranley-Patterson rotation for one lift, drawn from the seed."""
    return int(rng(seed).integers(0, 2 ** 32, dtype=np.uint64))


def random_particles(n: int, n_cells: int, seed: int, vth: float = 0.3,
                     w_mean: float = 1e-2, sort: bool = True, dead_fraction: float = 0.0):
    """Random FP32 particle state (cell int16, frac f32, v f32, w f32).

    Cells uniform on [0, n_cells), offsets uniform on [0, 1), Maxwellian
    velocities, weights uniform in [0.5, 1.5] w_mean.  A fraction of particles
    can be marked dead (cell = -1) to exercise absorbed-particle handling.
    """
    g = rng(seed)
    cell = g.integers(0, n_cells, n).astype(np.int16)
    if sort:
        cell = np.sort(cell)
    frac = g.random(n, dtype=np.float32)
    frac = np.minimum(frac, np.float32(1.0) - np.float32(2.0 ** -24)).astype(np.float32)
    v = (vth * g.standard_normal(n)).astype(np.float32)
    w = (w_mean * (0.5 + g.random(n))).astype(np.float32)
    if dead_fraction > 0.0:
        dead = g.random(n) < dead_fraction
        cell[dead] = -1
    return cell, frac, v, w


def random_coarse(n_coarse: int, seed: int, levels: int, mean_density: float = 1.0,
                  amp: float = 0.2, u_amp: float = 0.2):
    """Smooth random coarse (density, momentum) coefficients, shape (2, n_coarse)."""
    g = rng(seed)
    k = np.arange(n_coarse)
    dens = np.full(n_coarse, mean_density)
    mom = np.zeros(n_coarse)
    for m in range(1, 4):
        a, b, ph = g.standard_normal(3)
        dens += amp / m * a * np.cos(2 * np.pi * m * k / n_coarse + ph)
        mom += u_amp / m * b * np.cos(2 * np.pi * m * k / n_coarse + ph)
    scale = 2.0 ** (levels / 2.0)
    return np.stack([dens * scale, mom * dens * scale])


def random_coarse_efree(n_coarse: int, seed: int, levels: int, t_range=(0.05, 0.2)):
    """Three coarse moments (density n, momentum j, second moment s) of positive
    density and temperature, shape (3, n_coarse): the two of random_coarse and
    c^s = (c^j)^2 / c^n + c^n T for a block temperature T drawn uniformly in
    t_range.  Also returns T."""
    c = random_coarse(n_coarse, seed=seed, levels=levels)
    t = rng(seed + 1).uniform(t_range[0], t_range[1], n_coarse)
    return np.stack([c[0], c[1], c[1] ** 2 / c[0] + c[0] * t]), t


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Steele, Lea and Flood, 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def ensemble_sizes(n_replicas: int = 64, seed: int = SEED, target: float = 150e6,
                   lo: float = 140e6, hi: float = 160e6):
    """Uneven ensemble of ion-acoustic replicas: [(n_cells, ppc)] per replica.

    n_cells = 1024 * 2^(r mod 5) (1024 .. 16384), ppc from a uniform draw
    u_r in [0.5, 1.5) of SplitMix64(seed + r): ppc = clamp(round(2,343,750 u_r /
    n_cells), 100, 2000), rescaled once so that the total ion count lies in
    [lo, hi] (about 150 M ions).
    """
    cells = [1024 << (r % 5) for r in range(n_replicas)]
    u = [0.5 + splitmix64(seed + r) / 2.0 ** 64 for r in range(n_replicas)]

    def ppcs(scale):
        return [int(min(2000, max(100, round(2_343_750 * ur * scale / n)))) for ur, n in
                zip(u, cells)]

    scale = 1.0
    for _ in range(20):
        total = sum(n * p for n, p in zip(cells, ppcs(scale)))
        if lo <= total <= hi:
            break
        scale *= target / total
    return list(zip(cells, ppcs(scale)))
