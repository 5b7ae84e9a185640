"""Inputs of the phase-space lift parity cases, shared by the GPU parity tests and
the CPU check that the oracle's summation order does not decide them."""
from __future__ import annotations

import functools
import math

import numpy as np

import synth
from oracle import efpi as oefpi
from oracle import phase as ophase
from oracle import pic as opic

S3 = math.sqrt(3.0)
D4 = [(1 + S3) / (4 * math.sqrt(2)), (3 + S3) / (4 * math.sqrt(2)),
      (3 - S3) / (4 * math.sqrt(2)), (1 - S3) / (4 * math.sqrt(2))]

# (n_cells, levels, jf, jc, ions per cell, filter): the closed-form 4-tap
# Daubechies filter, and the oracle's order-4 Coiflet at the benchmark's 4096 cells
LIFT_CASES = [(128, 2, 6, 4, 40, "d4"), (256, 3, 7, 5, 24, "d4"), (128, 2, 11, 6, 24, "d4"),
              (4096, 4, 8, 5, 8, "coif12")]


@functools.lru_cache(maxsize=None)
def _coiflet() -> tuple:
    return tuple(ophase.coiflet_filter())


def taps(name: str) -> np.ndarray:
    return np.array(D4) if name == "d4" else np.array(_coiflet())


def phase_state(n, ppc, seed, ps, h):
    """Coarse phase-space coefficients of a quiet IAW start (oracle load and coarsening)."""
    g = opic.Grid(n, float(n))
    sch = oefpi.Scheme(ppc=ppc, vth=0.316)
    dens, u = synth.iaw_profile(n, float(n))
    c, f, v, w = oefpi.load_particles(dens, u, g, sch, synth.lift_shift(seed))
    x = oefpi.particles_to_x(c, f, g)
    return ophase.coarsen(ophase.phase_histogram(x, v, w, g, ps), ps, h)
