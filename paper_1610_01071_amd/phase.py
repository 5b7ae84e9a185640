"""Projective integration on phase-space coarse variables (the wavelet-based
scheme of Sec. 3.3), driven through the C ABI.

A macro step is: efpi_phase_lift (columns back to the fine velocity grid,
midpoint interpolation in x, CDF repair of App. C, inverse-CDF quiet start),
with kinetic electrons efpi_reset_electrons (Boltzmann electrons for the lifted
ions), efpi_store_field (E_n of the burst start), then for p = 0..N_e the phase-space
restriction along the co-evolving frame with tau = Delta t - p dt (App. B)
after p fine steps, and efpi_phase_project (eqs. 3.17-3.18) over the
snapshots.  Python only sequences the calls and owns the buffers.

The order-4 Coiflet filter of App. A comes from the library
(efpi_coiflet_taps), which derives it from its moment conditions.
"""
from __future__ import annotations

import numpy as np
import torch
from . import efpi as E


def coiflet_taps(n_taps: int = 12) -> np.ndarray:
    """The library's order-n_taps/3 Coiflet low-pass taps (12: the paper's order 4)."""
    return np.array(E.efpi_coiflet_taps(n_taps))


def _aligned(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off: off + nbytes]


class PhaseStepper:
    """Buffers and calls of phase-space macro steps for replica 0 of a context."""

    def __init__(self, ctx: E.Context, ph: E.Phase, replica: int = 0):
        spec = ctx.spec.replicas[replica]
        self.ctx, self.ph, self.replica, self.spec = ctx, ph, replica, spec
        dev = ctx.device
        self.n_coef = (spec.n_cells >> ph.levels) << ph.jc
        self.hist = _aligned(E.efpi_phase_work_size(ctx.ctx, replica, ph), dev)
        self.lift_work = _aligned(E.efpi_phase_lift_work_size(ctx.ctx, replica, ph), dev)
        self.snaps = torch.empty((spec.burst_steps + 1, self.n_coef), dtype=torch.float64,
                                 device=dev)

    def new_coarse(self) -> torch.Tensor:
        return torch.zeros(self.n_coef, dtype=torch.float64, device=self.ctx.device)

    def restrict(self, out: torch.Tensor, tau: float = 0.0, stored_field: bool = False):
        E.efpi_phase_restrict(self.ctx.ctx, self.replica, self.ph, tau, self.hist, out,
                              stored_field)

    def macro_step(self, coarse_in: torch.Tensor, coarse_out: torch.Tensor, shift: int):
        s = self.spec
        E.efpi_phase_lift(self.ctx.ctx, self.replica, self.ph, coarse_in, shift, self.lift_work)
        if s.closure == E.CLOSURE_KINETIC:
            # electrons in Boltzmann equilibrium with the lifted ions (their density
            # and mean velocity), as at every kinetic lift
            E.efpi_reset_electrons(self.ctx.ctx, [shift] * len(self.ctx.spec.replicas))
        E.efpi_store_field(self.ctx.ctx)
        for p in range(s.burst_steps + 1):
            if p > 0:
                E.efpi_pic_burst(self.ctx.ctx, 1, False)
            self.restrict(self.snaps[p], s.macro_dt - p * s.dt, True)
        E.efpi_phase_project(self.ctx.ctx, self.snaps, s.burst_steps + 1, s.dt, s.macro_dt,
                             coarse_out)
