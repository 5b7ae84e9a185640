"""Helpers shared by the GPU parity tests: build a library context, move seeded
inputs to the device, and run the oracle on the same inputs."""
from __future__ import annotations

import numpy as np
import torch

from oracle import efpi as oefpi
from oracle import pic as opic


def lib():
    import paper_1610_01071_amd.efpi as E
    return E


def oracle_grid(spec):
    return opic.Grid(spec.n_cells, spec.length, spec.bc, spec.closure, spec.dt)


def oracle_scheme(spec):
    return oefpi.Scheme(levels=spec.haar_levels, burst_steps=spec.burst_steps,
                        macro_dt=spec.macro_dt, coevolving=bool(spec.coevolving), ppc=spec.ppc,
                        vth=spec.vth, lift_linear=bool(spec.lift_linear), n_floor=spec.n_floor)


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def set_particles(ctx, replica, cell, frac, v, w):
    E = lib()
    E.efpi_set_particles(ctx.ctx, replica, to_dev(cell, torch.int16), to_dev(frac, torch.float32),
                         to_dev(v, torch.float32), to_dev(w, torch.float32))


def particles_np(ctx, replica=0):
    c, f, v, w = ctx.particles(replica)
    return (c.cpu().numpy(), f.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy())


def grid_np(ctx, replica=0):
    q, phi, e = ctx.grid(replica)
    torch.cuda.synchronize()
    return q.cpu().numpy(), phi.cpu().numpy(), e.cpu().numpy()


def x_of(cell, frac, h):
    return (cell.astype(np.float64) + frac.astype(np.float64)) * h


def periodic_dx(a, b, length):
    d = np.asarray(a) - np.asarray(b)
    return d - length * np.round(d / length)


def relmax(a, b):
    """max |a - b| / max |b| (normwise relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))
