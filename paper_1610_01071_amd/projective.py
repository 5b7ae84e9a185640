"""Higher-order and adaptive projective integration driven through the C ABI.

A macro step here is lift, restricting fine burst, snapshots, then
``efpi_project2``: the least-squares slope of eq. 3.18 and either the
forward-Euler projection of eq. 3.17 (order 1) or the second-order step that
extrapolates the slopes of the last two bursts to the middle of the projection
leap (order 2; include/efpi.h).  The adaptive integrator takes the difference of
the two projections of the coarse density (the error of eq. 4.2) as the local
error of a first-order step, which grows as Delta t^2, and sets the next Delta t
from it (the library's ``efpi_next_macro_dt``), with ``efpi_set_macro_dt`` between steps.

Python only chooses step sizes and calls the library; all arithmetic on the
coarse and fine states runs in the library's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import torch

from . import efpi as E
from .learned import lift_shift


@dataclass
class ProjectiveRun:
    states: list          # coarse states [2 N_c] at the step ends (first: the start)
    times: list           # times of the states
    steps: list           # Delta t of every step
    err: list             # Euler / second-order difference of the density per step
                          # (eq. 4.2; 0 on the first step, which has no previous slope)
    wall_ms: float


def run_projective(ctx: E.Context, c0: torch.Tensor, t_end: float, macro_dt: float, seed: int,
                   order: int = 2, tol: float = 0.0, dt_min: float = 0.0,
                   dt_max: float = 0.0, shift_of=None) -> ProjectiveRun:
    """Projective integration of a one-replica context from c0 (time 0) to t_end.

    order 1: forward-Euler steps (eq. 3.17); order 2: the second-order step from
    the second step on.  tol > 0 makes the step adaptive in [dt_min, dt_max]
    (raised to at least N_e dt), starting from macro_dt; otherwise every step is
    macro_dt.  The last step is shortened, or the last two are evened out, so
    that the run ends at t_end with every step in [dt_min, dt_max]; only when
    t_end itself or dt_max < 2 dt_min leaves a remainder below N_e dt does the
    last step (a burst without leap) pass t_end.
    shift_of(n) gives the lift rotation of step n (default: lift_shift(seed, n))."""
    if len(ctx.spec.replicas) != 1:
        raise ValueError("run_projective drives a context with one replica")
    if order not in (1, 2):
        raise ValueError("order must be 1 or 2")
    spec = ctx.spec.replicas[0]
    ne_dt = spec.burst_steps * spec.dt
    adaptive = tol > 0.0
    lo = max(dt_min if adaptive else macro_dt, ne_dt)
    hi = max(dt_max if adaptive else macro_dt, lo)
    if shift_of is None:
        shift_of = lambda n: lift_shift(seed, n)
    nc2 = c0.numel()
    dev = c0.device
    cur = c0.clone()
    snap = ctx.new_snap()
    slope = [torch.empty(nc2, dtype=torch.float64, device=dev) for _ in range(2)]
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    states, times, steps, errs = [c0.clone()], [0.0], [], []
    t, dt, gap, n = 0.0, min(hi, max(lo, macro_dt)), 0.0, 0
    set_dt = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < t_end - 1e-9:
        left = t_end - t
        if left <= dt * (1.0 + 1e-12):
            dt = max(left, ne_dt)
        elif left < dt + lo:
            # a full step would leave less than dt_min: split the rest in two
            # steps, or take it whole when two would fall below dt_min
            dt = left / 2.0 if left >= 2.0 * lo else min(left, hi)
        if dt != set_dt:
            E.efpi_set_macro_dt(ctx.ctx, dt)
            set_dt = dt
        E.efpi_lift(ctx.ctx, cur, [shift_of(n)])
        E.efpi_pic_burst(ctx.ctx, spec.burst_steps, True)
        E.efpi_restrict(ctx.ctx, snap)
        euler = torch.empty(nc2, dtype=torch.float64, device=dev)
        second = torch.empty(nc2, dtype=torch.float64, device=dev)
        # the previous slope always enters: the error estimate needs it at either order
        prev = slope[(n + 1) % 2] if n > 0 else None
        E.efpi_project2(ctx.ctx, snap, prev, gap, slope[n % 2], euler, second)
        e = 0.0
        if prev is not None:
            nd = nc2 // ctx.moments  # the density coefficients lead the state
            E.efpi_rel_l2(second[:nd], euler[:nd], eps, ctx.stream)
            with torch.cuda.stream(ctx.stream):      # read it back on the context's stream
                e = float(eps.item())
        cur = second if order == 2 else euler
        t += dt
        states.append(cur)
        times.append(t)
        steps.append(dt)
        errs.append(e)
        gap = dt
        # the first step has no error estimate and keeps its size
        if adaptive and n > 0:
            dt = E.efpi_next_macro_dt(dt, e, tol, lo, hi)
        n += 1
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return ProjectiveRun(states, times, steps, errs, wall)
