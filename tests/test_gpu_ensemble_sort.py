"""Ensembles (several replicas in one launch per step), the cell sort and
capacity handling, through the C ABI on the GPU."""
import numpy as np
import pytest
import torch

import synth
from helpers import lib, to_dev, set_particles, particles_np, grid_np

pytestmark = pytest.mark.gpu


def make_ctx(specs, **kw):
    E = lib()
    return E.Context(E.ConfigSpec(list(specs), **kw))


def test_sort_stable_and_drops_absorbed():
    E = lib()
    n = 50000 - 7
    spec = E.ReplicaSpec(1024, 1024.0, ppc=1, haar_levels=2, capacity=50000)
    ctx = make_ctx([spec], flags=E.FLAG_SORT_BUFFER)
    cell, frac, v, w = synth.random_particles(n, 1024, seed=31, sort=False, dead_fraction=0.1)
    set_particles(ctx, 0, cell, frac, v, w)
    E.efpi_deposit(ctx.ctx)
    q0, _, _ = grid_np(ctx)
    E.efpi_sort(ctx.ctx)
    gc, gf, gv, gw = particles_np(ctx)
    alive = cell >= 0
    order = np.argsort(cell[alive], kind="stable")
    assert np.array_equal(gc, cell[alive][order])
    assert np.array_equal(gf, frac[alive][order])
    assert np.array_equal(gv, v[alive][order])
    assert np.array_equal(gw, w[alive][order])
    E.efpi_deposit(ctx.ctx)
    q1, _, _ = grid_np(ctx)
    assert np.array_equal(q0, q1)


def test_sort_needs_buffer_flag():
    E = lib()
    ctx = make_ctx([E.ReplicaSpec(64, 64.0, ppc=2, haar_levels=2)])
    with pytest.raises(E.EfpiError):
        E.efpi_sort(ctx.ctx)


def _specs():
    E = lib()
    kw = dict(haar_levels=3, burst_steps=10, macro_dt=5.0)
    return [E.ReplicaSpec(256, 256.0, ppc=50, **kw),
            E.ReplicaSpec(512, 512.0, ppc=30, **kw),
            E.ReplicaSpec(256, 256.0, ppc=80, **kw),
            E.ReplicaSpec(2048, 2048.0, ppc=12, **kw)]


def test_ensemble_replicas_equal_single_runs():
    E = lib()
    specs = _specs()
    coarse = [synth.random_coarse(s.n_coarse, seed=40 + r, levels=s.haar_levels)
              for r, s in enumerate(specs)]
    shifts = [synth.lift_shift(50 + r) for r in range(len(specs))]
    ens = make_ctx(specs)
    cin = to_dev(np.concatenate([c.ravel() for c in coarse]), torch.float64)
    cout = ens.new_coarse()
    E.efpi_macro_step(ens.ctx, cin, cout, shifts)
    E.efpi_sync(ens.ctx)
    parts = ens.split_coarse(cout)
    for r, s in enumerate(specs):
        one = make_ctx([s])
        o = one.new_coarse()
        E.efpi_macro_step(one.ctx, to_dev(coarse[r].ravel(), torch.float64), o, [shifts[r]])
        E.efpi_sync(one.ctx)
        assert torch.equal(o.view(2, -1), parts[r]), r
        a = particles_np(one)
        b = particles_np(ens, r)
        assert all(np.array_equal(x, y) for x, y in zip(a, b)), r


def test_ensemble_mean_over_equal_grids():
    E = lib()
    specs = _specs()
    ens = make_ctx(specs)
    vals = [np.full(2 * s.n_coarse, float(r + 1)) for r, s in enumerate(specs)]
    c = to_dev(np.concatenate(vals), torch.float64)
    E.efpi_ensemble_mean(ens.ctx, c)
    torch.cuda.synchronize()
    parts = [p.cpu().numpy() for p in ens.split_coarse(c)]
    # replicas 0 and 2 share (256, 256.0): mean of 1 and 3; 1 and 3 are alone
    assert np.allclose(parts[0], 2.0) and np.allclose(parts[2], 2.0)
    assert np.allclose(parts[1], 2.0) and np.allclose(parts[3], 4.0)


def test_lift_capacity_overflow_flag():
    E = lib()
    spec = E.ReplicaSpec(128, 128.0, ppc=10, haar_levels=2, capacity=600)
    ctx = make_ctx([spec])
    coarse = synth.random_coarse(32, seed=3, levels=2)
    E.efpi_lift(ctx.ctx, to_dev(coarse.ravel(), torch.float64), [1])
    with pytest.raises(E.EfpiError) as ei:
        E.efpi_sync(ctx.ctx)
    assert ei.value.status == -7
    c, f, v, w = particles_np(ctx)
    assert c.size == 600 and np.all(np.diff(c) >= 0)
