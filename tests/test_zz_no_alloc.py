"""efpi_phase_restrict_static (histogram in the library's static device scratch,
no work buffer) against efpi_phase_restrict with a caller work buffer.

Both run the same kernels on an order-free int64 histogram, so the coarse
coefficients must agree bit for bit.  Two calls in a row, the second with a
smaller histogram on another context (the array keeps the first call's
contents, which the second must clear), then the first case again after it;
a co-evolving restriction after a burst; and a histogram beyond the array's
size rejected before anything is enqueued.
"""
import numpy as np
import pytest
import torch

import synth
from helpers import lib, set_particles
from phase_cases import D4, taps

pytestmark = pytest.mark.gpu

STATIC_BYTES = 8 << 20


def with_work(E, ctx, ph, tau=0.0, stored=False):
    nbytes = E.efpi_phase_work_size(ctx.ctx, 0, ph)
    work = torch.empty(nbytes // 8 + 32, dtype=torch.int64, device="cuda")
    off = (-work.data_ptr()) % 256 // 8
    out = torch.empty(nbytes // 8 >> (ph.jf - ph.jc), dtype=torch.float64, device="cuda")
    E.efpi_phase_restrict(ctx.ctx, 0, ph, tau, work[off: off + nbytes // 8], out, stored)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def static(E, ctx, ph, tau=0.0, stored=False):
    nbytes = E.efpi_phase_work_size(ctx.ctx, 0, ph)
    out = torch.full((nbytes // 8 >> (ph.jf - ph.jc),), np.nan, dtype=torch.float64,
                     device="cuda")
    E.efpi_phase_restrict_static(ctx.ctx, 0, ph, tau, out, stored)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def loaded(E, n_cells, ppc, seed):
    ctx = E.Context(E.ConfigSpec([E.ReplicaSpec(n_cells, float(n_cells), ppc=ppc,
                                                haar_levels=2)]))
    set_particles(ctx, 0, *synth.random_particles(n_cells * ppc, n_cells, seed=seed, vth=0.7,
                                                  w_mean=1.0 / ppc))
    return ctx


def test_static_matches_work_buffer_on_consecutive_calls():
    E = lib()
    big = loaded(E, 4096, 30, 11)
    ph_big = E.phase(-2.0, 2.0, 11, 6, 4, list(taps("coif12")))   # 256 x 2^11 int64: 4 MiB
    assert E.efpi_phase_work_size(big.ctx, 0, ph_big) == 4 << 20
    small = loaded(E, 512, 40, 12)
    ph_small = E.phase(-1.5, 1.5, 7, 4, 2, D4)                  # 128 x 2^7 int64: 128 KiB
    ref_big = with_work(E, big, ph_big)
    ref_small = with_work(E, small, ph_small)
    got_big = static(E, big, ph_big)
    got_small = static(E, small, ph_small)
    assert np.array_equal(got_big, ref_big)
    assert np.array_equal(got_small, ref_small)
    # and back to the larger histogram over what the smaller call left
    assert np.array_equal(static(E, big, ph_big), ref_big)
    E.efpi_sync(big.ctx)
    E.efpi_sync(small.ctx)


def test_static_coevolving_frame_after_a_burst():
    E = lib()
    n = 1024
    spec = E.ReplicaSpec(n, float(n), ppc=60, haar_levels=3, vth=0.316)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters_start=10))
    dens, u = synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(dens, device="cuda"),
                        torch.as_tensor(u, device="cuda"), 7)
    E.efpi_store_field(ctx.ctx)
    E.efpi_pic_burst(ctx.ctx, 5, False)
    ph = E.phase(-2.0, 2.0, 9, 5, 3, D4)
    for tau, stored in ((4.0, False), (2.5, True)):
        assert np.array_equal(static(E, ctx, ph, tau, stored), with_work(E, ctx, ph, tau, stored))
    E.efpi_sync(ctx.ctx)


def test_static_rejects_histograms_beyond_its_size():
    E = lib()
    ctx = E.Context(E.ConfigSpec([E.ReplicaSpec(16384, 16384.0, ppc=1, haar_levels=2)]))
    ok = E.phase(-1.0, 1.0, 11, 6, 6, D4)     # 256 x 2^11 int64: 4 MiB
    over = E.phase(-1.0, 1.0, 11, 6, 2, D4)   # 4096 x 2^11 int64: 64 MiB
    assert E.efpi_phase_work_size(ctx.ctx, 0, ok) <= STATIC_BYTES
    assert E.efpi_phase_work_size(ctx.ctx, 0, over) > STATIC_BYTES
    out = torch.zeros(4096 << 6, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EfpiError, match="static scratch"):
        E.efpi_phase_restrict_static(ctx.ctx, 0, over, 0.0, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0   # nothing was enqueued
    E.efpi_phase_restrict_static(ctx.ctx, 0, ok, 0.0, out)
    E.efpi_sync(ctx.ctx)
