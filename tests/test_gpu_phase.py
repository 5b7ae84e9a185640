"""Phase-space restriction on the GPU (efpi_phase_restrict) against the oracle.

Bars: the int64 restricted histogram bit-exact against the oracle's integer
form (same quantisation, fresh ions, tau = 0, power-of-two bin widths, 2^5 to
2^11 bins); the
coarse coefficients within 1e-13 of the oracle's transform of that histogram,
for the closed-form 4-tap Daubechies filter and for 12 seeded taps; after a
burst, along the co-evolving frame, within eps = 1e-4 (eq. 4.2) of the FP64
oracle (FP32 positions and velocities move a few ions across bin edges).  The
lift (cells and offsets bit-exact, velocities and weights within 1e-6) and the
macro step (eps 1e-3) with the 4-tap filter and with the oracle's order-4
Coiflet at 4096 cells.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import phase as ophase
from oracle import pic as opic
from oracle import metrics
from helpers import lib, oracle_grid, set_particles, particles_np, grid_np, x_of
from phase_cases import D4, LIFT_CASES, phase_state, taps

pytestmark = pytest.mark.gpu


def run(E, ctx, ph, tau=0.0, replica=0):
    nbytes = E.efpi_phase_work_size(ctx.ctx, replica, ph)
    work = torch.empty(nbytes // 8 + 32, dtype=torch.int64, device="cuda")
    off = (-work.data_ptr()) % 256 // 8
    work = work[off: off + nbytes // 8]
    nxc = ctx.spec.replicas[replica].n_cells >> ph.levels
    out = torch.empty(nxc * (1 << ph.jc), dtype=torch.float64, device="cuda")
    E.efpi_phase_restrict(ctx.ctx, replica, ph, tau, work, out)
    torch.cuda.synchronize()
    return work.view(nxc, 1 << ph.jf).cpu().numpy(), out.view(nxc, 1 << ph.jc).cpu().numpy()


@pytest.mark.parametrize("n_cells,levels,jf,jc,taps", [
    (256, 2, 6, 4, "d4"), (1024, 4, 8, 5, "taps12"), (64, 0, 5, 4, "d4"), (4096, 4, 10, 6, "d4"),
    (512, 2, 11, 6, "taps12")])
def test_histogram_bitexact_and_coefficients(n_cells, levels, jf, jc, taps):
    E = lib()
    spec = E.ReplicaSpec(n_cells, float(n_cells), ppc=30, haar_levels=2)
    ctx = E.Context(E.ConfigSpec([spec]))
    parts = synth.random_particles(n_cells * 30, n_cells, seed=n_cells + jf, vth=0.7,
                                   w_mean=1.0 / 30)
    set_particles(ctx, 0, *parts)
    # the transform is linear in the filter: any 12 taps exercise the 12-tap path
    h = D4 if taps == "d4" else list(np.random.default_rng(5).normal(0.0, 0.3, 12))
    ph = E.phase(-2.0, 2.0, jf, jc, levels, h)
    ps = ophase.PhaseScheme(levels=levels, v_min=-2.0, v_max=2.0, jf=jf, jc=jc)
    H, coarse = run(E, ctx, ph)
    ref_H = ophase.restricted_histogram_fx(parts[0], parts[1], parts[2], parts[3], n_cells, ps)
    assert np.array_equal(H, ref_H)
    ref = ophase.coarse_from_histogram_fx(ref_H, ps, spec.length / n_cells, np.array(h))
    assert np.max(np.abs(coarse - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_coevolving_frame_after_a_burst():
    E = lib()
    n = 512
    spec = E.ReplicaSpec(n, float(n), ppc=60, haar_levels=3, vth=0.316)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters_start=10))
    dens, u = synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(dens, device="cuda"),
                        torch.as_tensor(u, device="cuda"), 7)
    E.efpi_pic_burst(ctx.ctx, 5, False)
    ph = E.phase(-2.0, 2.0, 7, 5, 3, D4)
    _, coarse = run(E, ctx, ph, tau=4.0)
    c, f, v, w = particles_np(ctx)
    _, _, e = grid_np(ctx)
    g = oracle_grid(spec)
    x = x_of(c, f, g.h)
    ex = opic.gather(e.astype(np.float64), x, g)
    vc = v.astype(np.float64) + 0.5 * g.dt * ex
    ps = ophase.PhaseScheme(levels=3, v_min=-2.0, v_max=2.0, jf=7, jc=5)
    ref = ophase.restrict_phase(x, vc, ex, w.astype(np.float64), 4.0, g, ps, np.array(D4))
    assert metrics.rel_l2(coarse, ref) < 1e-4
    E.efpi_sync(ctx.ctx)


def test_phase_parameters_checked():
    E = lib()
    walls = E.Context(E.ConfigSpec([E.ReplicaSpec(64, 64.0, bc=1, ppc=4)]))
    with pytest.raises(E.EfpiError):
        E.efpi_phase_work_size(walls.ctx, 0, E.phase(-1, 1, 6, 4, 1, D4))
    per = E.Context(E.ConfigSpec([E.ReplicaSpec(64, 64.0, ppc=4)]))
    for bad in (E.phase(-1, 1, 3, 2, 1, D4), E.phase(1, -1, 6, 4, 1, D4),
                E.phase(-1, 1, 6, 7, 1, D4), E.phase(-1, 1, 6, 1, 1, D4),
                E.phase(-1, 1, 6, 4, 7, D4), E.phase(-1, 1, 6, 4, 1, D4[:3]),
                E.phase(-1, 1, 12, 6, 1, D4)):
        with pytest.raises(E.EfpiError):
            E.efpi_phase_work_size(per.ctx, 0, bad)
    # the int64 histogram's range: h 4^levels below 2^18
    big = E.Context(E.ConfigSpec([E.ReplicaSpec(16384, 16384.0, ppc=1)]))
    E.efpi_phase_work_size(big.ctx, 0, E.phase(-1, 1, 6, 4, 8, D4))      # 2^16: accepted
    with pytest.raises(E.EfpiError):
        E.efpi_phase_work_size(big.ctx, 0, E.phase(-1, 1, 6, 4, 9, D4))  # 2^18: rejected
    coarse = E.Context(E.ConfigSpec([E.ReplicaSpec(1024, 4096.0, ppc=1)]))   # h = 4
    with pytest.raises(E.EfpiError):
        E.efpi_phase_work_size(coarse.ctx, 0, E.phase(-1, 1, 6, 4, 8, D4))


@pytest.mark.parametrize("n,levels,jf,jc,ppc,filt", LIFT_CASES)
def test_phase_lift_matches_oracle(n, levels, jf, jc, ppc, filt):
    E = lib()
    spec = E.ReplicaSpec(n, float(n), ppc=ppc, haar_levels=2)
    ctx = E.Context(E.ConfigSpec([spec]))
    ps = ophase.PhaseScheme(levels=levels, v_min=-2.0, v_max=2.0, jf=jf, jc=jc, ppc=ppc)
    h = taps(filt)
    coarse = phase_state(n, 50, 3, ps, h)
    # the reconstruction of a sharp Maxwellian has negative wiggles: the repair runs
    refined = ophase.refine(coarse, ps, h)
    assert np.min(refined) < 0.0
    ph = E.phase(-2.0, 2.0, jf, jc, levels, list(h))
    work = torch.empty(E.efpi_phase_lift_work_size(ctx.ctx, 0, ph) + 256, dtype=torch.uint8,
                       device="cuda")
    work = work[(-work.data_ptr()) % 256:]
    E.efpi_phase_lift(ctx.ctx, 0, ph, torch.as_tensor(coarse.ravel(), device="cuda"), 4242, work)
    E.efpi_sync(ctx.ctx)
    gc, gf, gv, gw = particles_np(ctx)
    rc, rf, rv, rw = ophase.lift_phase(coarse, opic.Grid(n, float(n)), ps, h, 4242)
    assert np.array_equal(gc, rc) and np.array_equal(gf.astype(np.float64), rf)
    assert np.max(np.abs(gv - rv)) <= 1e-6 * np.max(np.abs(rv))     # FP32 store
    assert np.max(np.abs(gw - rw)) <= 1e-6 * np.max(np.abs(rw))


def test_phase_lift_matches_oracle_at_the_papers_resolution():
    """The lift at the paper's velocity resolution (2^11 bins, 2^6 Coiflet-12
    coefficients per node) on 1024 cells and l = 4: cells and offsets bit-exact,
    velocities and weights within 1e-6 (the CDF repair's decisions are the oracle's).
    The oracle's repair runs node by node in Python, about 20 s here."""
    test_phase_lift_matches_oracle(1024, 4, 11, 6, 8, "coif12")


@pytest.mark.parametrize("n,levels,jf,jc,ppc,filt", [(128, 2, 6, 4, 48, "d4"),
                                                     (4096, 4, 8, 5, 8, "coif12")])
def test_phase_macro_step_matches_oracle(n, levels, jf, jc, ppc, filt):
    from paper_1610_01071_amd.phase import PhaseStepper
    E = lib()
    spec = E.ReplicaSpec(n, float(n), ppc=ppc, haar_levels=2, burst_steps=6, macro_dt=3.0,
                         vth=0.316)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters_start=12))
    ps = ophase.PhaseScheme(levels=levels, v_min=-2.0, v_max=2.0, jf=jf, jc=jc, burst_steps=6,
                            macro_dt=3.0, ppc=ppc)
    h = taps(filt)
    coarse = phase_state(n, 50, 5, ps, h)
    stepper = PhaseStepper(ctx, E.phase(-2.0, 2.0, jf, jc, levels, list(h)))
    out = stepper.new_coarse()
    stepper.macro_step(torch.as_tensor(coarse.ravel(), device="cuda"), out, 777)
    E.efpi_sync(ctx.ctx)
    ref, _ = ophase.phase_macro_step(coarse, opic.Grid(n, float(n)), ps, h, 777)
    assert metrics.rel_l2(out.view(ref.shape).cpu().numpy(), ref) < 1e-3
