#!/usr/bin/env python3
"""Benchmark of the EFPI / PIC-burst hot path on one MI355X.

Headline workload: the batched ensemble of 64 seeded replicas of the ion-acoustic
wave (Sec. 4.1, eq. 4.1; delta = 0.2, T_i/T_e = 0.1, Boltzmann electrons, CIC,
dt = 0.1): 1024 .. 16384 cells, 100 .. 2000 ions per cell, 147,954,688 FP32 ions
in all, Haar level l = log2(N / 256) (256 coarse blocks per moment and replica),
N_e = 20, Delta t = 200 dt, co-evolving restriction, Maxwellian-corrected
quiet-start lift.  One step = one EFPI macro step of every replica (lift, 20
restricted fine steps, restriction, least squares and projection) plus the
ensemble mean over replicas of equal grids, from the same coarse state; every
fine step is one particle launch and one field launch for all replicas.  Inputs
are synthetic and seeded and reside in HBM before the timed region.

Printed: one JSON line with particle-updates/s (ions x N_e per macro step over
the macro-step wall time, lift included), the roofline of the dominant kernel
(the fused push / deposit / restriction pass, timed by HIP events on its own
launches inside a second pass over the same steps), the burst's fraction of the
HBM peak at 24 bytes per particle-update, and the CPU oracle timed on the host's
cores on a sample of the same replicas.  Further legs: the single 4096-cell
wave (4,096,000 ions) with EFPI against full PIC at fixed moment error (eq. 4.2),
Euler / second-order / adaptive projective steps, the plain 1000-step PIC run
of 25,600 ions, the expanding slab (16.8 M ions, walls), the kinetic-electron
solver, the phase-space wavelet coarse variables and the learned projection.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s + EFPI wall-time speedup vs full PIC at fixed moment error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 24  # read cell(2) frac v w (4 each), write cell frac v
TILE = 4096  # ions per work item of the particle pass (one workgroup per item)
# Full-PIC references run in contexts of their own at the tile that is fastest
# for the plain push-and-deposit step, with the cell-sort period from the
# autotuner (sort_period), so that EFPI is not compared with a slowed PIC.
PIC_TILE = 2048
CPU_WORKERS_MAX = 16  # the host share of one GPU on the benchmark box


def pic_context(E, spec, newton_iters, newton_iters_start):
    return E.Context(E.ConfigSpec([spec], newton_iters=newton_iters,
                                  newton_iters_start=newton_iters_start, tile=PIC_TILE,
                                  flags=E.FLAG_SORT_BUFFER))


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_particles_hbm_traffic_ensemble148m.md")


def measured_traffic():
    """HBM bytes per launch of the particle pass from the committed counter record.

    The record holds FETCH_SIZE and WRITE_SIZE of the pass on the headline
    workload, scaled by a plain copy of known size, and the hash of the kernel
    source they were taken on; the figure is reported only while the source is
    unchanged.
    """
    import hashlib
    try:
        rec = {}
        for line in open(TRAFFIC_RECORD):
            if ":" in line and not line.startswith(("#", "|", " ", "`")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        src = os.path.join(ROOT, rec["kernel_source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def ensemble_specs(E, synth):
    return [E.ReplicaSpec(n, float(n), ppc=p, haar_levels=int(round(math.log2(n // 256))),
                          burst_steps=20, macro_dt=20.0, dt=0.1, vth=math.sqrt(0.1))
            for n, p in synth.ensemble_sizes()]


def workload_spec(E):
    return E.ReplicaSpec(n_cells=4096, length=4096.0, ppc=1000, haar_levels=4, burst_steps=20,
                         macro_dt=20.0, dt=0.1, vth=math.sqrt(0.1), coevolving=1, lift_linear=1)


def host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _oracle_macro_step(job):
    """One EFPI macro step of one ensemble replica by the CPU oracle (FP64 numpy):
    quiet start of the wave, plain restriction, then the timed macro step."""
    n, ppc, seed = job
    import numpy as np
    import synth
    from oracle import efpi as oefpi, pic as opic
    g = opic.Grid(n, float(n))
    sch = oefpi.Scheme(levels=int(round(math.log2(n // 256))), burst_steps=20, macro_dt=20.0,
                       ppc=ppc, vth=math.sqrt(0.1))
    nn, uu = synth.iaw_profile(n, float(n))
    c, f, v, w = oefpi.load_particles(nn, uu, g, sch, synth.lift_shift(seed))
    x = oefpi.particles_to_x(c, f, g)
    c0 = oefpi.restrict_state(x, v, w, np.ones(x.size, bool), g, sch)
    t0 = time.perf_counter()
    oefpi.macro_step(c0, g, sch, synth.lift_shift(seed + 1))
    return n * ppc, time.perf_counter() - t0


def cpu_baseline(synth, workers=None):
    """The oracle on this host: the smallest replicas of the headline ensemble, one
    macro step each, in parallel processes (one per core, at most the GPU's host
    share) and then one of them in this process alone.  Run before the GPU is
    initialised: the workers are forked."""
    import multiprocessing as mp
    sizes = synth.ensemble_sizes()
    order = sorted(range(len(sizes)), key=lambda r: sizes[r][0] * sizes[r][1])
    cores = workers or min(CPU_WORKERS_MAX, os.cpu_count() or 1)
    jobs = [(sizes[r][0], sizes[r][1], 2016 + r) for r in order[:cores]]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_macro_step, jobs)
    wall = time.perf_counter() - t0
    ions = sum(r[0] for r in res)
    one_ions, one_s = _oracle_macro_step(jobs[0])
    return {
        "value": ions * 20 / wall,
        "unit": "particle-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"one EFPI macro step (quiet-start lift, 20-step restricted burst, "
                   f"projection) of each of the {cores} smallest replicas of the headline "
                   f"ensemble ({ions} ions, {min(r[0] for r in res)}..{max(r[0] for r in res)} "
                   f"each), one process per core, FP64 numpy/scipy, {wall:.1f} s wall on "
                   f"{host_cpu()} (nproc {os.cpu_count()}); the rate scales the replicas' "
                   f"particle-updates to the wall time"),
        "single_thread_value": one_ions * 20 / one_s,
        "single_thread_sample": f"the first of those replicas ({one_ions} ions) alone, {one_s:.1f} s",
    }


def timed(torch, fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed ensemble macro steps")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--horizon", type=float, default=200.0,
                    help="physical time of the EFPI-vs-full-PIC comparison (1/omega_pi)")
    ap.add_argument("--eps-max", type=float, default=1e-2,
                    help="coarse-density error (eq. 4.2) that defines the fixed-error point")
    ap.add_argument("--sort-period", type=int, default=0,
                    help="full-PIC steps between sorts (0: from the autotuner)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="the ensemble headline only (profiling runs)")
    ap.add_argument("--no-speedup", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-efree", action="store_true",
                    help="skip the three-moment (EFREE) wave")
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--no-phase", action="store_true",
                    help="skip the phase-space (wavelet) coarse-variable runs")
    ap.add_argument("--no-kinetic", action="store_true",
                    help="skip the kinetic-electron fine solver and its EFPI runs")
    ap.add_argument("--kinetic-horizon", type=float, default=60.0,
                    help="physical time of the kinetic-electron comparison")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the Euler / second-order / adaptive projective runs")
    ap.add_argument("--tile", type=int, default=0,
                    help="ions per work item of the ensemble's particle pass (0: autotuned)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB three times (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              f"decomposition is described in DESIGN.md and not measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth

    cpu = None if (args.no_cpu or args.headline_only) else cpu_baseline(synth)
    if cpu is not None:
        print(f"[bench] cpu_baseline done", file=sys.stderr, flush=True)

    import paper_1610_01071_amd.efpi as E

    torch.cuda.set_device(0)
    # a stream of our own: captured macro steps need a non-null stream
    with torch.cuda.stream(torch.cuda.Stream()):
        out = run_bench(args, np, torch, synth, E)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def headline(args, np, torch, synth, E):
    """The 64-replica ensemble: macro steps timed without and with per-launch
    events, replayed from captured graphs, and the lift alone."""
    from paper_1610_01071_amd import autotune
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    specs = ensemble_specs(E, synth)
    n_ions = sum(s.n_cells * s.ppc for s in specs)
    K = specs[0].burst_steps
    t0 = time.perf_counter()
    if args.tile > 0:  # a fixed launch shape (profiling runs: one shape per kernel record)
        choice = autotune.Choice(args.tile, 0, float("nan"), [])
    else:
        choice = autotune.autotune(specs, tiles=(2048, TILE, 8192), grids=(0,), steps=1, warmup=1)
    t_tune = time.perf_counter() - t0
    ctx = E.Context(E.ConfigSpec(specs, newton_iters=2, newton_iters_start=4, tile=choice.tile,
                                 grid_blocks=choice.grid_blocks))
    for r, sp in enumerate(specs):
        n0, u0 = synth.iaw_profile(sp.n_cells, sp.length)
        E.efpi_load_profile(ctx.ctx, r, torch.as_tensor(n0, device="cuda"),
                            torch.as_tensor(u0, device="cuda"), synth.lift_shift(2016 + r))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 30, cold=True)
    a = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, a)
    b = ctx.new_coarse()
    E.efpi_sync(ctx.ctx, raise_on_error=False)
    shifts = lambda i: [synth.lift_shift(30_000 + 64 * i + r) for r in range(len(specs))]

    # every timed step is one whole macro step of every replica from the same state
    def step(i, graph=False):
        (E.efpi_macro_step_graph if graph else E.efpi_macro_step)(ctx.ctx, a, b, shifts(i))
        E.efpi_ensemble_mean(ctx.ctx, b)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    status = E.efpi_sync(ctx.ctx, raise_on_error=False)
    t0 = time.perf_counter()
    ms_total = timed(torch, lambda: [step(args.warmup + i) for i in range(args.steps)])
    wall = time.perf_counter() - t0
    status |= E.efpi_sync(ctx.ctx, raise_on_error=False)
    ms_per_step = ms_total / args.steps

    # The same number of macro steps again with every burst-step particle launch
    # bracketed by its own start/end events (hipExtLaunchKernelGGL on the launch
    # stream): the kernel's average duration for the roofline.  The headline rate
    # above is taken without the events.
    E.efpi_timing(ctx.ctx, True)
    ms_total_ev = timed(torch, lambda: [step(100 + i) for i in range(args.steps)])
    kern_ms, kern_n = E.efpi_timing_read(ctx.ctx)
    E.efpi_timing(ctx.ctx, False)
    status |= E.efpi_sync(ctx.ctx, raise_on_error=False)

    # the same steps replayed from captured graphs
    step(0, graph=True)
    torch.cuda.synchronize()
    ms_graph = timed(torch, lambda: [step(200 + i, graph=True) for i in range(args.steps)]) / \
        args.steps
    status |= E.efpi_sync(ctx.ctx, raise_on_error=False)

    # the lift alone (profile, occupancy, quiet load, block correction)
    ms_lift = timed(torch, lambda: [E.efpi_lift(ctx.ctx, a, shifts(300 + i))
                                    for i in range(args.steps)]) / args.steps
    E.efpi_sync(ctx.ctx, raise_on_error=False)
    ctx.close()

    # the runtime's device copy of 1 GiB (its blit kernel, plain loads and stores):
    # a reference rate, not a ceiling (nontemporal streams go faster)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = timed(torch, lambda: [dst.copy_(src) for _ in range(5)]) / 5
    copy_gbs = 2 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9
    del src, dst
    value = n_ions * K / (ms_per_step * 1e-3)
    avg_launch_s = kern_ms / max(kern_n, 1) * 1e-3
    achieved = BYTES_PER_UPDATE * n_ions / avg_launch_s / 1e9
    burst_rate = n_ions * K / ((ms_per_step - ms_lift) * 1e-3)
    return {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("batched EFPI ensemble: 64 seeded replicas of the ion-acoustic wave "
                         "(eq. 4.1, delta 0.2, Ti/Te 0.1, Boltzmann electrons, CIC, dt=0.1), "
                         "1024..16384 cells, 100..2000 ions/cell, 147,954,688 ions; K=20 "
                         "burst, Haar l=log2(N/256) (256 coarse/moment), Delta t=200 dt, "
                         "co-evolving restriction, quiet-start lift; one step = one macro "
                         "step of every replica from the same coarse state plus the "
                         "ensemble mean; one particle launch and one field launch per fine "
                         "step for all replicas"),
            "n_ions": n_ions,
            "replicas": len(specs),
            "burst_steps": K,
            "newton_iters_per_step": 2,
            "tile": choice.tile,
            "grid_blocks": choice.grid_blocks,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "kernel": "k_particles<kRestrict|kPush> (burst step)",
            "bytes_per_launch": BYTES_PER_UPDATE * n_ions,
            "avg_launch_us": avg_launch_s * 1e6,
            "launches": kern_n,
            "runtime_copy_gbs": copy_gbs,
            "frac_of_runtime_copy": achieved / copy_gbs,
        },
        "burst_hbm_frac": BYTES_PER_UPDATE * burst_rate / (HBM_PEAK_GBS * 1e9),
        "macro_step_hbm_frac": BYTES_PER_UPDATE * value / (HBM_PEAK_GBS * 1e9),
        "burst_particle_updates_per_s": burst_rate,
        "ms_per_step_graph": ms_graph,
        "ms_per_step_with_launch_events": ms_total_ev / args.steps,
        "lift_ms": ms_lift,
        "autotune_s": t_tune,
        "autotune_table": choice.table,
        "wall_s_timed": wall,
        "device_status": status,
    }


def iaw_leg(args, np, torch, synth, E):
    """The single 4096-cell ion-acoustic wave (4,096,000 ions): its macro-step rate and
    roofline, then EFPI against full PIC at fixed error and the projective variants."""
    spec = workload_spec(E)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4, tile=TILE,
                                 flags=E.FLAG_SORT_BUFFER))
    n_ions = spec.n_cells * spec.ppc
    c0 = initial_coarse(E, ctx, spec, synth, torch)
    c1 = ctx.new_coarse()
    macro = lambda i: E.efpi_macro_step(ctx.ctx, c0, c1, [synth.lift_shift(10_000 + i)])
    for i in range(3):
        macro(i)
    steps = 20
    ms = timed(torch, lambda: [macro(3 + i) for i in range(steps)]) / steps
    E.efpi_timing(ctx.ctx, True)
    timed(torch, lambda: [macro(100 + i) for i in range(steps)])
    kern_ms, kern_n = E.efpi_timing_read(ctx.ctx)
    E.efpi_timing(ctx.ctx, False)
    status = E.efpi_sync(ctx.ctx, raise_on_error=False)
    us = kern_ms / max(kern_n, 1) * 1e3
    out = {"n_ions": n_ions, "ms_per_macro_step": ms,
           "particle_updates_per_s": n_ions * spec.burst_steps / (ms * 1e-3),
           "particle_pass_us": us,
           "particle_pass_hbm_frac": BYTES_PER_UPDATE * n_ions / (us * 1e-6) / (HBM_PEAK_GBS * 1e9),
           "note": "57 MB of particles: held in the 256 MB last-level cache, not an HBM figure",
           "device_status": status}
    if not args.no_speedup:
        out.update(speedup_sweep(E, torch, np, synth, ctx, spec, c0, args))
    ctx.close()
    return out, c0


def efree_leg(E, torch, np, synth, args):
    """EFREE coarse variables (Sec. 3.2: n, j = nV and s = nV^2 + P per block) on the
    benchmark wave: the three-moment macro-step rate, and EFPI with three moments
    against full PIC over the same horizon from the same lifted start, with eps
    (eq. 4.2) at the horizon on the density, the second moment and the block
    pressure P = s - j^2 / n."""
    spec = workload_spec(E)
    flags = E.FLAG_PRESSURE | E.FLAG_SORT_BUFFER
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4, tile=TILE,
                                 flags=flags))
    n_ions = spec.n_cells * spec.ppc
    c0 = initial_coarse(E, ctx, spec, synth, torch)
    c1 = ctx.new_coarse()
    macro = lambda i: E.efpi_macro_step(ctx.ctx, c0, c1, [synth.lift_shift(50_000 + i)])
    for i in range(3):
        macro(i)
    steps = 20
    ms = timed(torch, lambda: [macro(3 + i) for i in range(steps)]) / steps
    status = E.efpi_sync(ctx.ctx, raise_on_error=False)
    ctx.close()
    out = {"n_ions": n_ions, "ms_per_macro_step": ms,
           "particle_updates_per_s": n_ions * spec.burst_steps / (ms * 1e-3),
           "device_status": status}
    if args.no_speedup:
        return out

    fine = int(round(args.horizon / spec.dt))
    shift0 = synth.lift_shift(60_000)
    pctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4, tile=TILE,
                                  flags=flags))

    def pic_run():
        E.efpi_lift(pctx.ctx, c0, [shift0])
        done = 0
        while done < fine:
            k = min(args.sort_period, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    c_pic = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, c_pic)
    pic_bits = E.efpi_sync(pctx.ctx, raise_on_error=False)
    pctx.close()
    ref = c_pic.view(3, -1).cpu().numpy()

    def eps(a, b):
        return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(a * a + b * b)))

    def pressure(c):
        return c[2] - c[1] ** 2 / c[0]

    def pert_eps(a, b):
        # eq. 4.2 on the perturbations about their means: the wave itself
        da, db = a - a.mean(), b - b.mean()
        return float(np.sqrt(np.sum((da - db) ** 2) / np.sum(da * da + db * db)))

    rows = []
    for mult in (50, 75, 100, 200):
        sp = workload_spec(E)
        sp.macro_dt = mult * spec.dt
        cx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=4, tile=TILE,
                                    flags=E.FLAG_PRESSURE))
        m = int(round(args.horizon / sp.macro_dt))
        a, b = cx.new_coarse(), cx.new_coarse()
        a.copy_(c0)
        state = {"a": a, "b": b}

        def efpi_run():
            for i in range(m):
                sh = shift0 if i == 0 else synth.lift_shift(60_000 + i)
                E.efpi_macro_step(cx.ctx, state["a"], state["b"], [sh])
                state["a"], state["b"] = state["b"], state["a"]

        t_efpi = timed(torch, efpi_run)
        bits = E.efpi_sync(cx.ctx, raise_on_error=False)
        got = state["a"].view(3, -1).cpu().numpy()
        rows.append({"macro_dt_over_dt": mult, "macro_steps": m, "efpi_ms": t_efpi,
                     "speedup": t_pic / t_efpi, "eps_density": eps(got[0], ref[0]),
                     "eps_density_perturbation": pert_eps(got[0], ref[0]),
                     "eps_second_moment": eps(got[2], ref[2]),
                     "eps_pressure": eps(pressure(got), pressure(ref)), "device_status": bits})
        cx.close()
    ok = [r for r in rows if r["eps_density"] <= args.eps_max and r["device_status"] == 0]
    best = max(ok, key=lambda r: r["macro_dt_over_dt"]) if ok and pic_bits == 0 else None
    # the two-moment scheme from the same start (its n and j): its lift reloads the
    # fixed temperature vth^2 every macro step, so the pressure it implies is n vth^2
    sp = workload_spec(E)
    sp.macro_dt = 75 * spec.dt
    cx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=4, tile=TILE))
    a2, b2 = cx.new_coarse(), cx.new_coarse()
    a2.copy_(c0.view(3, -1)[:2].reshape(-1))
    for i in range(int(round(args.horizon / sp.macro_dt))):
        sh = shift0 if i == 0 else synth.lift_shift(60_000 + i)
        E.efpi_macro_step(cx.ctx, a2, b2, [sh])
        a2, b2 = b2, a2
    bits2 = E.efpi_sync(cx.ctx, raise_on_error=False)
    g2 = a2.view(2, -1).cpu().numpy()
    cx.close()
    two = {"macro_dt_over_dt": 75, "eps_density": eps(g2[0], ref[0]),
           "eps_density_perturbation": pert_eps(g2[0], ref[0]),
           "eps_pressure_of_n_vth2": eps(g2[0] * spec.vth ** 2, pressure(ref)),
           "device_status": bits2}
    out.update({
        "two_moment_same_start": two,
        "efree_speedup_vs_pic": best["speedup"] if best else None,
        "horizon": args.horizon, "eps_max": args.eps_max, "pic_fine_steps": fine,
        "pic_ms": t_pic, "device_status_pic": pic_bits,
        "fixed_error_macro_dt_over_dt": best["macro_dt_over_dt"] if best else None,
        "sweep": rows,
    })
    return out


def cfg1_leg(args, np, torch, synth, E):
    """Plain PIC of the small wave: L = 128, 128 cells, 200 ions per cell (25,600
    ions), 1000 steps, the cell sort every sort_period steps (autotuned)."""
    from paper_1610_01071_amd import autotune
    sp = E.ReplicaSpec(128, 128.0, ppc=200, haar_levels=3, dt=0.1, vth=math.sqrt(0.1))
    ctx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=8, tile=1024,
                                 flags=E.FLAG_SORT_BUFFER))
    c0 = initial_coarse(E, ctx, sp, synth, torch)
    period, table = autotune.sort_period(sp, c0, synth.lift_shift(1), periods=(50, 200, 0),
                                         steps=1000, tile=1024)

    def run():
        E.efpi_lift(ctx.ctx, c0, [synth.lift_shift(2)])
        done = 0
        while done < 1000:
            k = 1000 - done if period == 0 else min(period, 1000 - done)
            E.efpi_pic_burst(ctx.ctx, k, False)
            done += k
            if done < 1000:
                E.efpi_sort(ctx.ctx)

    run()
    ms = timed(torch, run)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    ctx.close()
    return {"n_ions": 25_600, "steps": 1000, "ms": ms, "us_per_step": ms,
            "particle_updates_per_s": 25_600 * 1000 / (ms * 1e-3), "sort_period": period,
            "sort_period_table": table, "device_status": bits,
            "note": "launch-latency bound: 25,600 ions fill 7 workgroups"}


def _progress(name, t0):
    """One line on stderr per finished leg (the JSON line stays alone on stdout)."""
    print(f"[bench] {name} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)


def run_bench(args, np, torch, synth, E):
    t0 = time.perf_counter()
    out = headline(args, np, torch, synth, E)
    _progress("headline", t0)
    if args.headline_only:
        return out
    from paper_1610_01071_amd import autotune
    spec = workload_spec(E)
    if args.sort_period <= 0:
        # sort period of the full-PIC references, tuned on the benchmark wave
        tctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4, tile=TILE))
        tc0 = initial_coarse(E, tctx, spec, synth, torch)
        tctx.close()
        args.sort_period, table = autotune.sort_period(spec, tc0, synth.lift_shift(3),
                                                       periods=(25, 50, 100, 200, 400),
                                                       steps=400)
        out["pic_sort_period_table"] = table
    out["pic_sort_period"] = args.sort_period
    iaw, c0 = iaw_leg(args, np, torch, synth, E)
    for key in ("efpi_speedup_vs_pic", "efpi_speedup_vs_pic_tuned_burst",
                "efpi_adaptive_speedup_vs_pic", "efpi_adaptive_speedup_vs_pic_short_burst"):
        if key in iaw:
            out[key] = iaw.pop(key)
    out["iaw4096"] = iaw
    _progress("iaw4096", t0)
    out["plain_pic_128"] = cfg1_leg(args, np, torch, synth, E)
    _progress("plain_pic_128", t0)
    if not args.no_efree:
        out["efree_iaw4096"] = efree_leg(E, torch, np, synth, args)
        _progress("efree_iaw4096", t0)
    if not args.no_phase:
        out["phase_space"] = phase_leg(E, torch, np, synth, c0, args)
        out["phase_space_nv2048"] = phase_leg(E, torch, np, synth, c0, args, jf=11, jc=6)
        out["phase_space_nv2048_ne6"] = phase_leg(E, torch, np, synth, c0, args, jf=11, jc=6,
                                                  burst=6)
        if not args.no_kinetic:
            out["phase_space_kinetic"] = phase_leg(E, torch, np, synth, c0, args, kinetic=True)
            out["phase_space_kinetic_nv2048"] = phase_leg(E, torch, np, synth, c0, args,
                                                          kinetic=True, jf=11, jc=6)
        _progress("phase_space", t0)
    if not args.no_kinetic:
        out["kinetic"] = kinetic_leg(E, torch, np, synth, c0, args)
        _progress("kinetic", t0)
    if not args.no_slab:
        out["slab"] = slab_leg(E, torch, np, synth, args)
        if not args.no_efree:
            out["slab_efree"] = slab_leg(E, torch, np, synth, args, pressure=True)
        out["slab_t2000"] = slab_leg(E, torch, np, synth, args, horizon=2000.0)
        _progress("slab", t0)
    if not args.no_learned:
        out["learned_vs_plain"] = learned_leg(E, torch, np, synth, args)
        if not args.no_kinetic:
            out["learned_kinetic"] = learned_leg(E, torch, np, synth, args, kinetic=True)
        if not args.no_slab:
            out["learned_slab"] = learned_slab_leg(E, torch, np, synth, args)
        _progress("learned", t0)
    return out


def initial_coarse(E, ctx, spec, synth, torch):
    """Quiet start of eq. 4.1, converged field, plain restriction: the coarse state at t = 0."""
    n0, u0 = synth.iaw_profile(spec.n_cells, spec.length)
    dn = torch.as_tensor(n0, dtype=torch.float64, device="cuda")
    du = torch.as_tensor(u0, dtype=torch.float64, device="cuda")
    E.efpi_load_profile(ctx.ctx, 0, dn, du, synth.lift_shift(2016))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 30, cold=True)
    c0 = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c0)
    E.efpi_sync(ctx.ctx)
    return c0


def speedup_sweep(E, torch, np, synth, ctx, spec, c0, args):
    """EFPI against full PIC over the same physical time from the same lifted state.

    Full PIC: the plain leapfrog burst with a cell sort every `sort_period` steps.
    EFPI: chained macro steps with Delta t in {50, 75, 100, 200} dt (K = 20).  The
    fixed-error point is the largest Delta t whose coarse density stays within
    eps_max of full PIC (eq. 4.2) at the horizon.
    """
    n_ions = spec.n_cells * spec.ppc
    fine = int(round(args.horizon / spec.dt))
    shift0 = synth.lift_shift(20_000)

    pctx = pic_context(E, spec, 2, 4)

    def pic_run(shift=shift0):
        E.efpi_lift(pctx.ctx, c0, [shift])
        done = 0
        while done < fine:
            k = min(args.sort_period, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    c_pic = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, c_pic)
    pic_bits = E.efpi_sync(pctx.ctx, raise_on_error=False)
    ref = c_pic.view(2, -1)[0].cpu().numpy()
    # the noise floor: full PIC from another quiet-start rotation of the same state
    pic_run(synth.lift_shift(20_999))
    E.efpi_restrict_state(pctx.ctx, c_pic)
    pic_bits_other = E.efpi_sync(pctx.ctx, raise_on_error=False)
    ref_other = c_pic.view(2, -1)[0].cpu().numpy()
    pctx.close()

    def pert_eps(a, b):
        # eq. 4.2 on the perturbations about their means: the wave itself
        da, db = a - a.mean(), b - b.mean()
        return float(np.sqrt(np.sum((da - db) ** 2) / np.sum(da * da + db * db)))

    rows = []
    for mult in (50, 75, 100, 200):
        sp = workload_spec(E)
        sp.macro_dt = mult * spec.dt
        cx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=4, tile=TILE))
        m = int(round(args.horizon / sp.macro_dt))
        a, b = cx.new_coarse(), cx.new_coarse()
        a.copy_(c0)
        state = {"a": a, "b": b}

        def efpi_run():
            for i in range(m):
                sh = shift0 if i == 0 else synth.lift_shift(20_000 + i)
                E.efpi_macro_step(cx.ctx, state["a"], state["b"], [sh])
                state["a"], state["b"] = state["b"], state["a"]

        t_efpi = timed(torch, efpi_run)
        bits = E.efpi_sync(cx.ctx, raise_on_error=False)
        got = state["a"].view(2, -1)[0].cpu().numpy()
        eps = float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(got * got + ref * ref)))
        rows.append({"macro_dt_over_dt": mult, "macro_steps": m, "efpi_ms": t_efpi,
                     "speedup": t_pic / t_efpi, "eps_density": eps,
                     "eps_density_perturbation": pert_eps(got, ref), "device_status": bits})
        cx.close()
    # a speedup is reported only against a clean reference and for clean EFPI runs
    ok = [r for r in rows if r["eps_density"] <= args.eps_max and r["device_status"] == 0]
    best = max(ok, key=lambda r: r["macro_dt_over_dt"]) if ok and pic_bits == 0 else None
    # the burst length N_e, which the paper tunes by the error it gives (Sec. 4.1): the
    # same runs with fewer fine steps per macro step, against the same reference
    ne_rows = []
    for ne in (2, 4, 6, 10, 14):
        for mult in (50, 75):
            sp = workload_spec(E)
            sp.burst_steps = ne
            sp.macro_dt = mult * spec.dt
            cx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=4, tile=TILE))
            m = int(round(args.horizon / sp.macro_dt))
            a, b = cx.new_coarse(), cx.new_coarse()
            a.copy_(c0)
            state = {"a": a, "b": b}

            def efpi_run():
                for i in range(m):
                    sh = shift0 if i == 0 else synth.lift_shift(20_000 + i)
                    E.efpi_macro_step(cx.ctx, state["a"], state["b"], [sh])
                    state["a"], state["b"] = state["b"], state["a"]

            t_efpi = timed(torch, efpi_run)
            bits = E.efpi_sync(cx.ctx, raise_on_error=False)
            got = state["a"].view(2, -1)[0].cpu().numpy()
            eps = float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(got * got + ref * ref)))
            ne_rows.append({"burst_steps": ne, "macro_dt_over_dt": mult, "macro_steps": m,
                            "efpi_ms": t_efpi, "speedup": t_pic / t_efpi, "eps_density": eps,
                            "eps_density_perturbation": pert_eps(got, ref),
                            "device_status": bits})
            cx.close()
    ok_ne = [r for r in ne_rows if r["eps_density"] <= args.eps_max and r["device_status"] == 0]
    best_ne = max(ok_ne, key=lambda r: r["speedup"]) if ok_ne and pic_bits == 0 else None
    extra = {}
    if not args.no_adaptive:
        pv = projective_leg(E, torch, np, synth, spec, c0, ref, t_pic, shift0, args)
        extra["efpi_adaptive_speedup_vs_pic"] = pv["adaptive_best_speedup"]
        extra["efpi_adaptive_speedup_vs_pic_short_burst"] = pv["adaptive_short_burst_best_speedup"]
        extra["projective_vs_pic"] = pv
    return {
        **extra,
        "efpi_speedup_vs_pic": best["speedup"] if best else None,
        "efpi_speedup_vs_pic_tuned_burst": best_ne["speedup"] if best_ne else None,
        "efpi_vs_pic": {
            "horizon": args.horizon,
            "eps_max": args.eps_max,
            "pic_fine_steps": fine,
            "pic_ms": t_pic,
            "pic_particle_updates_per_s": n_ions * fine / (t_pic * 1e-3),
            "pic_sort_period": args.sort_period,
            "device_status_pic": pic_bits,
            "pic_other_rotation_eps_density": float(np.sqrt(
                np.sum((ref_other - ref) ** 2) / np.sum(ref_other ** 2 + ref ** 2))),
            "pic_other_rotation_eps_density_perturbation": pert_eps(ref_other, ref),
            "device_status_pic_other_rotation": pic_bits_other,
            "fixed_error_macro_dt_over_dt": best["macro_dt_over_dt"] if best else None,
            "sweep": rows,
            "burst_length_sweep": ne_rows,
            "best_speedup_over_burst_lengths": best_ne["speedup"] if best_ne else None,
            "best_burst_length": ({k: best_ne[k] for k in ("burst_steps", "macro_dt_over_dt",
                                                           "eps_density")}
                                  if best_ne else None),
        },
    }


def projective_leg(E, torch, np, synth, spec, c0, ref, t_pic, shift0, args):
    """Forward-Euler, second-order and adaptive projective runs against the same
    full-PIC reference as the fixed-step sweep (same start and horizon).  Every
    setting runs with three sequences of lift rotations (the first lift is the
    reference's own); a row reports the largest eps (eq. 4.2, coarse density, at
    the horizon) and the mean wall time over them.  Each run goes through
    set_macro_dt / lift / restricting burst / restrict / project2 with the
    Euler-vs-second-order density difference read back every step (the adaptive
    controller's error estimate), so its wall time includes one host round trip
    per macro step that the fused chains above do not pay."""
    from paper_1610_01071_amd.projective import run_projective

    bases = (20_000, 30_000, 40_000)
    runs = [dict(order=1, macro_dt_over_dt=m) for m in (75, 100, 150, 200)]
    runs += [dict(order=2, macro_dt_over_dt=m) for m in (25, 50, 75, 100)]
    runs += [dict(order=o, tol=tol, dt_min_over_dt=50, dt_max_over_dt=400, macro_dt_over_dt=75)
             for o in (1, 2) for tol in (3e-4, 1e-3, 3e-3)]
    # adaptive Euler with the short bursts the fixed-step sweep finds as accurate
    runs += [dict(order=1, tol=tol, dt_min_over_dt=50, dt_max_over_dt=400, macro_dt_over_dt=75,
                  burst_steps=ne) for ne in (2, 6) for tol in (3e-4, 1e-3)]
    rows = []
    for r in runs:
        sp = workload_spec(E)
        sp.burst_steps = r.get("burst_steps", sp.burst_steps)
        sp.macro_dt = r["macro_dt_over_dt"] * spec.dt
        kw = {}
        if "tol" in r:
            kw = dict(tol=r["tol"], dt_min=r["dt_min_over_dt"] * spec.dt,
                      dt_max=r["dt_max_over_dt"] * spec.dt)
        eps_all, ms_all, steps_all, bits_all, first = [], [], [], 0, None
        for base in bases:
            cx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=4, tile=TILE))
            box = {}

            def go():
                box["run"] = run_projective(
                    cx, c0, args.horizon, sp.macro_dt, 0, order=r["order"],
                    shift_of=lambda i: shift0 if i == 0 else synth.lift_shift(base + i), **kw)

            ms_all.append(timed(torch, go))
            bits_all |= E.efpi_sync(cx.ctx, raise_on_error=False)
            run = box["run"]
            got = run.states[-1].view(2, -1)[0].cpu().numpy()
            eps_all.append(float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(got * got + ref * ref))))
            steps_all.append(len(run.steps))
            first = first or run
            cx.close()
        ms = float(np.mean(ms_all))
        row = dict(r, macro_steps=steps_all, efpi_ms=ms, speedup=t_pic / ms,
                   eps_density=max(eps_all), eps_density_per_rotation=eps_all,
                   device_status=bits_all)
        if "tol" in r:
            row["steps_over_dt_first_rotation"] = [round(x / spec.dt, 2) for x in first.steps]
        rows.append(row)

    def best(sel):
        ok = [x for x in rows
              if sel(x) and x["eps_density"] <= args.eps_max and x["device_status"] == 0]
        return max(ok, key=lambda x: x["speedup"]) if ok else None

    b1 = best(lambda x: x["order"] == 1 and "tol" not in x)
    b2 = best(lambda x: x["order"] == 2 and "tol" not in x)
    ba = best(lambda x: "tol" in x and "burst_steps" not in x)
    bs = best(lambda x: "tol" in x and "burst_steps" in x)
    return {
        "eps_max": args.eps_max,
        "euler_best_speedup": b1["speedup"] if b1 else None,
        "second_order_best_speedup": b2["speedup"] if b2 else None,
        "second_order_best_macro_dt_over_dt": b2["macro_dt_over_dt"] if b2 else None,
        "adaptive_best_speedup": ba["speedup"] if ba else None,
        "adaptive_best": ({k: ba[k] for k in ("order", "tol", "macro_steps", "eps_density")}
                          if ba else None),
        "adaptive_short_burst_best_speedup": bs["speedup"] if bs else None,
        "adaptive_short_burst_best": ({k: bs[k] for k in ("burst_steps", "tol", "macro_steps",
                                                          "eps_density")} if bs else None),
        "runs": rows,
    }


def kinetic_spec(E, macro_dt=7.5, burst=60):
    """The benchmark IAW with kinetic electrons: m_i / m_e = 1836, T_e = 1 (thermal
    speed sqrt(1836)), 1000 electrons per cell, dt = 0.25 / omega_pe."""
    mu = 1836.0
    return E.ReplicaSpec(n_cells=4096, length=4096.0, ppc=1000, haar_levels=4, burst_steps=burst,
                         macro_dt=macro_dt, dt=0.25 / math.sqrt(mu), vth=math.sqrt(0.1),
                         coevolving=1, lift_linear=1, closure=E.CLOSURE_KINETIC, qm_e=-mu,
                         vth_e=math.sqrt(mu), ppc_e=1000)


def kinetic_leg(E, torch, np, synth, c0, args):
    """The ion-acoustic wave with kinetic electrons (the two-species fine solver
    of Sec. 2 and 4.1): 4,096,000 ions and 4,096,000 electrons, linear Poisson.
    Full PIC (both species sorted by cell every 200 steps: at dt = 0.25 / omega_pe a
    thermal electron crosses a quarter cell per step, and an unsorted electron store
    spreads every workgroup's deposit over the whole grid) over the horizon from the lifted start
    (ions and Boltzmann electrons) against EFPI macro steps of N_e = 60 fine
    steps and Delta t in {2, 4, 5, 7.5, 10}, eps (eq. 4.2) on the coarse ion density,
    against full PIC and against the control run that resets the electrons to the
    Boltzmann equilibrium of the ions every 150 steps (Sec. 4.1)."""
    sp = kinetic_spec(E)
    n_ions = sp.n_cells * sp.ppc
    n_el = sp.n_cells * sp.ppc_e
    fine = int(round(args.kinetic_horizon / sp.dt))
    shift0 = synth.lift_shift(30_000)
    pctx = E.Context(E.ConfigSpec([sp], newton_iters=2, newton_iters_start=8, tile=PIC_TILE,
                                  flags=E.FLAG_SORT_BUFFER))

    def pic_run():
        E.efpi_lift(pctx.ctx, c0, [shift0])
        done = 0
        while done < fine:
            k = min(200, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    c_pic = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, c_pic)
    pic_bits = E.efpi_sync(pctx.ctx, raise_on_error=False)
    ref = c_pic.view(2, -1)[0].cpu().numpy()

    # live roofline of the electron pass: 200 further steps with every ion and
    # electron launch bracketed by events (outside the timed comparison above)
    E.efpi_sort(pctx.ctx)
    E.efpi_timing(pctx.ctx, True)
    E.efpi_pic_burst(pctx.ctx, 200, False)
    el_ms, el_n = E.efpi_timing_read_electrons(pctx.ctx)
    io_ms, io_n = E.efpi_timing_read(pctx.ctx)
    E.efpi_timing(pctx.ctx, False)
    el_us = el_ms * 1e3 / max(el_n, 1)
    el_bytes = BYTES_PER_UPDATE * n_el
    el_roofline = {"bound": "hbm", "kernel": "k_electrons (push + deposit)",
                   "achieved": el_bytes / (el_us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": el_bytes / (el_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                   "bytes_per_launch": el_bytes, "avg_launch_us": el_us, "launches": el_n,
                   "ion_pass_avg_launch_us": io_ms * 1e3 / max(io_n, 1)}

    # the control run of Sec. 4.1: full PIC with the electrons reset to the
    # Boltzmann equilibrium of the ions every 150 steps (the reset loads them in
    # cell order); both species are sorted every 600 steps, as the ions drift out
    # of their work items' field windows over thousands of steps
    def reset_run():
        E.efpi_lift(pctx.ctx, c0, [shift0])
        done, k = 0, 0
        while done < fine:
            n = min(150, fine - done)
            E.efpi_pic_burst(pctx.ctx, n, False)
            done += n
            k += 1
            if done < fine:
                if k % 4 == 0:
                    E.efpi_sort(pctx.ctx)
                E.efpi_reset_electrons(pctx.ctx, [synth.lift_shift(31_000 + k)])

    t_reset = timed(torch, reset_run)
    E.efpi_restrict_state(pctx.ctx, c_pic)
    reset_bits = E.efpi_sync(pctx.ctx, raise_on_error=False)
    pctx.close()
    ref_reset = c_pic.view(2, -1)[0].cpu().numpy()

    def eps_of(a, b):
        return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(a * a + b * b)))

    rows = []
    for macro_dt in (2.0, 4.0, 5.0, 7.5, 10.0):
        spm = kinetic_spec(E, macro_dt=macro_dt)
        cx = E.Context(E.ConfigSpec([spm], newton_iters=2, newton_iters_start=8, tile=TILE))
        m = int(round(args.kinetic_horizon / macro_dt))
        a, b = cx.new_coarse(), cx.new_coarse()
        a.copy_(c0)
        state = {"a": a, "b": b}

        def efpi_run():
            for i in range(m):
                sh = shift0 if i == 0 else synth.lift_shift(30_000 + i)
                E.efpi_macro_step(cx.ctx, state["a"], state["b"], [sh])
                state["a"], state["b"] = state["b"], state["a"]

        t_efpi = timed(torch, efpi_run)
        bits = E.efpi_sync(cx.ctx, raise_on_error=False)
        got = state["a"].view(2, -1)[0].cpu().numpy()
        rows.append({"macro_dt": macro_dt, "macro_dt_over_dt": round(macro_dt / sp.dt, 1),
                     "macro_steps": m, "time": m * macro_dt, "efpi_ms": t_efpi,
                     "speedup": t_pic / t_efpi, "eps_density": eps_of(got, ref),
                     "eps_density_vs_reset_pic": eps_of(got, ref_reset), "device_status": bits})
        cx.close()
    # adaptive projective steps (forward Euler, step from the Euler / second-order
    # gap) on the same workload
    from paper_1610_01071_amd.projective import run_projective
    adaptive = []
    for tol in (3e-4, 1e-3):
        cx = E.Context(E.ConfigSpec([kinetic_spec(E, macro_dt=5.0)], newton_iters=2,
                                    newton_iters_start=8, tile=TILE))
        box = {}

        def go():
            box["run"] = run_projective(
                cx, c0, args.kinetic_horizon, 5.0, 0, order=1, tol=tol, dt_min=2.0, dt_max=20.0,
                shift_of=lambda i: shift0 if i == 0 else synth.lift_shift(30_000 + i))

        t_ad = timed(torch, go)
        bits = E.efpi_sync(cx.ctx, raise_on_error=False)
        run = box["run"]
        got = run.states[-1].view(2, -1)[0].cpu().numpy()
        adaptive.append({"tol": tol, "macro_steps": len(run.steps),
                         "macro_dt_range": [min(run.steps), max(run.steps)], "efpi_ms": t_ad,
                         "speedup": t_pic / t_ad, "eps_density": eps_of(got, ref),
                         "eps_density_vs_reset_pic": eps_of(got, ref_reset),
                         "device_status": bits})
        cx.close()
    ok = [r for r in rows if r["eps_density"] <= args.eps_max]
    best = max(ok, key=lambda r: r["speedup"]) if ok else None
    ok_ad = [r for r in adaptive if r["eps_density"] <= args.eps_max]
    best_ad = max(ok_ad, key=lambda r: r["speedup"]) if ok_ad else None
    return {
        "efpi_adaptive_speedup_vs_pic": best_ad["speedup"] if best_ad else None,
        "adaptive": adaptive,
        "ions": n_ions, "electrons": n_el, "mass_ratio": -sp.qm_e, "dt": sp.dt,
        "burst_steps": sp.burst_steps, "horizon": args.kinetic_horizon, "pic_fine_steps": fine,
        "pic_ms": t_pic, "pic_ms_per_step": t_pic / fine,
        "pic_particle_updates_per_s": (n_ions + n_el) * fine / (t_pic * 1e-3),
        "pic_device_status": pic_bits,
        "roofline_electrons": el_roofline,
        "reset_pic_ms": t_reset, "reset_pic_device_status": reset_bits,
        "eps_density_reset_pic_vs_pic": eps_of(ref_reset, ref),
        "efpi_speedup_vs_pic": best["speedup"] if best else None,
        "sweep": rows,
    }


def phase_leg(E, torch, np, synth, c0, args, kinetic=False, jf=8, jc=5, burst=20):
    """Projective integration on phase-space coarse variables (Sec. 3.3): the
    benchmark wave, 4096 cells and 1000 ions per cell, l = 4 full-weighting levels
    (256 coarse x nodes), 2^jf velocity bins over [-2, 2) reduced to 2^jc order-4
    Coiflet scaling coefficients per node (2^8 -> 2^5: 8192 coarse variables; the
    paper's IAW runs use 2^11 -> 2^6), N_e = `burst` (20; the paper's IAW runs use 6),
    Delta t = 75 dt, 27 macro steps to t = 202.5.  The start is the phase-space
    restriction of the lifted benchmark state; full PIC runs from that lifted
    state.  The error compares the coarse density of the final state (its ions
    restricted onto the Haar blocks of the benchmark) with full PIC's (eq. 4.2).
    Also timed: one phase-space restriction of the 4,096,000 ions (histogram,
    transform) and one phase-space lift."""
    from paper_1610_01071_amd.phase import PhaseStepper, coiflet_taps
    steps = 27
    if kinetic:
        spec = kinetic_spec(E, macro_dt=7.5)
        mult = spec.macro_dt / spec.dt
        start_iters, sort_period = 8, 200
    else:
        mult = 75
        spec = workload_spec(E)
        spec.burst_steps = burst
        spec.macro_dt = mult * spec.dt
        start_iters, sort_period = 4, args.sort_period
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=start_iters,
                                 tile=TILE))
    taps = coiflet_taps()
    ph = E.phase(-2.0, 2.0, jf, jc, 4, taps)
    st = PhaseStepper(ctx, ph)
    shift0 = synth.lift_shift(40_000)
    E.efpi_lift(ctx.ctx, c0, [shift0])
    a, b = st.new_coarse(), st.new_coarse()
    st.restrict(a)
    # restriction and lift timings
    reps = 20
    t_r = timed(torch, lambda: [st.restrict(b) for _ in range(reps)]) / reps
    t_l = timed(torch, lambda: E.efpi_phase_lift(ctx.ctx, 0, ph, a, 5, st.lift_work))
    E.efpi_lift(ctx.ctx, c0, [shift0])
    st.restrict(a)
    n_ions = spec.n_cells * spec.ppc
    state = {"a": a, "b": b}

    def run():
        for i in range(steps):
            st.macro_step(state["a"], state["b"], synth.lift_shift(40_000 + i))
            state["a"], state["b"] = state["b"], state["a"]

    t_run = timed(torch, run)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    # density of the final state through a lift and the Haar restriction
    E.efpi_phase_lift(ctx.ctx, 0, ph, state["a"], 99, st.lift_work)
    cfin = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, cfin)
    got = cfin.view(2, -1)[0].cpu().numpy()

    fine = int(round(steps * mult))
    pctx = pic_context(E, spec, 2, start_iters)

    def pic_run():
        E.efpi_lift(pctx.ctx, c0, [shift0])
        done = 0
        while done < fine:
            k = min(sort_period, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    cp = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, cp)
    E.efpi_sync(pctx.ctx, raise_on_error=False)
    pctx.close()
    ctx.close()
    ref = cp.view(2, -1)[0].cpu().numpy()
    eps = float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(got * got + ref * ref)))
    dg, dr = got - got.mean(), ref - ref.mean()
    eps_wave = float(np.sqrt(np.sum((dg - dr) ** 2) / np.sum(dg * dg + dr * dr)))
    return {
        "workload": "ion-acoustic wave, kinetic electrons" if kinetic else
                    "ion-acoustic wave, Boltzmann electrons",
        "coarse_variables": st.n_coef, "velocity_bins": 1 << jf,
        "scaling_coefficients_per_node": 1 << jc,
        "x_levels": 4, "burst_steps": spec.burst_steps, "macro_dt_over_dt": mult,
        "macro_steps": steps,
        "ms_per_macro_step": t_run / steps, "efpi_ms": t_run, "pic_ms": t_pic,
        "speedup_vs_pic": t_pic / t_run, "eps_density_vs_pic": eps,
        "eps_density_perturbation_vs_pic": eps_wave,
        "restrict_us": t_r * 1e3, "restrict_ion_gbs": 14 * n_ions / (t_r * 1e-3) / 1e9,
        "lift_ms": t_l, "device_status": bits,
    }


def slab_leg(E, torch, np, synth, args, pressure=False, horizon=200.0):
    """Plasma slab expanding into vacuum (the setting of Sec. 4.2): 16384 cells,
    absorbing walls, n = 1 on the central quarter, 4096 ions per occupied cell
    (about 16.8 M ions), T_i/T_e = 0.01, l = 4 (1024 coarse points per moment),
    N_e = 20.  Full PIC (cell sort every sort_period steps) against EFPI with
    Delta t in {25, 50} dt over t = `horizon` (200, and the workload's stated 2000:
    20,000 fine steps) from the same lifted state; eps (eq. 4.2)
    on the coarse density.  The fixed-error point is the largest Delta t within
    eps_max; no speedup is reported when a run raised a device status bit.  With
    `pressure` the coarse state carries the EFREE variables (three moments, Sec. 3.2)."""
    n_cells, ppc = 16384, 4096
    nm = 3 if pressure else 2
    extra = E.FLAG_PRESSURE if pressure else 0

    def make(mult):
        sp = E.ReplicaSpec(n_cells, float(n_cells), bc=E.BC_WALLS, ppc=ppc, haar_levels=4,
                           burst_steps=20, macro_dt=mult * 0.1, dt=0.1, vth=0.1)
        return sp, E.Context(E.ConfigSpec([sp], newton_iters=3, newton_iters_start=6, tile=TILE,
                                          flags=E.FLAG_SORT_BUFFER | extra))

    spec, ctx = make(50)
    n0, u0 = synth.slab_profile(n_cells)
    E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(n0, device="cuda"),
                        torch.as_tensor(u0, device="cuda"), synth.lift_shift(2016))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 60, cold=True)
    c0 = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c0)
    n_ions = ctx.particles()[0].numel()
    ctx.close()
    fine = int(round(horizon / spec.dt))
    shift0 = synth.lift_shift(40_000)

    pctx = E.Context(E.ConfigSpec([spec], newton_iters=3, newton_iters_start=6, tile=PIC_TILE,
                                  flags=E.FLAG_SORT_BUFFER | extra))

    def pic_run():
        E.efpi_lift(pctx.ctx, c0, [shift0])
        done = 0
        while done < fine:
            k = min(args.sort_period, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    cp = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, cp)
    pic_bits = E.efpi_sync(pctx.ctx, raise_on_error=False)
    pctx.close()
    ref_both = cp.view(nm, -1).cpu().numpy()

    def eps(u, w):
        return float(np.sqrt(np.sum((u - w) ** 2) / np.sum(u * u + w * w)))

    rows = []
    for mult in (25, 50):
        sp, cx = make(mult)
        steps = int(round(horizon / sp.macro_dt))
        a, b = cx.new_coarse(), cx.new_coarse()
        a.copy_(c0)
        st = {"a": a, "b": b}

        def efpi_run():
            for i in range(steps):
                sh = shift0 if i == 0 else synth.lift_shift(40_000 + i)
                E.efpi_macro_step(cx.ctx, st["a"], st["b"], [sh])
                st["a"], st["b"] = st["b"], st["a"]

        t_efpi = timed(torch, efpi_run)
        bits = E.efpi_sync(cx.ctx, raise_on_error=False)
        got = st["a"].view(nm, -1).cpu().numpy()
        rows.append({"macro_dt_over_dt": mult, "macro_steps": steps, "efpi_ms": t_efpi,
                     "efpi_ms_per_macro_step": t_efpi / steps, "speedup": t_pic / t_efpi,
                     "eps_density": eps(got[0], ref_both[0]),
                     "eps_momentum": eps(got[1], ref_both[1]), "device_status": bits})
        if pressure:
            rows[-1]["eps_second_moment"] = eps(got[2], ref_both[2])
        cx.close()
    ok = [r for r in rows if r["eps_density"] <= args.eps_max and r["device_status"] == 0]
    best = max(ok, key=lambda r: r["macro_dt_over_dt"]) if ok and pic_bits == 0 else None
    return {
        "n_cells": n_cells, "ppc": ppc, "n_ions_t0": n_ions, "horizon": horizon,
        "pic_fine_steps": fine, "pic_ms": t_pic, "pic_sort_period": args.sort_period,
        "pic_particle_updates_per_s": n_ions * fine / (t_pic * 1e-3),
        "device_status_pic": pic_bits, "eps_max": args.eps_max,
        "speedup": best["speedup"] if best else None,
        "fixed_error_macro_dt_over_dt": best["macro_dt_over_dt"] if best else None,
        "sweep": rows,
    }


def learned_slab_leg(E, torch, np, synth, args):
    """Learned projection driving the expanding slab (16384 cells, walls, 4096 ions per
    occupied cell, l = 4, Delta t = 50 dt, 40 macro steps to t = 200).

    Cells are lifted where a node density exceeds 1e-3 (for plain and learned runs
    alike).  Training data: plain EFPI trajectories of slabs of 12 other widths (0.18 .. 0.32 of
    the domain); 10,000 Adam steps of batch 16 with input-state noise of one increment
    scale, so that chained learned steps stay on the trajectory.  Test: width 0.25,
    plain EFPI against the learned run with a fine burst every 2nd (and every 4th) step
    as judge and fallback (accumulated-error bound 2e-3 on the coarse density and on
    the momentum, eq. 4.2).
    """
    import paper_1610_01071_amd.learned as L
    n_cells, steps = 16384, 40
    # n_floor 1e-3: a lifted cell needs a node density of 1e-3 (of the bulk's 1); below
    # it, the mean velocity j / n of a learned state's noise-level density and
    # momentum at the plasma edge would launch ions at arbitrary speeds
    spec = E.ReplicaSpec(n_cells, float(n_cells), bc=E.BC_WALLS, ppc=4096, haar_levels=4,
                         burst_steps=20, macro_dt=5.0, dt=0.1, vth=0.1, n_floor=1e-3)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=3, newton_iters_start=6, tile=TILE))

    def c0_for(width, seed):
        n0, u0 = synth.slab_profile(n_cells, width)
        E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(n0, device="cuda"),
                            torch.as_tensor(u0, device="cuda"), synth.lift_shift(seed))
        E.efpi_deposit(ctx.ctx)
        E.efpi_solve_field(ctx.ctx, 60, cold=True)
        c = ctx.new_coarse()
        E.efpi_restrict_state(ctx.ctx, c)
        return c

    widths = [0.18, 0.2, 0.21, 0.22, 0.23, 0.24, 0.26, 0.27, 0.28, 0.29, 0.3, 0.32]
    t_gen = time.perf_counter()
    trajs = [L.plain_run(ctx, c0_for(w, 100 + k), steps, seed=500 + k)
             for k, w in enumerate(widths)]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    norm = L.fit_norm(trajs)
    states = torch.cat(trajs, 0).contiguous()
    T = steps + 1
    train_idx = np.concatenate([np.arange(2, T - 1) + r * T for r in range(len(trajs))])
    tr = L.Trainer(spec.n_coarse, False, batch=16)
    t_train = time.perf_counter()
    tr.train(states, train_idx, norm, 10_000, noise=1.0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train

    c0 = c0_for(0.25, 999)
    L.plain_run(ctx, c0, 3, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = L.plain_run(ctx, c0, steps, seed=77)
    torch.cuda.synchronize()
    wall_plain = (time.perf_counter() - t0) * 1e3
    b = ref[-1].cpu().numpy().reshape(2, -1)
    o = L.plain_run(ctx, c0, steps, seed=78)[-1].cpu().numpy().reshape(2, -1)

    def eps(u, w):
        return float(np.sqrt(np.sum((u - w) ** 2) / np.sum(u * u + w * w)))

    out = {"macro_dt_over_dt": 50, "macro_steps": steps, "threshold": 2e-3, "train_noise": 1.0,
           "plain_ms": wall_plain, "datagen_s": t_gen, "train_s": t_train, "train_iters": 10_000,
           "plain_spread_density": eps(o[0], b[0]), "plain_spread_momentum": eps(o[1], b[1])}
    for jp in (2, 4):
        run = L.run_learned(ctx, tr, norm, c0, steps, seed=77, judge_period=jp, threshold=2e-3)
        a = run.states[-1].cpu().numpy().reshape(2, -1)
        out[f"judge_period_{jp}"] = {
            "learned_ms": run.wall_ms, "speedup": wall_plain / run.wall_ms,
            "eps_density": eps(a[0], b[0]), "eps_momentum": eps(a[1], b[1]),
            "learned_steps": run.learned, "judged_steps": run.judged,
            "fallback_steps": run.fallback, "judge_eps_max": max(run.eps) if run.eps else None,
            "judge_eps_momentum_max": max(run.eps_momentum) if run.eps_momentum else None,
            "judge_bound_density": run.acc[-1] if run.acc else 0.0,
            "judge_bound_momentum": run.acc_momentum[-1] if run.acc_momentum else 0.0,
            "plain_from_step": run.fell_back_at}
    ctx.close()
    return out


def learned_leg(E, torch, np, synth, args, kinetic=False):
    """Learned projection against plain EFPI on the benchmark grid.

    With kinetic=True the same comparison runs on the kinetic-electron workload
    (kinetic_spec, Delta t = 7.5 = 1286 fine steps, 27 macro steps to t = 202.5),
    where every fine burst costs 60 two-species steps.

    Training data: plain EFPI trajectories (27 macro steps of Delta t = 75 dt,
    the largest stable step of the sweep, t = 202.5) of the ion-acoustic wave at
    six amplitudes other than 0.2; 2000 Adam steps of batch 32 on the GPU.  Test:
    delta = 0.2 from the benchmark's initial state, 27 macro steps, plain EFPI
    against the learned run (fine burst every 4th step as judge and fallback,
    accumulated-error bound 2e-3 on density and momentum, eq. 4.2), and both against full PIC
    over the same time from the same lifted start.
    """
    import paper_1610_01071_amd.learned as L
    if kinetic:
        spec = kinetic_spec(E, macro_dt=7.5)
        mult = spec.macro_dt / spec.dt
        sort_period = 200
        start_iters = 8
    else:
        mult = 75
        spec = workload_spec(E)
        spec.macro_dt = mult * spec.dt
        sort_period = args.sort_period
        start_iters = 4
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=start_iters, tile=TILE,
                                 flags=E.FLAG_SORT_BUFFER))
    steps = 27

    def c0_for(delta, seed):
        n0, u0 = synth.iaw_profile(spec.n_cells, spec.length, delta)
        E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(n0, device="cuda"),
                            torch.as_tensor(u0, device="cuda"), synth.lift_shift(seed))
        E.efpi_deposit(ctx.ctx)
        E.efpi_solve_field(ctx.ctx, 30, cold=True)
        c = ctx.new_coarse()
        E.efpi_restrict_state(ctx.ctx, c)
        return c

    t_gen = time.perf_counter()
    trajs = [L.plain_run(ctx, c0_for(d, 100 + k), steps, seed=500 + k)
             for k, d in enumerate([0.1, 0.15, 0.25, 0.3, 0.12, 0.28])]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    norm = L.fit_norm(trajs)
    states = torch.cat(trajs, 0).contiguous()
    T = steps + 1
    train_idx = np.concatenate([np.arange(2, T - 1) + r * T for r in range(len(trajs) - 1)])
    val_idx = np.arange(2, T - 1) + (len(trajs) - 1) * T
    tr = L.Trainer(spec.n_coarse, True, batch=32)
    t_train = time.perf_counter()
    tr.train(states, train_idx, norm, 2000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    val = tr.evaluate(states, val_idx, norm)

    c0 = c0_for(0.2, 2016)
    L.plain_run(ctx, c0, 4, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = L.plain_run(ctx, c0, steps, seed=77)
    torch.cuda.synchronize()
    wall_plain = (time.perf_counter() - t0) * 1e3
    run = L.run_learned(ctx, tr, norm, c0, steps, seed=77, judge_period=4, threshold=2e-3)
    other = L.plain_run(ctx, c0, steps, seed=78)
    a = run.states[-1].cpu().numpy().reshape(2, -1)
    b = ref[-1].cpu().numpy().reshape(2, -1)
    o = other[-1].cpu().numpy().reshape(2, -1)

    # full PIC over the same time from the same lifted start
    fine = int(round(steps * mult))

    pctx = pic_context(E, spec, 2, start_iters)

    def pic_run():
        E.efpi_lift(pctx.ctx, c0, [L.lift_shift(77, 0)])
        done = 0
        while done < fine:
            k = min(sort_period, fine - done)
            E.efpi_pic_burst(pctx.ctx, k, False)
            done += k
            if done < fine:
                E.efpi_sort(pctx.ctx)

    t_pic = timed(torch, pic_run)
    cp = pctx.new_coarse()
    E.efpi_restrict_state(pctx.ctx, cp)
    E.efpi_sync(pctx.ctx, raise_on_error=False)
    pctx.close()
    pc = cp.view(2, -1).cpu().numpy()

    def eps(u, w):
        return float(np.sqrt(np.sum((u - w) ** 2) / np.sum(u * u + w * w)))

    ctx.close()
    return {
        "workload": "ion-acoustic wave, kinetic electrons" if kinetic else
                    "ion-acoustic wave, Boltzmann electrons",
        "macro_dt_over_dt": mult, "macro_steps": steps, "judge_period": 4, "threshold": 2e-3,
        "plain_ms": wall_plain, "learned_ms": run.wall_ms, "speedup": wall_plain / run.wall_ms,
        "pic_ms": t_pic, "learned_speedup_vs_pic": t_pic / run.wall_ms,
        "plain_speedup_vs_pic": t_pic / wall_plain,
        "eps_density_learned_vs_pic": eps(a[0], pc[0]),
        "eps_density_plain_vs_pic": eps(b[0], pc[0]),
        "eps_density": eps(a[0], b[0]), "eps_momentum": eps(a[1], b[1]),
        "plain_spread_density": eps(o[0], b[0]), "plain_spread_momentum": eps(o[1], b[1]),
        "learned_steps": run.learned, "judged_steps": run.judged, "fallback_steps": run.fallback,
        "judge_eps_max": max(run.eps) if run.eps else None,
        "judge_eps_momentum_max": max(run.eps_momentum) if run.eps_momentum else None,
        "judge_bound_density": run.acc[-1] if run.acc else 0.0,
        "judge_bound_momentum": run.acc_momentum[-1] if run.acc_momentum else 0.0,
        "plain_from_step": run.fell_back_at,
        "datagen_s": t_gen, "train_s": t_train, "train_iters": 2000, "val_loss": val,
    }


if __name__ == "__main__":
    main()
