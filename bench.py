#!/usr/bin/env python3
"""Benchmark of the tempered + jittered SCH particle filter on one MI355X.

One step = one assimilation cycle of the whole hot path on the GPU: forecast
noise draw, forecast window (40 implicit-midpoint steps per particle),
likelihood, then adaptive tempering steps, each with ESS bisection, systematic
resampling, particle gathers and 5 pCN jitter moves (each a full rerun of the
window).  Workload: Nx = 4096 nodes, 1024 particles, 8 noise modes, 40 steps
per window, 256 observations (sigma 0.02), ESS threshold N/2, rho = 0.99;
synthetic twin-experiment data (truth from the same model with seed + 1).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 vector peak of MI355X (TFLOP/s) and HBM peak (GB/s).
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic floating-point operations per grid node:
# per implicit-solve iteration: dv (2) + rows of A (7) + tridiagonal
# factor-and-solve (9) + m* (1) + mass product (4) + Helmholtz solve with
# stored factors (5) + convergence test (3) = 31; per step: noise
# assembly (2 Q + 1) and the mass product of the right-hand side (4).
FLOPS_PER_NODE_ITER = 31
def flops_per_node_step(n_modes: int) -> int:
    return 2 * n_modes + 5


# The coarser per-node model of the step used for the headline roofline
# fraction: 60 flops per node per Picard iteration (about 25 for assembling
# the rows, 20 for the cyclic solve with one reciprocal per row, 11 for the
# Helmholtz solve, 2 for the test) and 20 per node per step outside it.
MODEL_FLOPS_PER_NODE_ITER = 60
MODEL_FLOPS_PER_NODE_STEP = 20


def host_cpu() -> dict:
    """The host's logical CPU count, the CPUs this process may use, and the
    CPU model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


# With the Matern-type noise the per-step noise assembly is the dv part (1),
# the load vector (2), k scan-form solves (5 each), k - 1 mass products (4
# each) and the sum into dv (1), plus the right-hand-side mass product (4);
# a pCN proposal adds 3 per cell.
def matern_flops_per_node_step(k: int, pcn: bool) -> int:
    return 1 + 2 + 5 * k + 4 * (k - 1) + 1 + 4 + (3 if pcn else 0)


# HBM traffic of one k_jitter launch at this workload from two rocprofv3
# counter runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors of a plain
# 1 GiB copy), valid for the kernel sources with the hash below.
TRAFFIC_JITTER_BYTES = (199964.40625 * 2.0 + 268370.109375 * 1.0) * 1024
# the same for the jitter kernel with the Matern-type noise (cells read and
# proposals written per step)
TRAFFIC_JITTER_MATERN_BYTES = (3907625.34375 * 2.0 + 7411383.984375 * 1.0) * 1024
TRAFFIC_THREADS = 256
# checkpoint interval of the adjoint passes of the pCN-Langevin jitter
PCNL_CKPT = 8
# Hybrid Monte Carlo jitter of the bench: leapfrog angle and steps per move
HMC_H = 0.5
HMC_LEAP = 3
TRAFFIC_SOURCES_HASH = "ee65545743aecf33"


def kernel_sources_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("device.hpp", "helm.hpp", "model.hpp"):
        with open(os.path.join(ROOT, "paper_2402_06927_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(wl, u_start, m_start, n_threads: int, psteps_per_cycle: float):
    """Oracle timed on the host: one forecast window of the whole ensemble
    (the same 1024 particles and 40 steps), scaled to cycles/s with the
    particle-steps per cycle measured on the GPU."""
    import oracle as O

    xi = __import__("paper_2402_06927_amd.workloads", fromlist=["x"]).mode_table(
        wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    om = O.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                 picard_tol=wl.picard_tol, picard_max=wl.picard_max)
    n = u_start.shape[0]
    if wl.noise == "matern":
        cells = O.draw_increments(wl.seed, n, wl.n_steps, wl.nx, 0, O.TAG_FORECAST, 0, wl.dt)
        mt = O.matern(wl.kappa, wl.eta, wl.k_solves)
        t0 = time.perf_counter()
        worst, _, _, _, _ = O.ensemble_window_matern(om, mt, m_start, u_start, cells,
                                                     n_threads=n_threads)
    else:
        dW = O.draw_increments(wl.seed, n, wl.n_steps, wl.n_modes, 0, O.TAG_FORECAST, 0, wl.dt)
        t0 = time.perf_counter()
        worst, _, _, _, _ = O.ensemble_window(om, m_start, u_start, dW, n_threads=n_threads)
    dt = time.perf_counter() - t0
    psteps = n * wl.n_steps
    ps_rate = psteps / dt
    # the plain single-threaded oracle on the first n1 particles of the same window
    n1 = min(n, 48)
    t0 = time.perf_counter()
    if wl.noise == "matern":
        O.ensemble_window_matern(om, mt, m_start[:n1], u_start[:n1], cells[:n1], n_threads=1)
    else:
        O.ensemble_window(om, m_start[:n1], u_start[:n1], dW[:n1], n_threads=1)
    dt1 = time.perf_counter() - t0
    ps1 = n1 * wl.n_steps / dt1
    return {
        "value": ps_rate / psteps_per_cycle,
        "unit": "cycles/s",
        "cores": n_threads,
        "kind": "oracle",
        "sample": (f"one forecast window of all {n} particles x {wl.n_steps} steps at Nx={wl.nx} "
                   f"on {n_threads} threads ({psteps} particle-steps, {dt:.1f} s, "
                   f"{ps_rate:.1f} particle-steps/s), scaled by the {psteps_per_cycle:.0f} "
                   f"particle-steps per cycle measured on the GPU; oracle status {worst}; "
                   f"single-threaded: {n1} particles of the same window, {dt1:.1f} s"),
        "particle_steps_per_s": ps_rate,
        "single_thread": {"value": ps1 / psteps_per_cycle, "unit": "cycles/s", "cores": 1,
                          "particle_steps_per_s": ps1},
        "host": host_cpu(),
    }


def copy_probe(nbytes: int):
    """A plain device-to-device copy of known size, for scaling the HBM
    traffic counters (FETCH_SIZE, WRITE_SIZE) of a profiled run."""
    import torch

    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "launches": 3}), flush=True)


def bench_nudging(args, matern=False):
    """One step = the sequential adapted nudging of one 40-step window for
    all 2048 particles at Nx = 2048 (8 modes, 256 observations, sigma 0.02,
    L-BFGS memory 8, checkpoints every 8 steps) plus the likelihood of the
    nudged ends.  matern: the Matern-type noise (eta = 1, k = 3, kappa = 1)
    with one control per cell, 2048 per step and particle."""
    import torch

    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    wl = W.NUDGING_MATERN_2048 if matern else W.NUDGING_2048
    if args.particles:
        wl = wl.scaled(n_particles=args.particles)
    dev = "cuda"
    n, nx, Q, S = wl.n_particles, wl.nx, wl.n_modes, wl.n_steps
    log(f"bench: {wl.name} n={n} nx={nx} Q={Q} S={S} windows={args.warmup}+{args.steps}")
    xi = torch.tensor(W.mode_table(wl.L, nx, Q, wl.mode_amp), device=dev)
    model = sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                      picard_tol=wl.picard_tol, picard_max=wl.picard_max)
    u_init = torch.tensor(W.initial_velocity(wl, n, wl.seed), device=dev)
    m_init = torch.empty_like(u_init)
    sch.sch_init_momentum(model, u_init, m_init)
    ts = W.truth_seed(wl)
    ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
    mt = torch.empty_like(ut)
    sch.sch_init_momentum(model, ut, mt)
    nq = nx if matern else Q  # controls per step
    mtn = sch.Matern(wl.kappa, wl.eta, wl.k_solves)
    dWt = torch.empty((1, S, nq), dtype=torch.float64, device=dev)
    sch.sch_draw_increments(ts, 0, 0, sch.TAG_FORECAST, dWt, wl.dt)
    if matern:
        sch.sch_ensemble_step_matern(model, mtn, mt, ut, dWt)
    else:
        sch.sch_ensemble_step(model, mt, ut, dWt)
    y = torch.empty((1, wl.n_obs), dtype=torch.float64, device=dev)
    sch.sch_observe(model, ut, y)
    y = y[0] + wl.sigma_obs * torch.tensor(W.obs_noise(wl, ts, 1)[0], device=dev)
    obs = sch.Obs(y.contiguous(), torch.full((wl.n_obs,), wl.sigma_obs, dtype=torch.float64,
                                             device=dev))
    dW = torch.empty((n, S, nq), dtype=torch.float64, device=dev)
    sch.sch_draw_increments(wl.seed, 0, 0, sch.TAG_NUDGE, dW, wl.dt)
    if matern:
        ws = sch.matern_workspace(sch.WS_NUDGE, model, n, S, 8)
    else:
        ws = sch.workspace(sch.WS_NUDGE, model, n, S, 8)
    dLam = torch.zeros_like(dW)
    logG = torch.empty(n, dtype=torch.float64, device=dev)
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    evals = torch.empty(n, dtype=torch.int32, device=dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)

    def run():
        m, u = m_init.clone(), u_init.clone()
        if matern:
            sch.sch_nudge_run_matern(model, mtn, obs, m, u, dW, dLam, logG, iters=iters,
                                     evals=evals, workspace=ws)
        else:
            sch.sch_nudge_run(model, obs, m, u, dW, dLam, logG, iters=iters, evals=evals,
                              workspace=ws)
        sch.sch_loglik(model, obs, u, phi)
        return u

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    sch.sch_timing_reset()
    sch.sch_timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sch.sch_timing_enable(False)
    tim = sch.sch_timing_read()
    ev = float(evals.double().mean())
    it = float(iters.double().mean())
    # step-equivalents per particle: each evaluation of stage s runs S - s
    # forward steps, recomputes them, and sweeps them backwards
    out = {
        "metric": "nudged windows/s (sequential adapted nudging, L-BFGS + adjoint)",
        "value": round(args.steps / elapsed, 4),
        "unit": "windows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "filter": "nudging", "nx": nx, "n_particles": n,
                   "n_modes": Q, "n_steps": S, "n_obs": wl.n_obs, "sigma_obs": wl.sigma_obs,
                   "lbfgs_mem": 8, "ckpt_every": 8, "noise": wl.noise,
                   "controls_per_step": nq},
        "lbfgs_evals_per_particle": round(ev, 2),
        "lbfgs_iters_per_particle": round(it, 2),
        "mean_phi_nudged": float(phi.mean()),
        "kernel_ms": {k: round(v["ms"], 3) for k, v in tim.items()},
        "nudge_launches": tim["nudge"]["launches"],
    }
    print(json.dumps(out), flush=True)


def bench_nudged(args, matern=False):
    """One step = one cycle of the nudged filter at the nudging workload
    (Nx = 2048, 2048 particles, 8 modes, 40 steps, 256 observations): the
    sequential adapted nudging of the window (L-BFGS on the adjoint gradient),
    then adaptive tempering on the weights exp(-dtheta J), J = phi - log G,
    with systematic resampling and 5 pCN moves of the increments per
    tempering step (controls fixed).  Observations of consecutive cycles come
    from one truth run."""
    import torch

    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    wl = W.NUDGING_MATERN_2048 if matern else W.NUDGING_2048
    if args.particles:
        wl = wl.scaled(n_particles=args.particles)
    dev = "cuda"
    n, nx, Q, S = wl.n_particles, wl.nx, wl.n_modes, wl.n_steps
    n_cycles = args.warmup + args.steps
    n_jitter, rho = 5, 0.99
    log(f"bench: nudged filter {wl.name} n={n} nx={nx} Q={Q} S={S} cycles={args.warmup}+{args.steps}")
    xi = torch.tensor(W.mode_table(wl.L, nx, Q, wl.mode_amp), device=dev)
    model = sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                      picard_tol=wl.picard_tol, picard_max=wl.picard_max)
    u = torch.tensor(W.initial_velocity(wl, n, wl.seed), device=dev)
    m = torch.empty_like(u)
    sch.sch_init_momentum(model, u, m)
    ts = W.truth_seed(wl)
    ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
    mt = torch.empty_like(ut)
    sch.sch_init_momentum(model, ut, mt)
    z = torch.tensor(W.obs_noise(wl, ts, n_cycles), device=dev)
    nq = nx if matern else Q  # increments and controls per step
    mtn = sch.Matern(wl.kappa, wl.eta, wl.k_solves)
    dWt = torch.empty((1, S, nq), dtype=torch.float64, device=dev)
    yobs = torch.empty((n_cycles, wl.n_obs), dtype=torch.float64, device=dev)
    for c in range(n_cycles):
        sch.sch_draw_increments(ts, c, 0, sch.TAG_FORECAST, dWt, wl.dt)
        if matern:
            sch.sch_ensemble_step_matern(model, mtn, mt, ut, dWt)
        else:
            sch.sch_ensemble_step(model, mt, ut, dWt)
        sch.sch_observe(model, ut, yobs[c:c + 1])
    yobs += wl.sigma_obs * z
    sigma = torch.full((wl.n_obs,), wl.sigma_obs, dtype=torch.float64, device=dev)
    dLam = torch.zeros((n, S, nq), dtype=torch.float64, device=dev)
    if matern:
        ws = sch.nudged_workspace_matern(model, n, S, n_jitter, 8)
    else:
        ws = sch.nudged_workspace(model, n, S, n_jitter, 8)
    # the tile of the window kernels, tuned as for the headline filter (the
    # adjoint takes its own from it); the Matern-noise kernels keep the
    # default, to which the noise operator's constants and its adjoint belong
    tuned = None
    if not matern and not args.threads:
        from paper_2402_06927_amd import autotune

        tuned, tile_ms = autotune.tune(model, m, u)
        log(f"autotuned threads per particle: {tuned} ({tile_ms})")
    elif args.threads:
        sch.sch_tune_set(sch.TUNE_THREADS, args.threads)
        tuned = args.threads

    def run_cycle(c):
        obs = sch.Obs(yobs[c].contiguous(), sigma)
        if matern:
            return sch.sch_pf_nudged_cycle_matern(model, mtn, obs, wl.seed, c, m, u, dLam, S,
                                                  0.5 * n, 50, rho, n_jitter, 100, ws)
        return sch.sch_pf_nudged_cycle(model, obs, wl.seed, c, m, u, dLam, S, 0.5 * n, 50, rho,
                                       n_jitter, 100, ws)

    for c in range(args.warmup):
        st = run_cycle(c)
        log(f"warmup cycle {c}: tempering steps {st['n_temper']}")
    torch.cuda.synchronize()
    sch.sch_timing_reset()
    sch.sch_timing_enable(True)
    stats = []
    t0 = time.perf_counter()
    for c in range(args.warmup, n_cycles):
        st = run_cycle(c)
        stats.append(st)
        log(f"cycle {c}: tempering steps {st['n_temper']}, ess {st['ess']:.1f}, "
            f"accept {st['n_accept']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sch.sch_timing_enable(False)
    tim = sch.sch_timing_read()
    out = {
        "metric": "nudged-filter assimilation cycles/s (nudging + tempering + jittering)",
        "value": round(args.steps / elapsed, 4),
        "unit": "cycles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "filter": "nudged+tempered+jittered", "nx": nx,
                   "n_particles": n, "n_modes": Q, "n_steps": S, "n_obs": wl.n_obs,
                   "noise": wl.noise, "controls_per_step": nq,
                   "sigma_obs": wl.sigma_obs, "ess_threshold": 0.5 * n, "n_jitter": n_jitter,
                   "rho": rho, "lbfgs_mem": 8, "ckpt_every": 8,
                   "threads_per_particle": tuned},
        "tempering_steps_per_cycle": [s_["n_temper"] for s_ in stats],
        "kernel_ms": {k: round(v["ms"], 3) for k, v in tim.items()},
    }
    print(json.dumps(out), flush=True)


PEAK_BF16_TFLOPS = 2500.0


def bench_warmstart(args):
    """The learned warm start of nudging against plain nudging, at 4096 nodes x
    4096 particles (8 modes, 40-step windows, 256 observations, sigma 0.02).
    The network (256 misfits + 4096 velocities -> 256 -> 256 -> 320 controls,
    BF16 on the matrix cores) is trained on the GPU on the plain-nudging
    solutions of --train-windows consecutive windows (25: 102400 pairs).  Then
    one step = one cycle of the nudged filter (nudging, tempering, jittering),
    run for --steps cycles by four ensembles from the same start on the same
    observations and seeds: plain nudging from zero controls; the network's
    controls as they are; the network's controls as the L-BFGS start with one
    accepted step per stage; and one step per stage from zero (the ablation
    that shows what the network adds).  The line's value is the third arm,
    the learned form that reaches plain nudging's likelihood; particles whose
    misfit lies outside the training range are nudged from zero in every
    learned arm.  The same four are also compared on identical inputs (mean
    likelihood and objective after nudging one window, objective evaluations
    per particle)."""
    import torch

    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import warmstart as WS
    from paper_2402_06927_amd import workloads as W

    wl = W.WARMSTART_4096
    if args.particles:
        wl = wl.scaled(n_particles=args.particles)
    dev = "cuda"
    n, nx, Q, S, nobs = wl.n_particles, wl.nx, wl.n_modes, wl.n_steps, wl.n_obs
    n_train, n_cycles = args.train_windows, args.steps
    n_jit, ckpt, thr = wl.n_jitter, 8, wl.ess_threshold
    log(f"bench: warm start, {wl.name}, {n_train} training windows, {n_cycles} cycles")
    xi = torch.tensor(W.mode_table(wl.L, nx, Q, wl.mode_amp), device=dev)
    model = sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi)
    ts = W.truth_seed(wl)
    ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
    mt = torch.empty_like(ut)
    sch.sch_init_momentum(model, ut, mt)
    u = torch.tensor(W.initial_velocity(wl, n, wl.seed), device=dev)
    m = torch.empty_like(u)
    sch.sch_init_momentum(model, u, m)
    z = torch.tensor(W.obs_noise(wl, ts, n_train + n_cycles), device=dev)
    sig = torch.full((nobs,), wl.sigma_obs, dtype=torch.float64, device=dev)

    def obs_for(c):
        dWt = torch.empty((1, S, Q), dtype=torch.float64, device=dev)
        sch.sch_draw_increments(ts, c, 0, sch.TAG_FORECAST, dWt, wl.dt)
        sch.sch_ensemble_step(model, mt, ut, dWt)
        y = torch.empty((1, nobs), dtype=torch.float64, device=dev)
        sch.sch_observe(model, ut, y)
        return sch.Obs((y[0] + wl.sigma_obs * z[c]).contiguous(), sig)

    def mean_phi(obs, uu):
        phi = torch.empty(uu.shape[0], dtype=torch.float64, device=dev)
        sch.sch_loglik(model, obs, uu, phi)
        return float(phi.mean())

    # ---- training data: plain nudging of consecutive windows
    ws = WS.WarmStart(nobs, nx, S, Q)
    nws = sch.workspace(sch.WS_NUDGE, model, n, S, ckpt)
    parts = []
    t0 = time.perf_counter()
    for c in range(n_train):
        obs = obs_for(c)
        dW = torch.empty((n, S, Q), dtype=torch.float64, device=dev)
        sch.sch_draw_increments(wl.seed, c, 0, sch.TAG_NUDGE, dW, wl.dt)
        parts.append(ws.collect(model, obs, m, u, dW, nws))
        log(f"training window {c} collected ({time.perf_counter() - t0:.0f} s)")
    del nws
    data = WS.concat(parts)
    del parts
    ws.fit_scaling(data)
    X, T = ws.encode(data)
    n_pairs = int(X.shape[0])
    del data
    B = 256
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    hist = ws.train(X, T, epochs=args.epochs, batch=B, lr=1e-3,
                    log=lambda s: log(s) if s.endswith("0") or True else None)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    steps_train = args.epochs * (n_pairs // B)
    F, H, O = ws.F, ws.H, ws.O
    flops_step = 3 * 2 * B * (F * H + H * H + H * O)
    del X, T

    # ---- the nudged forecasts on identical inputs (the first cycle's window)
    c0 = n_train
    ut0, mt0 = ut.clone(), mt.clone()  # the truth at the first filter cycle's start
    obs0 = obs_for(c0)
    dW = torch.empty((n, S, Q), dtype=torch.float64, device=dev)
    sch.sch_draw_increments(wl.seed, c0, 0, sch.TAG_NUDGE, dW, wl.dt)
    mm, uu = m.clone(), u.clone()
    sch.sch_ensemble_step(model, mm, uu, dW)
    same = {"none": mean_phi(obs0, uu)}
    nws = sch.workspace(sch.WS_NUDGE, model, n, S, ckpt)
    for arm in ("plain", "plain_1iter", "learned_1iter", "learned"):
        mm, uu = m.clone(), u.clone()
        dl = torch.zeros_like(dW)
        logG = torch.empty(n, dtype=torch.float64, device=dev)
        ev = torch.zeros(n, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        if arm in ("plain", "plain_1iter"):
            sch.sch_nudge_run(model, obs0, mm, uu, dW, dl, logG, evals=ev, workspace=nws,
                              max_iter=1 if arm == "plain_1iter" else sch.LBFGS_MAX_ITER)
        elif arm == "learned_1iter":
            ws.predict(model, obs0, uu, dl)
            sch.sch_nudge_run(model, obs0, mm, uu, dW, dl, logG, warm_start=True, max_iter=1,
                              evals=ev, workspace=nws)
        else:
            # the network's controls as they are (zero where the misfit is out of
            # range: this diagnostic leaves those particles un-nudged)
            ws.predict(model, obs0, uu, dl)
            sch.sch_ensemble_step(model, mm, uu, dW, dl)
            logG = -((0.5 * dl * dl + dl * dW).sum(dim=(1, 2)) / wl.dt)
        torch.cuda.synchronize()
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        sch.sch_loglik(model, obs0, uu, phi)
        same[arm] = {"mean_phi": float(phi.mean()), "mean_J": float((phi - logG).mean()),
                     "evals_per_particle": float(ev.double().mean()),
                     "seconds": round(time.perf_counter() - ta, 3)}
        log(f"same inputs, {arm}: {same[arm]}")
    del nws

    # ---- the nudged filter, arm by arm, cycle by cycle
    # plain: nudging from zero with the default stopping rule; learned_keep: the
    # network's controls as they are (plain nudging past the training range);
    # learned_1iter: the network's controls as the L-BFGS start, one accepted
    # step per stage; plain_1iter: the same optimiser budget from zero (what
    # the network adds over the method without it).
    arms = {"plain": (None, {}), "learned_keep": (sch.NUDGE_KEEP, {}),
            "learned_1iter": (sch.NUDGE_FROM_GIVEN, {"max_iter": 1}),
            "plain_1iter": (None, {"max_iter": 1})}
    cws = sch.nudged_workspace(model, n, S, n_jit, ckpt)
    res = {a: {"seconds": [], "n_temper": [], "final_phi": [], "fallback": []} for a in arms}
    for arm, (keep, lb) in arms.items():
        ut.copy_(ut0)
        mt.copy_(mt0)
        ma, ua = m.clone(), u.clone()
        for c in range(n_cycles):
            obs = obs_for(c0 + c)
            dl = torch.zeros((n, S, Q), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            if keep is None:
                st = sch.sch_pf_nudged_cycle(model, obs, wl.seed, c0 + c, ma, ua, dl, S, thr,
                                             wl.n_bisect, wl.rho, n_jit, wl.max_temper, cws,
                                             ckpt_every=ckpt, **lb)
                nfb = 0
            else:
                mode = torch.empty(n, dtype=torch.int32, device=dev)
                ws.predict(model, obs, ua, dl, True, mode, keep)
                st = sch.sch_pf_nudged_cycle_warm(model, obs, wl.seed, c0 + c, ma, ua, dl, mode,
                                                  S, thr, wl.n_bisect, wl.rho, n_jit,
                                                  wl.max_temper, cws, ckpt_every=ckpt, **lb)
                nfb = int((mode == sch.NUDGE_FROM_ZERO).sum())
            torch.cuda.synchronize()
            dt = time.perf_counter() - ta
            r = res[arm]
            r["seconds"].append(round(dt, 3))
            r["n_temper"].append(st["n_temper"])
            r["final_phi"].append(mean_phi(obs, ua))
            r["fallback"].append(nfb)
            log(f"{arm} cycle {c}: {dt:.2f} s, tempering steps {st['n_temper']}, "
                f"fallback {nfb}, final mean phi {r['final_phi'][-1]:.2f}")
        del ma, ua
    for arm in res:
        r = res[arm]
        r["cycles_per_s"] = n_cycles / sum(r["seconds"])
        r["mean_final_phi"] = sum(r["final_phi"]) / n_cycles
    def versus(a, b):
        return {"speedup": round(res[a]["cycles_per_s"] / res[b]["cycles_per_s"], 3),
                "final_phi_rel_diff": (res[a]["mean_final_phi"] - res[b]["mean_final_phi"])
                / res[b]["mean_final_phi"]}

    le = res["learned_1iter"]
    train_tflops = flops_step * steps_train / (train_ms * 1e-3) / 1e12
    out = {
        "metric": "nudged-filter assimilation cycles/s with the learned warm start "
                  "(plain nudging beside it)",
        "value": round(le["cycles_per_s"], 4),
        "unit": "cycles/s",
        "n_gpus": 1, "steps": n_cycles, "warmup": 0,
        "ms_per_step": round(1e3 / le["cycles_per_s"], 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 model, bf16/f32 network", "data": "synthetic",
        "config": {"workload": wl.name, "nx": nx, "n_particles": n, "n_modes": Q, "n_steps": S,
                   "n_obs": nobs, "network": [F, H, H, O], "training_pairs": n_pairs,
                   "epochs": args.epochs, "batch": B, "n_jitter": n_jit, "rho": wl.rho,
                   "value_arm": "learned_1iter"},
        "arms": res,
        "learned_keep_vs_plain": versus("learned_keep", "plain"),
        "learned_1iter_vs_plain": versus("learned_1iter", "plain"),
        "plain_1iter_vs_plain": versus("plain_1iter", "plain"),
        "network_gain_at_1iter": versus("learned_1iter", "plain_1iter"),
        "same_inputs": same,
        "same_inputs_phi_rel_diff": (same["learned"]["mean_phi"] - same["plain"]["mean_phi"])
        / same["plain"]["mean_phi"],
        "training": {"loss_first_last": [hist[0], hist[-1]], "ms": round(train_ms, 1),
                     "steps": steps_train, "tflops": round(train_tflops, 3)},
        "roofline": {"bound": "mfma", "achieved": round(train_tflops, 3),
                     "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(train_tflops / PEAK_BF16_TFLOPS, 5), "traffic": None,
                     "kernel": "network training step (k_gemm_bf16 forward + backward, Adam)",
                     "algorithmic_flops_per_step": flops_step},
    }
    print(json.dumps(out), flush=True)


def bench_mlp(args):
    """The warm-start network at its configured shape, 4352 (256 misfits +
    4096 velocities) -> 256 -> 256 -> 320, on 4096 particles: one step = one
    forward pass of the whole ensemble (inference), plus one training step
    (forward, backward, Adam) on a batch of 1024, both timed with events."""
    import numpy as np
    import torch

    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    F, H, O, B, Bt = 4352, 256, 320, 4096, 1024
    dev = "cuda"
    p = W.mlp_init_params(F, H, O, 1)
    net = sch.Mlp(F, H, O, torch.tensor(p, dtype=torch.float32, device=dev),
                  torch.empty(H * F + H * H + O * H, dtype=torch.bfloat16, device=dev))
    sch.sch_mlp_sync(net)
    g = np.random.default_rng(2)
    X = torch.tensor(g.standard_normal((B, F)), dtype=torch.float32, device=dev).to(torch.bfloat16)
    T = torch.tensor(g.standard_normal((B, O)), dtype=torch.float32, device=dev)
    Y = torch.empty((B, O), dtype=torch.float32, device=dev)
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, B), dtype=torch.uint8, device=dev)
    grad = torch.zeros_like(net.params)
    m, v = torch.zeros_like(grad), torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        sch.sch_mlp_forward(net, X, Y, ws)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        sch.sch_mlp_forward(net, X, Y, ws)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.steps
    flops_fwd = 2 * B * (F * H + H * H + H * O)
    Xt, Tt, Yt = X[:Bt], T[:Bt], Y[:Bt]
    e0.record()
    for k in range(args.steps):
        sch.sch_mlp_forward(net, Xt, Yt, ws)
        sch.sch_mlp_backward(net, Xt, Yt, Tt, loss, grad, ws)
        sch.sch_mlp_adam(net, grad, m, v, k + 1, 1e-4)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / args.steps
    flops_train = 3 * 2 * Bt * (F * H + H * H + H * O)
    tf = flops_fwd / (fwd_ms * 1e-3) / 1e12
    out = {
        "metric": "warm-start network inference, particles/s (4352-256-256-320, bf16 MFMA)",
        "value": round(B / (fwd_ms * 1e-3), 1), "unit": "particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fwd_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 x bf16 -> f32", "data": "synthetic",
        "config": {"workload": "warmstart_network_b4096", "network": [F, H, H, O], "batch": B,
                   "train_batch": Bt},
        "train_step_ms": round(train_ms, 4),
        "train_tflops": round(flops_train / (train_ms * 1e-3) / 1e12, 3),
        "roofline": {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(tf / PEAK_BF16_TFLOPS, 5), "traffic": None,
                     "kernel": "k_gemm_bf16 (three layers of one forward pass)",
                     "algorithmic_flops_per_launch": flops_fwd},
    }
    print(json.dumps(out), flush=True)


def paper_cpu_baseline(wl, n_da: int, n_threads: int):
    """The oracle's twin experiment (tempered + jittered, Matern noise) timed
    on the host for n_da assimilation steps from the same initial ensemble."""
    import oracle as O
    from paper_2402_06927_amd import workloads as W

    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    om = O.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                 picard_tol=wl.picard_tol, picard_max=wl.picard_max)
    omt = O.matern(wl.kappa, wl.eta, wl.k_solves)
    n, nx, S = wl.n_particles, wl.nx, wl.n_steps
    u = O.paper_init(nx, wl.L, wl.seed, n)
    m = O.momentum_from_velocity(om, u)
    ts = W.truth_seed(wl)
    ut = O.paper_init(nx, wl.L, ts, 1)[0]
    mt = O.momentum_from_velocity(om, ut)
    z = W.obs_noise(wl, ts, n_da)
    sig = W.sigma_vector(wl)
    t0 = time.perf_counter()
    for c in range(n_da):
        cells = O.draw_increments(ts, 1, S, nx, c * S, O.TAG_FORECAST, 0, wl.dt)[0]
        _, mt, ut, _ = O.window_matern(om, omt, mt, ut, cells)
        y = O.observe(ut, wl.n_obs) + wl.sigma_obs * z[c]
        _, out, _ = O.tempered_cycle_matern(om, omt, y, sig, wl.seed, c, m, u, S,
                                            wl.ess_threshold, wl.n_bisect, wl.rho, wl.n_jitter,
                                            wl.max_temper, n_threads=n_threads)
        m, u = out["m"], out["u"]
    dt = time.perf_counter() - t0
    return {"value": n_da / dt, "unit": "DA steps/s", "cores": n_threads, "kind": "oracle",
            "sample": f"the first {n_da} assimilation steps of experiment 1 (tempered + "
                      f"jittered, {n} particles) from the same initial ensemble, {dt:.1f} s"}


def bench_paper(args):
    """The paper's experiment 1 (section 4): nx = 100, 150 particles, Matern
    noise, observations every 5 steps at 80 points, tempering + jittering;
    args.steps assimilation steps timed after args.warmup untimed ones."""
    import torch

    from paper_2402_06927_amd import experiments as E
    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    sch.lib()
    wl = W.PAPER_SHAPE if args.exp == 1 else W.PAPER_HALF
    if args.warmup:
        E.run_twin(wl, "tempered", args.warmup)
    sch.sch_timing_reset()
    sch.sch_timing_enable(True)
    r = E.run_twin(wl, "tempered", args.steps)
    sch.sch_timing_enable(False)
    tim = sch.sch_timing_read()
    rb = E.run_twin(wl, "bootstrap", args.steps)
    summ, summ_b = E.summary(r), E.summary(rb)
    log(f"tempered: {summ}")
    log(f"bootstrap: {summ_b}")
    jt = tim["jitter"]
    j_launches = max(jt["launches"], 1)
    n, nx, S = wl.n_particles, wl.nx, wl.n_steps
    j_psteps = j_launches * n * S * wl.n_jitter
    j_flops = nx * (FLOPS_PER_NODE_ITER * jt["iters"]
                    + matern_flops_per_node_step(wl.k_solves, True) * j_psteps)
    j_ms = jt["ms"] / j_launches
    j_tflops = (j_flops / j_launches) / (j_ms * 1e-3) / 1e12 if jt["ms"] > 0 else 0.0
    out = {
        "metric": "assimilation steps/sec of the paper's experiment 1 (tempered + jittered)",
        "value": round(args.steps / r["seconds"], 3),
        "unit": "DA steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl.name, "filter": "tempered+jittered", "nx": nx,
                   "n_particles": n, "n_steps": S, "n_obs": wl.n_obs,
                   "n_observed": wl.n_observed or wl.n_obs, "sigma_obs": wl.sigma_obs,
                   "ess_threshold": wl.ess_threshold, "n_jitter": wl.n_jitter, "rho": wl.rho,
                   "noise": "matern", "kappa": wl.kappa, "eta": wl.eta, "k_solves": wl.k_solves},
        "statistics": {"tempered": summ, "bootstrap": summ_b},
        "kernel_ms": {k: round(v["ms"], 3) for k, v in tim.items()},
        "roofline": {
            "bound": "alu", "achieved": round(j_tflops, 4), "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": round(j_tflops / PEAK_FP64_TFLOPS, 5), "traffic": None,
            "kernel": "k_jitter<Matern> at nx = 100 (150 workgroups: under one per CU)",
            "avg_launch_ms": round(j_ms, 4),
        },
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = paper_cpu_baseline(wl, min(args.steps, 40), threads)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 independent bootstrap filters of uneven sizes (grids log-uniform in
    [512, 8192], ensembles log-uniform in [64, 2048]; physics of the Nx = 256
    bootstrap workload with per-instance seeds) advanced together: one step =
    one assimilation cycle of every instance as one HIP graph replay
    (forecast noise, persistent forecast kernels per tile class, likelihood,
    weights, conditional resampling, gathers).  Tiles come from the autotuner
    (one tuning per group of grids with the same tile options)."""
    import torch

    from paper_2402_06927_amd import autotune
    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    sch.lib()
    base = W.BOOTSTRAP_256
    insts = W.uneven_instances(64)
    dev = "cuda"
    Q, S, nobs = base.n_modes, base.n_steps, base.n_obs
    n_cycles = args.warmup + args.steps + 1
    node_states = sum(i.nx * i.n_particles for i in insts)
    G = sum(i.n_particles for i in insts)
    log(f"bench batch: {len(insts)} instances, {G} particles, {node_states} node-states")

    def make_model(nx, xi=None):
        if xi is None:
            xi = torch.tensor(W.mode_table(base.L, nx, Q, base.mode_amp), device=dev)
        return sch.Model(L=base.L, alpha=base.alpha, mu=base.mu, dt=base.dt, xi=xi,
                         picard_tol=base.picard_tol, picard_max=base.picard_max)

    t0 = time.perf_counter()
    tiles = autotune.tune_batch(make_model, [i.nx for i in insts])
    log(f"tiles per grid group: {sorted(set(tiles.values()))} ({time.perf_counter() - t0:.1f} s)")
    gi, models = [], []
    sig = torch.full((nobs,), base.sigma_obs, dtype=torch.float64, device=dev)
    for k, ins in enumerate(insts):
        wl = base.scaled(nx=ins.nx, n_particles=ins.n_particles, seed=ins.seed)
        xi = torch.tensor(W.mode_table(wl.L, wl.nx, Q, wl.mode_amp), device=dev)
        model = make_model(ins.nx, xi)
        u = torch.tensor(W.initial_velocity(wl, ins.n_particles, wl.seed), device=dev)
        m = torch.empty_like(u)
        sch.sch_init_momentum(model, u, m)
        # truth (seed + 1) and its observations for every cycle
        ts = W.truth_seed(wl)
        ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
        mt = torch.empty_like(ut)
        sch.sch_init_momentum(model, ut, mt)
        z = torch.tensor(W.obs_noise(wl, ts, n_cycles), device=dev)
        dWt = torch.empty((1, S, Q), dtype=torch.float64, device=dev)
        y = torch.empty((n_cycles, nobs), dtype=torch.float64, device=dev)
        for c in range(n_cycles):
            sch.sch_draw_increments(ts, c, 0, sch.TAG_FORECAST, dWt, wl.dt)
            sch.sch_ensemble_step(model, mt, ut, dWt)
            sch.sch_observe(model, ut, y[c:c + 1])
        y += wl.sigma_obs * z
        gi.append(sch.Instance(xi=xi, m=m, u=u, logw=torch.zeros(ins.n_particles,
                                                                 dtype=torch.float64, device=dev),
                               y=y, sigma=sig, seed=ins.seed, threads=tiles[ins.nx]))
        models.append(model)
    b = sch.Batch(base.L, base.alpha, base.mu, base.dt, Q, S, nobs, base.ess_frac, gi,
                  base.picard_tol, base.picard_max)
    torch.cuda.synchronize()
    log(f"set-up {time.perf_counter() - t0:.1f} s")
    for c in range(args.warmup):
        b.run(c, 1, use_graph=True)
    out0 = b.read()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e0.record()
    for c in range(args.warmup, args.warmup + args.steps):
        b.run(c, 1, use_graph=True)
    e1.record()
    out1 = b.read()
    elapsed = time.perf_counter() - t1
    ms = e0.elapsed_time(e1) / args.steps
    iters_graph = out1["picard_iters"] - out0["picard_iters"]
    # one more cycle with direct launches and timing events: the forecast
    # kernels' share
    sch.sch_timing_reset()
    sch.sch_timing_enable(True)
    b.run(args.warmup + args.steps, 1, use_graph=False)
    out2 = b.read()
    sch.sch_timing_enable(False)
    tim = sch.sch_timing_read()
    iters_direct = out2["picard_iters"] - out1["picard_iters"]
    b.close()
    node_steps = node_states * S
    kbar = iters_direct / (G * S)
    flops = node_steps * (FLOPS_PER_NODE_ITER * kbar + flops_per_node_step(Q))
    w_ms = tim["window"]["ms"]
    tf = flops / (w_ms * 1e-3) / 1e12 if w_ms > 0 else 0.0
    out = {
        "metric": "batched uneven filters: assimilation cycles/s of all 64 instances (one graph replay per cycle)",
        "value": round(1e3 / ms, 4), "unit": "cycles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch64_uneven", "instances": len(insts), "particles": G,
                   "node_states": node_states, "nx_range": [512, 8192],
                   "particles_range": [64, 2048], "n_modes": Q, "n_steps": S, "n_obs": nobs,
                   "filter": "bootstrap", "tiles": {str(k): v for k, v in sorted(tiles.items())}},
        "node_steps_per_s": round(node_steps * 1e3 / ms, 1),
        "particle_steps_per_s": round(G * S * 1e3 / ms, 1),
        "picard_iters_per_step": round(iters_graph / (G * S * args.steps), 3),
        "resamplings": out1["resampled"],
        "host_ms_per_cycle": round(1e3 * elapsed / args.steps, 3),
        "kernel_ms_direct_cycle": {k: round(v["ms"], 3) for k, v in tim.items()},
        "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "k_batch_window (persistent forecast, all tile classes of one cycle)",
                     "avg_launch_ms": round(w_ms, 3), "algorithmic_flops_per_launch": flops,
                     "picard_iters_per_step": round(kbar, 3)},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        import oracle as O

        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        order = sorted(range(len(insts)), key=lambda k: insts[k].nx * insts[k].n_particles)
        # forecast windows of instances from the median size upwards until
        # about 10 s of oracle work
        done_ns, spent, used, worst = 0, 0.0, [], 0
        for k in order[len(order) // 2:]:
            ins = insts[k]
            wl = base.scaled(nx=ins.nx, n_particles=ins.n_particles, seed=ins.seed)
            xi = W.mode_table(wl.L, wl.nx, Q, wl.mode_amp)
            om = O.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                         picard_tol=wl.picard_tol, picard_max=wl.picard_max)
            u = W.initial_velocity(wl, ins.n_particles, wl.seed)
            mo = O.momentum_from_velocity(om, u)
            dW = O.draw_increments(wl.seed, ins.n_particles, S, Q, 0, O.TAG_FORECAST, 0, wl.dt)
            log(f"cpu baseline: oracle forecast of instance {k} (nx {ins.nx}, "
                f"{ins.n_particles} particles), {threads} threads ...")
            t2 = time.perf_counter()
            st, _, _, _, _ = O.ensemble_window(om, mo, u, dW, n_threads=threads)
            spent += time.perf_counter() - t2
            worst = worst or st
            done_ns += ins.nx * ins.n_particles * S
            used.append(k)
            if spent >= 10.0:
                break
        rate = done_ns / spent
        out["cpu_baseline"] = {
            "value": rate / node_steps, "unit": "cycles/s", "cores": threads, "kind": "oracle",
            "sample": (f"forecast windows of {len(used)} instances from the median size up "
                       f"({done_ns} node-steps in {spent:.1f} s, {rate:.3g} node-steps/s), "
                       f"scaled by the {node_steps} node-steps of one cycle of all 64 "
                       f"instances; oracle status {worst}"),
            "node_steps_per_s": rate,
        }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed assimilation cycles")
    ap.add_argument("--warmup", type=int, default=1, help="untimed cycles before timing")
    ap.add_argument("--particles", type=int, default=None, help="override the ensemble size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=None)
    ap.add_argument("--workload", choices=("tempered", "matern", "pcnl", "hmc", "paper",
                                           "nudging", "nudging_matern", "nudged_matern",
                                           "nudged", "warmstart", "mlp", "batch"),
                    default="tempered",
                    help="tempered: the headline filter; matern: the same filter with the "
                         "Matern-type noise of section 2; pcnl: the same filter with "
                         "gradient-based (pCN-Langevin) jitter; hmc: the same filter with Hybrid "
                         "Monte Carlo jitter; paper: the paper's twin experiment "
                         "(--exp 1 or 2); nudging: one nudged window; nudging_matern: the same "
                         "with the Matern-type noise and one control per cell; "
                         "nudged: the nudged filter (nudging, tempering, jittering); nudged_matern: "
                         "the same with the Matern-type noise; "
                         "warmstart: plain vs learned warm-start nudging; mlp: the "
                         "warm-start network; batch: 64 uneven filters in one graph")
    ap.add_argument("--threads", type=int, default=0,
                    help="threads per particle of the model kernels (0 = automatic)")
    ap.add_argument("--exp", type=int, choices=(1, 2), default=1,
                    help="paper workload: 1 full domain observed, 2 half domain")
    ap.add_argument("--train-windows", type=int, default=25)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="run only a plain copy of BYTES (traffic-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.threads:
        from paper_2402_06927_amd import sch as _sch

        _sch.sch_tune_set(_sch.TUNE_THREADS, args.threads)
    if args.workload == "paper":
        bench_paper(args)
        return
    if args.workload in ("nudging", "nudging_matern"):
        bench_nudging(args, matern=args.workload == "nudging_matern")
        return
    if args.workload in ("nudged", "nudged_matern"):
        bench_nudged(args, matern=args.workload == "nudged_matern")
        return
    if args.workload == "warmstart":
        bench_warmstart(args)
        return
    if args.workload == "mlp":
        bench_mlp(args)
        return
    if args.workload == "batch":
        bench_batch(args)
        return

    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    sch.lib()
    matern = args.workload == "matern"
    hmc = args.workload == "hmc"
    pcnl = args.workload == "pcnl" or hmc
    wl = W.MATERN_4096 if matern else W.TEMPERED_4096
    mtn = sch.Matern(wl.kappa, wl.eta, wl.k_solves) if matern else None
    if args.particles:
        wl = wl.scaled(n_particles=args.particles)
    dev = "cuda"
    n, nx, Q, S = wl.n_particles, wl.nx, wl.n_modes, wl.n_steps
    n_cycles = args.warmup + args.steps
    log(f"bench: {wl.name} n={n} nx={nx} Q={Q} S={S} cycles={args.warmup}+{args.steps}")

    xi = torch.tensor(W.mode_table(wl.L, nx, Q, wl.mode_amp), device=dev)
    model = sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                      picard_tol=wl.picard_tol, picard_max=wl.picard_max)
    u0 = W.initial_velocity(wl, n, wl.seed)
    u = torch.tensor(u0, device=dev)
    m = torch.empty_like(u)
    sch.sch_init_momentum(model, u, m)

    # truth run (seed + 1) and observations for every cycle
    ts = W.truth_seed(wl)
    ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
    mt = torch.empty_like(ut)
    sch.sch_init_momentum(model, ut, mt)
    z = torch.tensor(W.obs_noise(wl, ts, n_cycles), device=dev)
    dWt = torch.empty((1, S, nx if matern else Q), dtype=torch.float64, device=dev)
    yobs = torch.empty((n_cycles, wl.n_obs), dtype=torch.float64, device=dev)
    for c in range(n_cycles):
        sch.sch_draw_increments(ts, c, 0, sch.TAG_FORECAST, dWt, wl.dt)
        if matern:
            sch.sch_ensemble_step_matern(model, mtn, mt, ut, dWt)
        else:
            sch.sch_ensemble_step(model, mt, ut, dWt)
        sch.sch_observe(model, ut, yobs[c:c + 1])
    yobs += wl.sigma_obs * z
    sigma = torch.full((wl.n_obs,), wl.sigma_obs, dtype=torch.float64, device=dev)
    if matern:
        ws = sch.matern_workspace(sch.WS_TEMPERED, model, n, S, wl.n_jitter)
    elif hmc:
        ws = sch.hmc_workspace(sch.WS_TEMPERED, model, n, S, wl.n_jitter, PCNL_CKPT)
    elif pcnl:
        ws = sch.pcnl_workspace(sch.WS_TEMPERED, model, n, S, wl.n_jitter, PCNL_CKPT)
    else:
        ws = sch.workspace(sch.WS_TEMPERED, model, n, S, wl.n_jitter)
    m_cpu0, u_cpu0 = None, None
    if not args.threads:
        from paper_2402_06927_amd import autotune

        tuned, tile_ms = autotune.tune(model, m, u)
        log(f"autotuned threads per particle: {tuned} ({tile_ms})")
    else:
        tuned, tile_ms = args.threads, {}

    def run_cycle(c):
        obs = sch.Obs(yobs[c].contiguous(), sigma)
        if matern:
            return sch.sch_pf_tempered_cycle_matern(model, mtn, obs, wl.seed, c, m, u, S,
                                                    wl.ess_threshold, wl.n_bisect, wl.rho,
                                                    wl.n_jitter, wl.max_temper, ws)
        if hmc:
            return sch.sch_pf_tempered_cycle_hmc(model, obs, wl.seed, c, m, u, S,
                                                 wl.ess_threshold, wl.n_bisect, HMC_H, HMC_LEAP,
                                                 wl.n_jitter, wl.max_temper, ws, PCNL_CKPT)
        if pcnl:
            return sch.sch_pf_tempered_cycle_pcnl(model, obs, wl.seed, c, m, u, S,
                                                  wl.ess_threshold, wl.n_bisect, wl.rho,
                                                  wl.n_jitter, wl.max_temper, ws, PCNL_CKPT)
        return sch.sch_pf_tempered_cycle(model, obs, wl.seed, c, m, u, S, wl.ess_threshold,
                                         wl.n_bisect, wl.rho, wl.n_jitter, wl.max_temper, ws)

    for c in range(args.warmup):
        st = run_cycle(c)
        log(f"warmup cycle {c}: tempering steps {st['n_temper']}")
    torch.cuda.synchronize()
    # the CPU baseline starts from the ensemble of the first timed cycle
    m_cpu0 = m.cpu().numpy().copy()
    u_cpu0 = u.cpu().numpy().copy()

    sch.sch_timing_reset()
    sch.sch_timing_enable(True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(args.warmup, n_cycles):
        st = run_cycle(c)
        stats.append(st)
        log(f"cycle {c}: tempering steps {st['n_temper']}, ess {st['ess']:.1f}, "
            f"accept {st['n_accept']}, particle-steps {st['particle_steps']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sch.sch_timing_enable(False)
    tim = sch.sch_timing_read()

    psteps = sum(s["particle_steps"] for s in stats)
    iters = sum(s["picard_iters"] for s in stats)
    n_temper = [s["n_temper"] for s in stats]
    cycles_per_s = args.steps / elapsed
    psteps_per_s = psteps / elapsed

    # dominant kernel: fused pCN jitter (5 window reruns per launch)
    jt = tim["jitter"]
    j_launches = max(jt["launches"], 1)
    j_psteps = j_launches * n * S * wl.n_jitter
    per_step = (matern_flops_per_node_step(wl.k_solves, True) if matern
                else flops_per_node_step(Q))
    adj_iters = 0
    if pcnl:
        # forward windows per stage: the gradient at the start, one per proposal
        # (n_leap per HMC move), the end-state rerun; jt["iters"] holds the Picard
        # iterations of all of them and of the adjoint's segment recomputations, the
        # adjoint class the transposed fixed-point iterations, counted at the minimal
        # forward count (the same operations, transposed); the reverse sweeps'
        # per-step work and the recomputations' are left out: a lower bound
        evals = wl.n_jitter * (HMC_LEAP if hmc else 1) + 2
        j_psteps = j_launches * n * S * evals
        adj_iters = tim["adjoint"]["iters"]
    j_min_flops = nx * (FLOPS_PER_NODE_ITER * (jt["iters"] + adj_iters) + per_step * j_psteps)
    # (the Matern-type noise's own per-step work exceeds the 20 of the modes form)
    model_step = max(MODEL_FLOPS_PER_NODE_STEP, per_step)
    j_flops = nx * (MODEL_FLOPS_PER_NODE_ITER * jt["iters"] + FLOPS_PER_NODE_ITER * adj_iters
                    + model_step * j_psteps)
    j_ms = jt["ms"] / j_launches
    j_tflops = (j_flops / j_launches) / (j_ms * 1e-3) / 1e12 if jt["ms"] > 0 else 0.0
    j_min_tflops = (j_min_flops / j_launches) / (j_ms * 1e-3) / 1e12 if jt["ms"] > 0 else 0.0
    traffic_ok = (kernel_sources_hash() == TRAFFIC_SOURCES_HASH and wl.nx == 4096 and n == 1024
                  and tuned == TRAFFIC_THREADS and not pcnl)
    roofline = {
        "bound": "alu",
        "achieved": round(j_tflops, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(j_tflops / PEAK_FP64_TFLOPS, 4),
        "traffic": ((TRAFFIC_JITTER_MATERN_BYTES if matern else TRAFFIC_JITTER_BYTES)
                    if traffic_ok else None),
        "flop_count": (f"achieved/frac: {MODEL_FLOPS_PER_NODE_ITER} flops per node per Picard "
                       f"iteration + {model_step} per node per step, with the "
                       f"iterations the launches took; achieved_min/frac_min: the minimal "
                       f"count {FLOPS_PER_NODE_ITER} per node per iteration + {per_step} per "
                       f"node per step"),
        "achieved_min": round(j_min_tflops, 3),
        "frac_min": round(j_min_tflops / PEAK_FP64_TFLOPS, 4),
        "traffic_source": ("constant from two rocprofv3 counter runs (FETCH_SIZE x 2.0 + "
                           "WRITE_SIZE x 1.0, the factors of a plain copy) on the kernel "
                           f"sources with hash {TRAFFIC_SOURCES_HASH}; null when the sources, "
                           "grid, ensemble or tile differ" if traffic_ok else
                           "null: kernel sources, grid, ensemble or tile differ from the "
                           "counter runs"),
        "kernel": ("k_jitter<Matern> (pCN proposal drawn per cell + noise field + window "
                   "rerun + likelihood + accept)" if matern else
                   "pCN-Langevin stage (k_nudge_grad x (moves + 1), proposals, accepts, "
                   "end-state window); the adjoint's transposed iterations at the minimal "
                   "count, its reverse sweeps' per-step work left out (lower bound)"
                   if pcnl and not hmc else
                   "Hybrid Monte Carlo stage (k_nudge_grad x (moves x leapfrog steps + 1), kicks "
                   "and rotations, accepts, end-state window); the adjoint's transposed "
                   "iterations at the minimal count, its reverse sweeps' per-step work left out "
                   "(lower bound)" if hmc else
                   "k_jitter (fused pCN proposal + window rerun + likelihood + accept)"),
        "avg_launch_ms": round(j_ms, 3),
        "algorithmic_flops_per_launch": j_flops / j_launches,
        "min_flops_per_launch": j_min_flops / j_launches,
        "picard_iters_per_step": jt["iters"] / max(j_psteps, 1),
    }
    if pcnl:
        ad = tim["adjoint"]
        roofline.update(adjoint_evals_per_launch=ad["launches"] / j_launches,
                        adjoint_ms_per_eval=round(ad["ms"] / max(ad["launches"], 1), 3),
                        transposed_iters_per_step=adj_iters / max(ad["launches"] * n * S, 1))

    config = {
        "workload": wl.name, "filter": "tempered+jittered", "nx": nx, "n_particles": n,
        "n_modes": Q, "n_steps": S, "n_obs": wl.n_obs, "sigma_obs": wl.sigma_obs,
        "ess_threshold": wl.ess_threshold, "n_bisect": wl.n_bisect,
        "n_jitter": wl.n_jitter, "rho": wl.rho, "threads_per_particle": tuned,
    }
    if matern:
        del config["n_modes"]
        config.update(noise="matern", kappa=wl.kappa, eta=wl.eta, k_solves=wl.k_solves)
    if hmc:
        del config["rho"]
        config.update(jitter="hybrid-monte-carlo", h=HMC_H, n_leap=HMC_LEAP,
                      ckpt_every=PCNL_CKPT)
        config["workload"] = wl.name + "_hmc"
    elif pcnl:
        config.update(jitter="pcn-langevin", ckpt_every=PCNL_CKPT)
        config["workload"] = wl.name + "_pcnl"
    out = {
        "metric": "assimilation cycles/sec + particle-steps/sec at N=1024, Nx=4096, vs plain",
        "value": round(cycles_per_s, 4),
        "unit": "cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": config,
        "particle_steps_per_s": round(psteps_per_s, 1),
        "tempering_steps_per_cycle": n_temper,
        "picard_iters_per_step": round(iters / max(psteps, 1), 3),
        "kernel_ms": {k: round(v["ms"], 3) for k, v in tim.items()},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline and not pcnl:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        log(f"cpu baseline: oracle, {threads} threads ...")
        cb = cpu_baseline(wl, u_cpu0, m_cpu0, threads, psteps / args.steps)
        out["cpu_baseline"] = cb
        log(f"cpu baseline: {cb['particle_steps_per_s']:.1f} particle-steps/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
