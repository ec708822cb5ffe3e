"""Shared set-up for the GPU-vs-oracle tests: the same seeded inputs handed
to both sides.  Inputs come from ``paper_2402_06927_amd.workloads`` only;
expected values come from the oracle only."""
from __future__ import annotations

import math

import numpy as np

import oracle as O
from paper_2402_06927_amd import workloads as W

REL_TOL = 1e-10  # relative L2 per cycle / per window


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def oracle_model(wl: W.Workload) -> O.Model:
    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    return O.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                   picard_tol=wl.picard_tol, picard_max=wl.picard_max)


def gpu_model(wl: W.Workload):
    import torch

    from paper_2402_06927_amd import sch

    xi = torch.tensor(W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp), device="cuda")
    return sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                     picard_tol=wl.picard_tol, picard_max=wl.picard_max)


def prior(wl: W.Workload, n: int | None = None):
    """Initial velocities of the ensemble and the truth (inputs), and the
    oracle's momenta for them."""
    n = n or wl.n_particles
    u = W.initial_velocity(wl, n, wl.seed)
    ut = W.initial_velocity(wl, 1, W.truth_seed(wl))[0]
    om = oracle_model(wl)
    return u, O.momentum_from_velocity(om, u), ut, O.momentum_from_velocity(om, ut)


def oracle_observations(wl: W.Workload, n_cycles: int):
    """Twin-experiment observations from the oracle's truth run: truth uses
    seed + 1 for its increments; y_c = P u_truth(t_c) + sigma z_c."""
    om = oracle_model(wl)
    _, _, ut, mt = prior(wl, 1)
    z = W.obs_noise(wl, W.truth_seed(wl), n_cycles)
    ys = []
    for c in range(n_cycles):
        dW = O.draw_increments(W.truth_seed(wl), 1, wl.n_steps, wl.n_modes, c * wl.n_steps,
                               O.TAG_FORECAST, 0, wl.dt)[0]
        st, mt, ut, _ = O.window(om, mt, ut, dW)
        assert st == 0
        ys.append(O.observe(ut, wl.n_obs) + wl.sigma_obs * z[c])
    return np.array(ys)


def sdt(wl) -> float:
    return math.sqrt(wl.dt)
