"""Seeded synthetic workloads for the SCH particle filter.

This module only produces inputs: parameter sets, the nodal values of the
noise modes, prior-ensemble and truth initial velocities, and the standard
normal draws that perturb the observations.  It holds none of the method's
arithmetic (no Helmholtz solve, no time step, no likelihood) and imports
neither the GPU library nor the oracle, so both can consume exactly the same
arrays.

The paper's experiments are synthetic twin experiments (section 4: the truth
is drawn from the same model as the particles), so no external dataset is
involved.  The workloads below follow the parameter sets of this project
(periodic domain of length 40, alpha = 1, mu = 0.01, dt = 0.025, sinusoidal
noise modes of amplitude 0.05); the paper's own shape (N = 100 cells, 150
particles, 5 steps per window, 81 observations) is available as ``paper``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

MASTER_SEED = 240206927


@dataclass(frozen=True)
class Workload:
    """One filter configuration.  All lengths in model units."""
    name: str
    nx: int
    n_particles: int
    n_modes: int
    n_steps: int            # model steps per assimilation window (N_s)
    n_cycles: int
    n_obs: int
    sigma_obs: float
    filter: str             # "bootstrap" or "tempered"
    L: float = 40.0
    alpha: float = 1.0
    mu: float = 0.01
    dt: float = 0.025
    mode_amp: float = 0.05
    ess_frac: float = 0.5   # resampling / tempering threshold as a fraction of N_p
    n_bisect: int = 50
    n_jitter: int = 5
    rho: float = 0.99
    max_temper: int = 100
    picard_tol: float = 1e-13
    picard_max: int = 50
    seed: int = MASTER_SEED
    # noise: "modes" (dU = sum_q xi_q dW_q) or "matern" (section 2: k solves
    # with M + kappa^-2 K on the DG0 white noise, amplitude eta)
    noise: str = "modes"
    kappa: float = 1.0
    eta: float = 1.0
    k_solves: int = 3
    # observed points: the first n_observed of the n_obs grid points (0 = all)
    n_observed: int = 0

    @property
    def h(self) -> float:
        return self.L / self.nx

    @property
    def ess_threshold(self) -> float:
        return self.ess_frac * self.n_particles

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


# Bootstrap filter, Nx = 256, 32 particles, 4 modes, 10 cycles of 20 steps,
# 40 observations with sigma 0.05.
BOOTSTRAP_256 = Workload(
    name="bootstrap_nx256_np32", nx=256, n_particles=32, n_modes=4, n_steps=20, n_cycles=10,
    n_obs=40, sigma_obs=0.05, filter="bootstrap")

# Tempered + jittered filter, Nx = 4096, 1024 particles, 8 modes, 50 cycles of
# 40 steps, 256 observations with sigma 0.02, ESS threshold N/2 with
# bisection tempering, 5 pCN steps per temperature at rho = 0.99.
TEMPERED_4096 = Workload(
    name="tempered_nx4096_np1024", nx=4096, n_particles=1024, n_modes=8, n_steps=40,
    n_cycles=50, n_obs=256, sigma_obs=0.02, filter="tempered")

# Nudging workload: Nx = 2048, 2048 particles, 8 modes, 40-step window,
# 256 observations with sigma 0.02.
NUDGING_2048 = Workload(
    name="nudging_nx2048_np2048", nx=2048, n_particles=2048, n_modes=8, n_steps=40,
    n_cycles=1, n_obs=256, sigma_obs=0.02, filter="nudging")

# The paper's experiment 1 (section 4): N = 100 cells, 150 particles,
# observations every 5 steps at 81 points (80 distinct on the periodic grid)
# with N(0, 0.5) errors, threshold 80, delta = 0.15 (rho = (2 - delta)/(2 + delta)),
# the Matern-type noise (eta = 1, k = 3, kappa = 1) and the initial ensemble of
# eq. init_solve.  The noise feeds energy into the solution (the transport
# noise conserves circulation, not energy): after about 900 assimilation steps
# the velocity has grown some thirtyfold and the implicit solve needs about 30
# Picard iterations per step, so the cap is raised to 200.
PAPER_SHAPE = Workload(
    name="paper_nx100_np150", nx=100, n_particles=150, n_modes=4, n_steps=5, n_cycles=1000,
    n_obs=80, sigma_obs=math.sqrt(0.5), filter="tempered", ess_frac=80.0 / 150.0,
    rho=(2.0 - 0.15) / (2.0 + 0.15), noise="matern", picard_max=200)

# Experiment 2: only [0, L/2] observed, at 41 points: the first 41 of the 80.
PAPER_HALF = replace(PAPER_SHAPE, name="paper_half_nx100_np150", n_observed=41)

# The tempered + jittered filter of TEMPERED_4096 with the paper's own noise:
# the Matern-type field of section 2 with eta = 1, k = 3 and kappa = 1 (the
# operator of the paper's initial-condition smoothing), nx = 4096 cell
# increments per step.
MATERN_4096 = replace(TEMPERED_4096, name="tempered_matern_nx4096_np1024", noise="matern")

# The nudging workload with the Matern-type noise: one control per DG0 cell
# and step (2048 per step and particle instead of 8).
NUDGING_MATERN_2048 = replace(NUDGING_2048, name="nudging_matern_nx2048_np2048", noise="matern")

# The learned warm start of nudging: the tempered workload's physics and
# observations (nx = 4096, 8 modes, 40 steps, 256 observations, sigma 0.02)
# with 4096 particles; the network is trained on plain-nudging solutions of
# consecutive windows (25 windows = 102400 pairs).
WARMSTART_4096 = replace(NUDGING_2048, name="warmstart_nx4096_np4096", nx=4096,
                         n_particles=4096)

WORKLOADS = {w.name: w for w in (BOOTSTRAP_256, TEMPERED_4096, NUDGING_2048, PAPER_SHAPE,
                                 PAPER_HALF, MATERN_4096, NUDGING_MATERN_2048, WARMSTART_4096)}


def node_positions(L: float, nx: int) -> np.ndarray:
    return np.arange(nx, dtype=np.float64) * (L / nx)


def mode_table(L: float, nx: int, n_modes: int, amp: float) -> np.ndarray:
    """Nodal values xi[q][i] of the sinusoidal noise modes:
    q = 2(j-1): amp sin(2 pi j x / L), q = 2(j-1)+1: amp cos(2 pi j x / L)."""
    x = node_positions(L, nx)
    xi = np.zeros((n_modes, nx), dtype=np.float64)
    for q in range(n_modes):
        j = q // 2 + 1
        arg = 2.0 * math.pi * j * x / L
        xi[q] = amp * (np.sin(arg) if q % 2 == 0 else np.cos(arg))
    return xi


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed) & 0xFFFFFFFFFFFFFFFF, stream]))


def initial_velocity(wl: Workload, n: int, seed: int) -> np.ndarray:
    """Initial velocities [n][nx]: 0.2 sech^2((x - L/2)/2) plus a smooth
    random perturbation p(x) = sum_{k=1..4} a_k cos(2 pi k x/L) + b_k sin(2 pi k x/L)
    with a_k, b_k ~ N(0, 0.01/4), so that p has pointwise variance 0.01."""
    x = node_positions(wl.L, wl.nx)
    base = 0.2 / np.cosh((x - 0.5 * wl.L) / 2.0) ** 2
    g = _rng(seed, 0)
    coef = g.standard_normal((n, 4, 2)) * math.sqrt(0.01 / 4.0)
    u = np.empty((n, wl.nx), dtype=np.float64)
    for p in range(n):
        pert = np.zeros(wl.nx)
        for k in range(1, 5):
            arg = 2.0 * math.pi * k * x / wl.L
            pert += coef[p, k - 1, 0] * np.cos(arg) + coef[p, k - 1, 1] * np.sin(arg)
        u[p] = base + pert
    return u


def obs_noise(wl: Workload, seed: int, n_cycles: int | None = None) -> np.ndarray:
    """Standard normal draws [cycles][n_obs] that perturb the observations."""
    g = _rng(seed, 5)
    return g.standard_normal((n_cycles or wl.n_cycles, wl.n_obs))


def sigma_vector(wl: Workload) -> np.ndarray:
    """Observation error std per point; +inf on the unobserved points (n_observed)."""
    s = np.full(wl.n_obs, wl.sigma_obs, dtype=np.float64)
    if wl.n_observed:
        s[wl.n_observed:] = np.inf
    return s


def truth_seed(wl: Workload) -> int:
    return wl.seed + 1


def random_weights(n: int, seed: int, spread: float = 3.0) -> np.ndarray:
    """Positive, normalised test weights with a log-normal spread."""
    g = _rng(seed, 9)
    w = np.exp(spread * g.standard_normal(n))
    return w / w.sum()


def random_phi(n: int, seed: int, scale: float = 50.0) -> np.ndarray:
    """Non-negative test negative-log-likelihoods with a chi-square-like spread."""
    g = _rng(seed, 10)
    return scale * g.chisquare(4, n)


def random_state_noise(shape, seed: int, stream: int = 11) -> np.ndarray:
    return _rng(seed, stream).standard_normal(shape)


@dataclass
class Instance:
    """Sizes of one filter instance of the batched-uneven workload."""
    nx: int
    n_particles: int
    seed: int


def uneven_instances(n_instances: int = 64, seed: int = MASTER_SEED,
                     nx_range=(512, 8192), np_range=(64, 2048), nx_multiple: int = 1):
    """Instance sizes drawn log-uniform in the given ranges (per-instance seeds
    seed + 2 i, truth seed + 2 i + 1)."""
    g = _rng(seed, 7)
    out = []
    for i in range(n_instances):
        nx = int(round(math.exp(g.uniform(math.log(nx_range[0]), math.log(nx_range[1])))))
        npart = int(round(math.exp(g.uniform(math.log(np_range[0]), math.log(np_range[1])))))
        if nx_multiple > 1:
            nx = max(nx_multiple, nx_multiple * round(nx / nx_multiple))
        out.append(Instance(nx=nx, n_particles=npart, seed=seed + 2 * i))
    return out


def mlp_init_params(n_in: int, n_hidden: int, n_out: int, seed: int) -> np.ndarray:
    """Initial parameters of the warm-start network as one vector in the order
    W1 [H][F], b1 [H], W2 [H][H], b2 [H], W3 [O][H], b3 [O] (weights
    He-normal with std sqrt(2 / fan_in), zero biases)."""
    g = _rng(seed, 12)
    F, H, O = n_in, n_hidden, n_out
    parts = [g.standard_normal(H * F) * math.sqrt(2.0 / F), np.zeros(H),
             g.standard_normal(H * H) * math.sqrt(2.0 / H), np.zeros(H),
             g.standard_normal(O * H) * math.sqrt(2.0 / H), np.zeros(O)]
    return np.concatenate(parts)
