"""GPU (C-ABI) versus oracle with the Matern-type noise of section 2 (eqs.
noise_solve and noise_solve2): the field of k elliptic solves on the DG0
white noise, the window driven by it, the pCN jitter of the cell increments
(proposals drawn inside the kernel) and the tempered cycle.

Floating point: relative L2 <= 1e-10 per window / cycle (the field alone:
k eps cond(M + kappa^-2 K), at least 1e-12); acceptance counts and tempering
steps: exact.  Sizes cover the
non-bordered tiles (one node per thread, odd chunk starts: nx = 100), ragged
tiles (nx = 600) and the full 4096-node tile."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import pairing as PR
from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06927_amd import sch as S

    S.lib()
    return S


def T(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _wl(nx, **kw):
    return W.MATERN_4096.scaled(nx=nx, **kw)


def _pair(sch, wl):
    return (O.matern(wl.kappa, wl.eta, wl.k_solves),
            sch.Matern(wl.kappa, wl.eta, wl.k_solves))


def _cells(wl, n, s, seed=None, step0=0):
    return O.draw_increments(wl.seed if seed is None else seed, n, s, wl.nx, step0,
                             O.TAG_FORECAST, 0, wl.dt)


@pytest.mark.parametrize("nx,kappa,eta,k", [
    (100, 1.0, 1.0, 3), (100, 30.0, 1.0, 1), (600, 0.5, 1.3, 2), (4096, 1.0, 1.0, 3),
])
def test_matern_field_parity(sch, nx, kappa, eta, k):
    # kappa = 30 at nx = 100 (h = 0.4) gives a positive off-diagonal h/6 - 1/(kappa^2 h)
    _say("matern field", nx, kappa, eta, k)
    wl = _wl(nx)
    gm = PR.gpu_model(wl)
    n = 3
    cells = _cells(wl, n, 1)[:, 0, :]
    ref = np.stack([O.matern_field(nx, wl.L, O.matern(kappa, eta, k), cells[p]) for p in range(n)])
    out = torch.zeros((n, nx), dtype=torch.float64, device="cuda")
    sch.sch_matern_field(gm, sch.Matern(kappa, eta, k), T(cells), out)
    # each solve may lose the condition number of M + kappa^-2 K, the ratio
    # of its largest eigenvalue (theta = pi: h/3 + 4 kappa^-2 / h) to its
    # smallest (theta = 0: h); the two sides round differently (scans on the
    # GPU, an LU in the oracle)
    h = wl.L / nx
    cond = (h / 3.0 + 4.0 / (kappa * kappa * h)) / h
    tol = max(1e-12, np.finfo(float).eps * k * cond)
    assert PR.rel_l2(N(out), ref) < tol


@pytest.mark.parametrize("nx,n,s", [(100, 5, 6), (600, 3, 5), (4096, 2, 4)])
def test_window_matern_parity(sch, nx, n, s):
    _say("matern window", nx, n, s)
    wl = _wl(nx, n_steps=s)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _pair(sch, wl)
    u0, m0, _, _ = PR.prior(wl, n)
    cells = _cells(wl, n, s)
    worst, m_ref, u_ref, _, it_ref = O.ensemble_window_matern(om, omt, m0, u0, cells)
    assert worst == 0
    m, u = T(m0), T(u0)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    iters = torch.zeros(n, dtype=torch.int32, device="cuda")
    sch.sch_ensemble_step_matern(gm, gmt, m, u, T(cells), status, iters)
    assert np.all(N(status) == 0)
    assert PR.rel_l2(N(m), m_ref) < PR.REL_TOL
    assert PR.rel_l2(N(u), u_ref) < PR.REL_TOL
    d = it_ref - N(iters)  # per step the oracle's change rule takes as many or one more
    assert d.min() >= -1 and d.max() <= s + 1


def test_window_matern_every_tile(sch):
    from paper_2402_06927_amd import autotune as A

    wl = _wl(2048, n_steps=4)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _pair(sch, wl)
    n = 2
    u0, m0, _, _ = PR.prior(wl, n)
    cells = _cells(wl, n, wl.n_steps)
    worst, m_ref, u_ref, _, _ = O.ensemble_window_matern(om, omt, m0, u0, cells)
    assert worst == 0
    try:
        for nt in A.candidates(wl.nx):
            _say("matern tile", nt)
            sch.sch_tune_set(sch.TUNE_THREADS, nt)
            m, u = T(m0), T(u0)
            sch.sch_ensemble_step_matern(gm, gmt, m, u, T(cells))
            assert PR.rel_l2(N(m), m_ref) < PR.REL_TOL, nt
            assert PR.rel_l2(N(u), u_ref) < PR.REL_TOL, nt
    finally:
        sch.sch_tune_set(sch.TUNE_THREADS, 0)


def test_window_matern_full_size_sampled(sch):
    """Nx = 4096, 1024 particles, 40 steps (the launch the Matern bench
    times); four particles recomputed by the oracle."""
    wl = W.MATERN_4096
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _pair(sch, wl)
    n = wl.n_particles
    u0 = W.initial_velocity(wl, n, wl.seed)
    gu = T(u0)
    gmm = torch.zeros_like(gu)
    sch.sch_init_momentum(gm, gu, gmm)
    cells = torch.zeros((n, wl.n_steps, wl.nx), dtype=torch.float64, device="cuda")
    sch.sch_draw_increments(wl.seed, 0, 0, sch.TAG_FORECAST, cells, wl.dt)
    status = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    sch.sch_ensemble_step_matern(gm, gmt, gmm, gu, cells, status)
    assert np.all(N(status) == 0)
    for p in (0, 1, 517, n - 1):
        _say("sampled particle", p)
        ref_cells = O.draw_increments_rows(wl.seed, p, 1, wl.n_steps, wl.nx, 0, O.TAG_FORECAST,
                                           0, wl.dt)[0]
        mr = O.momentum_from_velocity(om, u0[p])
        st, m_ref, u_ref, _ = O.window_matern(om, omt, mr, u0[p], ref_cells)
        assert st == 0
        assert PR.rel_l2(N(gmm[p]), m_ref) < PR.REL_TOL, p
        assert PR.rel_l2(N(gu[p]), u_ref) < PR.REL_TOL, p


def _jitter_setup(wl, n, theta):
    om = PR.oracle_model(wl)
    omt = O.matern(wl.kappa, wl.eta, wl.k_solves)
    u0, m0, ut, _ = PR.prior(wl, n)
    cells = _cells(wl, n, wl.n_steps)
    _, m1, u1, _, _ = O.ensemble_window_matern(om, omt, m0, u0, cells)
    y = O.observe(ut, wl.n_obs) + wl.sigma_obs * W.random_state_noise(wl.n_obs, 3)
    sig = np.full(wl.n_obs, wl.sigma_obs)
    phi = O.ensemble_nll(u1, y, sig)
    return om, omt, u0, m0, cells, m1, u1, y, sig, phi


@pytest.mark.parametrize("nx,n,s,theta", [(100, 7, 6, 0.4), (600, 5, 5, 1.0)])
def test_jitter_matern_parity(sch, nx, n, s, theta):
    _say("matern jitter", nx, n, s)
    wl = _wl(nx, n_steps=s, n_obs=40, sigma_obs=0.02)
    gm = PR.gpu_model(wl)
    gmt = sch.Matern(wl.kappa, wl.eta, wl.k_solves)
    om, omt, u0, m0, cells, m1, u1, y, sig, phi = _jitter_setup(wl, n, theta)
    ref = O.jitter_pcn_matern(om, omt, y, sig, wl.seed, 2, 3, m0, u0, cells, phi, m1, u1, theta,
                              0.9, 4)
    gc, gphi, gm1, gu1 = T(cells), T(phi), T(m1), T(u1)
    acc = torch.zeros(n, dtype=torch.int32, device="cuda")
    sch.sch_jitter_pcn_matern(gm, gmt, sch.Obs(T(y), T(sig)), wl.seed, 2, 3, T(m0), T(u0), gc,
                              gphi, gm1, gu1, T([theta]), 0.9, 4, acc)
    assert np.array_equal(N(acc), ref[4])
    assert 0 < ref[4].sum() < 4 * n
    assert PR.rel_l2(N(gc), ref[0]) < 1e-12
    assert PR.rel_l2(N(gphi), ref[1]) < PR.REL_TOL
    assert PR.rel_l2(N(gm1), ref[2]) < PR.REL_TOL and PR.rel_l2(N(gu1), ref[3]) < PR.REL_TOL


def _truth_obs(wl, n_cycles):
    """Twin-experiment observations from the oracle's Matern-noise truth run."""
    om = PR.oracle_model(wl)
    omt = O.matern(wl.kappa, wl.eta, wl.k_solves)
    _, _, ut, mt = PR.prior(wl, 1)
    z = W.obs_noise(wl, W.truth_seed(wl), n_cycles)
    ys = []
    for c in range(n_cycles):
        cells = _cells(wl, 1, wl.n_steps, seed=W.truth_seed(wl), step0=c * wl.n_steps)[0]
        st, mt, ut, _ = O.window_matern(om, omt, mt, ut, cells)
        assert st == 0
        ys.append(O.observe(ut, wl.n_obs) + wl.sigma_obs * z[c])
    return np.array(ys)


def test_tempered_cycle_matern_parity(sch):
    """The paper's grid (nx = 100, L = 40) with 40 particles, 5-step windows,
    40 observations, two cycles."""
    wl = _wl(100, n_particles=40, n_steps=5, n_obs=40, sigma_obs=0.05, n_cycles=2)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _pair(sch, wl)
    n = wl.n_particles
    u0, m0, _, _ = PR.prior(wl, n)
    ys = _truth_obs(wl, wl.n_cycles)
    sig = np.full(wl.n_obs, wl.sigma_obs)
    m_o, u_o = m0.copy(), u0.copy()
    m, u = T(m0), T(u0)
    ws = sch.matern_workspace(sch.WS_TEMPERED, gm, n, wl.n_steps, wl.n_jitter)
    for c in range(wl.n_cycles):
        _say("matern tempered cycle", c)
        rc, out, st_o = O.tempered_cycle_matern(om, omt, ys[c], sig, wl.seed, c, m_o, u_o,
                                                wl.n_steps, wl.ess_threshold, wl.n_bisect,
                                                wl.rho, wl.n_jitter, wl.max_temper)
        assert rc == 0
        m_o, u_o = out["m"], out["u"]
        st = sch.sch_pf_tempered_cycle_matern(gm, gmt, sch.Obs(T(ys[c]), T(sig)), wl.seed, c, m,
                                              u, wl.n_steps, wl.ess_threshold, wl.n_bisect,
                                              wl.rho, wl.n_jitter, wl.max_temper, ws)
        assert st["n_temper"] == st_o.n_temper and st_o.n_temper >= 2
        assert st["n_accept"] == st_o.n_accept
        assert PR.rel_l2(N(m), m_o) < PR.REL_TOL, c
        assert PR.rel_l2(N(u), u_o) < PR.REL_TOL, c


def test_matern_argument_errors(sch):
    wl = _wl(256)
    gm = PR.gpu_model(wl)
    cells = torch.zeros((1, 256), dtype=torch.float64, device="cuda")
    out = torch.zeros_like(cells)
    for bad in (sch.Matern(0.0, 1.0, 3), sch.Matern(-1.0, 1.0, 3), sch.Matern(1.0, 1.0, 0),
                sch.Matern(1.0, float("nan"), 3), sch.Matern(1.0, 1.0, 17)):
        with pytest.raises(sch.SchError):
            sch.sch_matern_field(gm, bad, cells, out)
    assert sch.lib().sch_matern_workspace_bytes(sch.WS_BOOTSTRAP, None, 4, 4, 1) == 0
