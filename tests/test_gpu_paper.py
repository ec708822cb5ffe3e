"""GPU (C-ABI) versus oracle for the paper's twin experiments (section 4): the
initial ensemble of eq. init_solve, the statistics EMRE / RB / RES, the
half-domain likelihood (sigma = inf off the observed half), the bootstrap
cycle with the Matern-type noise, and short runs of both experiments end to
end (truth, observations, filter, statistics per assimilation step).

Bars: relative L2 <= 1e-12 for the initial ensemble (well-conditioned solves
at h = 0.4) and the statistics, 1e-10 for states after cycles; decisions
(tempering steps, resampling) identical."""
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


@pytest.mark.parametrize("nx,n", [(100, 150), (600, 7), (4096, 3)])
def test_paper_init_parity(sch, nx, n):
    _say("paper init", nx, n)
    wl = W.PAPER_SHAPE.scaled(nx=nx)
    gm = PR.gpu_model(wl)
    u = torch.zeros((n, nx), dtype=torch.float64, device="cuda")
    sch.sch_paper_init(gm, 1234, u)
    ref = O.paper_init(nx, wl.L, 1234, n)
    h = wl.L / nx
    cond = (h / 3.0 + 4.0 / h) / h          # of M + K, as in the Matern field tests
    assert PR.rel_l2(N(u), ref) < max(1e-12, 3 * np.finfo(float).eps * cond)
    assert np.all(N(u) > 0)


@pytest.mark.parametrize("n,nx", [(150, 100), (1, 64), (1024, 4096), (7, 333)])
def test_ensemble_stats_parity(sch, n, nx):
    rng = np.random.default_rng(n + nx)
    ua = rng.standard_normal(nx) + 1.0
    u = ua + 0.3 * rng.standard_normal((n, nx))
    out = N(sch.sch_ensemble_stats(T(u), T(ua)))
    ref = O.ensemble_stats(u, ua)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-300)


def test_half_domain_loglik(sch):
    wl = W.PAPER_HALF
    gm = PR.gpu_model(wl)
    rng = np.random.default_rng(6)
    u = rng.standard_normal((5, wl.nx))
    y = rng.standard_normal(wl.n_obs)
    sig = W.sigma_vector(wl)
    assert np.isinf(sig[41:]).all() and np.isfinite(sig[:41]).all()
    phi = torch.zeros(5, dtype=torch.float64, device="cuda")
    sch.sch_loglik(gm, sch.Obs(T(y), T(sig)), T(u), phi)
    ref = O.ensemble_nll(u, y, sig)
    np.testing.assert_allclose(N(phi), ref, rtol=1e-13)


def test_bootstrap_cycle_matern_parity(sch):
    wl = W.PAPER_SHAPE.scaled(n_particles=40, sigma_obs=0.2)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = O.matern(), sch.Matern()
    n = wl.n_particles
    u0 = O.paper_init(wl.nx, wl.L, wl.seed, n)
    m0 = O.momentum_from_velocity(om, u0)
    ut = O.paper_init(wl.nx, wl.L, W.truth_seed(wl), 1)[0]
    y = O.observe(ut, wl.n_obs) + 0.2 * W.random_state_noise(wl.n_obs, 4)
    sig = np.full(wl.n_obs, 0.2)
    m_o, u_o, lw_o = m0.copy(), u0.copy(), np.zeros(n)
    m, u, lw = T(m0), T(u0), torch.zeros(n, dtype=torch.float64, device="cuda")
    ws = sch.matern_workspace(sch.WS_BOOTSTRAP, gm, n, wl.n_steps, 0)
    n_res = 0
    for c in range(3):
        _say("matern bootstrap cycle", c)
        rc, m_o, u_o, lw_o, st_o = O.bootstrap_cycle_matern(om, omt, y, sig, wl.seed, c, m_o, u_o,
                                                            lw_o, wl.n_steps, 0.5)
        assert rc == 0
        st = sch.sch_pf_bootstrap_cycle_matern(gm, gmt, sch.Obs(T(y), T(sig)), wl.seed, c, m, u,
                                               lw, wl.n_steps, 0.5, ws)
        assert st["resampled"] == st_o.resampled
        n_res += st["resampled"]
        assert PR.rel_l2(N(m), m_o) < PR.REL_TOL and PR.rel_l2(N(u), u_o) < PR.REL_TOL
        np.testing.assert_allclose(N(lw), lw_o, rtol=1e-9, atol=1e-9)
    assert n_res >= 1


def _oracle_twin(wl, filt, n_da):
    om = PR.oracle_model(wl)
    omt = O.matern(wl.kappa, wl.eta, wl.k_solves)
    n, nx, S = wl.n_particles, wl.nx, wl.n_steps
    u = O.paper_init(nx, wl.L, wl.seed, n)
    m = O.momentum_from_velocity(om, u)
    ts = W.truth_seed(wl)
    ut = O.paper_init(nx, wl.L, ts, 1)[0]
    mt = O.momentum_from_velocity(om, ut)
    z = W.obs_noise(wl, ts, n_da)
    sig = W.sigma_vector(wl)
    lw = np.zeros(n)
    rows = []
    for c in range(n_da):
        cells = O.draw_increments(ts, 1, S, nx, c * S, O.TAG_FORECAST, 0, wl.dt)[0]
        st, mt, ut, _ = O.window_matern(om, omt, mt, ut, cells)
        assert st == 0
        y = O.observe(ut, wl.n_obs) + wl.sigma_obs * z[c]
        if filt == "tempered":
            rc, out, so = O.tempered_cycle_matern(om, omt, y, sig, wl.seed, c, m, u, S,
                                                  wl.ess_threshold, wl.n_bisect, wl.rho,
                                                  wl.n_jitter, wl.max_temper)
            m, u = out["m"], out["u"]
            dec = so.n_temper
        elif filt == "nudged":
            rc, out, so = O.nudged_cycle_matern(om, omt, y, sig, wl.seed, c, m, u, S,
                                                wl.ess_threshold, wl.n_bisect, wl.rho,
                                                wl.n_jitter, wl.max_temper)
            m, u = out["m"], out["u"]
            dec = so.n_temper
        else:
            rc, m, u, lw, so = O.bootstrap_cycle_matern(om, omt, y, sig, wl.seed, c, m, u, lw, S,
                                                        wl.ess_frac)
            dec = so.resampled
        assert rc == 0
        rows.append((O.ensemble_stats(u, ut), dec))
    return rows, u, ut


@pytest.mark.parametrize("exp,filt", [(1, "tempered"), (2, "bootstrap"), (2, "tempered")])
def test_twin_experiment_parity(sch, exp, filt):
    """Three assimilation steps of the paper's experiments (nx = 100, L = 40,
    5 steps per observation, 80 points or the first 41 of them, sigma^2 = 0.5)
    with 40 particles."""
    from paper_2402_06927_amd import experiments as E

    _say("twin experiment", exp, filt)
    wl = (W.PAPER_SHAPE if exp == 1 else W.PAPER_HALF).scaled(n_particles=40)
    n_da = 3
    rows, u_o, ut_o = _oracle_twin(wl, filt, n_da)
    r = E.run_twin(wl, filt, n_da)
    assert PR.rel_l2(r["u_truth"], ut_o) < PR.REL_TOL
    assert PR.rel_l2(r["u"], u_o) < PR.REL_TOL
    for c, (s_o, dec) in enumerate(rows):
        np.testing.assert_allclose([r["emre"][c], r["rb"][c], r["res"][c]], s_o, rtol=1e-9)
        if filt == "tempered":
            assert r["n_temper"][c] == dec
        else:
            assert r["resampled"][c] == dec


def test_paper_init_errors(sch):
    wl = W.PAPER_SHAPE
    gm = PR.gpu_model(wl)
    with pytest.raises(sch.SchError):
        sch.sch_paper_init(gm, 1, torch.zeros((0, wl.nx), dtype=torch.float64, device="cuda"))
    assert sch.lib().sch_ensemble_stats(0, 10, None, None, None, None, None) != 0


@pytest.mark.parametrize("kind", ["bootstrap", "tempered", "tempered_matern",
                                  "bootstrap_matern"])
def test_failed_particle_gets_zero_weight(sch, kind):
    """A particle whose forecast fails (here: a non-finite start state) gets
    zero weight on both sides and is replaced by the resampling; the call
    succeeds and counts it."""
    matern = kind.endswith("matern")
    if matern:
        wl = W.PAPER_SHAPE.scaled(n_particles=24, sigma_obs=0.2)
        u0 = O.paper_init(wl.nx, wl.L, wl.seed, wl.n_particles)
        ut = O.paper_init(wl.nx, wl.L, W.truth_seed(wl), 1)[0]
    else:
        wl = W.BOOTSTRAP_256.scaled(n_particles=24, n_steps=5)
        u0, _, ut, _ = PR.prior(wl, wl.n_particles)
    _say("failed particle", kind)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    n = wl.n_particles
    m0 = O.momentum_from_velocity(om, u0)
    u0[3] = np.nan
    m0[3] = np.nan
    y = O.observe(ut, wl.n_obs) + wl.sigma_obs * W.random_state_noise(wl.n_obs, 9)
    sig = np.full(wl.n_obs, wl.sigma_obs)
    obs = sch.Obs(T(y), T(sig))
    m, u = T(m0), T(u0)
    omt, gmt = O.matern(), sch.Matern()
    if kind.startswith("bootstrap"):
        lw = torch.zeros(n, dtype=torch.float64, device="cuda")
        if matern:
            rc, m_o, u_o, _, st_o = O.bootstrap_cycle_matern(om, omt, y, sig, wl.seed, 0, m0, u0,
                                                             np.zeros(n), wl.n_steps, 1.01)
            ws = sch.matern_workspace(sch.WS_BOOTSTRAP, gm, n, wl.n_steps, 0)
            st = sch.sch_pf_bootstrap_cycle_matern(gm, gmt, obs, wl.seed, 0, m, u, lw,
                                                   wl.n_steps, 1.01, ws)
        else:
            rc, m_o, u_o, _, st_o = O.bootstrap_cycle(om, y, sig, wl.seed, 0, m0, u0,
                                                      np.zeros(n), wl.n_steps, 1.01)
            ws = sch.workspace(sch.WS_BOOTSTRAP, gm, n, wl.n_steps)
            st = sch.sch_pf_bootstrap_cycle(gm, obs, wl.seed, 0, m, u, lw, wl.n_steps, 1.01, ws)
        assert st["resampled"] == 1 == st_o.resampled
    else:
        if matern:
            rc, out, st_o = O.tempered_cycle_matern(om, omt, y, sig, wl.seed, 0, m0, u0,
                                                    wl.n_steps, n / 2, 50, 0.9, 3, 100)
            m_o, u_o = out["m"], out["u"]
            ws = sch.matern_workspace(sch.WS_TEMPERED, gm, n, wl.n_steps, 3)
            st = sch.sch_pf_tempered_cycle_matern(gm, gmt, obs, wl.seed, 0, m, u, wl.n_steps,
                                                  n / 2, 50, 0.9, 3, 100, ws)
        else:
            rc, m_o, u_o, st_o = O.tempered_cycle(om, y, sig, wl.seed, 0, m0, u0, wl.n_steps,
                                                  n / 2, 50, 0.9, 3, 100)
            ws = sch.workspace(sch.WS_TEMPERED, gm, n, wl.n_steps, 3)
            st = sch.sch_pf_tempered_cycle(gm, obs, wl.seed, 0, m, u, wl.n_steps, n / 2, 50,
                                           0.9, 3, 100, ws)
        assert st["n_temper"] == st_o.n_temper
    assert rc == 0 and st["status"] == 0 and st["n_failed"] == 1
    assert np.all(np.isfinite(u_o)) and np.all(np.isfinite(N(u)))
    assert PR.rel_l2(N(m), m_o) < PR.REL_TOL and PR.rel_l2(N(u), u_o) < PR.REL_TOL


def test_twin_experiment_nudged(sch):
    """Two assimilation steps of experiment 1 with the nudged filter (nudging
    with one control per cell, then tempering and jittering), 16 particles:
    equal tempering-step counts; states and statistics at the L-BFGS bar of
    the nudging tests (controls within 1e-6 of their scale)."""
    from paper_2402_06927_amd import experiments as E

    wl = W.PAPER_SHAPE.scaled(n_particles=16)
    n_da = 2
    rows, u_o, ut_o = _oracle_twin(wl, "nudged", n_da)
    r = E.run_twin(wl, "nudged", n_da)
    assert PR.rel_l2(r["u_truth"], ut_o) < PR.REL_TOL
    assert PR.rel_l2(r["u"], u_o) < 1e-6
    for c, (s_o, dec) in enumerate(rows):
        np.testing.assert_allclose([r["emre"][c], r["rb"][c], r["res"][c]], s_o, rtol=1e-5)
        assert r["n_temper"][c] == dec

