"""Pins of the oracle's gradient-based jitter: the preconditioned
Crank-Nicolson Langevin move (pCNL; Cotter, Roberts, Stuart & White 2013),
the Metropolis-adjusted Langevin sampler in the form that keeps the N(0, dt)
prior of the increments invariant.  The paper names MALA/HMC jittering as
future work (section 5).

The acceptance ratio is pinned against Gaussian densities evaluated by
scipy (target exp(-theta Phi) N(0, dt I), proposal N(rho x - (1 - rho) dt
theta g(x), (1 - rho^2) dt I)) for an arbitrary drift, which also fixes its
antisymmetry; the linear-Gaussian toy chain with the exact gradient samples
the closed-form tempered posterior, mixes faster than pCN at the same rho
while its drift step (1 - rho) dt theta |H| stays below about 1 (and
overshoots beyond), and equals the pCN chain at theta = 0; on the SCH model the moves keep every
particle's end state and potential consistent with its final increments."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from paper_2402_06927_amd import workloads as W


def _log_target(x, phi, theta, dt):
    return -theta * phi + multivariate_normal(np.zeros(len(x)), dt * np.eye(len(x))).logpdf(x)


def _log_q(frm, to, g, theta, rho, dt):
    mean = rho * frm - (1 - rho) * dt * theta * g
    return multivariate_normal(mean, (1 - rho * rho) * dt * np.eye(len(frm))).logpdf(to)


def test_pcnl_ratio_is_metropolis_hastings(orc):
    rng = np.random.default_rng(3)
    d, dt = 6, 0.025
    for theta, rho in [(1.0, 0.9), (0.3, 0.5), (0.7, 0.99)]:
        x, v = rng.standard_normal(d) * 0.2, rng.standard_normal(d) * 0.2
        gx, gv = rng.standard_normal(d) * 5, rng.standard_normal(d) * 5
        px, pv = 3.7, 2.2
        want = (_log_target(v, pv, theta, dt) + _log_q(v, x, gv, theta, rho, dt)
                - _log_target(x, px, theta, dt) - _log_q(x, v, gx, theta, rho, dt))
        got = orc.pcnl_log_ratio(x, px, gx, v, pv, gv, theta, rho, dt)
        assert got == pytest.approx(want, rel=1e-10, abs=1e-10)
        back = orc.pcnl_log_ratio(v, pv, gv, x, px, gx, theta, rho, dt)
        assert back == pytest.approx(-got, rel=1e-12, abs=1e-12)


def _toy(d=4, n_obs=3, dt=0.025, sigma=0.05, theta=0.6, seed=0):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n_obs, d))
    y = rng.standard_normal(n_obs) * 0.1
    Sinv = np.eye(d) / dt + theta * G.T @ G / sigma ** 2
    S = np.linalg.inv(Sinv)
    mu = S @ (theta * G.T @ y / sigma ** 2)
    return G, y, S, mu


def test_pcnl_targets_tempered_gaussian_posterior(orc):
    d, dt, sigma, theta = 4, 0.025, 0.05, 0.6
    G, y, S, mu = _toy(d, 3, dt, sigma, theta)
    n_iter = 200000
    s, acc = orc.pcnl_linear_chain(21, 2, 2, G, y, sigma, theta, 0.9, dt, n_iter)
    x = s[10000:]
    assert 0.05 < acc / n_iter < 0.999
    nb = 100
    bm = x.reshape(nb, -1, d).mean(axis=1)
    se = bm.std(axis=0) / math.sqrt(nb)
    assert np.all(np.abs(x.mean(axis=0) - mu) < 5 * se + 1e-4)
    np.testing.assert_allclose(np.cov(x.T), S, rtol=0.1, atol=0.1 * np.abs(S).max())


@pytest.mark.parametrize("sigma,rho", [(0.2, 0.6), (0.05, 0.99)])
def test_pcnl_mixes_faster_than_pcn(orc, sigma, rho):
    # while the drift step (1 - rho) dt theta |H| (H the likelihood's Hessian)
    # stays below about 1, the Langevin drift moves the chain along the
    # likelihood: higher acceptance and a lower lag-1 autocorrelation in the
    # posterior's most constrained direction than pCN at the same rho
    d, dt, theta = 4, 0.025, 1.0
    G, y, S, mu = _toy(d, 3, dt, sigma, theta, seed=1)
    n_iter = 60000
    sl, al = orc.pcnl_linear_chain(7, 2, 2, G, y, sigma, theta, rho, dt, n_iter)
    sp, ap = orc.pcn_linear_chain(7, 2, 2, G, y, sigma, theta, rho, dt, n_iter)
    assert al > 1.15 * ap
    e = np.linalg.eigh(S)[1][:, 0]
    lag = lambda s: np.corrcoef((s[1000:] @ e)[:-1], (s[1000:] @ e)[1:])[0, 1]
    assert lag(sl) < lag(sp) - 0.1


def test_pcnl_overshoots_when_the_drift_step_is_large(orc):
    # (1 - rho) dt theta |H| = 11 here: the drift overshoots the mode and
    # the chain rejects almost everything (pCN's limit is the noise, not this)
    G, y, _, _ = _toy(4, 3, 0.025, 0.05, 1.0, seed=1)
    _, al = orc.pcnl_linear_chain(7, 2, 2, G, y, 0.05, 1.0, 0.6, 0.025, 20000)
    _, ap = orc.pcn_linear_chain(7, 2, 2, G, y, 0.05, 1.0, 0.6, 0.025, 20000)
    assert al < 0.2 * ap


def test_pcnl_is_pcn_at_theta_zero(orc):
    G, y, _, _ = _toy()
    a, acc_a = orc.pcnl_linear_chain(5, 2, 2, G, y, 0.05, 0.0, 0.8, 0.025, 3000)
    b, acc_b = orc.pcn_linear_chain(5, 2, 2, G, y, 0.05, 0.0, 0.8, 0.025, 3000)
    assert acc_b == 3000 and acc_a >= 2990
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)


def _model(orc, wl):
    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    return orc.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                     picard_tol=wl.picard_tol, picard_max=wl.picard_max)


def test_jitter_pcnl_consistency(orc):
    wl = W.TEMPERED_4096.scaled(nx=48, n_particles=6, n_modes=4, n_steps=5, n_obs=12,
                                sigma_obs=0.002)
    om = _model(orc, wl)
    n = wl.n_particles
    u0 = W.initial_velocity(wl, n, wl.seed)
    m0 = orc.momentum_from_velocity(om, u0)
    dW = orc.draw_increments(wl.seed, n, wl.n_steps, wl.n_modes, 0, orc.TAG_FORECAST, 0, wl.dt)
    _, m1, u1, _, _ = orc.ensemble_window(om, m0, u0, dW)
    ut = W.initial_velocity(wl, 1, W.truth_seed(wl))[0]
    y = orc.observe(ut, wl.n_obs)
    phi = orc.ensemble_nll(u1, y, wl.sigma_obs)
    dW2, phi2, me, ue, acc = orc.jitter_pcnl(om, y, wl.sigma_obs, 3, 1, 2, m0, u0, dW, phi, 1.0,
                                             0.9, 4)
    assert 0 < acc.sum() < 4 * n
    worst, mr, ur, _, _ = orc.ensemble_window(om, m0, u0, dW2)
    assert worst == 0
    np.testing.assert_array_equal(me, mr)
    np.testing.assert_array_equal(ue, ur)
    np.testing.assert_allclose(phi2, orc.ensemble_nll(ur, y, wl.sigma_obs), rtol=1e-12)
    for p in range(n):
        if acc[p] == 0:
            np.testing.assert_array_equal(dW2[p], dW[p])
            assert phi2[p] == phi[p]


def test_tempered_cycle_pcnl(orc):
    wl = W.TEMPERED_4096.scaled(nx=48, n_particles=10, n_modes=4, n_steps=5, n_obs=12,
                                sigma_obs=0.05)
    om = _model(orc, wl)
    u0 = W.initial_velocity(wl, wl.n_particles, wl.seed)
    m0 = orc.momentum_from_velocity(om, u0)
    ut = W.initial_velocity(wl, 1, W.truth_seed(wl))[0]
    y = orc.observe(ut, wl.n_obs)
    rc, m, u, st = orc.tempered_cycle_pcnl(om, y, wl.sigma_obs, 3, 0, m0, u0, wl.n_steps,
                                           wl.n_particles / 2, 50, 0.9, 3, 100)
    assert rc == 0 and st.n_temper >= 2 and st.n_accept > 0
    assert np.all(np.isfinite(u))
