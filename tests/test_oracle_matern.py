"""Pins of the oracle's Matern-type noise (section 2, eqs. noise_solve and
noise_solve2): the DG0 white-noise increment Delta W_h (one N(0, dt) value per
cell, scaled by h^{-1/2}) is smoothed by k P1 elliptic solves with the operator
M + kappa^{-2} K.

On a uniform periodic grid every matrix in the construction is circulant, so
a discrete Fourier mode goes through it unchanged up to a factor: cell input
cos(theta (i + 1/2)) gives the load vector eta sqrt(h) cos(theta/2) cos(theta n),
and each solve multiplies by 1 / A(theta), each mass product by M(theta), with
M(theta) = h (2 + cos theta) / 3 and A(theta) = M(theta) + kappa^{-2} 2 (1 -
cos theta) / h.  Cosine and sine inputs at every frequency determine the linear
map, so the closed form pins it completely (a shifted load vector, a wrong
sign of the stiffness, a dropped sqrt(h) or eta, one solve too many or too
few each change the factor or the phase).  Independently, the mean is
conserved: the rows of K sum to zero and those of M to h, so
h sum_n Delta U_n = eta sqrt(h) sum_i Delta W_i for every kappa and k."""
import math

import numpy as np
import pytest

from paper_2402_06927_amd import workloads as W


def _gain(theta, h, kappa, eta, k):
    """Factor of the k solves on a Fourier mode, without the load vector's cos(theta/2)."""
    Mh = h * (2.0 + math.cos(theta)) / 3.0
    Ah = Mh + (2.0 * (1.0 - math.cos(theta)) / h) / kappa ** 2
    return eta * math.sqrt(h) * Mh ** (k - 1) / Ah ** k


@pytest.mark.parametrize("nx,L,kappa,eta,k", [
    (16, 40.0, 1.0, 1.0, 3),
    (100, 40.0, 1.0, 1.0, 3),
    (37, 5.0, 2.5, 0.7, 1),
    (64, 40.0, 0.3, 1.3, 2),
])
def test_matern_fourier_closed_form(orc, nx, L, kappa, eta, k):
    h = L / nx
    mt = orc.matern(kappa, eta, k)
    i = np.arange(nx)
    # rounding is relative to the largest gain (theta = 0: eta / sqrt(h)), not
    # to the attenuated high-frequency output
    g0 = _gain(0.0, h, kappa, eta, k)
    for q in sorted({0, 1, 2, nx // 3, nx // 2 - 1, nx // 2}):
        theta = 2.0 * math.pi * q / nx
        g = _gain(theta, h, kappa, eta, k)
        s = g * math.cos(theta / 2.0)    # zero at theta = pi: the load vector cancels
        for trig in (np.cos, np.sin):
            dU = orc.matern_field(nx, L, mt, trig(theta * (i + 0.5)))
            want = s * trig(theta * i)
            assert np.max(np.abs(dU - want)) <= 1e-13 * g0, (q, trig.__name__)
            assert abs(g) > 1e-9 * g0        # the mode is not attenuated below the bar


def test_matern_conserves_mean(orc):
    rng = np.random.default_rng(3)
    for nx, L, kappa, eta, k in [(50, 40.0, 1.0, 1.0, 3), (33, 7.0, 0.5, 2.0, 2)]:
        h = L / nx
        dWc = rng.standard_normal(nx) * 0.15
        dU = orc.matern_field(nx, L, orc.matern(kappa, eta, k), dWc)
        assert h * dU.sum() == pytest.approx(eta * math.sqrt(h) * dWc.sum(), rel=1e-12,
                                             abs=1e-14)


def test_matern_large_kappa_is_l2_projection(orc):
    # kappa^{-2} -> 0 with k = 1: Delta U is the L2 projection of Delta W_h onto
    # P1, i.e. M U = b; checked through the residual with a mass product built
    # here from the element integrals (h/6, 2h/3, h/6).
    nx, L = 24, 3.0
    h = L / nx
    rng = np.random.default_rng(5)
    dWc = rng.standard_normal(nx)
    dU = orc.matern_field(nx, L, orc.matern(1e9, 1.0, 1), dWc)
    MU = (h / 6.0) * (np.roll(dU, 1) + np.roll(dU, -1)) + (2.0 * h / 3.0) * dU
    b = math.sqrt(h) * 0.5 * (np.roll(dWc, 1) + dWc)
    assert np.max(np.abs(MU - b)) <= 1e-12 * np.max(np.abs(b))


def _model(orc, nx=32, n_modes=4, dt=0.025):
    wl = W.TEMPERED_4096.scaled(nx=nx, n_modes=n_modes, dt=dt)
    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    return wl, orc.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                         picard_tol=wl.picard_tol, picard_max=wl.picard_max)


def test_step_field_matches_modes_step(orc):
    # The modes form is the field form with Delta U = sum_q xi_q dW_q.
    wl, om = _model(orc)
    u = W.initial_velocity(wl, 1, wl.seed)[0]
    m = orc.momentum_from_velocity(om, u)
    dW = np.random.default_rng(1).standard_normal(wl.n_modes) * math.sqrt(wl.dt)
    st0, m0, u0, it0 = orc.step(om, m, u, dW)
    dU = np.zeros(wl.nx)
    for q in range(wl.n_modes):
        dU += om.xi[q] * dW[q]
    st1, m1, u1, it1 = orc.step_field(om, m, u, dU)
    assert st0 == st1 == 0 and it0 == it1
    np.testing.assert_allclose(m1, m0, rtol=0, atol=1e-15 * np.max(np.abs(m0)))
    np.testing.assert_allclose(u1, u0, rtol=0, atol=1e-15 * np.max(np.abs(u0)))


def test_window_matern_is_field_steps(orc):
    wl, om = _model(orc)
    mt = orc.matern(1.0, 1.0, 3)
    u = W.initial_velocity(wl, 1, wl.seed)[0]
    m = orc.momentum_from_velocity(om, u)
    dWc = orc.draw_increments(7, 1, 5, wl.nx, 0, orc.TAG_FORECAST, 0, wl.dt)[0]
    st, mw, uw, _ = orc.window_matern(om, mt, m, u, dWc)
    assert st == 0
    mm, uu = m.copy(), u.copy()
    for s in range(5):
        dU = orc.matern_field(wl.nx, wl.L, mt, dWc[s])
        st, mm, uu, _ = orc.step_field(om, mm, uu, dU)
        assert st == 0
    np.testing.assert_array_equal(mw, mm)
    np.testing.assert_array_equal(uw, uu)
    assert np.max(np.abs(uw - u)) > 1e-6   # the noise moved the state


def _cycle_setup(orc, nx=32, n=8, n_steps=6, n_obs=8, sigma=0.05):
    wl, om = _model(orc, nx=nx)
    wl = wl.scaled(n_particles=n, n_steps=n_steps, n_obs=n_obs, sigma_obs=sigma)
    u = W.initial_velocity(wl, n, wl.seed)
    m = orc.momentum_from_velocity(om, u)
    y = orc.observe(W.initial_velocity(wl, 1, W.truth_seed(wl))[0], n_obs)
    return wl, om, m, u, y


def test_tempered_cycle_matern_draw(orc):
    # Without jitter the window's cell increments are the FORECAST draw with
    # nx values per step, resampled as whole rows.
    wl, om, m, u, y = _cycle_setup(orc)
    mt = orc.matern()
    rc, out, st = orc.tempered_cycle_matern(om, mt, y, wl.sigma_obs, 11, 2, m, u, wl.n_steps,
                                            wl.ess_threshold, n_jitter=0, rho=wl.rho)
    assert rc == 0 and st.n_temper >= 1
    draw = orc.draw_increments(11, wl.n_particles, wl.n_steps, wl.nx, 2 * wl.n_steps,
                               orc.TAG_FORECAST, 0, wl.dt)
    for p in range(wl.n_particles):
        hit = [r for r in range(wl.n_particles) if np.array_equal(out["dWc"][p], draw[r])]
        assert hit, p
        np.testing.assert_array_equal(out["m0"][p], m[hit[0]])


def test_tempered_cycle_matern_consistency(orc):
    # Every particle's window end and potential follow from its window-start
    # state and its (jittered) increments.
    wl, om, m, u, y = _cycle_setup(orc)
    mt = orc.matern()
    rc, out, st = orc.tempered_cycle_matern(om, mt, y, wl.sigma_obs, 11, 0, m, u, wl.n_steps,
                                            wl.ess_threshold, n_jitter=4, rho=0.9)
    assert rc == 0 and st.n_temper >= 2 and st.n_accept > 0
    worst, me, ue, status, _ = orc.ensemble_window_matern(om, mt, out["m0"], out["u0"],
                                                          out["dWc"])
    assert worst == 0
    np.testing.assert_array_equal(me, out["m"])
    np.testing.assert_array_equal(ue, out["u"])
    np.testing.assert_allclose(out["phi"], orc.ensemble_nll(ue, y, wl.sigma_obs), rtol=1e-14)
    # the cell increments stay N(0, dt) under pCN (loose moment check)
    v = out["dWc"].ravel()
    assert abs(v.var() / wl.dt - 1.0) < 0.25


def test_bootstrap_cycle_matern(orc):
    # Without resampling (threshold 0) the cycle is the Matern window of the
    # FORECAST draw plus the likelihood weights; with threshold 1 it resamples.
    wl, om, m, u, y = _cycle_setup(orc)
    mt = orc.matern()
    n = wl.n_particles
    rc, m1, u1, lw, st = orc.bootstrap_cycle_matern(om, mt, y, wl.sigma_obs, 5, 3, m, u,
                                                    np.zeros(n), wl.n_steps, ess_frac=0.0)
    assert rc == 0 and st.resampled == 0
    cells = orc.draw_increments(5, n, wl.n_steps, wl.nx, 3 * wl.n_steps, orc.TAG_FORECAST, 0,
                                wl.dt)
    worst, me, ue, _, _ = orc.ensemble_window_matern(om, mt, m, u, cells)
    assert worst == 0
    np.testing.assert_array_equal(m1, me)
    np.testing.assert_array_equal(u1, ue)
    phi = orc.ensemble_nll(ue, y, wl.sigma_obs)
    w = np.exp(-(phi - phi.min()))
    np.testing.assert_allclose(np.exp(lw), w / w.sum(), rtol=1e-12, atol=1e-300)
    rc, m2, u2, lw2, st2 = orc.bootstrap_cycle_matern(om, mt, y, wl.sigma_obs, 5, 3, m, u,
                                                      np.zeros(n), wl.n_steps, ess_frac=1.01)
    assert rc == 0 and st2.resampled == 1 and np.all(lw2 == 0)
    for p in range(n):
        assert any(np.array_equal(u2[p], ue[r]) for r in range(n))
