"""Pins of the oracle's nudging with the Matern-type noise (section 3.1.3 with
the noise of section 2): the control is a DG0 field per step, entering the
load vector beside the white-noise cells (eq. "SCH nudge"), and the Girsanov
term sums over the cells.

The gradient's new part is the transpose of the Matern map, pinned by the
adjoint identity <T w, v> = <w, T^T v>; the whole gradient is checked against
central differences of the objective in random directions, reduces to the
Girsanov gradient (dLambda + dW)/dt when the observations carry no weight,
and nudging lowers the misfit (and leaves zero controls alone when the
observations carry no weight)."""
import numpy as np
import pytest

from paper_2402_06927_amd import workloads as W


@pytest.mark.parametrize("nx,L,kappa,eta,k", [(37, 5.0, 1.3, 0.7, 3), (100, 40.0, 1.0, 1.0, 3),
                                             (64, 40.0, 0.4, 1.0, 2)])
def test_matern_transpose_adjoint_identity(orc, nx, L, kappa, eta, k):
    rng = np.random.default_rng(nx)
    mt = orc.matern(kappa, eta, k)
    for _ in range(3):
        w, v = rng.standard_normal(nx), rng.standard_normal(nx)
        lhs = orc.matern_field(nx, L, mt, w) @ v
        rhs = w @ orc.matern_transpose(nx, L, mt, v)
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-15)


def _setup(orc, nx=24, n_steps=2, sigma=0.05, seed=3):
    wl = W.PAPER_SHAPE.scaled(nx=nx, n_steps=n_steps, n_obs=12, sigma_obs=sigma)
    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    om = orc.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                   picard_tol=1e-14, picard_max=200)
    u0 = orc.paper_init(nx, wl.L, wl.seed, 1)[0]
    m0 = orc.momentum_from_velocity(om, u0)
    ut = orc.paper_init(nx, wl.L, W.truth_seed(wl), 1)[0]
    y = orc.observe(ut, wl.n_obs)
    rng = np.random.default_rng(seed)
    dW = rng.standard_normal((n_steps, nx)) * np.sqrt(wl.dt)
    lam = rng.standard_normal((n_steps, nx)) * 0.05
    return wl, om, orc.matern(), m0, u0, y, dW, lam


def test_matern_nudge_gradient_central_differences(orc):
    wl, om, mt, m0, u0, y, dW, lam = _setup(orc)
    st, J, g = orc.nudge_grad_matern(om, mt, y, wl.sigma_obs, m0, u0, dW, lam)
    assert st == 0 and np.isfinite(J)
    rng = np.random.default_rng(9)
    for _ in range(4):
        d = rng.standard_normal(lam.shape)
        eps = 1e-6
        _, jp, _ = orc.nudge_grad_matern(om, mt, y, wl.sigma_obs, m0, u0, dW, lam + eps * d)
        _, jm, _ = orc.nudge_grad_matern(om, mt, y, wl.sigma_obs, m0, u0, dW, lam - eps * d)
        fd = (jp - jm) / (2 * eps)
        assert fd == pytest.approx(np.sum(g * d), rel=1e-6)


def test_matern_nudge_gradient_without_observation_weight(orc):
    wl, om, mt, m0, u0, y, dW, lam = _setup(orc, sigma=1e30)
    st, J, g = orc.nudge_grad_matern(om, mt, y, 1e30, m0, u0, dW, lam)
    assert st == 0
    np.testing.assert_allclose(g, (lam + dW) / wl.dt, rtol=1e-12, atol=1e-12)
    want = np.sum(0.5 * lam * lam + lam * dW) / wl.dt
    assert J == pytest.approx(want, rel=1e-12)


def test_matern_nudging_lowers_the_misfit(orc):
    wl, om, mt, m0, u0, y, dW, _ = _setup(orc, nx=32, n_steps=3)
    m0s, u0s = np.tile(m0, (2, 1)), np.tile(u0, (2, 1))
    dWs = np.stack([dW, -dW])
    r = orc.nudge_ensemble_matern(om, mt, y, wl.sigma_obs, m0s, u0s, dWs)
    assert r["worst"] == 0
    # the same window without controls
    cells = dWs
    worst, _, ue, _, _ = orc.ensemble_window_matern(om, mt, m0s, u0s, cells)
    assert worst == 0
    phi_plain = orc.ensemble_nll(ue, y, wl.sigma_obs)
    phi_nudged = orc.ensemble_nll(r["u"], y, wl.sigma_obs)
    assert np.all(phi_nudged < phi_plain)
    assert np.all(r["logG"] < 0) or np.all(np.abs(r["dLam"]) > 0)
    # no observation weight: the zero controls are optimal and stay
    r0 = orc.nudge_ensemble_matern(om, mt, y, 1e30, m0s, u0s, dWs)
    assert np.all(r0["dLam"] == 0.0) and np.all(r0["logG"] == 0.0)
