"""Pins of the oracle's nudging objective, its reverse-sweep adjoint, the
L-BFGS optimiser and the sequential adapted nudging scheme (section 3.1.3).

The reverse sweep (transposed solves, backwards in time) is checked against an
independent forward-mode derivative built from dense Jacobians and dense LU,
against central finite differences, by the Taylor remainder test, and in the
no-data limit where only the Girsanov term is left and the gradient has a
closed form.  L-BFGS is checked on problems with known minimisers and on the
real objective against scipy's BFGS."""
import numpy as np
import pytest
from scipy import optimize

from paper_2402_06927_amd import workloads as W

SMALL = W.NUDGING_2048.scaled(nx=32, n_particles=3, n_modes=4, n_steps=6, n_obs=8,
                              sigma_obs=0.05)


def _model(orc, wl):
    xi = W.mode_table(wl.L, wl.nx, wl.n_modes, wl.mode_amp)
    return orc.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi,
                     picard_tol=wl.picard_tol, picard_max=wl.picard_max)


def _problem(orc, wl, n=1, seed_shift=0):
    """State of n particles, a truth observed at the end of the window, noise
    increments and a random control of the size of the increments."""
    om = _model(orc, wl)
    u = W.initial_velocity(wl, n, wl.seed + seed_shift)
    m = orc.momentum_from_velocity(om, u)
    ut = W.initial_velocity(wl, 1, W.truth_seed(wl))[0]
    mt = orc.momentum_from_velocity(om, ut)
    dWt = orc.draw_increments(W.truth_seed(wl), 1, wl.n_steps, wl.n_modes, 0,
                              orc.TAG_FORECAST, 0, wl.dt)[0]
    st, mt, ut, _ = orc.window(om, mt, ut, dWt)
    assert st == 0
    z = W.obs_noise(wl, W.truth_seed(wl), 1)[0]
    y = orc.observe(ut, wl.n_obs) + wl.sigma_obs * z
    dW = orc.draw_increments(wl.seed, n, wl.n_steps, wl.n_modes, 0, orc.TAG_NUDGE, 0, wl.dt)
    rng = np.random.default_rng(11 + seed_shift)
    dLam = 0.5 * np.sqrt(wl.dt) * rng.standard_normal(dW.shape)
    return om, m, u, y, dW, dLam


def test_objective_is_likelihood_plus_girsanov(orc):
    wl = SMALL
    om, m, u, y, dW, dLam = _problem(orc, wl)
    st, J = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0])
    assert st == 0
    st, _, uN, _ = orc.window(om, m[0], u[0], dW[0], dLam[0])
    phi = orc.nll(uN, y, wl.sigma_obs)
    girs = np.sum(0.5 * dLam[0] ** 2 + dLam[0] * dW[0]) / wl.dt
    assert J == pytest.approx(phi + girs, rel=1e-14)
    # no control: J is the likelihood of the plain forecast
    st, J0 = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], None)
    st, _, uN0, _ = orc.window(om, m[0], u[0], dW[0])
    assert J0 == pytest.approx(orc.nll(uN0, y, wl.sigma_obs), rel=1e-14)


@pytest.mark.parametrize("nx,S,Q", [(32, 6, 4), (17, 3, 2), (48, 9, 8)])
def test_reverse_sweep_matches_dense_forward_mode(orc, nx, S, Q):
    wl = SMALL.scaled(nx=nx, n_steps=S, n_modes=Q)
    om, m, u, y, dW, dLam = _problem(orc, wl)
    st, J, g = orc.nudge_grad(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0])
    assert st == 0
    st, gt = orc.nudge_grad_tangent(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0])
    assert st == 0
    # the Girsanov part is common; compare the data part on its own scale too
    gir = (dLam[0] + dW[0]) / wl.dt
    np.testing.assert_allclose(g, gt, rtol=0, atol=1e-10 * np.abs(g).max())
    np.testing.assert_allclose(g - gir, gt - gir, rtol=0,
                               atol=1e-9 * np.abs(gt - gir).max())
    assert np.abs(g - gir).max() > 1e-3 * np.abs(gir).max()  # data term is not negligible


def test_central_differences(orc):
    wl = SMALL
    om, m, u, y, dW, dLam = _problem(orc, wl)
    st, J, g = orc.nudge_grad(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0])
    assert st == 0
    h = 1e-6
    rng = np.random.default_rng(5)
    for k in range(4):
        d = rng.standard_normal(dLam[0].shape)
        d /= np.linalg.norm(d)
        _, Jp = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] + h * d)
        _, Jm = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] - h * d)
        fd = (Jp - Jm) / (2 * h)
        ad = float(np.sum(g * d))
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), np.abs(g).max()), (k, fd, ad)
    # single components, including the first and the last step
    for (n, q) in [(0, 0), (wl.n_steps - 1, wl.n_modes - 1), (2, 1)]:
        e = np.zeros_like(dLam[0])
        e[n, q] = 1.0
        _, Jp = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] + h * e)
        _, Jm = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] - h * e)
        assert (Jp - Jm) / (2 * h) == pytest.approx(g[n, q], rel=1e-6, abs=1e-6 * np.abs(g).max())


def test_taylor_remainder_is_second_order(orc):
    wl = SMALL
    om, m, u, y, dW, dLam = _problem(orc, wl)
    st, J, g = orc.nudge_grad(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0])
    d = np.random.default_rng(9).standard_normal(dLam[0].shape) * np.sqrt(wl.dt)
    rem = []
    eps = [2.0 ** -k for k in range(2, 8)]
    for e in eps:
        _, Je = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] + e * d)
        rem.append(abs(Je - J - e * float(np.sum(g * d))))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.1), rates
    # with a wrong gradient the remainder is only first order
    gw = g.copy()
    gw[1, 0] += 0.1 * np.abs(g).max()
    remw = []
    for e in [2.0 ** -k for k in range(12, 15)]:
        _, Je = orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], dW[0], dLam[0] + e * d)
        remw.append(abs(Je - J - e * float(np.sum(gw * d))))
    ratew = np.log2(remw[-2] / remw[-1])
    assert abs(ratew - 1.0) < 0.2


def test_no_data_limit_gradient_is_girsanov_closed_form(orc):
    wl = SMALL
    om, m, u, y, dW, dLam = _problem(orc, wl)
    st, J, g = orc.nudge_grad(om, y, 1e30, m[0], u[0], dW[0], dLam[0])
    assert st == 0
    np.testing.assert_allclose(g, (dLam[0] + dW[0]) / wl.dt, rtol=1e-14, atol=0)
    assert J == pytest.approx(np.sum(0.5 * dLam[0] ** 2 + dLam[0] * dW[0]) / wl.dt, rel=1e-14)


def test_lbfgs_quadratic_and_rosenbrock(orc):
    rng = np.random.default_rng(3)
    B = rng.standard_normal((8, 8))
    A = B @ B.T + 8 * np.eye(8)
    b = rng.standard_normal(8)

    def quad(x):
        return 0, 0.5 * x @ A @ x - b @ x, A @ x - b

    st, x, f, it, ev = orc.lbfgs(quad, np.zeros(8), h0=0.1, gtol=1e-12, max_iter=100)
    assert st == 0
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    assert it <= 20

    def rosen(x):
        f = (1 - x[0]) ** 2 + 100 * (x[1] - x[0] ** 2) ** 2
        g = np.array([-2 * (1 - x[0]) - 400 * x[0] * (x[1] - x[0] ** 2),
                      200 * (x[1] - x[0] ** 2)])
        return 0, f, g

    st, x, f, it, ev = orc.lbfgs(rosen, np.array([-1.2, 1.0]), h0=1e-3, gtol=1e-10,
                                 max_iter=500)
    assert st == 0
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-8)
    # iteration cap and a failed line search report their status
    st, x, f, it, ev = orc.lbfgs(rosen, np.array([-1.2, 1.0]), h0=1e-3, gtol=1e-10, max_iter=3)
    assert st == 1 and it == 3

    def bad(x):
        return 0, float(np.sum(x)), np.full_like(x, -1.0)  # gradient points uphill

    st, x, f, it, ev = orc.lbfgs(bad, np.zeros(2), h0=1.0, max_back=5)
    assert st == 2 and it == 0 and ev == 1 + 6


def test_single_stage_optimum_matches_scipy(orc):
    """One step: the stage objective Phi(step(x)) + |x|^2/(2 dt) with zero
    increment; the scheme's control must be its minimiser."""
    wl = SMALL.scaled(n_steps=1)
    om, m, u, y, dW, dLam = _problem(orc, wl)
    res = orc.nudge_ensemble(om, y, wl.sigma_obs, m[:1], u[:1], dW[:1])
    assert res["worst"] == 0 and res["lbfgs_status"][0] == 0
    xs = res["dLam"][0, 0]
    zero = np.zeros((1, wl.n_modes))

    def f(x):
        return orc.nudge_objective(om, y, wl.sigma_obs, m[0], u[0], zero, x[None, :])[1]

    ref = optimize.minimize(f, np.zeros(wl.n_modes), method="Nelder-Mead",
                            options=dict(xatol=1e-12, fatol=1e-14, maxiter=20000,
                                         maxfev=40000))
    assert f(xs) <= ref.fun + 1e-10 * abs(ref.fun)
    np.testing.assert_allclose(xs, ref.x, atol=1e-5 * max(1.0, np.abs(ref.x).max()))
    st, J, g = orc.nudge_grad(om, y, wl.sigma_obs, m[0], u[0], zero, xs[None, :])
    assert np.abs(g).max() <= 1e-8 * (1 + abs(J))


def test_nudging_no_data_keeps_zero_control(orc):
    wl = SMALL
    om, m, u, y, dW, dLam = _problem(orc, wl, n=2)
    res = orc.nudge_ensemble(om, y, 1e30, m, u, dW, dLam0=dLam)
    assert res["worst"] == 0
    # from a nonzero warm start the optimiser returns to the prior's minimiser 0
    assert np.abs(res["dLam"]).max() <= 1e-8 * wl.dt * 10
    # and the state equals the plain forecast with the revealed increments
    st, mF, uF, _, _ = orc.ensemble_window(om, m, u, dW)
    np.testing.assert_allclose(res["u"], uF, rtol=0, atol=1e-10 * np.abs(uF).max())


def test_nudging_pulls_towards_observations(orc):
    wl = SMALL
    om, m, u, y, dW, _ = _problem(orc, wl, n=3)
    res = orc.nudge_ensemble(om, y, wl.sigma_obs, m, u, dW)
    assert res["worst"] == 0
    assert np.all(res["lbfgs_status"] <= 1)
    phi_n = orc.ensemble_nll(res["u"], y, wl.sigma_obs)
    _, _, uF, _, _ = orc.ensemble_window(om, m, u, dW)
    phi_f = orc.ensemble_nll(uF, y, wl.sigma_obs)
    assert np.all(phi_n < phi_f)
    # log Girsanov factor of the realised path
    lg = -np.sum(0.5 * res["dLam"] ** 2 + res["dLam"] * dW, axis=(1, 2)) / wl.dt
    np.testing.assert_allclose(res["logG"], lg, rtol=1e-13)
    # the nudged path stays a solution of the model with increments dW + dLam
    st, mW, uW, _, _ = orc.ensemble_window(om, m, u, dW + res["dLam"])
    np.testing.assert_allclose(res["u"], uW, rtol=0, atol=1e-12 * np.abs(uW).max())
