"""Pins of the oracle's linear algebra, P1 operators, Helmholtz relation and
implicit-midpoint step (section 2, eqs. sde1 and fde1) against things other
than itself: LAPACK solves, quadrature-assembled weak forms, circulant
eigenvalues, conservation laws the scheme satisfies exactly, symmetries and
convergence to the peakon travelling wave."""
import math

import numpy as np
import pytest

import fem_quadrature as fq
from paper_2402_06927_amd import workloads as W


def _model(orc, nx, n_modes=0, amp=0.05, L=40.0, alpha=1.0, mu=0.01, dt=0.025, tol=1e-13):
    xi = W.mode_table(L, nx, n_modes, amp) if n_modes else np.zeros((1, nx))
    return orc.Model(L=L, alpha=alpha, mu=mu, dt=dt, xi=xi, picard_tol=tol)


# ----------------------------------------------------------------------------- linear algebra
def test_tridiag_pivot_matches_lapack(orc):
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 7, 40):
        dl, d, du = rng.standard_normal(n - 1), rng.standard_normal(n) * 0.1, rng.standard_normal(n - 1)
        A = np.diag(d) + np.diag(dl, -1) + np.diag(du, 1)
        b = rng.standard_normal((2, n))
        st, x = orc.tridiag_pivot_solve(dl, d, du, b)
        assert st == 0
        ref = np.linalg.solve(A, b.T).T
        np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_tridiag_pivot_detects_singular(orc):
    st, _ = orc.tridiag_pivot_solve([0.0], [0.0, 1.0], [0.0], [1.0, 1.0])
    assert st == orc.ORC_E_SINGULAR


def test_cyclic_solve_matches_dense_lapack(orc):
    rng = np.random.default_rng(2)
    for n in (3, 4, 9, 64):
        a, b, c = rng.standard_normal(n), rng.standard_normal(n) + 4.0, rng.standard_normal(n)
        d = rng.standard_normal(n)
        A = np.zeros((n, n))
        for i in range(n):
            A[i, (i - 1) % n] += a[i]
            A[i, i] += b[i]
            A[i, (i + 1) % n] += c[i]
        st, x = orc.cyclic_solve(a, b, c, d)
        assert st == 0
        np.testing.assert_allclose(x, np.linalg.solve(A, d), rtol=1e-12, atol=1e-12)


def test_dense_solve_matches_lapack(orc):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 30))
    b = rng.standard_normal(30)
    st, x = orc.dense_solve(A, b)
    assert st == 0
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


# ----------------------------------------------------------------------------- operators
@pytest.mark.parametrize("nx", [5, 16, 101])
def test_operators_match_quadrature(orc, nx):
    L = 40.0
    rng = np.random.default_rng(nx)
    f, v = rng.standard_normal(nx), rng.standard_normal(nx)
    h = L / nx
    np.testing.assert_allclose(orc.apply_mass(h, f), fq.mass(L, f), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(orc.apply_stiff(h, f), fq.stiff(L, f), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.apply_advect(v, f), fq.advect(L, v, f), rtol=1e-12, atol=1e-12)


def test_advection_identities(orc):
    # v . C(v) f = 0 for any f (energy), and 1 . C(v) f = 1/2 sum f_i (v_{i+1} - v_{i-1})
    rng = np.random.default_rng(5)
    v, f = rng.standard_normal(64), rng.standard_normal(64)
    c = orc.apply_advect(v, f)
    assert abs(v @ c) < 1e-12 * np.abs(v).sum() * np.abs(f).sum()
    assert abs(c.sum() - 0.5 * f @ (np.roll(v, -1) - np.roll(v, 1))) < 1e-12 * np.abs(c).sum()


# ----------------------------------------------------------------------------- Helmholtz
@pytest.mark.parametrize("nx,k", [(64, 1), (64, 7), (256, 3), (4096, 5), (4096, 2047)])
def test_helmholtz_fourier_closed_form(orc, nx, k):
    """For m_i = cos(2 pi k i/nx) the circulant system H u = M m gives u = lam m,
    lam = Mhat/(Mhat + alpha^2 Khat), Mhat = h(2 + cos t)/3, Khat = 2(1 - cos t)/h."""
    md = _model(orc, nx)
    t = 2 * math.pi * k / nx
    m = np.cos(t * np.arange(nx))
    h = md.h
    mh, kh = h * (2 + math.cos(t)) / 3, 2 * (1 - math.cos(t)) / h
    lam = mh / (mh + md.alpha ** 2 * kh)
    u = orc.velocity_from_momentum(md, m)
    # forward error of a backward-stable solve: a few eps times cond(H),
    # cond(H) = (h/3 + 4 alpha^2/h) / h
    cond = (h / 3 + 4 * md.alpha ** 2 / h) / h
    np.testing.assert_allclose(u, lam * m, rtol=0, atol=20 * 2.2e-16 * cond * max(lam, 1e-3))


def test_helmholtz_residual_and_inverse(orc):
    md = _model(orc, 4096)
    rng = np.random.default_rng(7)
    m = rng.standard_normal(4096)
    u = orc.velocity_from_momentum(md, m)
    L = md.L
    res = fq.mass(L, u) + md.alpha ** 2 * fq.stiff(L, u) - fq.mass(L, m)
    assert np.linalg.norm(res) / np.linalg.norm(fq.mass(L, m)) < 1e-12
    m2 = orc.momentum_from_velocity(md, u)
    np.testing.assert_allclose(m2, m, rtol=0, atol=1e-9 * np.abs(m).max())


# ----------------------------------------------------------------------------- step
def _fde1_residuals(md, m0, u0, m1, u1, dW):
    """Residuals of the two lines of eq. fde1, assembled by quadrature."""
    L, dt, mu = md.L, md.dt, md.mu
    dU = md.xi.T @ dW if md.xi.shape[0] == len(dW) else 0.0
    dv = dt * 0.5 * (u0 + u1) + dU
    mh = 0.5 * (m0 + m1)
    r_mom = fq.mass(L, m1 - m0) + mu * dt * fq.stiff(L, mh) + fq.advect(L, dv, mh)
    r_helm = fq.mass(L, u1) + md.alpha ** 2 * fq.stiff(L, u1) - fq.mass(L, m1)
    scale = np.abs(fq.mass(L, m0)).max()
    # backward-error scale of the Helmholtz line: |H| |u| + |M| |m|
    h = md.h
    hnorm = h + 4 * md.alpha ** 2 / h
    scale_h = hnorm * np.abs(u1).max() + h * np.abs(m1).max()
    return np.abs(r_mom).max() / scale, np.abs(r_helm).max() / scale_h


@pytest.mark.parametrize("nx,n_modes", [(64, 4), (256, 4), (4096, 8)])
def test_step_solves_fde1(orc, nx, n_modes):
    """The returned pair satisfies the discrete equations to the Picard tolerance."""
    wl = W.BOOTSTRAP_256.scaled(nx=nx, n_modes=n_modes)
    md = _model(orc, nx, n_modes)
    u0 = W.initial_velocity(wl, 1, 11)[0]
    m0 = orc.momentum_from_velocity(md, u0)
    dW = W.random_state_noise(n_modes, 3) * math.sqrt(md.dt)
    st, m1, u1, it = orc.step(md, m0, u0, dW)
    assert st == 0 and 1 <= it < 20
    r1, r2 = _fde1_residuals(md, m0, u0, m1, u1, dW)
    assert r1 < 1e-11 and r2 < 1e-14


def test_linear_heat_closed_form(orc):
    """Tiny amplitude, no noise: every Fourier mode is multiplied per step by
    (Mhat - mu dt Khat/2)/(Mhat + mu dt Khat/2) (midpoint rule for M m' = -mu K m)."""
    nx, k = 128, 5
    md = _model(orc, nx, mu=0.3)
    t = 2 * math.pi * k / nx
    m0 = 1e-20 * np.cos(t * np.arange(nx))
    u0 = orc.velocity_from_momentum(md, m0)
    h, dt, mu = md.h, md.dt, md.mu
    mh, kh = h * (2 + math.cos(t)) / 3, 2 * (1 - math.cos(t)) / h
    g = (mh - 0.5 * mu * dt * kh) / (mh + 0.5 * mu * dt * kh)
    st, m, u, _ = orc.window(md, m0, u0, np.zeros((10, 1)))
    assert st == 0
    np.testing.assert_allclose(m, g ** 10 * m0, rtol=0, atol=1e-13 * 1e-20)


def _energy(md, m, u):
    return 0.5 * float(u @ orc_mass(md, m))


def orc_mass(md, f):
    return fq.mass(md.L, f)


def test_energy_conserved_inviscid_noise_free(orc):
    nx = 256
    md = _model(orc, nx, mu=0.0)
    wl = W.BOOTSTRAP_256
    u0 = W.initial_velocity(wl, 1, 21)[0]
    m0 = orc.momentum_from_velocity(md, u0)
    E0 = _energy(md, m0, u0)
    st, m, u, _ = orc.window(md, m0, u0, np.zeros((400, 1)))
    assert st == 0
    assert abs(_energy(md, m, u) - E0) / E0 < 1e-12


def test_energy_decays_with_viscosity(orc):
    nx = 256
    md = _model(orc, nx, mu=0.05)
    u = W.initial_velocity(W.BOOTSTRAP_256, 1, 22)[0]
    m = orc.momentum_from_velocity(md, u)
    E = _energy(md, m, u)
    for _ in range(20):
        st, m, u, _ = orc.step(md, m, u, np.zeros(1))
        assert st == 0
        E1 = _energy(md, m, u)
        assert E1 < E
        E = E1


def test_momentum_integral_conserved_noise_free(orc):
    """Without noise, 1^T M (m^{n+1} - m^n) = 0 at any mu: 1^T K = 0, and
    1^T C(dt u) s = (dt/2) s^T D u with D the central difference, which vanishes
    for s = 2 M^{-1} H u because M^{-1} H D is an antisymmetric circulant.
    With noise the integral is not conserved (the check below also shows it moves)."""
    nx = 256
    md = _model(orc, nx, mu=0.05)
    u = W.initial_velocity(W.BOOTSTRAP_256, 1, 23)[0]
    m = orc.momentum_from_velocity(md, u)
    I0 = md.h * m.sum()
    st, m1, _, _ = orc.window(md, m, u, np.zeros((30, 1)))
    assert st == 0
    assert abs(md.h * m1.sum() - I0) < 1e-12 * np.abs(md.h * m).sum()
    mdn = _model(orc, nx, 4, amp=0.3)
    dW = W.random_state_noise((30, 4), 4) * math.sqrt(md.dt)
    st, m2, _, _ = orc.window(mdn, m, u, dW)
    assert st == 0 and abs(md.h * m2.sum() - I0) > 1e-9


def test_shift_and_reflection_symmetry(orc):
    nx = 128
    md = _model(orc, nx)
    u = W.initial_velocity(W.BOOTSTRAP_256.scaled(nx=nx), 1, 24)[0]
    m = orc.momentum_from_velocity(md, u)
    z = np.zeros((8, 1))
    _, m1, u1, _ = orc.window(md, m, u, z)
    # one-node shift
    _, ms, us, _ = orc.window(md, np.roll(m, 1), np.roll(u, 1), z)
    np.testing.assert_allclose(ms, np.roll(m1, 1), rtol=0, atol=1e-13 * np.abs(m1).max())
    # x -> -x (node i -> -i), u -> -u, m -> -m
    rev = (-np.arange(nx)) % nx
    _, mr, ur, _ = orc.window(md, -m[rev], -u[rev], z)
    np.testing.assert_allclose(mr, -m1[rev], rtol=0, atol=1e-13 * np.abs(m1).max())
    np.testing.assert_allclose(ur, -u1[rev], rtol=0, atol=1e-13 * np.abs(u1).max())


def test_second_order_in_time(orc):
    nx = 128
    wl = W.BOOTSTRAP_256.scaled(nx=nx)
    u0 = W.initial_velocity(wl, 1, 25)[0]
    T = 0.4
    sols = []
    for n in (4, 8, 16, 32):
        md = _model(orc, nx, dt=T / n)
        m0 = orc.momentum_from_velocity(md, u0)
        st, m, u, _ = orc.window(md, m0, u0, np.zeros((n, 1)))
        assert st == 0
        sols.append(u)
    e1 = np.abs(sols[0] - sols[1]).max()
    e2 = np.abs(sols[1] - sols[2]).max()
    e3 = np.abs(sols[2] - sols[3]).max()
    assert 3.5 < e1 / e2 < 4.5 and 3.5 < e2 / e3 < 4.5


def _periodic_peakon(x, a, t, L, alpha):
    d = np.mod(x - a * t, L)
    return a * np.cosh((d - L / 2) / alpha) / np.cosh(L / (2 * alpha))


@pytest.mark.slow
def test_peakon_convergence(orc):
    """Noise-free inviscid single peakon u = a cosh((d - L/2)/alpha)/cosh(L/(2 alpha)),
    d = (x - a t) mod L (the periodic form of a e^{-|x - a t|/alpha}).  P1 does
    not resolve the kink exactly, so the pin is first-order convergence in h
    with dt proportional to h."""
    L, alpha, a, T = 40.0, 1.0, 0.2, 2.0
    errs = []
    for nx in (256, 512, 1024):
        h = L / nx
        n = int(round(T / (0.5 * h)))
        md = _model(orc, nx, mu=0.0, dt=T / n)
        x = np.arange(nx) * h
        u0 = _periodic_peakon(x, a, 0.0, L, alpha)
        m0 = orc.momentum_from_velocity(md, u0)
        st, m, u, _ = orc.window(md, m0, u0, np.zeros((n, 1)))
        assert st == 0
        exact = _periodic_peakon(x, a, T, L, alpha)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
        # the peak has moved by a*T to within two cells
        assert abs(x[np.argmax(u)] - a * T) <= 2 * h
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.01
    assert min(orders) > 1.0, (errs, orders)
