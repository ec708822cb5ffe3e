"""Pins of the oracle's RNG, observation operator, likelihood, ESS, adaptive
tempering, systematic resampling and pCN jittering (section 3) against
closed forms, invariants, brute force and a linear-Gaussian posterior.

Parity unpinned: the Philox4x32-10 bit stream itself (no known-answer vectors
are available here).  It is checked statistically below and must agree bit
for bit with the GPU library's independent implementation."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2402_06927_amd import workloads as W


# ----------------------------------------------------------------------------- RNG
def test_u01_exact_and_in_range(orc):
    assert orc.u01(0, 0) == 0.0
    assert orc.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u01(0x80000000, 0) == 0.5
    # the low 11 bits are dropped
    assert orc.u01(0, 0x7FF) == 0.0 and orc.u01(0, 0x800) == 2.0 ** -53


def test_philox_counters_and_keys_distinct(orc):
    seen = set()
    for ctr in ([0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]):
        for seed in (0, 1, 1 << 32):
            seen.add(tuple(orc.philox4x32_10(ctr, seed)))
    assert len(seen) == 15


def test_normals_statistics(orc):
    z = orc.draw_increments(7, 200, 50, 8, 0, orc.TAG_FORECAST, 0, 1.0).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / n)
    assert abs(stats.skew(z)) < 0.03 and abs(stats.kurtosis(z)) < 0.06
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # neighbouring modes and steps uncorrelated
    zz = orc.draw_increments(8, 400, 20, 2, 0, orc.TAG_FORECAST, 0, 1.0)
    c_mode = np.corrcoef(zz[:, :, 0].ravel(), zz[:, :, 1].ravel())[0, 1]
    c_step = np.corrcoef(zz[:, :-1, 0].ravel(), zz[:, 1:, 0].ravel())[0, 1]
    assert abs(c_mode) < 0.03 and abs(c_step) < 0.03


def test_increments_scaled_by_sqrt_dt(orc):
    a = orc.draw_increments(3, 4, 5, 6, 10, orc.TAG_FORECAST, 0, 1.0)
    b = orc.draw_increments(3, 4, 5, 6, 10, orc.TAG_FORECAST, 0, 0.025)
    np.testing.assert_allclose(b, a * math.sqrt(0.025), rtol=1e-15)
    c = orc.draw_increments(3, 4, 5, 6, 10, orc.TAG_PCN, 0, 1.0)
    assert not np.allclose(a, c)


# ----------------------------------------------------------------------------- observation
@pytest.mark.parametrize("nx,n_obs", [(256, 40), (4096, 256), (100, 81), (50, 7)])
def test_observe_is_p1_point_evaluation(orc, nx, n_obs):
    L = 40.0
    rng = np.random.default_rng(nx + n_obs)
    u = rng.standard_normal(nx)
    xn = np.arange(nx + 1) * (L / nx)
    xo = np.arange(n_obs) * (L / n_obs)
    ref = np.interp(xo, xn, np.append(u, u[0]))
    np.testing.assert_allclose(orc.observe(u, n_obs), ref, rtol=1e-13, atol=1e-13)


def test_nll_pins(orc):
    rng = np.random.default_rng(4)
    u = rng.standard_normal(256)
    y = orc.observe(u, 40)
    assert orc.nll(u, y, 0.05) == 0.0
    y2 = y.copy()
    y2[7] += 0.3
    assert orc.nll(u, y2, 0.05) == pytest.approx(0.5 * (0.3 / 0.05) ** 2, rel=1e-13)
    y3 = y + 0.01 * rng.standard_normal(40)
    assert orc.nll(u, y3, 0.025) == pytest.approx(4 * orc.nll(u, y3, 0.05), rel=1e-13)


# ----------------------------------------------------------------------------- weights / ESS
def test_ess_pins(orc):
    n = 64
    ess, w, lo = orc.weights(np.full(n, 3.7), 1.0)
    assert ess == pytest.approx(n, rel=1e-14)
    np.testing.assert_allclose(w, 1 / n, rtol=1e-14)
    phi = np.full(n, np.inf)
    phi[5] = 10.0
    ess, w, _ = orc.weights(phi, 0.5)
    assert ess == 1.0 and w[5] == 1.0 and w.sum() == 1.0
    # two-point closed form: weights (1, e^{-b d})
    d, b = 2.3, 0.7
    ess, w, _ = orc.weights(np.array([1.0, 1.0 + d]), b)
    e = math.exp(-b * d)
    assert ess == pytest.approx((1 + e) ** 2 / (1 + e * e), rel=1e-14)
    # shift invariance, log-weights, monotonicity in beta
    phi = W.random_phi(500, 1)
    e1, w1, lo1 = orc.weights(phi, 0.03)
    e2, w2, _ = orc.weights(phi + 1234.5, 0.03)
    assert e1 == pytest.approx(e2, rel=1e-12)
    np.testing.assert_allclose(np.exp(lo1), w1, rtol=1e-12)
    betas = np.linspace(0, 0.2, 41)
    ess_b = [orc.weights(phi, b)[0] for b in betas]
    assert all(ess_b[i + 1] <= ess_b[i] * (1 + 1e-12) for i in range(40))
    # carried log-weights combine with the tempered likelihood
    extra = np.random.default_rng(2).standard_normal(500)
    e3, w3, _ = orc.weights(phi, 0.03, extra)
    ref = np.exp(extra - 0.03 * phi - (extra - 0.03 * phi).max())
    np.testing.assert_allclose(w3, ref / ref.sum(), rtol=1e-12)


def test_temper_bisection_brackets_threshold(orc):
    phi = W.random_phi(1024, 3, scale=200.0)
    thr = 512.0
    dth, w, ess = orc.temper(phi, 0.0, thr, 50)
    assert 0 < dth < 1
    assert ess >= thr
    # one more bisection quantum (2^-50 of the remaining interval) fails
    e_next = orc.weights(phi, dth + 2.0 ** -50)[0]
    assert e_next < thr
    assert orc.weights(phi, dth)[0] == pytest.approx(ess, rel=1e-15)


def test_temper_sequence_reaches_one_exactly(orc):
    phi = W.random_phi(256, 5, scale=3.0)
    theta, k = 0.0, 0
    while theta < 1.0:
        dth, _, ess = orc.temper(phi, theta, 128.0, 50)
        theta = 1.0 if dth == 1.0 - theta else theta + dth
        k += 1
        assert k < 100
    assert theta == 1.0 and k > 2
    # no bisection needed when the full step keeps the ESS
    dth, _, _ = orc.temper(np.full(10, 1.0), 0.3, 5.0, 50)
    assert dth == 0.7


# ----------------------------------------------------------------------------- resampling
def _counts(idx, n):
    return np.bincount(idx, minlength=n)


def test_resample_brute_force_four_particles(orc):
    """For four particles, over a fine grid of u0: every particle is copied
    floor(N w) or ceil(N w) times, indices never decrease, and the mean count
    over u0 equals N w_p."""
    w = np.array([0.1, 0.45, 0.05, 0.4])
    n = 4
    grid = (np.arange(20000) + 0.5) / 20000
    total = np.zeros(n)
    for u0 in grid:
        st, idx = orc.resample_systematic(w, u0)
        assert st == 0
        assert np.all(np.diff(idx) >= 0)
        c = _counts(idx, n)
        assert np.all(c >= np.floor(n * w) - 1e-12) and np.all(c <= np.ceil(n * w) + 1e-12)
        total += c
    np.testing.assert_allclose(total / len(grid), n * w, atol=2e-4)


def test_resample_integer_form_equals_textbook_on_dyadic_weights(orc):
    rng = np.random.default_rng(11)
    for n in (4, 32, 1000):
        k = rng.integers(0, 64, n).astype(float)
        k[0] += 1
        w = k / k.sum()
        # make the weights exact dyadic rationals
        w = np.round(w * 2.0 ** 20) / 2.0 ** 20
        w[-1] = 1.0 - w[:-1].sum()
        for u0 in rng.random(20):
            _, a = orc.resample_systematic(w, u0)
            _, b = orc.resample_textbook(w, u0)
            assert np.array_equal(a, b), (n, u0)


def test_resample_degenerate_and_zero_weights(orc):
    st, _ = orc.resample_systematic(np.zeros(5), 0.3)
    assert st == orc.ORC_E_DEGENERATE
    w = np.array([0.0, 1.0, 0.0])
    st, idx = orc.resample_systematic(w, 0.99)
    assert st == 0 and np.all(idx == 1)
    st, _ = orc.resample_systematic(np.array([0.5, np.nan]), 0.3)
    assert st == orc.ORC_E_ARG


# ----------------------------------------------------------------------------- pCN
def test_pcn_accept_rule(orc):
    # min(1, exp(theta (phi_old - phi_new))): the paper's printed max() is read as min
    assert orc.pcn_accept(0.5, 10.0, 9.0, 0.999999)
    assert not orc.pcn_accept(0.5, 10.0, 12.0, math.exp(-1.0) + 1e-9)
    assert orc.pcn_accept(0.5, 10.0, 12.0, math.exp(-1.0) - 1e-9)
    assert not orc.pcn_accept(0.5, 10.0, np.inf, 0.0)
    assert orc.pcn_accept(0.0, 1.0, 1e300, 0.9)


def test_pcn_prior_preserved_at_theta_zero(orc):
    """At theta = 0 every proposal is accepted and the chain is an AR(1) with
    coefficient rho whose stationary law is the prior N(0, dt)."""
    rho, dt, n_iter = 0.8, 0.025, 20000
    G = np.zeros((1, 4))
    s, acc = orc.pcn_linear_chain(5, 2, 2, G, np.zeros(1), 1.0, 0.0, rho, dt, n_iter)
    assert acc == n_iter
    x = s[2000:, 0]
    assert abs(x.var() / dt - 1) < 0.1
    lag1 = np.corrcoef(x[:-1], x[1:])[0, 1]
    lag3 = np.corrcoef(x[:-3], x[3:])[0, 1]
    assert abs(lag1 - rho) < 0.03 and abs(lag3 - rho ** 3) < 0.04


def test_pcn_targets_tempered_gaussian_posterior(orc):
    """Linear forward map y = G x + N(0, sigma^2): the pCN chain with the
    Metropolis rule at temperature theta samples N(mu, S) with
    S^{-1} = I/dt + theta G^T G / sigma^2, mu = S theta G^T y / sigma^2."""
    rng = np.random.default_rng(0)
    d, n_obs, dt, sigma, theta = 4, 3, 0.025, 0.05, 0.6
    G = rng.standard_normal((n_obs, d))
    y = rng.standard_normal(n_obs) * 0.1
    Sinv = np.eye(d) / dt + theta * G.T @ G / sigma ** 2
    S = np.linalg.inv(Sinv)
    mu = S @ (theta * G.T @ y / sigma ** 2)
    s, acc = orc.pcn_linear_chain(21, 2, 2, G, y, sigma, theta, 0.9, dt, 400000)
    x = s[20000:]
    assert 0.05 < acc / 400000 < 0.95
    # batch-means error estimate
    nb = 100
    bm = x.reshape(nb, -1, d).mean(axis=1)
    se = bm.std(axis=0) / math.sqrt(nb)
    assert np.all(np.abs(x.mean(axis=0) - mu) < 5 * se + 1e-4)
    np.testing.assert_allclose(np.cov(x.T), S, rtol=0.15, atol=0.15 * np.abs(S).max())
