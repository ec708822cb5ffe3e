"""Pins of the oracle's parts of the paper's twin experiments (section 4): the
initial ensemble of eq. init_solve, the ensemble statistics EMRE, RB and RES,
and the half-domain observation of experiment 2 (points outside the observed
half carry an infinite error standard deviation, so they add nothing)."""
import math

import numpy as np
import pytest


def _gain(theta, h, k=3):
    # (M + K)^-1 applied k times with k - 1 mass products in between, on a
    # Fourier mode, with the load factor h/2 of the cell pair (kappa = 1)
    Mh = h * (2.0 + math.cos(theta)) / 3.0
    Ah = Mh + 2.0 * (1.0 - math.cos(theta)) / h
    return h * math.cos(theta / 2.0) * Mh ** (k - 1) / Ah ** k


def test_init_constant_cells(orc):
    # |W| = c everywhere: (M + K) U = h c 1 has U = c (rows of M sum to h, of
    # K to 0), and every later solve keeps it, so u = alpha^2 c + beta^2
    nx, L = 100, 40.0
    for c, a, b in [(0.7, 1.3, -0.4), (-2.0, 0.2, 1.1)]:
        u = orc.paper_init_from(nx, L, np.full(nx, c), a, b)
        np.testing.assert_allclose(u, a * a * abs(c) + b * b, rtol=1e-14)


@pytest.mark.parametrize("q", [1, 3, 17, 49])
def test_init_fourier_mode(orc, q):
    # W = c + d cos(theta (i + 1/2)) with c > |d| (so |W| = W): the constant
    # passes unchanged and the mode is multiplied by the three solves' factor
    nx, L = 100, 40.0
    h = L / nx
    theta = 2.0 * math.pi * q / nx
    i = np.arange(nx)
    c, d, a, b = 1.5, 0.8, 0.9, 0.3
    u = orc.paper_init_from(nx, L, c + d * np.cos(theta * (i + 0.5)), a, b)
    U3 = c + d * _gain(theta, h) * np.cos(theta * i)
    np.testing.assert_allclose(u, a * a * U3 + b * b, rtol=0, atol=1e-13)


def test_init_positive_and_mean(orc):
    # M + K is an M-matrix for h < sqrt(6) (negative off-diagonals) and M is
    # nonnegative, so U^{0,3} >= 0; its mean is that of |W|
    nx, L = 100, 40.0
    rng = np.random.default_rng(4)
    W = rng.standard_normal(nx) * math.sqrt(L / nx)
    a, b = 1.7, 0.6
    U3 = (orc.paper_init_from(nx, L, W, a, b) - b * b) / (a * a)
    assert U3.min() > 0
    assert U3.mean() == pytest.approx(np.abs(W).mean(), rel=1e-12)


def test_init_draws(orc):
    # the drawing form uses tag INIT: cells from the counter (p, 0, pair | tag << 24, 0)
    # with N(0, h) values, (alpha, beta) from (p, 1, tag << 24, 0)
    nx, L, seed = 100, 40.0, 99
    h = L / nx
    u = orc.paper_init(nx, L, seed, 3, p0=5)
    for r in range(3):
        p = 5 + r
        W = orc.draw_increments_rows(seed, p, 1, 1, nx, 0, orc.TAG_INIT, 0, h)[0, 0]
        ab = orc.normal_pair(seed, p, 1, orc.TAG_INIT << 24, 0)
        np.testing.assert_array_equal(u[r], orc.paper_init_from(nx, L, W, ab[0], ab[1]))
    assert np.all(u > 0)


def test_stats_hand_values(orc):
    # two particles mirrored about the truth: mean = truth
    ua = np.array([2.0, 1.0])
    u = np.array([[1.0, 2.0], [3.0, 0.0]])
    emre, rb, res = orc.ensemble_stats(u, ua)
    assert emre == pytest.approx(math.sqrt(2) / math.sqrt(5), rel=1e-15)
    assert rb == 0.0
    assert res == pytest.approx(2 * math.sqrt(2) / math.sqrt(5), rel=1e-15)
    # one particle: RB = EMRE, no spread
    emre, rb, res = orc.ensemble_stats(np.array([[3.0, 5.0]]), np.array([0.0, 1.0]))
    assert emre == pytest.approx(5.0, rel=1e-15) and rb == pytest.approx(5.0, rel=1e-15)
    assert res == 0.0
    # the whole ensemble on the truth
    assert np.all(orc.ensemble_stats(np.tile(ua, (4, 1)), ua) == 0.0)


def test_stats_structure(orc):
    # u_n = ua + d_n with sum d_n = 0: RB = 0, RES = N/(N-1) EMRE; a common
    # offset e moves RB to |e|/|ua|; scaling u and ua together changes nothing
    rng = np.random.default_rng(8)
    n, nx = 7, 50
    ua = rng.standard_normal(nx) + 2.0
    d = rng.standard_normal((n, nx))
    d -= d.mean(axis=0)
    emre, rb, res = orc.ensemble_stats(ua + d, ua)
    assert rb < 1e-15 and res == pytest.approx(n / (n - 1) * emre, rel=1e-13)
    e = np.full(nx, 0.3)
    _, rb2, res2 = orc.ensemble_stats(ua + d + e, ua)
    assert rb2 == pytest.approx(0.3 * math.sqrt(nx) / np.linalg.norm(ua), rel=1e-13)
    assert res2 == pytest.approx(res, rel=1e-13)
    np.testing.assert_allclose(orc.ensemble_stats(5.0 * (ua + d), 5.0 * ua), [emre, rb, res],
                               rtol=1e-13, atol=1e-15)


def test_half_domain_mask(orc):
    # experiment 2 observes the first 41 of the 80 full-domain points; the
    # others carry sigma = inf and equal their interpolated value's weight of
    # zero: the likelihood equals that of data matching the model there
    nx, n_obs = 100, 80
    rng = np.random.default_rng(2)
    u = rng.standard_normal(nx)
    y = rng.standard_normal(n_obs)
    sig = np.full(n_obs, math.sqrt(0.5))
    masked = sig.copy()
    masked[41:] = np.inf
    matched = y.copy()
    matched[41:] = orc.observe(u, n_obs)[41:]
    assert orc.nll(u, y, masked) == pytest.approx(orc.nll(u, matched, sig), rel=1e-15)
    assert orc.nll(u, y, masked) < orc.nll(u, y, sig)
