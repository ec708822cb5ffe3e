"""Pin of the oracle's tempering loop (section 3.1.2: adaptive tempering,
resampling with the incremental weights, jittering at the new cumulative
temperature) against the Kalman filter.

Every tempered driver of the oracle (modes form, pCN-Langevin, Matern-type
noise, nudged) runs the same loop; `orc_tempered_cycle_linear` runs it with
the forward window replaced by a linear-Gaussian map (end state
e = F s + B xi, increments xi ~ N(0, dt) per entry, potential
Phi = |G e - y|^2 / (2 sigma^2)).  With those ingredients the exact filtering
law of the end state is the Kalman filter's Gaussian, written out below from
its textbook recursion, so the ensemble's mean and covariance must agree with
it within Monte Carlo error.  Two planted mistakes of the loop (a jitter that
targets the temperature before the step; resampling with the cumulative
temperature instead of its increment) are run through the same checks to show
that they fail them.
"""
import numpy as np
import pytest

DT = 0.025
N_STEPS, N_MODES = 2, 2


def _system():
    """A damped rotation observed through a full-rank map; B mixes the four
    increments into the two state components."""
    r = np.random.default_rng(7)
    th = 0.3
    F = 0.95 * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    B = r.normal(size=(2, N_STEPS * N_MODES))
    G = np.array([[1.0, 0.0], [0.5, 1.0]])
    return F, B, G


def _kalman(mu, P, F, B, G, y, sigma):
    """One forecast + analysis of the Kalman filter for x' = F x + B xi,
    xi ~ N(0, dt I), y = G x' + N(0, sigma^2 I)."""
    mp = F @ mu
    Pp = F @ P @ F.T + DT * (B @ B.T)
    S = G @ Pp @ G.T + sigma ** 2 * np.eye(len(y))
    K = np.linalg.solve(S, G @ Pp).T  # Pp G^T S^{-1} (S, Pp symmetric)
    return mp + K @ (y - G @ mp), (np.eye(len(mu)) - K @ G) @ Pp


def _run(orc, n, cycles, sigma, n_jitter, rho, plant):
    """The filter and the Kalman filter side by side; per cycle: the number
    of tempering steps, the mean error in units of the posterior standard
    deviation, and the eigenvalues of P^{-1} (ensemble covariance)."""
    F, B, G = _system()
    r = np.random.default_rng(11)
    mu = np.array([0.3, -0.2])
    P = np.array([[0.04, 0.01], [0.01, 0.02]])
    x = r.multivariate_normal(mu, P, size=n)
    truth = r.multivariate_normal(mu, P)
    out = []
    for c in range(cycles):
        truth = F @ truth + B @ (np.sqrt(DT) * r.normal(size=N_STEPS * N_MODES))
        y = G @ truth + sigma * r.normal(size=2)
        rc, x, st = orc.tempered_cycle_linear(F, B, G, y, sigma, DT, 99, c, x, N_STEPS, N_MODES,
                                              0.5 * n, rho=rho, n_jitter=n_jitter, plant=plant)
        assert rc == 0 and st.status == 0
        mu, P = _kalman(mu, P, F, B, G, y, sigma)
        dev = (x.mean(axis=0) - mu) / np.sqrt(np.diag(P))
        eig = np.linalg.eigvals(np.linalg.solve(P, np.cov(x.T))).real
        out.append((st.n_temper, dev, eig))
    return out


# Jittered filter: 4000 particles, 10 pCN moves of rho = 0.5 per tempering
# step, three cycles.  The moves mix the increments well, so the ensemble is
# close to an independent sample: mean error within 4 standard errors of
# 4000 draws, covariance within 10 % in every direction.
JIT = dict(n=4000, cycles=3, sigma=0.05, n_jitter=10, rho=0.5)


def _jittered_ok(out, n):
    return all(abs(d).max() <= 4.0 / np.sqrt(n) and 0.9 <= e.min() and e.max() <= 1.1
               for _, d, e in out)


def test_tempered_jittered_cycle_matches_kalman(orc):
    out = _run(orc, plant=orc.PLANT_NONE, **JIT)
    for k, d, e in out:
        print("tempering steps", k, "mean error / sd", d, "cov eigenvalue ratios", e)
        assert k >= 3  # several tempering steps: each part of the loop is exercised
    assert _jittered_ok(out, JIT["n"])


def test_jitter_at_the_old_temperature_fails_the_kalman_pin(orc):
    out = _run(orc, plant=orc.PLANT_JITTER_PRE_THETA, **JIT)
    assert not _jittered_ok(out, JIT["n"])
    # the last moves target exp(-theta_old Phi): the spread stays too wide
    assert max(e.max() for _, _, e in out) > 1.15


# Without jitter the cycle is tempered importance sampling: the ensemble is
# the forecast resampled K times with the incremental weights exp(-dtheta
# Phi), whose product is the full likelihood.  Each resampling keeps an ESS of
# at least half the ensemble, so the error bound counts n / 2^K independent
# draws; covariance within 15 %.
NOJIT = dict(n=20000, cycles=1, sigma=0.05, n_jitter=0, rho=0.5)


def _nojit_ok(out, n):
    k, d, e = out[0]
    return abs(d).max() <= 4.0 * np.sqrt(2.0 ** k / n) and 0.85 <= e.min() and e.max() <= 1.15


def test_tempered_resampling_alone_matches_kalman(orc):
    out = _run(orc, plant=orc.PLANT_NONE, **NOJIT)
    k, d, e = out[0]
    print("tempering steps", k, "mean error / sd", d, "cov eigenvalue ratios", e)
    assert k >= 3
    assert _nojit_ok(out, NOJIT["n"])


def test_cumulative_resampling_weights_fail_the_kalman_pin(orc):
    out = _run(orc, plant=orc.PLANT_CUMULATIVE_WEIGHTS, **NOJIT)
    assert not _nojit_ok(out, NOJIT["n"])
    # the weights multiply to exp(-(sum of cumulative thetas) Phi): too narrow
    assert out[0][2].max() < 0.8


@pytest.mark.parametrize("plant", [0, 1, 2])
def test_single_step_when_the_data_are_uninformative(orc, plant):
    """sigma -> large: the whole increment 1 passes the ESS test at once, so one
    tempering step, and the ensemble is the prior forecast (the Kalman gain
    vanishes)."""
    out = _run(orc, n=4000, cycles=1, sigma=1e6, n_jitter=5, rho=0.5, plant=plant)
    k, d, e = out[0]
    assert k == 1
    if plant != orc.PLANT_JITTER_PRE_THETA:
        assert abs(d).max() <= 4.0 / np.sqrt(4000) and 0.9 <= e.min() and e.max() <= 1.1
