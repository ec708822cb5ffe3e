"""GPU nudged filter versus the oracle: the nudging of section 3.1.3 followed
by the tempering and jittering of section 3.1.2 with the weights W~ (last
paragraph of section 3.1.3), through the C-ABI.

Bars: pCN moves with fixed controls (sch_jitter_pcn with dLambda) match the
oracle's to relative L2 1e-10 in the potentials and states, with identical
acceptance decisions, at a ragged grid and at Nx = 4096 on the 256 x 16 tile.
The whole cycle (sch_pf_nudged_cycle) matches the oracle's at 1e-10 in the
no-data limit, where both optimisers keep the zero control exactly; with
data the L-BFGS controls agree to 1e-6 of their scale (the bar of the
nudging tests: two runs of the same optimiser can stop one step apart), so
the states are compared at 1e-6 and the tempering-step counts exactly."""
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


@pytest.mark.parametrize("nx,n,q,s,theta,tile", [(100, 8, 4, 6, 0.7, 0), (600, 6, 8, 5, 1.0, 0),
                                                 (4096, 16, 8, 40, 0.5, 256)])
def test_jitter_with_controls_parity(sch, nx, n, q, s, theta, tile):
    _say("jitter with controls", nx, n, q, s, theta, tile)
    wl = W.NUDGING_2048.scaled(nx=nx, n_modes=q, n_steps=s, n_obs=min(nx, 64), sigma_obs=0.05)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    u0, m0, ut, _ = PR.prior(wl, n)
    dW = O.draw_increments(wl.seed, n, s, q, 0, O.TAG_NUDGE, 0, wl.dt)
    rng = np.random.default_rng(nx + n)
    dLam = 0.3 * PR.sdt(wl) * rng.standard_normal(dW.shape)
    _, m1, u1, _, _ = O.ensemble_window(om, m0, u0, dW, dLam)
    y = O.observe(ut, wl.n_obs) + wl.sigma_obs * W.random_state_noise(wl.n_obs, 3)
    sig = np.full(wl.n_obs, wl.sigma_obs)
    phi = O.ensemble_nll(u1, y, sig)
    J = np.array([O.nudged_potential(phi[p], wl.dt, dW[p], dLam[p]) for p in range(n)])
    ref = O.jitter_pcn_ctrl(om, y, sig, wl.seed, 2, 3, m0, u0, dW, dLam, J, m1, u1, theta,
                            0.9, 4)
    if tile:
        sch.sch_tune_set(sch.TUNE_THREADS, tile)
    try:
        gdW, gJ, gm1, gu1 = T(dW), T(J), T(m1), T(u1)
        acc = torch.zeros(n, dtype=torch.int32, device="cuda")
        gl = T(dLam)
        sch.sch_jitter_pcn(gm, sch.Obs(T(y), T(sig)), wl.seed, 2, 3, T(m0), T(u0), gdW, gJ,
                           gm1, gu1, T([theta]), 0.9, 4, acc, dLambda=gl)
        acc, gdW, gJ, gm1, gu1 = N(acc), N(gdW), N(gJ), N(gm1), N(gu1)
    finally:
        if tile:
            sch.sch_tune_set(sch.TUNE_THREADS, 0)
    assert np.array_equal(acc, ref[4])
    assert 0 < ref[4].sum() < 4 * n
    assert PR.rel_l2(gdW, ref[0]) < 1e-12
    assert PR.rel_l2(gJ, ref[1]) < PR.REL_TOL
    assert PR.rel_l2(gm1, ref[2]) < PR.REL_TOL and PR.rel_l2(gu1, ref[3]) < PR.REL_TOL
    np.testing.assert_array_equal(N(gl), dLam)  # the controls are read only


def _cycle_inputs(wl):
    u0, m0, _, _ = PR.prior(wl, wl.n_particles)
    y = PR.oracle_observations(wl, 1)[0]
    return m0, u0, y


def _gpu_cycle(sch, wl, m0, u0, y, sigma, n_jitter=3):
    gm = PR.gpu_model(wl)
    n, s, q = wl.n_particles, wl.n_steps, wl.n_modes
    m, u = T(m0), T(u0)
    dl = torch.full((n, s, q), np.nan, dtype=torch.float64, device="cuda")
    ws = sch.nudged_workspace(gm, n, s, n_jitter, 4)
    obs = sch.Obs(T(y), T(np.full(wl.n_obs, sigma)))
    st = sch.sch_pf_nudged_cycle(gm, obs, wl.seed, 0, m, u, dl, s, n / 2, 50, 0.9, n_jitter,
                                 50, ws, ckpt_every=4)
    return st, N(m), N(u), N(dl)


def test_nudged_cycle_without_data(sch):
    """sigma -> infinity: both sides keep every control at exactly zero, so the
    cycle is the tempered cycle on the revealed increments: one tempering
    step, states at the 1e-10 bar."""
    wl = W.NUDGING_2048.scaled(nx=64, n_particles=12, n_modes=4, n_steps=6, n_obs=8)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    rc, ref, st_o = O.nudged_cycle(om, y, 1e7, wl.seed, 0, m0, u0, wl.n_steps,
                                   wl.n_particles / 2, 50, 0.9, 3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_cycle(sch, wl, m0, u0, y, 1e7)
    assert st["status"] == 0
    assert st["n_temper"] == st_o.n_temper == 1
    assert st["n_accept"] == st_o.n_accept
    np.testing.assert_array_equal(dl, 0.0)
    assert np.all(ref["dLam"] == 0.0)
    assert PR.rel_l2(m, ref["m"]) < PR.REL_TOL and PR.rel_l2(u, ref["u"]) < PR.REL_TOL


@pytest.mark.parametrize("nx,n,q,s", [(64, 16, 4, 6), (130, 10, 8, 5)])
def test_nudged_cycle_parity(sch, nx, n, q, s):
    _say("nudged cycle", nx, n, q, s)
    wl = W.NUDGING_2048.scaled(nx=nx, n_particles=n, n_modes=q, n_steps=s, n_obs=min(nx, 16),
                               sigma_obs=0.05)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    rc, ref, st_o = O.nudged_cycle(om, y, wl.sigma_obs, wl.seed, 0, m0, u0, s, n / 2, 50, 0.9,
                                   3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_cycle(sch, wl, m0, u0, y, wl.sigma_obs)
    assert st["status"] == 0
    _say("n_temper", st["n_temper"], st_o.n_temper, "accept", st["n_accept"], st_o.n_accept)
    assert st["n_temper"] == st_o.n_temper
    scale = np.abs(ref["dLam"]).max()
    assert scale > 0
    np.testing.assert_allclose(dl, ref["dLam"], rtol=0, atol=1e-6 * scale)
    assert PR.rel_l2(m, ref["m"]) < 1e-6 and PR.rel_l2(u, ref["u"]) < 1e-6


def test_nudged_cycle_argument_errors(sch):
    wl = W.NUDGING_2048.scaled(nx=64, n_particles=4, n_modes=4, n_steps=3, n_obs=8)
    gm = PR.gpu_model(wl)
    m0, u0, y = _cycle_inputs(wl)
    ws = sch.nudged_workspace(gm, 4, 3, 2, 4)
    obs = sch.Obs(T(y), T(np.full(wl.n_obs, 0.05)))
    with pytest.raises(sch.SchError) as e:
        sch.sch_pf_nudged_cycle(gm, obs, wl.seed, 0, T(m0), T(u0), None, 3, 2.0, 50, 0.9, 2, 50,
                                ws, ckpt_every=4)
    assert e.value.code == sch.SCH_E_ARG
    with pytest.raises(sch.SchError) as e:  # sized for checkpoints every 4 steps, not 8
        sch.sch_pf_nudged_cycle(gm, obs, wl.seed, 0, T(m0), T(u0),
                                torch.zeros((4, 3, 4), dtype=torch.float64, device="cuda"), 3,
                                2.0, 50, 0.9, 2, 50, ws, ckpt_every=8)
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError):
        sch.sch_pf_nudged_cycle(gm, obs, wl.seed, 0, T(m0), T(u0),
                                torch.zeros((4, 3, 4), dtype=torch.float64, device="cuda"), 3,
                                2.0, 50, 0.9, 2, 50, ws, ckpt_every=0)


def _gpu_cycle_warm(sch, wl, m0, u0, y, sigma, lam0, mode, n_jitter=3):
    gm = PR.gpu_model(wl)
    n, s = wl.n_particles, wl.n_steps
    m, u, dl = T(m0), T(u0), T(lam0)
    ws = sch.nudged_workspace(gm, n, s, n_jitter, 4)
    obs = sch.Obs(T(y), T(np.full(wl.n_obs, sigma)))
    st = sch.sch_pf_nudged_cycle_warm(gm, obs, wl.seed, 0, m, u, dl, T(mode, torch.int32), s,
                                      n / 2, 50, 0.9, n_jitter, 50, ws, ckpt_every=4)
    return st, N(m), N(u), N(dl)


def test_warm_cycle_keep_matches_at_the_tight_bar(sch):
    """Every particle KEEP: no optimiser runs on either side, so the nudged
    forecast is a deterministic window with increments plus the given controls
    and the whole cycle (tempering steps, acceptances, states) matches at the
    1e-10 bar; the final controls are rows of the given ones."""
    wl = W.NUDGING_2048.scaled(nx=130, n_particles=12, n_modes=8, n_steps=5, n_obs=16,
                               sigma_obs=0.05)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    lam0 = 0.02 * W.random_state_noise((wl.n_particles, wl.n_steps, wl.n_modes), 6)
    mode = np.full(wl.n_particles, sch.NUDGE_KEEP, dtype=np.int32)
    rc, ref, st_o = O.nudged_cycle_warm(om, y, wl.sigma_obs, wl.seed, 0, m0, u0, lam0, mode,
                                        wl.n_steps, wl.n_particles / 2, 50, 0.9, 3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_cycle_warm(sch, wl, m0, u0, y, wl.sigma_obs, lam0, mode)
    assert st["status"] == 0
    assert st["n_temper"] == st_o.n_temper and st["n_accept"] == st_o.n_accept
    np.testing.assert_array_equal(dl, ref["dLam"])
    assert PR.rel_l2(m, ref["m"]) < PR.REL_TOL and PR.rel_l2(u, ref["u"]) < PR.REL_TOL


@pytest.mark.parametrize("nx,n,q,s", [(64, 16, 4, 6), (130, 10, 8, 5)])
def test_warm_cycle_mixed_modes_parity(sch, nx, n, q, s):
    """A third of the particles KEEP their given controls, a third start
    their L-BFGS from them, a third nudge from zero (the fallback); bars of
    the plain nudged cycle."""
    _say("warm nudged cycle", nx, n, q, s)
    wl = W.NUDGING_2048.scaled(nx=nx, n_particles=n, n_modes=q, n_steps=s, n_obs=min(nx, 16),
                               sigma_obs=0.05)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    lam0 = 0.02 * W.random_state_noise((n, s, q), 7)
    mode = (np.arange(n) % 3).astype(np.int32)
    rc, ref, st_o = O.nudged_cycle_warm(om, y, wl.sigma_obs, wl.seed, 0, m0, u0, lam0, mode, s,
                                        n / 2, 50, 0.9, 3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_cycle_warm(sch, wl, m0, u0, y, wl.sigma_obs, lam0, mode)
    assert st["status"] == 0
    _say("n_temper", st["n_temper"], st_o.n_temper, "accept", st["n_accept"], st_o.n_accept)
    assert st["n_temper"] == st_o.n_temper
    scale = np.abs(ref["dLam"]).max()
    np.testing.assert_allclose(dl, ref["dLam"], rtol=0, atol=1e-6 * scale)
    assert PR.rel_l2(m, ref["m"]) < 1e-6 and PR.rel_l2(u, ref["u"]) < 1e-6
