"""GPU (C-ABI) versus oracle for nudging and the nudged filter with the
Matern-type noise (section 3.1.3 with the noise of section 2): one control per
cell and step, the objective's gradient through the transpose of the Matern
map, the stage-wise L-BFGS nudging with per-cell controls, the pCN moves of
the cells with the controls fixed, and the whole nudged cycle.

Bars as for the modes form: J and the gradient within relative L2 1e-10 of
the oracle's reverse sweep; the L-BFGS controls within 1e-6 of their scale
(two runs of one deterministic optimiser whose gradients differ by rounding
can stop one iteration apart), the window-end states within 1e-8 after
nudging and 1e-6 after a nudged cycle with data; the controlled moves with
identical acceptance decisions and potentials and states at 1e-10; the
no-data cycle at 1e-10."""
import sys
from dataclasses import replace

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


def _wl(nx, s, **kw):
    return replace(W.NUDGING_2048, noise="matern").scaled(nx=nx, n_steps=s,
                                                          n_obs=min(nx, 64), **kw)


def _problem(wl, n, ctrl_scale=0.2):
    """Prior particles, observations of the truth, revealed cell increments
    (tag NUDGE, nx per step) and a random per-cell control."""
    u, m, _, _ = PR.prior(wl, n)
    y = PR.oracle_observations(wl, 1)[0]
    dW = O.draw_increments(wl.seed, n, wl.n_steps, wl.nx, 0, O.TAG_NUDGE, 0, wl.dt)
    rng = np.random.default_rng(wl.nx + n)
    dLam = ctrl_scale * np.sqrt(wl.dt) * rng.standard_normal(dW.shape)
    return m, u, y, dW, dLam


def _mt(sch, wl):
    return O.matern(wl.kappa, wl.eta, wl.k_solves), sch.Matern(wl.kappa, wl.eta, wl.k_solves)


def _obs(sch, wl, y, sigma=None):
    s = wl.sigma_obs if sigma is None else sigma
    return sch.Obs(T(y), T(np.full(wl.n_obs, s)))


GRAD_CASES = [
    # nx, n, S, ckpt: several segments with a ragged last one, ragged node
    # chunks, one step per segment, full-row tiles of 8 and 16 nodes per thread
    (100, 3, 5, 2),
    (130, 2, 4, 8),
    (600, 2, 6, 4),
    (64, 2, 3, 1),
    (2048, 1, 5, 8),
    (4096, 1, 3, 2),
]


@pytest.mark.parametrize("nx,n,s,ce", GRAD_CASES)
def test_nudge_grad_matern_parity(sch, nx, n, s, ce):
    _say("nudge_grad_matern", nx, n, s, ce)
    wl = _wl(nx, s)
    m, u, y, dW, dLam = _problem(wl, n)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _mt(sch, wl)
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((n, s, nx), dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    sch.sch_nudge_grad_matern(gm, gmt, _obs(sch, wl, y), T(m), T(u), T(dW), T(dLam), J, g, ce,
                              st)
    assert np.all(N(st) == 0)
    Jg, gg = N(J), N(g)
    for p in range(n):
        rs, Jr, gr = O.nudge_grad_matern(om, omt, y, wl.sigma_obs, m[p], u[p], dW[p], dLam[p])
        assert rs == 0
        assert abs(Jg[p] - Jr) <= 1e-10 * abs(Jr)
        assert PR.rel_l2(gg[p], gr) < PR.REL_TOL, (p, PR.rel_l2(gg[p], gr))
        gir = (dLam[p] + dW[p]) / wl.dt
        # the data part alone (the transpose of the Matern map), on its own scale
        assert PR.rel_l2(gg[p] - gir, gr - gir) < 1e-9, (p, PR.rel_l2(gg[p] - gir, gr - gir))


def test_nudge_grad_matern_null_inputs_and_no_data(sch):
    wl = _wl(100, 4)
    n = 2
    m, u, y, dW, dLam = _problem(wl, n)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _mt(sch, wl)
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((n, wl.n_steps, wl.nx), dtype=torch.float64, device="cuda")
    # no increment and no control: J is the plain likelihood
    sch.sch_nudge_grad_matern(gm, gmt, _obs(sch, wl, y), T(m), T(u), None, None, J, g)
    zero = np.zeros_like(dW[0])
    for p in range(n):
        _, Jr, gr = O.nudge_grad_matern(om, omt, y, wl.sigma_obs, m[p], u[p], zero, None)
        assert abs(N(J)[p] - Jr) <= 1e-10 * abs(Jr)
        assert PR.rel_l2(N(g)[p], gr) < PR.REL_TOL
    # sigma -> infinity: only the Girsanov term is left
    sch.sch_nudge_grad_matern(gm, gmt, _obs(sch, wl, y, 1e30), T(m), T(u), T(dW), T(dLam), J, g)
    np.testing.assert_allclose(N(g), (dLam + dW) / wl.dt, rtol=1e-13, atol=0)
    np.testing.assert_allclose(N(J), np.sum(0.5 * dLam ** 2 + dLam * dW, axis=(1, 2)) / wl.dt,
                               rtol=1e-13)


def test_nudge_grad_matern_sampled_at_nx4096(sch):
    """64 particles at nx = 4096 (the Matern filter's row), 10 steps with
    checkpoints every 4: three particles checked against the oracle."""
    wl = _wl(4096, 10)
    n = 64
    _say("nudge_grad_matern sampled", wl.nx, n, wl.n_steps)
    m, u, y, dW, dLam = _problem(wl, n)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _mt(sch, wl)
    J = torch.empty(n, dtype=torch.float64, device="cuda")
    g = torch.empty((n, wl.n_steps, wl.nx), dtype=torch.float64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    sch.sch_nudge_grad_matern(gm, gmt, _obs(sch, wl, y), T(m), T(u), T(dW), T(dLam), J, g, 4, st)
    assert np.all(N(st) == 0)
    Jg, gg = N(J), N(g)
    for p in (0, 37, n - 1):
        _, Jr, gr = O.nudge_grad_matern(om, omt, y, wl.sigma_obs, m[p], u[p], dW[p], dLam[p])
        assert abs(Jg[p] - Jr) <= 1e-10 * abs(Jr)
        assert PR.rel_l2(gg[p], gr) < PR.REL_TOL


@pytest.mark.parametrize("nx,n,s,warm", [(64, 4, 3, False), (100, 3, 3, True)])
def test_nudge_run_matern_parity(sch, nx, n, s, warm):
    _say("nudge_run_matern", nx, n, s, warm)
    wl = _wl(nx, s)
    m, u, y, dW, dLam = _problem(wl, n, ctrl_scale=0.1)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _mt(sch, wl)
    ref = O.nudge_ensemble_matern(om, omt, y, wl.sigma_obs, m, u, dW,
                                  dLam0=dLam if warm else None)
    assert ref["worst"] == 0
    mg, ug = T(m), T(u)
    dl = T(dLam) if warm else torch.zeros((n, s, nx), dtype=torch.float64, device="cuda")
    logG = torch.empty(n, dtype=torch.float64, device="cuda")
    ls = torch.empty(n, dtype=torch.int32, device="cuda")
    its = torch.empty(n, dtype=torch.int32, device="cuda")
    evs = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    sch.sch_nudge_run_matern(gm, gmt, _obs(sch, wl, y), mg, ug, T(dW), dl, logG,
                             warm_start=warm, lbfgs_status=ls, iters=its, evals=evs, status=st)
    assert np.all(N(st) == 0)
    _say("iters", N(its), ref["iters"], "evals", N(evs), ref["evals"])
    np.testing.assert_array_equal(N(ls), ref["lbfgs_status"])
    scale = np.abs(ref["dLam"]).max()
    np.testing.assert_allclose(N(dl), ref["dLam"], rtol=0, atol=1e-6 * scale)
    np.testing.assert_allclose(N(logG), ref["logG"], rtol=1e-6, atol=1e-8)
    assert PR.rel_l2(N(ug), ref["u"]) < 1e-8
    assert PR.rel_l2(N(mg), ref["m"]) < 1e-8
    assert np.all(np.abs(N(its) - ref["iters"]) <= s)


def test_nudge_matern_argument_errors(sch):
    wl = _wl(64, 2)
    gm = PR.gpu_model(wl)
    n, s = 2, 2
    z = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    obs = sch.Obs(z(wl.n_obs) + 1.0, z(wl.n_obs) + 1.0)
    ws = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(sch.SchError):   # k = 0 solves
        sch.sch_nudge_grad_matern(gm, sch.Matern(1.0, 1.0, 0), obs, z(n, 64), z(n, 64), None,
                                  None, z(n), z(n, s, 64), 4, workspace=ws)
    with pytest.raises(sch.SchError):   # L-BFGS memory beyond 16 pairs
        sch.sch_nudge_run_matern(gm, sch.Matern(), obs, z(n, 64), z(n, 64), z(n, s, 64),
                                 z(n, s, 64), z(n), mem=17, workspace=ws)
    lib = sch.lib()
    mc = gm.c()
    import ctypes as C

    assert lib.sch_matern_workspace_bytes(sch.WS_NUDGE_GRAD, C.byref(mc), n, s, 0) == 0
    a = lib.sch_matern_workspace_bytes(sch.WS_NUDGE_GRAD, C.byref(mc), n, s, 4)
    b = lib.sch_matern_workspace_bytes(sch.WS_NUDGE, C.byref(mc), n, s, 4)
    assert 0 < a < b


@pytest.mark.parametrize("nx,n,s,theta", [(100, 8, 5, 0.7), (600, 6, 4, 1.0), (4096, 4, 6, 0.5)])
def test_jitter_matern_with_controls_parity(sch, nx, n, s, theta):
    """pCN moves of the cells with per-cell controls fixed: identical
    acceptance counts, cells at 1e-12, potentials and states at 1e-10."""
    _say("matern jitter with controls", nx, n, s, theta)
    wl = _wl(nx, s, sigma_obs=0.02)
    om, gm = PR.oracle_model(wl), PR.gpu_model(wl)
    omt, gmt = _mt(sch, wl)
    u0, m0, ut, _ = PR.prior(wl, n)
    dW = O.draw_increments(wl.seed, n, s, nx, 0, O.TAG_NUDGE, 0, wl.dt)
    dLam = 0.1 * np.sqrt(wl.dt) * np.random.default_rng(nx + n).standard_normal(dW.shape)
    worst, m1, u1, _, _ = O.ensemble_window_matern(om, omt, m0, u0, dW + dLam)
    assert worst == 0
    y = O.observe(ut, wl.n_obs) + wl.sigma_obs * W.random_state_noise(wl.n_obs, 3)
    sig = np.full(wl.n_obs, wl.sigma_obs)
    phi = O.ensemble_nll(u1, y, sig)
    J = np.array([O.nudged_potential(phi[p], wl.dt, dW[p], dLam[p]) for p in range(n)])
    ref = O.jitter_pcn_matern_ctrl(om, omt, y, sig, wl.seed, 2, 3, m0, u0, dW, dLam, J, m1, u1,
                                   theta, 0.95, 4)
    assert 0 < ref[4].sum() < 4 * n
    gdW, gJ, gm1, gu1, gl = T(dW), T(J), T(m1), T(u1), T(dLam)
    acc = torch.zeros(n, dtype=torch.int32, device="cuda")
    sch.sch_jitter_pcn_matern_ctrl(gm, gmt, sch.Obs(T(y), T(sig)), wl.seed, 2, 3, T(m0), T(u0),
                                   gdW, gl, gJ, gm1, gu1, T([theta]), 0.95, 4, acc)
    assert np.array_equal(N(acc), ref[4])
    assert PR.rel_l2(N(gdW), ref[0]) < 1e-12
    assert PR.rel_l2(N(gJ), ref[1]) < PR.REL_TOL
    assert PR.rel_l2(N(gm1), ref[2]) < PR.REL_TOL and PR.rel_l2(N(gu1), ref[3]) < PR.REL_TOL
    np.testing.assert_array_equal(N(gl), dLam)  # the controls are read only


def _gpu_nudged_cycle(sch, wl, m0, u0, y, sigma, n_jitter=3):
    gm = PR.gpu_model(wl)
    _, gmt = _mt(sch, wl)
    n, s = wl.n_particles, wl.n_steps
    m, u = T(m0), T(u0)
    dl = torch.full((n, s, wl.nx), np.nan, dtype=torch.float64, device="cuda")
    ws = sch.nudged_workspace_matern(gm, n, s, n_jitter, 4)
    obs = sch.Obs(T(y), T(np.full(wl.n_obs, sigma)))
    st = sch.sch_pf_nudged_cycle_matern(gm, gmt, obs, wl.seed, 0, m, u, dl, s, n / 2, 50, 0.9,
                                        n_jitter, 50, ws, ckpt_every=4)
    return st, N(m), N(u), N(dl)


def _cycle_inputs(wl):
    u0, m0, _, _ = PR.prior(wl, wl.n_particles)
    y = PR.oracle_observations(wl, 1)[0]
    return m0, u0, y


def test_nudged_cycle_matern_without_data(sch):
    """sigma -> infinity: both sides keep every control at exactly zero: one
    tempering step, states at the 1e-10 bar."""
    wl = _wl(64, 3, n_particles=12)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    omt, _ = _mt(sch, wl)
    rc, ref, st_o = O.nudged_cycle_matern(om, omt, y, 1e7, wl.seed, 0, m0, u0, wl.n_steps,
                                          wl.n_particles / 2, 50, 0.9, 3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_nudged_cycle(sch, wl, m0, u0, y, 1e7)
    assert st["status"] == 0
    assert st["n_temper"] == st_o.n_temper == 1
    assert st["n_accept"] == st_o.n_accept
    np.testing.assert_array_equal(dl, 0.0)
    assert np.all(ref["dLam"] == 0.0)
    assert PR.rel_l2(m, ref["m"]) < PR.REL_TOL and PR.rel_l2(u, ref["u"]) < PR.REL_TOL


@pytest.mark.parametrize("nx,n,s", [(64, 12, 3), (130, 8, 3)])
def test_nudged_cycle_matern_parity(sch, nx, n, s):
    _say("matern nudged cycle", nx, n, s)
    wl = _wl(nx, s, n_particles=n, sigma_obs=0.05)
    m0, u0, y = _cycle_inputs(wl)
    om = PR.oracle_model(wl)
    omt, _ = _mt(sch, wl)
    rc, ref, st_o = O.nudged_cycle_matern(om, omt, y, wl.sigma_obs, wl.seed, 0, m0, u0, s, n / 2,
                                          50, 0.9, 3, 50)
    assert rc == 0
    st, m, u, dl = _gpu_nudged_cycle(sch, wl, m0, u0, y, wl.sigma_obs)
    assert st["status"] == 0
    _say("n_temper", st["n_temper"], st_o.n_temper, "accept", st["n_accept"], st_o.n_accept)
    assert st["n_temper"] == st_o.n_temper
    scale = np.abs(ref["dLam"]).max()
    assert scale > 0
    np.testing.assert_allclose(dl, ref["dLam"], rtol=0, atol=1e-6 * scale)
    assert PR.rel_l2(m, ref["m"]) < 1e-6 and PR.rel_l2(u, ref["u"]) < 1e-6
