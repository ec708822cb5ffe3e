"""Learned warm start of nudging: trained on the GPU on plain-nudging
solutions, it must not change what nudging converges to (plain nudging
decides through its own stopping rule) and should save objective
evaluations; with the fallback forced for every particle it reduces to plain
nudging exactly."""
import sys

import numpy as np
import pytest

from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06927_amd import sch
    from paper_2402_06927_amd import warmstart as WS

    sch.lib()
    wl = W.NUDGING_2048.scaled(nx=256, n_particles=512, n_steps=10, n_obs=32)
    dev = "cuda"
    S, Q, nobs, npart = wl.n_steps, wl.n_modes, wl.n_obs, wl.n_particles
    xi = torch.tensor(W.mode_table(wl.L, wl.nx, Q, wl.mode_amp), device=dev)
    model = sch.Model(L=wl.L, alpha=wl.alpha, mu=wl.mu, dt=wl.dt, xi=xi)
    ts = W.truth_seed(wl)
    ut = torch.tensor(W.initial_velocity(wl, 1, ts), device=dev)
    mt = torch.empty_like(ut)
    sch.sch_init_momentum(model, ut, mt)
    u = torch.tensor(W.initial_velocity(wl, npart, wl.seed), device=dev)
    m = torch.empty_like(u)
    sch.sch_init_momentum(model, u, m)
    n_train = 8
    z = torch.tensor(W.obs_noise(wl, ts, n_train + 1), device=dev)
    sig = torch.full((nobs,), wl.sigma_obs, dtype=torch.float64, device=dev)

    def obs_for(c):
        dWt = torch.empty((1, S, Q), dtype=torch.float64, device=dev)
        sch.sch_draw_increments(ts, c, 0, sch.TAG_FORECAST, dWt, wl.dt)
        sch.sch_ensemble_step(model, mt, ut, dWt)
        y = torch.empty((1, nobs), dtype=torch.float64, device=dev)
        sch.sch_observe(model, ut, y)
        return sch.Obs((y[0] + wl.sigma_obs * z[c]).contiguous(), sig)

    ws = WS.WarmStart(nobs, wl.nx, S, Q)
    nws = sch.workspace(sch.WS_NUDGE, model, npart, S, 8)
    parts = []
    for c in range(n_train):
        obs = obs_for(c)
        dW = torch.empty((npart, S, Q), dtype=torch.float64, device=dev)
        sch.sch_draw_increments(wl.seed, c, 0, sch.TAG_NUDGE, dW, wl.dt)
        parts.append(ws.collect(model, obs, m, u, dW, nws))
    data = WS.concat(parts)
    ws.fit_scaling(data)
    X, T = ws.encode(data)
    hist = ws.train(X, T, epochs=40, batch=256, lr=1e-3)
    _say("warm-start training loss", hist[0], hist[-1])
    obs = obs_for(n_train)
    dW = torch.empty((npart, S, Q), dtype=torch.float64, device=dev)
    sch.sch_draw_increments(wl.seed, n_train, 0, sch.TAG_NUDGE, dW, wl.dt)
    return dict(sch=sch, ws=ws, model=model, obs=obs, m=m, u=u, dW=dW, nws=nws, hist=hist,
                npart=npart)


def _nudge(s, warm, threshold=None):
    sch, ws = s["sch"], s["ws"]
    mm, uu = s["m"].clone(), s["u"].clone()
    dl = torch.zeros_like(s["dW"])
    if warm:
        if threshold is not None:
            old, ws.threshold = ws.threshold, threshold
        ws.predict(s["model"], s["obs"], uu, dl)
        if threshold is not None:
            ws.threshold = old
    logG = torch.empty(s["npart"], dtype=torch.float64, device="cuda")
    ev = torch.empty(s["npart"], dtype=torch.int32, device="cuda")
    sch.sch_nudge_run(s["model"], s["obs"], mm, uu, s["dW"], dl, logG, warm_start=warm,
                      evals=ev, workspace=s["nws"])
    phi = torch.empty(s["npart"], dtype=torch.float64, device="cuda")
    sch.sch_loglik(s["model"], s["obs"], uu, phi)
    torch.cuda.synchronize()
    return dict(dl=dl.cpu().numpy(), u=uu.cpu().numpy(), phi=phi.cpu().numpy(),
                evals=ev.cpu().numpy(), logG=logG.cpu().numpy())


def test_training_learns(setup):
    h = setup["hist"]
    assert h[-1] < 0.5 * h[0]


def test_warm_start_saves_evaluations_at_equal_likelihood(setup):
    plain = _nudge(setup, False)
    warm = _nudge(setup, True)
    _say("evaluations per particle: plain", plain["evals"].mean(), "warm", warm["evals"].mean())
    _say("mean phi: plain", plain["phi"].mean(), "warm", warm["phi"].mean())
    assert abs(warm["phi"].mean() - plain["phi"].mean()) <= 0.01 * plain["phi"].mean()
    assert warm["evals"].mean() < plain["evals"].mean()


def test_fallback_everywhere_is_plain_nudging(setup):
    plain = _nudge(setup, False)
    fb = _nudge(setup, True, threshold=-1.0)
    np.testing.assert_array_equal(fb["dl"], plain["dl"])
    np.testing.assert_array_equal(fb["u"], plain["u"])
    np.testing.assert_array_equal(fb["evals"], plain["evals"])
