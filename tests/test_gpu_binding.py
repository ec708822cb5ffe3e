"""The Python binding refuses arrays whose shapes or workspace sizes do not
match the call before anything reaches the library: the kernels index the
caller's device arrays from the sizes passed, so a mismatch would otherwise
read or write outside them on the GPU."""
import numpy as np
import pytest

import pairing as PR
from paper_2402_06927_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_06927_amd import sch as S

    S.lib()
    return S


def z(*shape):
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def test_matern_nudged_cycle_rejects_modes_workspace_and_controls(sch):
    wl = W.NUDGING_MATERN_2048.scaled(nx=128, n_particles=4, n_modes=4, n_steps=3, n_obs=8)
    gm = PR.gpu_model(wl)
    n, s, nx, q = 4, 3, 128, 4
    obs = sch.Obs(z(8) + 1.0, z(8) + 1.0)
    mt = sch.Matern()
    ws_modes = sch.nudged_workspace(gm, n, s, 2, 4)        # sized for n_modes controls
    ws_cells = sch.nudged_workspace_matern(gm, n, s, 2, 4)
    assert ws_modes.numel() < ws_cells.numel()
    with pytest.raises(sch.SchError) as e:
        sch.sch_pf_nudged_cycle_matern(gm, mt, obs, 1, 0, z(n, nx), z(n, nx), z(n, s, nx), s,
                                       2.0, 50, 0.9, 2, 50, ws_modes, ckpt_every=4)
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError) as e:   # controls shaped for the modes form
        sch.sch_pf_nudged_cycle_matern(gm, mt, obs, 1, 0, z(n, nx), z(n, nx), z(n, s, q), s,
                                       2.0, 50, 0.9, 2, 50, ws_cells, ckpt_every=4)
    assert e.value.code == sch.SCH_E_SHAPE


def test_window_and_jitter_reject_mismatched_arrays(sch):
    wl = W.BOOTSTRAP_256.scaled(nx=256, n_modes=4)
    gm = PR.gpu_model(wl)
    n, s = 3, 5
    obs = sch.Obs(z(40) + 1.0, z(40) + 1.0)
    with pytest.raises(sch.SchError) as e:   # state rows of another grid
        sch.sch_ensemble_step(gm, z(n, 128), z(n, 128), z(n, s, 4))
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError) as e:   # increments with the wrong number of modes
        sch.sch_ensemble_step(gm, z(n, 256), z(n, 256), z(n, s, 8))
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError) as e:   # workspace for fewer moves than asked
        ws = sch.workspace(sch.WS_JITTER, gm, n, s, 1)
        sch.sch_jitter_pcn(gm, obs, 1, 0, 0, z(n, 256), z(n, 256), z(n, s, 4), z(n), z(n, 256),
                           z(n, 256), z(1), 0.9, 5, workspace=ws)
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError) as e:   # sigma and y of different lengths
        sch.sch_loglik(gm, sch.Obs(z(40), z(39)), z(n, 256), z(n))
    assert e.value.code == sch.SCH_E_SHAPE


def test_network_rejects_mismatched_batches(sch):
    F, H, O, B = 24, 16, 8, 5
    k = sch.sch_mlp_param_count(F, H, O)
    net = sch.Mlp(F, H, O, torch.zeros(k, dtype=torch.float32, device="cuda"),
                  torch.zeros(H * F + H * H + O * H, dtype=torch.bfloat16, device="cuda"))
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, B), dtype=torch.uint8, device="cuda")
    X = torch.zeros((B, F), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(sch.SchError) as e:
        sch.sch_mlp_forward(net, X, torch.zeros((B, O + 1), dtype=torch.float32, device="cuda"), ws)
    assert e.value.code == sch.SCH_E_SHAPE
    with pytest.raises(sch.SchError) as e:   # workspace for a smaller batch
        Xb = torch.zeros((4 * B, F), dtype=torch.bfloat16, device="cuda")
        sch.sch_mlp_forward(net, Xb, torch.zeros((4 * B, O), dtype=torch.float32, device="cuda"),
                            ws)
    assert e.value.code == sch.SCH_E_SHAPE


def test_window_and_jitter_are_bitwise_deterministic(sch):
    """Two runs of the forecast window and of the pCN jitter on the same inputs
    (headline grid and window, 32 particles, the benchmark's tile) give the
    same bits: no atomics or run-dependent orders in the kernels' arithmetic."""
    import oracle as O

    wl = W.TEMPERED_4096.scaled(n_particles=32)
    gm = PR.gpu_model(wl)
    n, s, q = 32, wl.n_steps, wl.n_modes
    u0, m0, ut, _ = PR.prior(wl, n)
    dW = O.draw_increments(wl.seed, n, s, q, 0, O.TAG_FORECAST, 0, wl.dt)
    y = O.observe(ut, wl.n_obs) + wl.sigma_obs * W.random_state_noise(wl.n_obs, 3)
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    obs = sch.Obs(T(y), T(np.full(wl.n_obs, wl.sigma_obs)))
    try:
        sch.sch_tune_set(sch.TUNE_THREADS, 256)
        runs = []
        for _ in range(2):
            m, u = T(m0), T(u0)
            sch.sch_ensemble_step(gm, m, u, T(dW))
            phi = torch.empty(n, dtype=torch.float64, device="cuda")
            sch.sch_loglik(gm, obs, u, phi)
            gdW, m1, u1 = T(dW), m.clone(), u.clone()
            acc = torch.zeros(n, dtype=torch.int32, device="cuda")
            sch.sch_jitter_pcn(gm, obs, wl.seed, 0, 0, T(m0), T(u0), gdW, phi, m1, u1, T([0.5]),
                               wl.rho, wl.n_jitter, acc)
            torch.cuda.synchronize()
            runs.append([t.cpu().numpy() for t in (m, u, phi, gdW, m1, u1, acc)])
        assert 0 < runs[0][-1].sum() < n * wl.n_jitter
        for a, b in zip(*runs):
            assert np.array_equal(a, b)
    finally:
        sch.sch_tune_set(sch.TUNE_THREADS, 0)


def test_network_products_are_bitwise_deterministic(sch):
    """Two forward and backward passes of the configured network (4096-row
    inference on 128 x 128 tiles with K split 4 ways, a 1024-row training step
    with split first layer and weight gradients) give the same outputs and
    gradients bit for bit: the split-K slices are summed in slice order and
    no product uses atomics.  (The loss sums its workgroups' shares with
    atomics, so it is compared to rounding.)"""
    F, H, O = 4352, 256, 320
    g = np.random.default_rng(7)
    k = sch.sch_mlp_param_count(F, H, O)
    theta = torch.tensor(W.mlp_init_params(F, H, O, 2), dtype=torch.float32, device="cuda")
    net = sch.Mlp(F, H, O, theta, torch.empty(H * F + H * H + O * H, dtype=torch.bfloat16,
                                              device="cuda"))
    sch.sch_mlp_sync(net)
    X = torch.tensor(g.standard_normal((4096, F)), dtype=torch.float32,
                     device="cuda").to(torch.bfloat16)
    T = torch.tensor(g.standard_normal((1024, O)), dtype=torch.float32, device="cuda")
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, 4096), dtype=torch.uint8, device="cuda")
    runs = []
    for _ in range(2):
        Y = torch.empty((4096, O), dtype=torch.float32, device="cuda")
        sch.sch_mlp_forward(net, X, Y, ws)
        Y1 = torch.empty((1024, O), dtype=torch.float32, device="cuda")
        sch.sch_mlp_forward(net, X[:1024], Y1, ws)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        grad = torch.zeros(k, dtype=torch.float32, device="cuda")
        sch.sch_mlp_backward(net, X[:1024], Y1, T, loss, grad, ws)
        torch.cuda.synchronize()
        runs.append([t.cpu().numpy() for t in (Y, Y1, grad, loss)])
    for a, b in zip(runs[0][:3], runs[1][:3]):
        assert np.array_equal(a, b)
    np.testing.assert_allclose(runs[0][3], runs[1][3], rtol=1e-12, atol=0)
