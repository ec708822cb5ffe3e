"""Warm-start network kernels (sch_mlp_*) versus the oracle's bfloat16-emulating
path (same rounding points, exact accumulation).  The GPU accumulates in
float32 on the matrix cores, so products agree to float32 accumulation error
and an occasional one-ulp bfloat16 flip of an activation: relative error
<= 1e-3 in norm and <= 1e-2 of the array's scale elementwise."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
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


def N(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 \
        else t.detach().cpu().numpy().astype(np.float64)


def net_on_gpu(sch, theta, dims):
    F, H, Oo = dims
    nw = H * F + H * H + Oo * H
    net = sch.Mlp(F, H, Oo, torch.tensor(theta, dtype=torch.float32, device="cuda"),
                  torch.empty(nw, dtype=torch.bfloat16, device="cuda"))
    sch.sch_mlp_sync(net)
    return net


def bf16_tensor(x):
    return torch.tensor(M.bf16(x), dtype=torch.float32, device="cuda").to(torch.bfloat16)


def close(a, b, norm=1e-3, elem=1e-2):
    scale = max(np.abs(b).max(), 1e-30)
    assert np.linalg.norm(a - b) <= norm * max(np.linalg.norm(b), 1e-30), \
        np.linalg.norm(a - b) / np.linalg.norm(b)
    assert np.abs(a - b).max() <= elem * scale, np.abs(a - b).max() / scale


# the first cases take the element-wise and register-prefetch products (K
# below, inside and past one 128-wide chunk); the fourth one's first layer
# (K = 2048) the products that load straight to LDS, over a ragged 200 rows;
# the fifth one (batch a multiple of 8, widths not) has the element-wise
# products of the backward pass write the transposed copies as well; in the
# sixth one (K = 1024 over the batch) the three weight gradients split K four
# ways on the register-prefetch loader, over a ragged 72-wide hidden layer;
# in the seventh one the first layer takes 128 x 128 tiles (16 x 5 of them,
# ragged both ways) with K = 2048 split 2 ways; in the last one the first
# layer's split product is 66 wide (ragged tiles of 64, split 8 ways)
CASES = [((100, 256, 40), 77), ((64, 32, 8), 5), ((300, 96, 50), 130), ((2048, 64, 24), 200),
         ((40, 36, 5), 64), ((96, 72, 20), 1024), ((2048, 520, 24), 2000), ((2048, 66, 24), 200)]


@pytest.mark.parametrize("dims,B", CASES)
def test_forward_backward_match_emulated(sch, dims, B):
    _say("mlp", dims, B)
    theta = W.mlp_init_params(*dims, 3) + 0.01 * np.random.default_rng(1).standard_normal(
        M.layout(*dims)[1])
    theta = M.f32(theta)
    g = np.random.default_rng(2)
    X = M.bf16(g.standard_normal((B, dims[0])))
    T = M.f32(g.standard_normal((B, dims[2])))
    net = net_on_gpu(sch, theta, dims)
    # the bfloat16 weight copy is the rounded master copy
    p = M.unpack(theta, *dims)
    wref = np.concatenate([M.bf16(p["W1"]).ravel(), M.bf16(p["W2"]).ravel(),
                           M.bf16(p["W3"]).ravel()])
    np.testing.assert_array_equal(N(net.weights_bf16), wref)
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, B), dtype=torch.uint8, device="cuda")
    Xg = bf16_tensor(X)
    Y = torch.empty((B, dims[2]), dtype=torch.float32, device="cuda")
    sch.sch_mlp_forward(net, Xg, Y, ws)
    Yr, _ = M.forward_bf16(theta, X, dims)
    close(N(Y), Yr)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(theta.size, dtype=torch.float32, device="cuda")
    sch.sch_mlp_backward(net, Xg, Y, torch.tensor(T, dtype=torch.float32, device="cuda"), loss,
                         grad, ws)
    lr_, gr = M.loss_grad_bf16(theta, X, T, dims)
    assert abs(N(loss)[0] - lr_) <= 1e-4 * lr_
    gg = N(grad)
    lay, _ = M.layout(*dims)
    for name, (off, shape) in lay.items():
        size = int(np.prod(shape))
        close(gg[off:off + size], gr[off:off + size], norm=3e-3, elem=3e-2)


def test_full_size_forward(sch):
    """The configured network 4352 -> 256 -> 256 -> 320 on 512 particles."""
    dims = (4352, 256, 320)
    theta = M.f32(W.mlp_init_params(*dims, 5))
    X = M.bf16(np.random.default_rng(4).standard_normal((512, dims[0])))
    net = net_on_gpu(sch, theta, dims)
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, 512), dtype=torch.uint8, device="cuda")
    Y = torch.empty((512, dims[2]), dtype=torch.float32, device="cuda")
    sch.sch_mlp_forward(net, bf16_tensor(X), Y, ws)
    Yr, _ = M.forward_bf16(theta, X, dims)
    close(N(Y), Yr)


def test_bench_shapes(sch):
    """The configured network at the benchmark's shapes: inference of 4096
    particles (the first layer on 128 x 128 tiles, K split 4 ways) and a
    training step's loss and gradient on 1024 rows (the first layer on
    64 x 64 tiles split 4 ways, the small weight gradients split on the
    register-prefetch loader)."""
    dims = (4352, 256, 320)
    theta = M.f32(W.mlp_init_params(*dims, 5))
    g = np.random.default_rng(4)
    X = M.bf16(g.standard_normal((4096, dims[0])))
    net = net_on_gpu(sch, theta, dims)
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, 4096), dtype=torch.uint8, device="cuda")
    Xg = bf16_tensor(X)
    Y = torch.empty((4096, dims[2]), dtype=torch.float32, device="cuda")
    _say("mlp inference 4096")
    sch.sch_mlp_forward(net, Xg, Y, ws)
    Yr, _ = M.forward_bf16(theta, X, dims)
    close(N(Y), Yr)
    B = 1024
    T = M.f32(g.standard_normal((B, dims[2])))
    Y1 = torch.empty((B, dims[2]), dtype=torch.float32, device="cuda")
    _say("mlp training step 1024")
    sch.sch_mlp_forward(net, Xg[:B], Y1, ws)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(theta.size, dtype=torch.float32, device="cuda")
    sch.sch_mlp_backward(net, Xg[:B], Y1, torch.tensor(T, dtype=torch.float32, device="cuda"),
                         loss, grad, ws)
    lr_, gr = M.loss_grad_bf16(theta, X[:B], T, dims)
    assert abs(N(loss)[0] - lr_) <= 1e-4 * lr_
    gg = N(grad)
    lay, _ = M.layout(*dims)
    for name, (off, shape) in lay.items():
        size = int(np.prod(shape))
        close(gg[off:off + size], gr[off:off + size], norm=3e-3, elem=3e-2)


def test_adam_matches_oracle(sch):
    dims = (40, 24, 6)
    theta = M.f32(W.mlp_init_params(*dims, 9))
    g = np.random.default_rng(3)
    net = net_on_gpu(sch, theta, dims)
    m = torch.zeros(theta.size, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    th, mo, vo = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for t in range(1, 6):
        grad = M.f32(g.standard_normal(theta.size) * 0.1)
        sch.sch_mlp_adam(net, torch.tensor(grad, dtype=torch.float32, device="cuda"), m, v, t,
                         lr=1e-2)
        th, mo, vo = M.adam(th, grad, mo, vo, t, lr=1e-2)
    np.testing.assert_allclose(N(net.params), th, rtol=1e-5, atol=1e-6)
    # float32 moments: rounding of terms of the gradient size (0.1 x 2^-24 per update)
    np.testing.assert_allclose(N(m), mo, rtol=1e-5, atol=5e-8)
    p = M.unpack(N(net.params), *dims)
    wref = np.concatenate([M.bf16(p["W1"]).ravel(), M.bf16(p["W2"]).ravel(),
                           M.bf16(p["W3"]).ravel()])
    np.testing.assert_array_equal(N(net.weights_bf16), wref)


def test_training_on_the_gpu_reduces_the_loss(sch):
    """Teacher-student regression with the GPU kernels: forward, backward and
    Adam steps cut the loss by an order of magnitude."""
    dims = (64, 64, 16)
    teacher = W.mlp_init_params(*dims, 100)
    g = np.random.default_rng(8)
    X = M.bf16(g.standard_normal((512, dims[0])))
    T, _ = M.forward_f64(teacher, X, dims)
    net = net_on_gpu(sch, M.f32(W.mlp_init_params(*dims, 1)), dims)
    B = 128
    ws = torch.empty(sch.sch_mlp_workspace_bytes(net, B), dtype=torch.uint8, device="cuda")
    Xg, Tg = bf16_tensor(X), torch.tensor(T, dtype=torch.float32, device="cuda")
    Y = torch.empty((B, dims[2]), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.zeros(net.params.numel(), dtype=torch.float32, device="cuda")
    m, v = torch.zeros_like(grad), torch.zeros_like(grad)
    losses = []
    step = 0
    for ep in range(150):
        tot = 0.0
        for s0 in range(0, 512, B):
            sch.sch_mlp_forward(net, Xg[s0:s0 + B], Y, ws)
            sch.sch_mlp_backward(net, Xg[s0:s0 + B], Y, Tg[s0:s0 + B], loss, grad, ws)
            step += 1
            sch.sch_mlp_adam(net, grad, m, v, step, lr=3e-3)
            tot += float(N(loss)[0])
        losses.append(tot / 4)
    _say("training loss", losses[0], losses[-1])
    assert losses[-1] < 0.1 * losses[0]


def test_features_scaling_and_controls(sch):
    wl = W.NUDGING_2048.scaled(nx=300, n_obs=40, n_modes=4, n_steps=5)
    from paper_2402_06927_amd import sch as S
    import pairing as PR

    n = 9
    u = W.initial_velocity(wl, n, 3)
    y = W.obs_noise(wl, 4, 1)[0] * 0.1
    gm = PR.gpu_model(wl)
    obs = S.Obs(torch.tensor(y, device="cuda"), torch.ones(wl.n_obs, dtype=torch.float64,
                                                           device="cuda"))
    F = wl.n_obs + wl.nx
    raw = torch.empty((n, F), dtype=torch.float32, device="cuda")
    mis = torch.empty(n, dtype=torch.float64, device="cuda")
    S.sch_mlp_features(gm, obs, torch.tensor(u, device="cuda"), None, None, None, raw, mis)
    pu = np.array([O.observe(u[p], wl.n_obs) for p in range(n)])
    ref = np.concatenate([y - pu, u], axis=1)
    np.testing.assert_allclose(N(raw), M.f32(ref), rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(N(mis), np.linalg.norm(y - pu, axis=1), rtol=1e-12)
    # column statistics and the scaled bfloat16 inputs
    mean = torch.empty(F, dtype=torch.float32, device="cuda")
    sdev = torch.empty_like(mean)
    S.sch_mlp_colstats(raw, mean, sdev)
    rr = N(raw)
    np.testing.assert_allclose(N(mean), rr.mean(axis=0), rtol=1e-5, atol=1e-7)
    sd = rr.std(axis=0)
    np.testing.assert_allclose(N(sdev), np.where(sd > 1e-12, sd, 1.0), rtol=1e-4, atol=1e-7)
    X = torch.empty((n, F), dtype=torch.bfloat16, device="cuda")
    S.sch_mlp_encode(raw, mean, sdev, X)
    X2 = torch.empty_like(X)
    S.sch_mlp_features(gm, obs, torch.tensor(u, device="cuda"), mean, sdev, X2, None, None)
    np.testing.assert_array_equal(N(X), N(X2))
    np.testing.assert_array_equal(N(X), M.bf16(M.f32((rr - N(mean)) / N(sdev))))
    # controls: denormalised outputs, zero where the misfit is above the threshold
    Oo = wl.n_steps * wl.n_modes
    Y = torch.tensor(np.random.default_rng(1).standard_normal((n, Oo)), dtype=torch.float32,
                     device="cuda")
    ym = torch.linspace(-1, 1, Oo, dtype=torch.float32, device="cuda")
    ys = torch.linspace(0.5, 2, Oo, dtype=torch.float32, device="cuda")
    dl = torch.empty((n, wl.n_steps, wl.n_modes), dtype=torch.float64, device="cuda")
    thr = float(np.median(N(mis)))
    mode = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    S.sch_mlp_controls(Y, ym, ys, mis, thr, dl, mode, S.NUDGE_FROM_GIVEN)
    expect = N(Y) * N(ys) + N(ym)
    expect[N(mis) > thr] = 0.0
    np.testing.assert_allclose(N(dl).reshape(n, Oo), expect, rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(
        N(mode), np.where(N(mis) > thr, S.NUDGE_FROM_ZERO, S.NUDGE_FROM_GIVEN))
