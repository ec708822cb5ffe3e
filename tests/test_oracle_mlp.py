"""Pins of the MLP oracle of the learned warm start: bfloat16 rounding (ties
to even), the float64 gradient against central differences, the
mixed-precision path against the float64 path, Adam's first step in closed
form, and descent of the loss on a regression the network can represent."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2402_06927_amd import workloads as W

DIMS = (7, 5, 3)


def test_bf16_round_to_nearest_even():
    one = 1.0
    assert M.bf16(one)[()] == 1.0
    # spacing at 1 is 2^-7: halfway points go to the even neighbour
    assert M.bf16(1 + 2 ** -8)[()] == 1.0
    assert M.bf16(1 + 3 * 2 ** -8)[()] == 1 + 2 ** -6
    assert M.bf16(1 + 2 ** -8 + 2 ** -20)[()] == 1 + 2 ** -7
    assert M.bf16(-(1 + 3 * 2 ** -8))[()] == -(1 + 2 ** -6)
    # representable values are fixed points; overflow gives infinity
    for v in (0.0, -0.0, 2.0 ** -130, 3.0, 0.15625, -1024.0):
        assert M.bf16(v)[()] == np.float32(v)
    assert np.isinf(M.bf16(3.4e38)[()])
    assert np.isnan(M.bf16(np.nan)[()])
    # bit patterns round-trip
    x = np.random.default_rng(0).standard_normal(1000)
    np.testing.assert_array_equal(M.from_bf16_bits(M.bf16_bits(x)), M.bf16(x))
    # relative error at most 2^-8
    assert np.all(np.abs(M.bf16(x) - np.float32(x)) <= 2.0 ** -8 * np.abs(np.float32(x)))


def _problem(B=4, dims=DIMS, seed=1):
    g = np.random.default_rng(seed)
    theta = W.mlp_init_params(*dims, seed) + 0.1 * g.standard_normal(M.layout(*dims)[1])
    X = g.standard_normal((B, dims[0]))
    T = g.standard_normal((B, dims[2]))
    return theta, X, T


def test_gradient_central_differences():
    theta, X, T = _problem()
    loss, g = M.loss_grad_f64(theta, X, T, DIMS)
    h = 1e-6
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.standard_normal(theta.shape)
        d /= np.linalg.norm(d)
        lp, _ = M.loss_grad_f64(theta + h * d, X, T, DIMS)
        lm, _ = M.loss_grad_f64(theta - h * d, X, T, DIMS)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(g @ d), np.abs(g).max())
    # every parameter block, one component each
    lay, _ = M.layout(*DIMS)
    for name, (off, _) in lay.items():
        e = np.zeros_like(theta)
        e[off] = 1.0
        lp, _ = M.loss_grad_f64(theta + h * e, X, T, DIMS)
        lm, _ = M.loss_grad_f64(theta - h * e, X, T, DIMS)
        assert (lp - lm) / (2 * h) == pytest.approx(g[off], rel=1e-6, abs=1e-9), name


def test_planted_wrong_gradient_is_caught():
    """A dropped ReLU mask in the backward pass fails the difference check."""
    theta, X, T = _problem(B=6, seed=5)
    p = M.unpack(theta, *DIMS)
    Y, (Z1, H1, Z2, H2) = M.forward_f64(theta, X, DIMS)
    B, O = Y.shape
    dY = 2 * (Y - T) / (B * O)
    dZ2_wrong = dY @ p["W3"]  # mask dropped
    gW2_wrong = dZ2_wrong.T @ H1
    _, g = M.loss_grad_f64(theta, X, T, DIMS)
    off, shape = M.layout(*DIMS)[0]["W2"]
    assert (Z2 <= 0).any()
    assert not np.allclose(gW2_wrong.ravel(), g[off:off + gW2_wrong.size])


def test_mixed_precision_tracks_float64():
    dims = (64, 32, 8)
    g = np.random.default_rng(7)
    theta = W.mlp_init_params(*dims, 7)
    X = g.standard_normal((50, 64))
    T = g.standard_normal((50, 8))
    Y64, _ = M.forward_f64(theta, X, dims)
    Yb, _ = M.forward_bf16(theta, X, dims)
    assert np.linalg.norm(Yb - Y64) <= 3e-2 * np.linalg.norm(Y64)
    l64, g64 = M.loss_grad_f64(theta, X, T, dims)
    lb, gb = M.loss_grad_bf16(theta, X, T, dims)
    assert abs(lb - l64) <= 3e-2 * l64
    assert np.linalg.norm(gb - g64) <= 5e-2 * np.linalg.norm(g64)


def test_adam_first_step_closed_form():
    theta, X, T = _problem()
    _, g = M.loss_grad_f64(theta, X, T, DIMS)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t1, m1, v1 = M.adam(theta, g, m, v, 1, lr=1e-3, eps=1e-8)
    np.testing.assert_allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_fits_a_representable_map():
    """Targets produced by a network of the same shape: Adam drives the loss
    down by orders of magnitude (float64 and mixed precision)."""
    dims = (16, 32, 4)
    g = np.random.default_rng(11)
    teacher = W.mlp_init_params(*dims, 100)
    X = g.standard_normal((256, 16))
    T, _ = M.forward_f64(teacher, X, dims)
    for grad_fn in (M.loss_grad_f64, M.loss_grad_bf16):
        theta = W.mlp_init_params(*dims, 3)
        m = np.zeros_like(theta)
        v = np.zeros_like(theta)
        l0, _ = grad_fn(theta, X, T, dims)
        for t in range(1, 801):
            loss, grad = grad_fn(theta, X, T, dims)
            theta, m, v = M.adam(theta, grad, m, v, t, lr=3e-3)
        assert loss < 0.05 * l0, (grad_fn.__name__, l0, loss)
