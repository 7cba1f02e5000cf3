"""Pins of the FP64 surrogate-network reference: backward against central
finite differences of the loss (brute force), SiLU derivative against its
closed form at known points, and Adam's first step against its closed form
(a step of exactly lr * sign(g) when eps is negligible)."""
import numpy as np

from oracle import mlp_ref as M


def test_silu_closed_form():
    z = np.array([0.0, 1.0, -2.0])
    np.testing.assert_allclose(M.silu(z), z / (1 + np.exp(-z)), rtol=0)
    assert M.silu(0.0) == 0.0 and abs(M.silu_grad(0.0) - 0.5) < 1e-15
    h = 1e-6
    for x in (-3.0, -0.5, 0.7, 4.0):
        assert abs(M.silu_grad(x) - (M.silu(x + h) - M.silu(x - h)) / (2 * h)) < 1e-9


def test_backward_matches_finite_differences():
    widths = [5, 7, 6, 4]
    theta = M.he_uniform(widths, 1) + 0.05 * np.random.default_rng(2).standard_normal(M.num_params(widths))
    x = np.random.default_rng(3).standard_normal((3, 5))
    t = np.random.default_rng(4).standard_normal((3, 4))
    y, cache = M.forward(theta, widths, x)
    loss, dy = M.mse(y, t)
    g = M.backward(theta, widths, cache, dy)
    rng = np.random.default_rng(5)
    for idx in rng.choice(theta.size, 25, replace=False):
        e = np.zeros_like(theta); e[idx] = 1e-6
        lp = M.mse(M.forward(theta + e, widths, x)[0], t)[0]
        lm = M.mse(M.forward(theta - e, widths, x)[0], t)[0]
        assert abs(g[idx] - (lp - lm) / 2e-6) <= 1e-7 * max(1.0, abs(g[idx]))


def test_pack_roundtrip_and_count():
    widths = [64, 512, 512, 512, 24576]
    assert M.num_params(widths) == 13_166_080
    small = [3, 4, 2]
    th = np.arange(M.num_params(small), dtype=float)
    np.testing.assert_array_equal(M.pack(M.unpack(th, small)), th)


def test_adam_first_step():
    th = np.array([1.0, -2.0, 0.5]); g = np.array([0.3, -4.0, 1e-3])
    th1, m, v = M.adam(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(th1, th - 0.01 * np.sign(g), rtol=0, atol=1e-9)


def test_forward_backward_match_torch_autograd():
    """The layer composition, the MSE loss and the gradient against PyTorch's
    own FP64 CPU layers (nn.functional.linear, silu) and autograd on the
    same packed weights: an error mirrored in forward and backward (say SiLU
    on the output layer, a transposed W, a dropped bias) fails here."""
    import torch
    widths = [6, 9, 7, 5]
    rng = np.random.default_rng(11)
    theta = M.he_uniform(widths, 4) + 0.1 * rng.standard_normal(M.num_params(widths))
    x = rng.standard_normal((4, widths[0]))
    t = rng.standard_normal((4, widths[-1]))
    params = [(torch.tensor(W, dtype=torch.float64, requires_grad=True),
               torch.tensor(b, dtype=torch.float64, requires_grad=True)) for W, b in M.unpack(theta, widths)]
    h = torch.tensor(x, dtype=torch.float64)
    for l, (W, b) in enumerate(params):
        h = torch.nn.functional.linear(h, W, b)
        if l < len(params) - 1:
            h = torch.nn.functional.silu(h)
    loss_t = torch.mean((h - torch.tensor(t, dtype=torch.float64)) ** 2)
    loss_t.backward()
    g_t = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy().ravel()]) for W, b in params])

    y, cache = M.forward(theta, widths, x)
    loss, dy = M.mse(y, t)
    g = M.backward(theta, widths, cache, dy)
    np.testing.assert_allclose(y, h.detach().numpy(), rtol=1e-13, atol=1e-14)
    assert abs(loss - loss_t.item()) <= 1e-14 * abs(loss)
    np.testing.assert_allclose(g, g_t, rtol=1e-11, atol=1e-14)
