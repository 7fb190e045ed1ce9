"""Pins of the FP64 MLP oracle (learned flux correction): finite-difference gradients, closed forms of
degenerate networks, and the first Adam step."""
import numpy as np


def _silu(z):
    return z / (1.0 + np.exp(-z))


def test_param_count(oracle_mod):
    # 32x128 + 128 + 2 (128x128 + 128) + 8x128 + 8
    assert oracle_mod.mlp_n_params(128) == 38280


def test_gradient_matches_finite_differences(oracle_mod):
    H = 8
    rng = np.random.default_rng(0)
    p = rng.normal(scale=0.4, size=oracle_mod.mlp_n_params(H))
    x = rng.normal(size=(5, 32))
    t = rng.normal(size=(5, 8))
    loss, g = oracle_mod.mlp_loss_grad(p, H, x, t)
    idx = rng.choice(p.size, 60, replace=False)
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle_mod.mlp_loss_grad(pp, H, x, t)[0] - oracle_mod.mlp_loss_grad(pm, H, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])
    y = oracle_mod.mlp_forward(p, H, x)
    assert np.isclose(loss, np.mean((y - t) ** 2), rtol=1e-14)


def test_degenerate_network_closed_form(oracle_mod):
    """With W1..W3 = 0 every hidden unit is silu(bias); the output is W4 silu(b3) + b4."""
    H = 16
    rng = np.random.default_rng(1)
    n = oracle_mod.mlp_n_params(H)
    p = np.zeros(n)
    o = 0
    o += H * 32
    p[o:o + H] = rng.normal(size=H); o += H
    o += H * H
    p[o:o + H] = rng.normal(size=H); o += H
    o += H * H
    b3 = rng.normal(size=H); p[o:o + H] = b3; o += H
    W4 = rng.normal(size=(8, H)); p[o:o + 8 * H] = W4.ravel(); o += 8 * H
    b4 = rng.normal(size=8); p[o:o + 8] = b4; o += 8
    assert o == n
    x = rng.normal(size=(3, 32))
    y = oracle_mod.mlp_forward(p, H, x)
    ref = W4 @ _silu(b3) + b4
    assert np.allclose(y, ref[None, :], rtol=1e-14, atol=1e-14)


def test_first_adam_step(oracle_mod):
    """At t = 1 the bias-corrected moments are g and g^2: the step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    p0 = p.copy()
    oracle_mod.mlp_adam(p, m, v, g, 1e-3, 1)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-16)
