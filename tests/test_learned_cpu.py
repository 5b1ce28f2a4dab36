"""The fp64 CPU references for the learned split models, pinned by central
finite differences (the GPU training kernels are checked against them)."""
import numpy as np
import pytest


def fd_grad(f, theta, h):
    g = np.empty_like(theta)
    for k in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[k] += h
        tm[k] -= h
        g[k] = (f(tp) - f(tm)) / (2 * h)
    return g


def test_pwl_gradient_matches_finite_differences(oracle):
    rng = np.random.default_rng(0)
    K = 16
    p = rng.random(K + 1)
    x = np.sort(rng.random(200))
    t = np.sqrt(x) + 0.01 * rng.standard_normal(200)
    loss, g = oracle.pwl_loss_grad(p, x, t)
    fd = fd_grad(lambda q: oracle.pwl_loss_grad(q, x, t)[0], p, 1e-6)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)
    # closed form: a PWL through the exact knot values of a linear target has zero loss
    p_lin = np.linspace(0.0, 2.0, K + 1)
    l0, g0 = oracle.pwl_loss_grad(p_lin, x, 2.0 * x)
    assert l0 < 1e-28 and np.abs(g0).max() < 1e-13


def test_mlp_gradient_matches_finite_differences(oracle):
    rng = np.random.default_rng(1)
    th = 0.3 * rng.standard_normal(oracle.MLP_PARAMS)
    x = rng.random(50)
    t = x ** 2
    loss, g = oracle.mlp_loss_grad(th, x, t)
    fd = fd_grad(lambda q: oracle.mlp_loss_grad(q, x, t)[0], th, 1e-6)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-8)
    # forward: a network with W3 = 0 is the constant b3
    th0 = th.copy()
    th0[64 + 1024 + 32: 64 + 1024 + 64] = 0.0
    th0[-1] = 0.25
    assert np.allclose(oracle.mlp_forward(th0, x), 0.25)
    # forward equals the loss's prediction: loss with t = f(x) is zero
    y = oracle.mlp_forward(th, x)
    assert oracle.mlp_loss_grad(th, x, y)[0] < 1e-28
