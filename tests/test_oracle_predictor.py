"""Pins of the oracle's learned-predictor pieces: transfer operators, moments,
network gradients (finite differences), Adam on a convex problem."""

import numpy as np
import pytest

from oracle import predictor as pr


def test_restriction_of_constant_and_prolongation_of_constant():
    n = (32, 48, 64)
    f = np.full((64, 48, 32), 2.5)
    assert np.allclose(pr.restrict(f, n), 2.5)
    assert np.allclose(pr.prolong(np.full((16, 16, 16), -1.25), n), -1.25)


def test_prolongation_reproduces_smooth_periodic_waves_and_restriction_averages():
    n = (48, 32, 64)
    nx, ny, nz = n
    c = np.arange(16)
    # a coarse plane wave sampled at cell centres; trilinear interpolation of a
    # linear function along the non-varying axes is exact, and along z the
    # interpolant is the chord between neighbouring centres
    g = np.cos(2 * np.pi * c / 16)[:, None, None] * np.ones((16, 16, 16))
    f = pr.prolong(g, n)
    zc = (np.arange(nz) + 0.5) / (nz // 16) - 0.5
    c0 = np.floor(zc).astype(int)
    w = zc - c0
    ref = (1 - w) * np.cos(2 * np.pi * c0 / 16) + w * np.cos(2 * np.pi * (c0 + 1) / 16)
    assert np.allclose(f[:, 3, 7], ref)
    # block average of a fine field that is constant on blocks returns the block values
    blocks = np.random.default_rng(0).standard_normal((16, 16, 16))
    fine = np.kron(blocks, np.ones((nz // 16, ny // 16, nx // 16)))
    assert np.allclose(pr.restrict(fine, n), blocks)


def test_moments_of_a_point_charge():
    h = 0.5
    q = [np.array([1.0, -2.0]), np.array([0.5, 0.5]), np.array([3.0, 0.0])]
    d = np.array([1.0, 0.0]) / h ** 3
    m = pr.moments(d, q, h)
    np.testing.assert_allclose(m[:3], [1.0, 0.5, 3.0])
    np.testing.assert_allclose(m[3:], [1.0, 0.5, 3.0, 0.25, 1.5, 9.0])


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = pr.init_params(2, n_in=11, n_h=7, n_out=5)
    for k in p:
        p[k] = p[k] + 0.1 * rng.standard_normal(p[k].shape)
    X = rng.standard_normal((4, 11))
    T = rng.standard_normal((4, 5))
    loss, g = pr.loss_and_grads(p, X, T)
    eps = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = pr.loss_and_grads(p, X, T)
            flat[idx] = old - eps
            lm, _ = pr.loss_and_grads(p, X, T)
            flat[idx] = old
            assert abs((lp - lm) / (2 * eps) - g[k].ravel()[idx]) < 1e-8, k


def test_adam_fits_a_linear_map():
    rng = np.random.default_rng(3)
    p = pr.init_params(4, n_in=6, n_h=16, n_out=3)
    A = rng.standard_normal((3, 6)) * 0.3
    X = rng.standard_normal((64, 6))
    T = X @ A.T
    st = {}
    l0, _ = pr.loss_and_grads(p, X, T)
    for _ in range(1500):
        _, g = pr.loss_and_grads(p, X, T)
        pr.adam(p, g, st, lr=3e-3)
    l1, _ = pr.loss_and_grads(p, X, T)
    assert l1 < 0.02 * l0
