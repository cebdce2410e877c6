"""Pins of the FP64 warm-start network reference (oracle.mlp) against facts
that do not come from the reference itself: values of the normal CDF, finite
differences, the C oracle's block-tridiagonal product and direct solve, and
the closed form of Adam's first step."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2309_06427_amd import inputs


def test_gelu_values():
    # gelu(z) = z * Phi(z); Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    z = np.array([0.0, 1.0, -1.0, 8.0, -8.0])
    g = mlp.gelu(z)
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15
    assert abs(g[3] - 8.0) < 1e-12 and abs(g[4]) < 1e-12


def test_gelu_grad_matches_central_differences():
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) < 1e-8
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def _problems(nx, nu, Ns, seed):
    rng = np.random.default_rng(seed)
    out = []
    for N in Ns:
        pr = inputs.draw_problem(rng, N, nx, nu)
        st, D, L, Di, M = oracle.build(pr["A"], pr["B"], pr["Q"], pr["R"], "sym")
        assert st == 0
        st, lam = oracle.direct(D, L, pr["gamma"])
        out.append((D, L, pr["gamma"], lam))
    return out


def test_block_product_matches_c_oracle():
    for (D, L, g, lam) in _problems(3, 2, [1, 4, 7], 1):
        N, nx = D.shape[:2]
        x = np.random.default_rng(2).standard_normal((N, nx))
        assert np.allclose(mlp.block_tridiag_mul(D, L, x).ravel(), oracle.btmv(D, L, x.ravel()), rtol=0, atol=1e-13)


def test_features_layout():
    (D, L, g, lam), = _problems(3, 1, [4], 3)
    X = mlp.features(D, L, g)
    assert X.shape == (4, 2 * 9 + 3)
    assert np.array_equal(X[2, :9], D[2].ravel())
    assert np.array_equal(X[2, 9:18], L[2].ravel())
    assert np.array_equal(X[2, 18:], g.reshape(4, 3)[2])
    assert np.all(X[0, 9:18] == 0.0)


def test_loss_is_mean_squared_residual_of_the_start():
    nx, H = 3, 8
    probs = _problems(nx, 2, [5, 3], 4)
    theta = inputs.mlp_init(nx, H, seed=5)
    X = np.concatenate([mlp.features(D, L, g) for (D, L, g, _) in probs])
    mu, isd = mlp.feature_stats(X)
    loss, _ = mlp.loss_and_grad(theta, probs, mu, isd, 0.7, nx, H)
    lam0, _ = mlp.forward(theta, X, mu, isd, 0.7, nx, H)
    res, r0 = 0.0, 0
    for (D, L, g, _) in probs:
        N = D.shape[0]
        r = g - oracle.btmv(D, L, lam0[r0:r0 + N].ravel())
        res += float(r @ r)
        r0 += N
    assert abs(loss - res / len(probs)) <= 1e-9 * res


@pytest.mark.parametrize("seed", [6, 7])
def test_gradient_matches_central_differences(seed):
    nx, H = 2, 5
    probs = _problems(nx, 1, [4, 3], seed)
    theta = inputs.mlp_init(nx, H, seed=seed)
    theta += 0.3 * np.random.default_rng(seed).standard_normal(theta.size)  # non-zero biases too
    X = np.concatenate([mlp.features(D, L, g) for (D, L, g, _) in probs])
    mu, isd = mlp.feature_stats(X)
    ys = 0.8
    _, grad = mlp.loss_and_grad(theta, probs, mu, isd, ys, nx, H)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (mlp.loss_and_grad(tp, probs, mu, isd, ys, nx, H)[0] -
                 mlp.loss_and_grad(tm, probs, mu, isd, ys, nx, H)[0]) / (2 * h)
    err = np.linalg.norm(fd - grad) / np.linalg.norm(fd)
    assert err < 1e-6, err


def test_adam_first_step_is_signed_learning_rate():
    # from zero moments, m_hat = g and v_hat = g^2, so the step is lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, -2e-2])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_standardisation_floor():
    X = np.array([[1.0, 2.0], [1.0, 4.0]])
    mu, isd = mlp.feature_stats(X)
    assert np.array_equal(mu, [1.0, 3.0])
    assert isd[0] == 1e6 and isd[1] == 1.0
