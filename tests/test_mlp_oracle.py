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


# ------------------------------------------------------------ forward pass pins
#
# Tiny networks whose output is written out below with scalar arithmetic and
# math.erf only (no matrix product), so that the forward pass is fixed by
# values that do not come from oracle.mlp itself.  Each case names the
# mistakes it catches.

def _gelu(z: float) -> float:
    return 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))


def _pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in (W1, b1, W2, b2, W3, b3)])


def test_forward_output_layer_is_linear_with_bias_and_scale():
    """nx = 1 (3 inputs), H = 2, W1 = W2 = 0: h1 = gelu(b1), h2 = gelu(W2 h1 + b2)
    = gelu(b2), output y_scale (W3^T h2 + b3).  Catches a GELU on the output
    layer, a dropped b2 or b3, and a missing y_scale."""
    nx, H = 1, 2
    b1, b2 = np.array([0.3, -0.2]), np.array([0.7, -1.1])
    W3, b3 = np.array([[1.5], [-0.5]]), np.array([0.25])
    theta = _pack(np.zeros((3, H)), b1, np.zeros((H, H)), b2, W3, b3)
    X = np.array([[4.0, -2.0, 1.0]])
    lam0, _ = mlp.forward(theta, X, np.zeros(3), np.ones(3), 3.0, nx, H)
    want = 3.0 * (1.5 * _gelu(0.7) - 0.5 * _gelu(-1.1) + 0.25)
    assert abs(lam0[0, 0] - want) < 1e-14


def test_forward_standardisation_and_layer_order():
    """Non-zero mean / scale and every layer in use.  xh = (x - mu) * inv_sd
    (not x * inv_sd - mu), z1 = xh W1 + b1, h1 = gelu(z1), z2 = h1 W2 + b2 with
    W2 applied as h1 (row) times W2 (W2[i][j] feeds hidden j from i, so the
    transpose gives a different value), h2 = gelu(z2).  Catches a swapped
    standardisation, a transposed W2, a skipped hidden GELU and a dropped b1."""
    nx, H = 1, 2
    mu, inv_sd = np.array([1.0, 2.0, 3.0]), np.array([0.5, 2.0, 0.25])
    X = np.array([[3.0, 1.0, 7.0]])
    xh = [(3.0 - 1.0) * 0.5, (1.0 - 2.0) * 2.0, (7.0 - 3.0) * 0.25]      # = 1, -2, 1
    W1 = np.array([[0.5, -0.3], [0.1, 0.2], [-0.4, 0.6]])
    b1 = np.array([0.05, -0.15])
    W2 = np.array([[0.0, 1.2], [0.0, 0.0]])                              # hidden 0 -> hidden 1 only
    b2 = np.array([0.4, -0.3])
    W3 = np.array([[2.0], [-1.0]])
    b3 = np.array([0.1])
    theta = _pack(W1, b1, W2, b2, W3, b3)
    z1 = [sum(xh[i] * W1[i][j] for i in range(3)) + b1[j] for j in range(H)]
    h1 = [_gelu(v) for v in z1]
    z2 = [sum(h1[i] * W2[i][j] for i in range(H)) + b2[j] for j in range(H)]
    h2 = [_gelu(v) for v in z2]
    want = 0.5 * (sum(h2[i] * W3[i][0] for i in range(H)) + b3[0])
    lam0, act = mlp.forward(theta, X, mu, inv_sd, 0.5, nx, H)
    assert abs(lam0[0, 0] - want) < 1e-14
    assert np.allclose(act["xh"][0], xh, rtol=0, atol=1e-15)
    # the transposed W2 gives another number, so the pin separates the two
    z2t = [sum(h1[i] * W2[j][i] for i in range(H)) + b2[j] for j in range(H)]
    want_t = 0.5 * (sum(_gelu(z2t[i]) * W3[i][0] for i in range(H)) + b3[0])
    assert abs(want_t - want) > 1e-3


def test_forward_feature_layout_and_rows():
    """nx = 2 (10 inputs: vec D_k row-major, vec L_k with L_0 = 0, gamma_k):
    a W1 column that reads only D_k[0][1] and one that reads gamma_k[1], with
    identity-like later layers, shows each feature lands where the layout says
    and each knot (row of X) is independent."""
    nx, H = 2, 2
    D = np.array([[[2.0, 0.5], [0.5, 3.0]], [[4.0, -1.0], [-1.0, 5.0]]])
    L = np.array([[[9.0, 9.0], [9.0, 9.0]], [[0.1, 0.2], [0.3, 0.4]]])   # L_0 must be ignored
    g = np.array([1.0, -2.0, 0.5, 0.25])
    X = mlp.features(D, L, g)
    assert X.shape == (2, 10)
    assert np.array_equal(X[0], [2.0, 0.5, 0.5, 3.0, 0, 0, 0, 0, 1.0, -2.0])
    assert np.array_equal(X[1], [4.0, -1.0, -1.0, 5.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.25])
    W1 = np.zeros((10, H))
    W1[1, 0] = 1.0      # D_k[0][1]
    W1[9, 1] = 1.0      # gamma_k[1]
    W2 = np.eye(H)
    W3 = np.array([[1.0, 0.0], [0.0, 1.0]])
    theta = _pack(W1, np.zeros(H), W2, np.zeros(H), W3, np.zeros(nx))
    lam0, _ = mlp.forward(theta, X, np.zeros(10), np.ones(10), 1.0, nx, H)
    for k, (d01, g1) in enumerate(((0.5, -2.0), (-1.0, 0.25))):
        assert abs(lam0[k, 0] - _gelu(_gelu(d01))) < 1e-15
        assert abs(lam0[k, 1] - _gelu(_gelu(g1))) < 1e-15
