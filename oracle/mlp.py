"""FP64 reference of the learned per-knot warm start (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module; the GPU library never calls it and shares no code with it.

The network maps one knot's local blocks to a guess of that knot's part of
the solution lambda of S lambda = gamma (Sec. II-A, Eq. (schur)):

    x_k  = [vec D_k, vec L_k, gamma_k]        (2 nx^2 + nx inputs, L_0 = 0,
                                               L_k = S[k][k-1], row-major)
    xh   = (x_k - mu) * inv_sd                (per-feature standardisation)
    z1   = xh W1 + b1,   h1 = gelu(z1)        (hidden width H)
    z2   = h1 W2 + b2,   h2 = gelu(z2)
    o    = h2 W3 + b3,   lambda0_k = y_scale * o

with the exact GELU, gelu(z) = z * Phi(z) and Phi the standard normal CDF.

Training loss over a set of problems p (each with its exact solution
lambda*_p):

    loss = (1 / P) * sum_p || S_p (lambda0_p - lambda*_p) ||^2

which equals the mean squared residual ||gamma_p - S_p lambda0_p||^2 of the
warm start when lambda*_p is exact, i.e. the quantity PCG's stopping test
measures.  Gradients are plain reverse-mode differentiation of the formulas
above; the optimiser is Adam (Kingma & Ba, 2015) with bias correction.

Parameters travel as one flat FP64/FP32 vector in the order
W1 (n_in x H, row-major), b1 (H), W2 (H x H), b2 (H), W3 (H x nx), b3 (nx).
"""
from __future__ import annotations

import math

import numpy as np

SQRT_HALF = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def n_inputs(nx: int) -> int:
    return 2 * nx * nx + nx


def n_params(nx: int, hidden: int = 128) -> int:
    ni = n_inputs(nx)
    return ni * hidden + hidden + hidden * hidden + hidden + hidden * nx + nx


def unpack(theta: np.ndarray, nx: int, hidden: int = 128) -> dict:
    """Views of the flat parameter vector (see module docstring for the order)."""
    ni, H = n_inputs(nx), hidden
    shapes = [("W1", (ni, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, nx)), ("b3", (nx,))]
    out, o = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size
    return out


def erf(x: np.ndarray) -> np.ndarray:
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def gelu(z: np.ndarray) -> np.ndarray:
    return 0.5 * z * (1.0 + erf(z * SQRT_HALF))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d gelu / dz = Phi(z) + z * phi(z)."""
    return 0.5 * (1.0 + erf(z * SQRT_HALF)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def features(D: np.ndarray, L: np.ndarray, gamma: np.ndarray) -> np.ndarray:
    """Per-knot inputs of one problem: (N, 2 nx^2 + nx)."""
    N, nx = D.shape[0], D.shape[1]
    Lz = L.copy()
    Lz[0] = 0.0
    return np.concatenate([D.reshape(N, -1), Lz.reshape(N, -1), np.asarray(gamma).reshape(N, nx)], axis=1)


def feature_stats(X: np.ndarray, sd_floor: float = 1e-6):
    """Per-feature mean and 1 / max(population std, sd_floor) over the rows of X."""
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    return mu, 1.0 / np.maximum(sd, sd_floor)


def forward(theta, X, mu, inv_sd, y_scale, nx, hidden=128):
    """Returns lambda0 (rows of X, nx) and the activations needed by backward."""
    p = unpack(theta, nx, hidden)
    xh = (X - mu) * inv_sd
    z1 = xh @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    o = h2 @ p["W3"] + p["b3"]
    return y_scale * o, dict(xh=xh, z1=z1, h1=h1, z2=z2, h2=h2)


def block_tridiag_mul(D, L, x):
    """(S x)_k = D_k x_k + L_k x_{k-1} + L_{k+1}^T x_{k+1}  (x: (N, nx))."""
    N = D.shape[0]
    y = np.einsum("kij,kj->ki", D, x)
    for k in range(1, N):
        y[k] += L[k] @ x[k - 1]
        y[k - 1] += L[k].T @ x[k]
    return y


def loss_and_grad(theta, probs, mu, inv_sd, y_scale, nx, hidden=128):
    """Residual loss over problems [(D, L, gamma, lam_star)] and its gradient."""
    P = len(probs)
    X = np.concatenate([features(D, L, g) for (D, L, g, _) in probs])
    lam0, act = forward(theta, X, mu, inv_sd, y_scale, nx, hidden)
    loss = 0.0
    dlam = np.zeros_like(lam0)
    r0 = 0
    for (D, L, g, ls) in probs:
        N = D.shape[0]
        e = lam0[r0:r0 + N] - np.asarray(ls).reshape(N, nx)
        r = block_tridiag_mul(D, L, e)
        loss += float((r * r).sum())
        dlam[r0:r0 + N] = (2.0 / P) * block_tridiag_mul(D, L, r)  # S is symmetric
        r0 += N
    loss /= P
    p = unpack(theta, nx, hidden)
    do = y_scale * dlam
    g = {}
    g["W3"] = act["h2"].T @ do
    g["b3"] = do.sum(axis=0)
    dz2 = (do @ p["W3"].T) * gelu_grad(act["z2"])
    g["W2"] = act["h1"].T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(act["z1"])
    g["W1"] = act["xh"].T @ dz1
    g["b1"] = dz1.sum(axis=0)
    grad = np.concatenate([g[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    return loss, grad


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
