"""Seeded synthetic inputs: per-knot dynamics and cost blocks of a trajectory-
optimization QP, packed into the ragged layout the library consumes.

This module draws random numbers and packs arrays. It contains none of the
method's arithmetic (no Schur complement, no preconditioner, no solve), so the
CPU oracle and the GPU path can both be fed from it.

Problem model (Sec. II-A, Eq. dynamics / cost and the integrator form
A = I + hM, B = hN): a problem with ``N`` knots has linearised dynamics
A_k (nx x nx), B_k (nx x nu) and cost Hessians Q_k (nx x nx, SPD), R_k
(nu x nu, SPD) for k = 0..N-1, plus a right-hand side gamma (N*nx).  The
last A and B are drawn but do not enter the N-block-row Schur complement.

Distributions:

* ``A_k = I + 0.05 * G_k``, ``G_k`` iid N(0,1)/sqrt(nx)  (h = 0.05)
* ``B_k`` iid N(0, 0.1^2)  (0.1 read as the standard deviation)
* ``Q_k = I + W_k W_k^T / nx`` with ``W_k`` nx x nx iid N(0,1)   (``qmode="wishart"``)
  or ``Q_k = U_k diag(c_k^(i/(nx-1))) U_k^T`` with ``c_k = 10^U(0, log10 cmax)``
  and ``U_k`` the sign-fixed QR factor of a Gaussian matrix (``qmode="logcond"``)
* ``R_k = 0.1 I``
* ``gamma`` iid N(0, 1)

Per problem the draws happen in the order G, B, (W | c, U), gamma from
``numpy.random.default_rng`` seeded with a child of ``SeedSequence(seed)``.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import os
from typing import Sequence

import numpy as np

H_STEP = 0.05          # integrator step in A = I + h*M
B_STD = 0.1            # standard deviation of the entries of B
R_SCALE = 0.1          # R_k = R_SCALE * I


@dataclasses.dataclass
class Batch:
    """Ragged batch of problems in packed row-major FP64 layout.

    Problem p occupies, in each flat array, a contiguous range starting at the
    matching offset: ``A[off_nn[p] : off_nn[p] + N*nx*nx]`` holds A_0..A_{N-1}
    row-major, likewise Q (same offsets), B (``off_nu``, nx x nu blocks),
    R (``off_uu``, nu x nu blocks) and gamma / lambda (``off_v``, N*nx).
    """

    N: np.ndarray       # int32 [P]
    nx: np.ndarray      # int32 [P]
    nu: np.ndarray      # int32 [P]
    A: np.ndarray       # float64 flat
    B: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    gamma: np.ndarray
    off_nn: np.ndarray  # int64 [P+1]
    off_nu: np.ndarray
    off_uu: np.ndarray
    off_v: np.ndarray

    @property
    def P(self) -> int:
        return int(self.N.shape[0])

    def problem(self, p: int) -> dict:
        """Views of problem ``p`` reshaped to per-knot blocks."""
        N, nx, nu = int(self.N[p]), int(self.nx[p]), int(self.nu[p])
        sl = lambda arr, off, blk: arr[off[p]:off[p + 1]].reshape((N,) + blk)
        return dict(
            N=N, nx=nx, nu=nu,
            A=sl(self.A, self.off_nn, (nx, nx)),
            B=sl(self.B, self.off_nu, (nx, nu)),
            Q=sl(self.Q, self.off_nn, (nx, nx)),
            R=sl(self.R, self.off_uu, (nu, nu)),
            gamma=self.gamma[self.off_v[p]:self.off_v[p + 1]],
        )

    def subset(self, idx: Sequence[int]) -> "Batch":
        """A new packed batch holding problems ``idx`` in that order."""
        probs = [self.problem(int(i)) for i in idx]
        return pack(probs)


def _sign_fixed_qr(M: np.ndarray) -> np.ndarray:
    q, r = np.linalg.qr(M)
    d = np.sign(np.diagonal(r, axis1=-2, axis2=-1)).copy()
    d[d == 0] = 1.0
    return q * d[..., None, :]


def draw_problem(rng: np.random.Generator, N: int, nx: int, nu: int,
                 qmode: str = "wishart", qcond_max: float = 1e4) -> dict:
    """Draw one problem's blocks (see module docstring for the recipe)."""
    G = rng.standard_normal((N, nx, nx)) / np.sqrt(nx)
    A = np.eye(nx)[None] + H_STEP * G
    B = rng.normal(0.0, B_STD, size=(N, nx, nu))
    if qmode == "wishart":
        W = rng.standard_normal((N, nx, nx))
        Q = np.eye(nx)[None] + W @ np.swapaxes(W, 1, 2) / nx
    elif qmode == "logcond":
        c = 10.0 ** rng.uniform(0.0, np.log10(qcond_max), size=N)
        U = _sign_fixed_qr(rng.standard_normal((N, nx, nx)))
        expo = np.arange(nx) / max(nx - 1, 1)
        ev = c[:, None] ** expo[None, :]
        Q = (U * ev[:, None, :]) @ np.swapaxes(U, 1, 2)
        Q = 0.5 * (Q + np.swapaxes(Q, 1, 2))
    else:
        raise ValueError(f"unknown qmode {qmode!r}")
    R = np.broadcast_to(R_SCALE * np.eye(nu), (N, nu, nu)).copy()
    gamma = rng.standard_normal(N * nx)
    return dict(N=N, nx=nx, nu=nu, A=A, B=B, Q=Q, R=R, gamma=gamma)


def pack(probs: Sequence[dict]) -> Batch:
    """Pack per-problem dicts into one ragged :class:`Batch`."""
    P = len(probs)
    N = np.array([p["N"] for p in probs], dtype=np.int32)
    nx = np.array([p["nx"] for p in probs], dtype=np.int32)
    nu = np.array([p["nu"] for p in probs], dtype=np.int32)

    def offs(sizes):
        o = np.zeros(P + 1, dtype=np.int64)
        o[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64))
        return o

    Ni, xi, ui = N.astype(np.int64), nx.astype(np.int64), nu.astype(np.int64)
    off_nn, off_nu = offs(Ni * xi * xi), offs(Ni * xi * ui)
    off_uu, off_v = offs(Ni * ui * ui), offs(Ni * xi)
    cat = lambda key: (np.concatenate([np.ascontiguousarray(p[key], dtype=np.float64).ravel() for p in probs])
                       if P else np.zeros(0))
    return Batch(N=N, nx=nx, nu=nu, A=cat("A"), B=cat("B"), Q=cat("Q"), R=cat("R"),
                 gamma=cat("gamma"), off_nn=off_nn, off_nu=off_nu, off_uu=off_uu, off_v=off_v)


@dataclasses.dataclass
class BlockBatch:
    """Ragged batch of symmetric block-tridiagonal matrices given by blocks:
    ``D[off_nn[p] : off_nn[p+1]]`` holds S[k][k] (k = 0..N-1) and ``L`` at the
    same offsets S[k][k-1] (block 0 zero), nx x nx row-major; ``gamma`` at
    ``off_v`` as in :class:`Batch`."""

    N: np.ndarray       # int32 [P]
    nx: np.ndarray      # int32 [P]
    D: np.ndarray       # float64 flat
    L: np.ndarray
    gamma: np.ndarray
    off_nn: np.ndarray  # int64 [P+1]
    off_v: np.ndarray

    @property
    def P(self) -> int:
        return int(self.N.shape[0])

    def problem(self, p: int) -> dict:
        N, nx = int(self.N[p]), int(self.nx[p])
        sl = lambda arr, off, blk: arr[off[p]:off[p + 1]].reshape((N,) + blk)
        return dict(N=N, nx=nx, D=sl(self.D, self.off_nn, (nx, nx)), L=sl(self.L, self.off_nn, (nx, nx)),
                    gamma=self.gamma[self.off_v[p]:self.off_v[p + 1]])


def draw_block_tridiag(rng: np.random.Generator, N: int, nx: int, margin: float = 0.5) -> dict:
    """Blocks of a random SPD block-tridiagonal matrix not built from dynamics:
    L_k (k >= 1) with iid N(0, 1/nx) entries, D_k = W_k W_k^T / nx + c_k I with
    W_k iid N(0,1) and c_k = ||L_k||_2 + ||L_{k+1}||_2 + margin, so every block
    row is diagonally dominant in the 2-norm (block Gershgorin) and the matrix
    is SPD.  Draw order: L, W, gamma."""
    L = rng.standard_normal((N, nx, nx)) / np.sqrt(nx)
    L[0] = 0.0
    W = rng.standard_normal((N, nx, nx))
    nrm = np.linalg.norm(L, ord=2, axis=(1, 2))
    c = nrm + np.append(nrm[1:], 0.0) + margin
    D = W @ np.swapaxes(W, 1, 2) / nx + c[:, None, None] * np.eye(nx)[None]
    D = 0.5 * (D + np.swapaxes(D, 1, 2))
    gamma = rng.standard_normal(N * nx)
    return dict(N=N, nx=nx, D=D, L=L, gamma=gamma)


def block_batch(Ns: Sequence[int], nxs: Sequence[int], seed: int, margin: float = 0.5) -> BlockBatch:
    """Problems of sizes (Ns[i], nxs[i]) from :func:`draw_block_tridiag`, problem i
    seeded with child i of ``SeedSequence(seed)``."""
    kids = np.random.SeedSequence(seed).spawn(len(Ns))
    probs = [draw_block_tridiag(np.random.default_rng(k), int(n), int(x), margin) for k, n, x in zip(kids, Ns, nxs)]
    P = len(probs)
    N = np.array([q["N"] for q in probs], dtype=np.int32)
    nx = np.array([q["nx"] for q in probs], dtype=np.int32)
    off_nn = np.zeros(P + 1, dtype=np.int64)
    off_nn[1:] = np.cumsum(N.astype(np.int64) * nx * nx)
    off_v = np.zeros(P + 1, dtype=np.int64)
    off_v[1:] = np.cumsum(N.astype(np.int64) * nx)
    cat = lambda key: np.concatenate([q[key].ravel() for q in probs]) if P else np.zeros(0)
    return BlockBatch(N=N, nx=nx, D=cat("D"), L=cat("L"), gamma=cat("gamma"), off_nn=off_nn, off_v=off_v)


def single(N: int, nx: int, nu: int, seed: int, qmode: str = "wishart",
           qcond_max: float = 1e4) -> Batch:
    """One problem drawn from ``default_rng(seed)`` (the plain single solve)."""
    rng = np.random.default_rng(seed)
    return pack([draw_problem(rng, N, nx, nu, qmode, qcond_max)])


def batch(P: int, seed: int, N_range=(32, 256), nx_choices=(6, 14, 26),
          qmode: str = "wishart", qcond_max: float = 1e4, first: int = 0,
          count: int | None = None) -> Batch:
    """Ragged batch: problem i draws its sizes from a dedicated child stream
    (N uniform on the inclusive range, nx uniform over ``nx_choices``,
    nu = nx // 2) and its blocks from child i of ``SeedSequence(seed)``.

    ``first``/``count`` select a contiguous slice of the P problems without
    drawing the others' blocks, so a sample can be regenerated cheaply.
    """
    children = np.random.SeedSequence(seed).spawn(P + 1)
    srng = np.random.default_rng(children[P])
    Ns = srng.integers(N_range[0], N_range[1] + 1, size=P)
    nxs = np.asarray(nx_choices)[srng.integers(0, len(nx_choices), size=P)]
    count = P - first if count is None else count

    def one(i):
        rng = np.random.default_rng(children[i])
        n, x = int(Ns[i]), int(nxs[i])
        return draw_problem(rng, n, x, x // 2, qmode, qcond_max)

    idx = range(first, first + count)
    if count >= 64:
        # each problem owns its generator, so threads do not change the draws
        with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            probs = list(ex.map(one, idx))
    else:
        probs = [one(i) for i in idx]
    return pack(probs)


def uniform_batch(P: int, N: int, nx: int, nu: int, seed: int,
                  qmode: str = "wishart", qcond_max: float = 1e4) -> Batch:
    """P problems of one shape, problem i from child i of ``SeedSequence(seed)``."""
    children = np.random.SeedSequence(seed).spawn(P)
    return pack([draw_problem(np.random.default_rng(children[i]), N, nx, nu, qmode, qcond_max)
                 for i in range(P)])


# Named workloads (sizes and generator settings of the benchmark cases).
WORKLOADS = {
    "single_n50_nx14": dict(kind="single", N=50, nx=14, nu=7, seed=0, qmode="wishart",
                            tol=1e-8, precision="fp64"),
    "single_n512_nx36": dict(kind="single", N=512, nx=36, nu=12, seed=1, qmode="logcond",
                             qcond_max=1e4, tol=1e-6, precision="fp32_refine64"),
    "batch4096_ragged": dict(kind="batch", P=4096, seed=2, qmode="wishart",
                             tol=1e-6, precision="fp32_refine64"),
    "batch1024_n128_nx26_cond1e6": dict(kind="uniform", P=1024, N=128, nx=26, nu=12, seed=3,
                                        qmode="logcond", qcond_max=1e6, tol=1e-6),
    # one state size at a time (the ragged batch's classes at its mean horizon)
    "batch1365_n144_nx26": dict(kind="uniform", P=1365, N=144, nx=26, nu=13, seed=5, qmode="wishart",
                                tol=1e-6, precision="fp32_refine64"),
    "batch1365_n144_nx14": dict(kind="uniform", P=1365, N=144, nx=14, nu=7, seed=6, qmode="wishart",
                                tol=1e-6, precision="fp32_refine64"),
    "batch1365_n144_nx6": dict(kind="uniform", P=1365, N=144, nx=6, nu=3, seed=7, qmode="wishart",
                               tol=1e-6, precision="fp32_refine64"),
}


def make(name: str, **over) -> Batch:
    """Generate a named workload (keyword overrides allowed, e.g. ``P=64``)."""
    w = dict(WORKLOADS[name])
    w.update(over)
    kind = w["kind"]
    if kind == "single":
        return single(w["N"], w["nx"], w["nu"], w["seed"], w["qmode"], w.get("qcond_max", 1e4))
    if kind == "batch":
        return batch(w["P"], w["seed"], qmode=w["qmode"], qcond_max=w.get("qcond_max", 1e4),
                     first=w.get("first", 0), count=w.get("count"))
    if kind == "uniform":
        return uniform_batch(w["P"], w["N"], w["nx"], w["nu"], w["seed"], w["qmode"],
                             w.get("qcond_max", 1e4))
    raise ValueError(kind)


def mlp_init(nx: int, hidden: int = 128, seed: int = 0) -> np.ndarray:
    """Initial weights of the per-knot warm-start network (random draws only).

    Flat FP64 vector W1 (n_in x H), b1, W2 (H x H), b2, W3 (H x nx), b3 with
    n_in = 2 nx^2 + nx: weights Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)),
    biases zero.
    """
    rng = np.random.default_rng(seed)
    ni, H = 2 * nx * nx + nx, hidden
    parts = []
    for fan_in, fan_out in ((ni, H), (H, H), (H, nx)):
        a = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-a, a, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
