"""CPU FP64 oracle for symmetric-stair PCG (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it.  The arithmetic lives in ``ssp_oracle.c`` (plain loops, FP64); this module
compiles it with gcc and marshals numpy arrays through ctypes.  The MLP
reference lives in :mod:`oracle.mlp`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssp_oracle.c")
_LIB = os.path.join(_HERE, "libssp_oracle.so")

OK, NOT_SPD, MAXITER, NONFINITE, BREAKDOWN, INACCURATE = 0, 1, 2, 3, 4, 5
WARM_FALLBACK = 8  # OR-ed onto a status: the warm start was replaced by zero
PC_FALLBACK = 16   # OR-ed: the refinement went on with block-Jacobi after a float breakdown
# bj: block-Jacobi, add / sym: additive / symmetric stair, jacobi: scalar
# Jacobi, poly2 / poly3: Neumann polynomial of degree 2 / 3 with Psi = D
PC = {"bj": 0, "add": 1, "sym": 2, "jacobi": 3, "poly2": 4, "poly3": 5}
POLY_DEGREE = {"poly2": 2, "poly3": 3}
PREC = {"fp64": 0, "fp32": 1, "fp32_refine64": 2}
# refinement constants: inner tolerance tau_j = clamp(THETA*tol*|g|/|r_j|, TAU_MIN, 1)
THETA, TAU_MIN, MAX_OUTER = 0.5, 1e-6, 5


def build_lib() -> str:
    """Compile the oracle with gcc (-O2, OpenMP over problems)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_lib()
        L = C.CDLL(_LIB)
        d, i, i64 = C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int64)
        ip = C.POINTER(C.c_int)
        L.ssp_oracle_build.argtypes = [i, i, i, d, d, d, d, i, d, d, d, d]
        L.ssp_oracle_build.restype = i
        L.ssp_oracle_precond.argtypes = [i, i, i, d, d, d, d]
        L.ssp_oracle_precond.restype = i
        L.ssp_oracle_btmv.argtypes = [i, i, d, d, d, d]
        L.ssp_oracle_pcg.argtypes = [i, i, d, d, d, d, i, d, C.c_double, i, d, ip]
        L.ssp_oracle_pcg.restype = i
        L.ssp_oracle_pcg_mixed.argtypes = [i, i, d, d, d, d, i, d, C.c_double, i, i, i,
                                           C.c_double, C.c_double, d, ip, ip]
        L.ssp_oracle_pcg_mixed.restype = i
        L.ssp_oracle_relres.argtypes = [i, i, d, d, d, d]
        L.ssp_oracle_relres.restype = C.c_double
        L.ssp_oracle_direct.argtypes = [i, i, d, d, d, d]
        L.ssp_oracle_direct.restype = i
        L.ssp_oracle_apply_precond.argtypes = [i, i, d, d, d, i, d, d]
        L.ssp_oracle_kkt_rhs.argtypes = [i, i, i, d, d, d, d, d, d, d, d]
        L.ssp_oracle_kkt_rhs.restype = i
        L.ssp_oracle_kkt_recover.argtypes = [i, i, i, d, d, d, d, d, d, d, d, d]
        L.ssp_oracle_kkt_recover.restype = i
        L.ssp_oracle_solve_batch.argtypes = [i, ip, ip, ip, i64, i64, i64, i64, d, d, d, d, d,
                                             i, i, C.c_double, i, i, C.c_double, C.c_double,
                                             i, d, ip, ip, d, ip]
        L.ssp_oracle_build_batch.argtypes = [i, ip, ip, ip, i64, i64, i64, d, d, d, d, i, ip]
        L.ssp_oracle_set_threads.argtypes = [i]
        L.ssp_oracle_get_threads.restype = i
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def build(A, B, Q, R, pc: str = "sym"):
    """Blocks of S and Phi^-1 for one problem.

    A, Q: (N, nx, nx); B: (N, nx, nu); R: (N, nu, nu).
    Returns (status, D, L, Dinv, M), each block array (N, nx, nx), where
    L[k] = S[k][k-1] and M[k] = Phi^-1[k][k-1] (L[0] = M[0] = 0).
    """
    A, B, Q, R = map(_f64, (A, B, Q, R))
    N, nx = A.shape[0], A.shape[1]
    nu = B.shape[2]
    D, L, Di, M = (np.zeros((N, nx, nx)) for _ in range(4))
    st = lib().ssp_oracle_build(N, nx, nu, _dp(A), _dp(B), _dp(Q), _dp(R), PC[pc],
                                _dp(D), _dp(L), _dp(Di), _dp(M))
    return st, D, L, Di, M


def precond(D, L, pc: str = "sym"):
    """Preconditioner of a block-tridiagonal S given by blocks (N, nx, nx):
    D[k] = S[k][k], L[k] = S[k][k-1] (L[0] unused), with D[k] taken as
    (D[k] + D[k]^T) / 2.  Returns (status, Dinv, M) with M[k] = Phi^-1[k][k-1].
    """
    D, L = map(_f64, (D, L))
    D = _f64(0.5 * (D + D.transpose(0, 2, 1)))
    N, nx = D.shape[0], D.shape[1]
    Di, M = np.zeros((N, nx, nx)), np.zeros((N, nx, nx))
    st = lib().ssp_oracle_precond(N, nx, PC[pc], _dp(D), _dp(L), _dp(Di), _dp(M))
    return st, Di, M


def btmv(Dg, Sb, x):
    """y = T x for the symmetric block-tridiagonal T = (Dg diagonal, Sb sub-diagonal)."""
    Dg, Sb, x = map(_f64, (Dg, Sb, x))
    N, nx = Dg.shape[0], Dg.shape[1]
    y = np.zeros(N * nx)
    lib().ssp_oracle_btmv(N, nx, _dp(Dg), _dp(Sb), _dp(x.ravel()), _dp(y))
    return y


def pcg(D, L, Dinv, M, gamma, tol=1e-8, max_iter=None, lam0=None, poly=0):
    """FP64 PCG; returns (status, lam, iters).  poly = 0: Phi^-1 is the
    block-tridiagonal (Dinv, M); poly = m >= 1: the Neumann polynomial of
    degree m with Psi = D (M ignored)."""
    D, L, Dinv, M, gamma = map(_f64, (D, L, Dinv, M, gamma))
    N, nx = D.shape[0], D.shape[1]
    lam = np.zeros(N * nx) if lam0 is None else _f64(lam0).copy()
    it = C.c_int(0)
    mi = 10 * N * nx if max_iter is None else max_iter
    st = lib().ssp_oracle_pcg(N, nx, _dp(D), _dp(L), _dp(Dinv), _dp(M), int(poly), _dp(gamma), tol, mi,
                              _dp(lam), C.byref(it))
    return st, lam, it.value


def pcg_mixed(D, L, Dinv, M, gamma, tol=1e-6, max_iter=None, refine=True, lam0=None,
              max_outer=MAX_OUTER, theta=THETA, tau_min=TAU_MIN, poly=0):
    """Float inner PCG with optional FP64 refinement; returns (status, lam, iters, outer)."""
    D, L, Dinv, M, gamma = map(_f64, (D, L, Dinv, M, gamma))
    N, nx = D.shape[0], D.shape[1]
    lam = np.zeros(N * nx) if lam0 is None else _f64(lam0).copy()
    it, ou = C.c_int(0), C.c_int(0)
    mi = 10 * N * nx if max_iter is None else max_iter
    st = lib().ssp_oracle_pcg_mixed(N, nx, _dp(D), _dp(L), _dp(Dinv), _dp(M), int(poly), _dp(gamma), tol, mi,
                                    int(refine), max_outer, theta, tau_min, _dp(lam),
                                    C.byref(it), C.byref(ou))
    return st, lam, it.value, ou.value


def apply_precond(L, Dinv, M, r, poly=0):
    """z = Phi^-1 r exactly as the oracle's PCG applies it (L: S's
    sub-diagonal blocks, used by the polynomial forms)."""
    L, Dinv, M, r = map(_f64, (L, Dinv, M, r))
    N, nx = Dinv.shape[0], Dinv.shape[1]
    z = np.zeros(N * nx)
    lib().ssp_oracle_apply_precond(N, nx, _dp(Dinv), _dp(M), _dp(L), int(poly), _dp(r.ravel()), _dp(z))
    return z


def kkt_rhs(A, B, Q, R, q, r, c):
    """gamma = c - C G^-1 g for one problem (Eq. schur with the zeta blocks);
    A, Q: (N, nx, nx), B: (N, nx, nu), R: (N, nu, nu); q, c: N*nx; r: N*nu
    (block N-1 unused).  Returns (status, gamma)."""
    A, B, Q, R, q, r, c = map(_f64, (A, B, Q, R, q, r, c))
    N, nx, nu = A.shape[0], A.shape[1], B.shape[2]
    g = np.zeros(N * nx)
    st = lib().ssp_oracle_kkt_rhs(N, nx, nu, _dp(A), _dp(B), _dp(Q), _dp(R), _dp(q.ravel()), _dp(r.ravel()),
                                  _dp(c.ravel()), _dp(g))
    return st, g


def kkt_recover(A, B, Q, R, q, r, lam):
    """dz* = G^-1 (g - C^T lambda*) with lambda* = -lam (the library's sign);
    returns (status, dx (N*nx), du (N*nu, block N-1 zero))."""
    A, B, Q, R, q, r, lam = map(_f64, (A, B, Q, R, q, r, lam))
    N, nx, nu = A.shape[0], A.shape[1], B.shape[2]
    dx, du = np.zeros(N * nx), np.zeros(max(N * nu, 1))
    st = lib().ssp_oracle_kkt_recover(N, nx, nu, _dp(A), _dp(B), _dp(Q), _dp(R), _dp(q.ravel()),
                                      _dp(r.ravel() if r.size else np.zeros(1)), _dp(lam.ravel()), _dp(dx), _dp(du))
    return st, dx, du[:N * nu]


def relres(D, L, gamma, lam) -> float:
    D, L, gamma, lam = map(_f64, (D, L, gamma, lam))
    return lib().ssp_oracle_relres(D.shape[0], D.shape[1], _dp(D), _dp(L), _dp(gamma), _dp(lam))


def direct(D, L, gamma):
    """Block-tridiagonal Cholesky solve; returns (status, lam)."""
    D, L, gamma = map(_f64, (D, L, gamma))
    N, nx = D.shape[0], D.shape[1]
    lam = np.zeros(N * nx)
    st = lib().ssp_oracle_direct(N, nx, _dp(D), _dp(L), _dp(gamma), _dp(lam))
    return st, lam


def set_threads(n: int) -> None:
    """OpenMP threads of the batch drivers (timing)."""
    lib().ssp_oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().ssp_oracle_get_threads())


def build_batch(b, pc: str = "sym") -> np.ndarray:
    """The build alone for every problem of a packed batch (timing); returns
    the per-problem build status."""
    P = b.P
    ip = lambda a: np.ascontiguousarray(a, dtype=np.int32).ctypes.data_as(C.POINTER(C.c_int))
    N32, nx32, nu32 = (np.ascontiguousarray(a, dtype=np.int32) for a in (b.N, b.nx, b.nu))
    offs = [np.ascontiguousarray(o, dtype=np.int64) for o in (b.off_nn, b.off_nu, b.off_uu)]
    i64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
    A, B, Q, R = map(_f64, (b.A, b.B, b.Q, b.R))
    status = np.zeros(P, dtype=np.int32)
    lib().ssp_oracle_build_batch(P, ip(N32), ip(nx32), ip(nu32), *(i64(o) for o in offs), _dp(A), _dp(B), _dp(Q),
                                 _dp(R), PC[pc], ip(status))
    return status


def solve_batch(b, pc: str = "sym", precision: str = "fp64", tol: float = 1e-8,
                max_iter: int | None = None, lam0=None, max_outer=MAX_OUTER, theta=THETA,
                tau_min=TAU_MIN, fallback: bool = False):
    """Build + solve every problem of a packed batch (OpenMP over problems).

    Returns dict(lam, iters, outer, relres, status).  ``max_iter`` defaults to
    10 * N * nx per problem (the largest problem's value is used for all).
    With ``fallback``, a start ``lam0`` whose residual is not below ||gamma||
    is replaced by zero and the status carries WARM_FALLBACK.
    """
    P = b.P
    ip = lambda a: np.ascontiguousarray(a, dtype=np.int32).ctypes.data_as(C.POINTER(C.c_int))
    i64 = lambda a: np.ascontiguousarray(a, dtype=np.int64).ctypes.data_as(C.POINTER(C.c_int64))
    N32, nx32, nu32 = (np.ascontiguousarray(a, dtype=np.int32) for a in (b.N, b.nx, b.nu))
    offs = [np.ascontiguousarray(o, dtype=np.int64) for o in (b.off_nn, b.off_nu, b.off_uu, b.off_v)]
    lam = np.zeros(b.gamma.shape[0]) if lam0 is None else _f64(lam0).copy()
    iters, outer, status = (np.zeros(P, dtype=np.int32) for _ in range(3))
    rel = np.zeros(P)
    if max_iter is None:
        max_iter = int(10 * np.max(b.N.astype(np.int64) * b.nx)) if P else 0
    A, B, Q, R, g = map(_f64, (b.A, b.B, b.Q, b.R, b.gamma))
    lib().ssp_oracle_solve_batch(P, ip(N32), ip(nx32), ip(nu32), *(i64(o) for o in offs),
                                 _dp(A), _dp(B), _dp(Q), _dp(R), _dp(g), PC[pc], PREC[precision],
                                 tol, max_iter, max_outer, theta, tau_min, int(fallback), _dp(lam), ip(iters),
                                 ip(outer), _dp(rel), ip(status))
    return dict(lam=lam, iters=iters, outer=outer, relres=rel, status=status)
