"""Pins of the oracle's scalar-Jacobi and polynomial preconditioners, its
statuses without refinement, and the KKT step around the solve.

Each test compares oracle output with an independent dense construction
(numpy inverses and solves of matrices built from the paper's definitions), a
closed form, or a special case.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2309_06427_amd import inputs
from tests import dense


def small(N=7, nx=4, nu=2, seed=11, qmode="wishart", cmax=1e4):
    return inputs.single(N, nx, nu, seed, qmode, cmax).problem(0)


def built(p, pc):
    st, D, L, Di, M = oracle.build(p["A"], p["B"], p["Q"], p["R"], pc)
    assert st == oracle.OK
    return D, L, Di, M


def dense_precond(L, Di, M, poly, n):
    """The oracle's Phi^-1 as a dense matrix: its application to unit vectors."""
    cols = [oracle.apply_precond(L, Di, M, e, poly) for e in np.eye(n)]
    return np.array(cols).T


# ------------------------------------------------- scalar Jacobi (Eq. jacobi)

@pytest.mark.parametrize("N,nx", [(1, 3), (5, 4), (8, 6)])
def test_scalar_jacobi_is_the_inverse_diagonal(N, nx):
    """Phi = diag(S): the stored D^-1 slots hold 1 / S_ii and nothing else."""
    p = small(N, nx, 2, 700 + N)
    D, L, Di, M = built(p, "jacobi")
    S = dense.assemble(D, L)
    want = np.diag(1.0 / np.diag(S))
    got = dense_precond(L, Di, M, 0, S.shape[0])
    assert np.abs(got - want).max() <= 1e-15 * np.abs(want).max()


def test_scalar_jacobi_pcg_matches_dense_and_is_slowest():
    b = inputs.make("single_n50_nx14")
    p = b.problem(0)
    its = {}
    for pc in ("jacobi", "bj", "sym"):
        D, L, Di, M = built(p, pc)
        S = dense.assemble(D, L)
        x = sla.cho_solve(sla.cho_factor(S), p["gamma"])
        st, lam, it = oracle.pcg(D, L, Di, M, p["gamma"], tol=1e-10)
        assert st == oracle.OK
        assert np.linalg.norm(lam - x) / np.linalg.norm(x) <= np.linalg.cond(S) * 1e-10
        its[pc] = it
    # the ordering the paper's Sec. V reports (scalar Jacobi needs the most iterations)
    assert its["sym"] < its["bj"] < its["jacobi"]


# ---------------------------------- polynomial preconditioner (Eq. polynomial_precon)

@pytest.mark.parametrize("N,poly", [(2, 1), (5, 1), (6, 2), (7, 3), (9, 2), (4, 4)])
def test_neumann_polynomial_equals_dense_series(N, poly):
    """(I + Psi^-1 P + ... + (Psi^-1 P)^m) Psi^-1 with Psi = block-diag(S),
    P = Psi - S, built densely; degree 1 is the symmetric stair (Sec. IV)."""
    nx = 3
    p = small(N, nx, 2, 800 + N)
    D, L, Di, M = built(p, "bj")
    S = dense.assemble(D, L)
    Psi = dense.block_diag_part(S, nx)
    Pm = Psi - S
    Pinv = np.linalg.inv(Psi)
    K = Pinv @ Pm
    want = sum(np.linalg.matrix_power(K, i) for i in range(poly + 1)) @ Pinv
    got = dense_precond(L, Di, M, poly, S.shape[0])
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
    assert np.abs(got - got.T).max() <= 1e-11 * np.abs(got).max()  # symmetric for every degree
    if poly == 1:
        Pl, Pr = dense.stair(S, nx, "l"), dense.stair(S, nx, "r")
        sym = np.linalg.inv(Pl) + np.linalg.inv(Pr) - Pinv
        assert np.abs(got - sym).max() <= 1e-11 * np.abs(sym).max()


def test_neumann_pin_detects_a_missing_inverse_on_the_right_hand_side():
    """A Horner step z = D^-1 r - O z (D^-1 dropped on the O z term) differs
    from the dense series, so the pin above would catch it."""
    nx, N = 3, 6
    p = small(N, nx, 2, 811)
    D, L, Di, M = built(p, "bj")
    S = dense.assemble(D, L)
    Psi = dense.block_diag_part(S, nx)
    Pinv = np.linalg.inv(Psi)
    O = S - Psi
    bad = Pinv - O @ Pinv
    good = dense_precond(L, Di, M, 1, S.shape[0])
    assert np.abs(bad - good).max() > 1e-3


@pytest.mark.parametrize("N", [4, 7])
def test_neumann_spectrum_closed_form(N):
    """With nu the eigenvalues of K = D^-1 (S - D) (block-Jacobi iteration
    matrix), the degree-m preconditioned spectrum is 1 - (-nu)^(m+1): in
    (0, 1] for odd m, (0, 2) for even m."""
    nx = 3
    p = small(N, nx, 2, 820 + N, "logcond", 1e3)
    D, L, Di, M = built(p, "bj")
    S = dense.assemble(D, L)
    Psi = dense.block_diag_part(S, nx)
    nu = np.real(np.linalg.eigvals(np.linalg.solve(Psi, S - Psi)))
    for m in (1, 2, 3):
        Phi = dense_precond(L, Di, M, m, S.shape[0])
        sp = dense.precond_spectrum(0.5 * (Phi + Phi.T), S)
        pred = np.sort(1 - (-nu) ** (m + 1))
        assert np.allclose(sp, pred, atol=1e-9), m
        if m % 2:
            assert sp.max() <= 1 + 1e-10
        assert sp.min() > 0


@pytest.mark.parametrize("pc", ["poly2", "poly3"])
def test_polynomial_pcg_matches_dense_cholesky(pc):
    b = inputs.make("single_n50_nx14")
    p = b.problem(0)
    D, L, Di, M = built(p, pc)
    assert not M.any()
    S = dense.assemble(D, L)
    x = sla.cho_solve(sla.cho_factor(S), p["gamma"])
    st, lam, it = oracle.pcg(D, L, Di, M, p["gamma"], tol=1e-10, poly=oracle.POLY_DEGREE[pc])
    assert st == oracle.OK
    assert np.linalg.norm(lam - x) / np.linalg.norm(x) <= np.linalg.cond(S) * 1e-10


def test_degree_three_needs_fewer_iterations_than_the_symmetric_stair():
    """1 - nu^4 is more clustered than 1 - nu^2 (same bytes per iteration in
    a fused pass); degree 2 is worse than degree 1 (spectrum 1 + nu^3)."""
    b = inputs.make("single_n50_nx14")
    p = b.problem(0)
    its = {}
    for pc, poly in (("sym", 0), ("poly2", 2), ("poly3", 3)):
        D, L, Di, M = built(p, pc)
        its[pc] = oracle.pcg(D, L, Di, M, p["gamma"], tol=1e-8, poly=poly)[2]
    assert its["poly3"] < its["sym"] < its["poly2"]


def test_batch_driver_runs_every_preconditioner():
    b = inputs.make("batch4096_ragged", P=5)
    for pc in oracle.PC:
        r = oracle.solve_batch(b, pc, "fp32_refine64", tol=1e-6)
        assert ((r["status"] & ~oracle.PC_FALLBACK) == 0).all(), pc
        assert r["relres"].max() <= 1e-6, pc
        r64 = oracle.solve_batch(b, pc, "fp64", tol=1e-9)
        assert (r64["status"] == 0).all() and r64["relres"].max() <= 1e-9, pc


# ------------------------------------------------ statuses without refinement

def test_one_float_solve_that_misses_the_true_tolerance_is_reported():
    """FP32 without refinement: the recurrence residual meets tol but the true
    FP64 residual does not (float storage error ~ eps32 kappa) -> INACCURATE."""
    b = inputs.make("batch1024_n128_nx26_cond1e6", P=4)
    r32 = oracle.solve_batch(b, "sym", "fp32", tol=1e-6)
    miss = r32["relres"] > 1e-6
    assert miss.any()
    assert (r32["status"][miss] & 7 != oracle.OK).all()
    st_ok = r32["status"][~miss]
    assert (st_ok == oracle.OK).all()
    assert ((r32["status"][miss] & 7) == oracle.INACCURATE).any()


# --------------------------------------------------- KKT step (Eq. schur, zeta)

def kkt_dense(p, q, r, c):
    """Solve [G C^T; C 0] [dz; lambda*] = [g; c] densely.  C's sign is the
    one the paper's block form of gamma fixes (row 0: +I on x_0; row k+1:
    -A_k, -B_k, +I on x_k, u_k, x_{k+1}); z = (x_0, u_0, ..., u_{N-2}, x_{N-1})."""
    A, B, Q, R = p["A"], p["B"], p["Q"], p["R"]
    N, nx, nu = A.shape[0], A.shape[1], B.shape[2]
    xpos = [k * (nx + nu) for k in range(N)]
    upos = [k * (nx + nu) + nx for k in range(N - 1)]
    nz = N * nx + (N - 1) * nu
    G = np.zeros((nz, nz))
    g = np.zeros(nz)
    Cm = np.zeros((N * nx, nz))
    for k in range(N):
        G[xpos[k]:xpos[k] + nx, xpos[k]:xpos[k] + nx] = Q[k]
        g[xpos[k]:xpos[k] + nx] = q[k * nx:(k + 1) * nx]
        if k < N - 1:
            G[upos[k]:upos[k] + nu, upos[k]:upos[k] + nu] = R[k]
            g[upos[k]:upos[k] + nu] = r[k * nu:(k + 1) * nu]
    Cm[0:nx, 0:nx] = np.eye(nx)
    for k in range(N - 1):
        rows = slice((k + 1) * nx, (k + 2) * nx)
        Cm[rows, xpos[k]:xpos[k] + nx] = -A[k]
        Cm[rows, upos[k]:upos[k] + nu] = -B[k]
        Cm[rows, xpos[k + 1]:xpos[k + 1] + nx] = np.eye(nx)
    K = np.block([[G, Cm.T], [Cm, np.zeros((N * nx, N * nx))]])
    sol = np.linalg.solve(K, np.concatenate([g, c]))
    dz, lam_star = sol[:nz], sol[nz:]
    gamma = c - Cm @ np.linalg.solve(G, g)
    dx = np.concatenate([dz[xpos[k]:xpos[k] + nx] for k in range(N)])
    du = np.concatenate([dz[upos[k]:upos[k] + nu] for k in range(N - 1)] + [np.zeros(nu)])
    return gamma, lam_star, dx, du, Cm, G


@pytest.mark.parametrize("N,nx,nu,seed", [(1, 3, 2, 0), (2, 4, 2, 1), (6, 4, 2, 2), (9, 6, 3, 3)])
def test_kkt_step_equals_the_dense_kkt_solve(N, nx, nu, seed):
    """gamma = c - C G^-1 g, the library-sign solution lambda = -lambda*, and
    dz* = G^-1 (g - C^T lambda*) all agree with one dense KKT solve; S of the
    same C is the oracle's S (the negated Schur complement)."""
    p = small(N, nx, nu, 900 + seed)
    rng = np.random.default_rng(seed)
    q, r, c = rng.standard_normal(N * nx), rng.standard_normal(N * nu), rng.standard_normal(N * nx)
    gamma_d, lam_star, dx_d, du_d, Cm, G = kkt_dense(p, q, r, c)
    st, gamma = oracle.kkt_rhs(p["A"], p["B"], p["Q"], p["R"], q, r, c)
    assert st == oracle.OK
    assert np.abs(gamma - gamma_d).max() <= 1e-12 * np.abs(gamma_d).max()
    D, L, _, _ = built(p, "sym")
    S_neg = Cm @ np.linalg.solve(G, Cm.T)
    assert np.abs(dense.assemble(D, L) - S_neg).max() <= 1e-12 * np.abs(S_neg).max()
    st, lam = oracle.direct(D, L, gamma)
    assert st == oracle.OK
    assert np.abs(lam + lam_star).max() <= 1e-10 * np.abs(lam_star).max()
    st, dx, du = oracle.kkt_recover(p["A"], p["B"], p["Q"], p["R"], q, r, lam)
    assert st == oracle.OK
    assert np.abs(dx - dx_d).max() <= 1e-9 * np.abs(dx_d).max()
    if nu:
        assert np.abs(du - du_d).max() <= 1e-9 * max(np.abs(du_d).max(), 1e-300)
        assert not du[(N - 1) * nu:].any()


def test_kkt_pin_detects_a_flipped_multiplier_sign():
    """Recovering with lambda* itself instead of -lambda* (the sign the
    negated system introduces) misses the dense solution."""
    N, nx, nu = 5, 4, 2
    p = small(N, nx, nu, 931)
    rng = np.random.default_rng(5)
    q, r, c = rng.standard_normal(N * nx), rng.standard_normal(N * nu), rng.standard_normal(N * nx)
    _, lam_star, dx_d, _, _, _ = kkt_dense(p, q, r, c)
    _, dx_bad, _ = oracle.kkt_recover(p["A"], p["B"], p["Q"], p["R"], q, r, lam_star)
    assert np.abs(dx_bad - dx_d).max() > 1e-3 * np.abs(dx_d).max()


def test_kkt_rhs_flags_an_indefinite_cost_block():
    N, nx, nu = 4, 3, 2
    p = small(N, nx, nu, 940)
    Q = p["Q"].copy()
    Q[2] = -np.eye(nx)
    z = np.zeros(N * nx)
    st, _ = oracle.kkt_rhs(p["A"], p["B"], Q, p["R"], z, np.zeros(N * nu), z)
    assert st == oracle.NOT_SPD
