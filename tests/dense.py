"""Dense numpy constructions used to pin the oracle (tests only).

Each function builds a matrix straight from a definition in the paper with
dense numpy linear algebra, independently of the oracle's block formulas.
"""
import numpy as np


def kkt_schur(A, B, Q, R):
    """C G^-1 C^T of the trajectory QP with N states and N-1 controls.

    Decision vector z = (x_0, u_0, x_1, u_1, ..., u_{N-2}, x_{N-1}); cost
    Hessian G = blkdiag(Q_0, R_0, ..., R_{N-2}, Q_{N-1}); constraints
    x_0 = x_s and x_{k+1} = A_k x_k + B_k u_k written as rows of C
    (Sec. II-A, Eq. schur).  This is the negated (SPD) Schur complement.
    """
    N, nx, nu = A.shape[0], A.shape[1], B.shape[2]
    sizes = []
    for k in range(N):
        sizes.append(nx)
        if k < N - 1:
            sizes.append(nu)
    off = np.concatenate([[0], np.cumsum(sizes)])
    nz = int(off[-1])
    G = np.zeros((nz, nz))
    xpos = lambda k: int(off[2 * k])
    upos = lambda k: int(off[2 * k + 1])
    for k in range(N):
        G[xpos(k):xpos(k) + nx, xpos(k):xpos(k) + nx] = Q[k]
        if k < N - 1:
            G[upos(k):upos(k) + nu, upos(k):upos(k) + nu] = R[k]
    Cm = np.zeros((N * nx, nz))
    Cm[0:nx, xpos(0):xpos(0) + nx] = -np.eye(nx)
    for k in range(N - 1):
        rows = slice((k + 1) * nx, (k + 2) * nx)
        Cm[rows, xpos(k):xpos(k) + nx] = A[k]
        Cm[rows, upos(k):upos(k) + nu] = B[k]
        Cm[rows, xpos(k + 1):xpos(k + 1) + nx] = -np.eye(nx)
    return Cm @ np.linalg.solve(G, Cm.T)


def assemble(Dg, Sb):
    """Dense symmetric block-tridiagonal matrix (diagonal Dg, sub-diagonal Sb)."""
    N, nx = Dg.shape[0], Dg.shape[1]
    T = np.zeros((N * nx, N * nx))
    for k in range(N):
        T[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = Dg[k]
        if k > 0:
            T[k * nx:(k + 1) * nx, (k - 1) * nx:k * nx] = Sb[k]
            T[(k - 1) * nx:k * nx, k * nx:(k + 1) * nx] = Sb[k].T
    return T


def block_diag_part(S, nx):
    n = S.shape[0] // nx
    Dm = np.zeros_like(S)
    for k in range(n):
        sl = slice(k * nx, (k + 1) * nx)
        Dm[sl, sl] = S[sl, sl]
    return Dm


def stair(S, nx, side):
    """Left or right stair matrix of Eq. (stair).

    Psi_l keeps the full block rows 2, 4, ... (1-indexed) of S and only the
    diagonal block elsewhere; Psi_r keeps the full rows 1, 3, 5, ....
    """
    n = S.shape[0] // nx
    Psi = block_diag_part(S, nx)
    full_parity = 1 if side == "l" else 0      # 0-indexed parity of the full rows
    for i in range(n):
        if i % 2 != full_parity:
            continue
        rs = slice(i * nx, (i + 1) * nx)
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                cs = slice(j * nx, (j + 1) * nx)
                Psi[rs, cs] = S[rs, cs]
    return Psi


def block_pattern(Mat, nx, tol):
    n = Mat.shape[0] // nx
    pat = np.zeros((n, n), dtype=bool)
    for i in range(n):
        for j in range(n):
            pat[i, j] = np.abs(Mat[i * nx:(i + 1) * nx, j * nx:(j + 1) * nx]).max() > tol
    return pat


def precond_spectrum(Phi_inv, S):
    """Eigenvalues of Phi^-1 S through the SPD similar matrix L^T S L, Phi^-1 = L L^T."""
    Lc = np.linalg.cholesky(Phi_inv)
    return np.linalg.eigvalsh(Lc.T @ S @ Lc)


def kappa(D, L):
    """2-norm condition number of the SPD block-tridiagonal S with diagonal
    blocks D_k and sub-diagonal blocks L_k = S[k][k-1] (L_0 unused): dense
    eigenvalues for small S, else the extreme eigenvalues of the sparse S by
    Lanczos (the smallest by shift-invert about zero)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    N, nx = D.shape[0], D.shape[1]
    if N * nx <= 600:
        ev = np.linalg.eigvalsh(assemble(D, L))
        return float(ev[-1] / ev[0])
    blocks = [[None] * N for _ in range(N)]
    for k in range(N):
        blocks[k][k] = sp.csr_matrix(D[k])
        if k:
            blocks[k][k - 1] = sp.csr_matrix(L[k])
            blocks[k - 1][k] = sp.csr_matrix(L[k].T)
    S = sp.bmat(blocks, format="csc")
    lmax = sla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    lmin = sla.eigsh(S, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    return float(lmax / lmin)
