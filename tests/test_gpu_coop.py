"""GPU parity of the cooperative single-problem solve (a batch of one problem
with N >= 24 knots spreads its knots over the grid, a few per workgroup, each
workgroup also carrying two ghost knots on each side)
against the CPU oracle and against the batched fused kernel on the same
problem.

Tolerances are those of the batched parity tests: FP64 to 1e-8 agrees with
the oracle's PCG to 1e-10 in lambda and +-1 in iterations (same recurrences,
different summation order); FP32 storage with FP64 refinement to 1e-6 meets
the FP64 residual on the problem and lands within kappa_2(S) * 1e-6 of the
oracle's direct solution.
"""
import numpy as np
import pytest

import oracle
from paper_2309_06427_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solve(b, pc, prec, tol, kernel=0, max_iter=0, lam0=None, fallback=False):
    """kernel 0: automatic (cooperative for one problem of >= 64 knots),
    2: the batched fused kernel, 3: cooperative at any length."""
    from paper_2309_06427_amd import solver
    db = solver.DeviceBatch(b)
    if kernel:
        db.solver.set_mapping(256, 0, kernel)
    db.build(pc, prec)
    l0 = None if lam0 is None else torch.from_numpy(lam0).cuda()
    db.solve(tol, max_iter, l0, fallback=fallback)
    return db.results()


def _one(N, nx, nu, seed):
    return inputs.pack([inputs.draw_problem(np.random.default_rng(seed), N, nx, nu)])


def _kappa(D, L):
    """2-norm condition number of the block-tridiagonal S from its extreme
    eigenvalues (sparse Lanczos; shift-invert at zero for the smallest)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh
    N = D.shape[0]
    rows = [[None] * N for _ in range(N)]
    for k in range(N):
        rows[k][k] = sp.csr_matrix(D[k])
        if k:
            rows[k][k - 1] = sp.csr_matrix(L[k])
            rows[k - 1][k] = sp.csr_matrix(L[k].T)
    S = sp.bmat(rows, format="csc")
    hi = eigsh(S, k=1, which="LA", return_eigenvectors=False)[0]
    lo = eigsh(S, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    return hi / lo


@pytest.mark.parametrize("pc", ["sym", "add", "bj"])
@pytest.mark.parametrize("N,nx,nu", [(64, 6, 3), (129, 14, 7), (66, 26, 13), (150, 5, 2)])
def test_coop_fp64_matches_oracle(N, nx, nu, pc):
    """Several workgroups, a partial last workgroup (N % 4 != 0), runtime nx."""
    b = _one(N, nx, nu, seed=N + nx)
    out = _solve(b, pc, "fp64", 1e-8)
    ref = oracle.solve_batch(b, pc, "fp64", tol=1e-8)
    assert out["status"][0] == 0 and ref["status"][0] == 0
    assert out["relres"][0] <= 1.0001e-8
    assert abs(int(out["iters"][0]) - int(ref["iters"][0])) <= 1
    err = np.linalg.norm(out["lam"] - ref["lam"]) / np.linalg.norm(ref["lam"])
    assert err <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
@pytest.mark.parametrize("N,nx,nu", [(1, 6, 3), (2, 14, 7), (3, 5, 2), (5, 26, 13), (9, 36, 12), (17, 14, 7)])
def test_coop_short_problems(N, nx, nu, prec):
    """Forced cooperative solve of short problems: ghost knots past both ends,
    one or two workgroups, a partial last workgroup."""
    b = _one(N, nx, nu, seed=100 + N)
    tol = 1e-8 if prec == "fp64" else 1e-6
    out = _solve(b, "sym", prec, tol, kernel=3)
    ref = oracle.solve_batch(b, "sym", prec, tol=tol)
    assert out["status"][0] & ~16 == 0 and out["relres"][0] <= tol * 1.0001
    if prec == "fp64":
        assert abs(int(out["iters"][0]) - int(ref["iters"][0])) <= 1
        err = np.linalg.norm(out["lam"] - ref["lam"]) / np.linalg.norm(ref["lam"])
        assert err <= 1e-10
    if N == 1:
        assert out["iters"][0] == 1  # Phi^-1 = S^-1


def test_coop_long_horizon_nx36_matches_fused_and_oracle():
    """N = 512, nx = 36: the single-problem workload at its full size."""
    b = inputs.make("single_n512_nx36")
    ref = oracle.solve_batch(b, "sym", "fp64", tol=1e-8)
    for kernel in (0, 2):
        out = _solve(b, "sym", "fp64", 1e-8, kernel=kernel)
        assert out["status"][0] == 0 and out["relres"][0] <= 1.0001e-8
        assert abs(int(out["iters"][0]) - int(ref["iters"][0])) <= 1
        err = np.linalg.norm(out["lam"] - ref["lam"]) / np.linalg.norm(ref["lam"])
        assert err <= 1e-10, (kernel, err)


@pytest.mark.parametrize("N,nx,nu", [(96, 14, 7), (512, 36, 12), (77, 26, 13)])
def test_coop_fp32_refine_reaches_fp64_residual(N, nx, nu):
    b = _one(N, nx, nu, seed=3 * N + nx)
    tol = 1e-6
    out = _solve(b, "sym", "fp32_refine64", tol)
    assert out["status"][0] & ~16 == 0, out["status"]
    assert out["relres"][0] <= tol * 1.0001
    ref = oracle.solve_batch(b, "sym", "fp32_refine64", tol=tol)
    assert ref["status"][0] & ~16 == 0
    p = b.problem(0)
    st, D, L, Di, M = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
    st, lam = oracle.direct(D, L, p["gamma"])
    kappa = _kappa(D, L)
    err = np.linalg.norm(out["lam"] - lam) / np.linalg.norm(lam)
    assert err <= kappa * tol * 1.01
    # the same refinement schedule as the batched kernel on this problem
    fused = _solve(b, "sym", "fp32_refine64", tol, kernel=2)
    assert abs(int(out["outer"][0]) - int(fused["outer"][0])) <= 1


def test_coop_status_codes_and_edge_cases():
    rng = np.random.default_rng
    cases = {
        "ok": inputs.draw_problem(rng(1), 80, 6, 3),
        "not_spd": inputs.draw_problem(rng(2), 80, 6, 3),
        "nonfinite": inputs.draw_problem(rng(3), 80, 6, 3),
        "zero": inputs.draw_problem(rng(4), 80, 6, 3),
    }
    cases["not_spd"]["Q"][40] = -np.eye(6)
    cases["nonfinite"]["gamma"][70] = np.nan
    cases["zero"]["gamma"][:] = 0.0
    want = {"ok": 2, "not_spd": 1, "nonfinite": 3, "zero": 0}
    for name, prob in cases.items():
        b = inputs.pack([prob])
        out = _solve(b, "sym", "fp64", 1e-12, max_iter=3)
        ref = oracle.solve_batch(b, "sym", "fp64", tol=1e-12, max_iter=3)
        assert out["status"][0] == want[name] == ref["status"][0], name
        if name == "zero":
            assert out["iters"][0] == 0 and not out["lam"].any()
        if name == "not_spd":
            assert np.isnan(out["relres"][0]) and not out["lam"].any()


def test_coop_warm_starts():
    b = _one(200, 14, 7, seed=11)
    ref = oracle.solve_batch(b, "sym", "fp64", tol=1e-12)
    out = _solve(b, "sym", "fp64", 1e-8, lam0=ref["lam"])
    assert out["iters"][0] == 0 and out["status"][0] == 0
    # a warm start worse than zero is dropped for lambda = 0 (status bit 8)
    bad = 1e3 * np.random.default_rng(0).standard_normal(ref["lam"].shape)
    out = _solve(b, "sym", "fp64", 1e-8, lam0=bad, fallback=True)
    cold = _solve(b, "sym", "fp64", 1e-8)
    assert out["status"][0] == 8 and out["relres"][0] <= 1.0001e-8
    assert out["iters"][0] == cold["iters"][0]
    np.testing.assert_array_equal(out["lam"], cold["lam"])


def test_solve_kernel_reports_the_path():
    from paper_2309_06427_amd import solver
    b = _one(100, 14, 7, seed=9)
    db = solver.DeviceBatch(b)
    assert db.solver.solve_kernel() == (0, 0, 0)
    db.build("sym", "fp32_refine64")
    db.solve(1e-6)
    k, W, G = db.solver.solve_kernel()
    assert k == 3 and 2 <= W <= 4 and G == -(-100 // W)
    db.solver.set_mapping(256, 0, 2)
    db.solve(1e-6)
    assert db.solver.solve_kernel() == (2, 0, 0)
    db.solver.set_mapping(256, 0, 1)
    db.solve(1e-6)
    assert db.solver.solve_kernel() == (1, 0, 0)
    short = solver.DeviceBatch(_one(10, 6, 3, seed=1))  # below the automatic threshold
    short.build("sym", "fp64")
    short.solve(1e-8)
    assert short.solver.solve_kernel()[0] == 2


def test_coop_is_deterministic():
    b = _one(300, 26, 13, seed=5)
    a = _solve(b, "sym", "fp32_refine64", 1e-6)
    c = _solve(b, "sym", "fp32_refine64", 1e-6)
    np.testing.assert_array_equal(a["lam"], c["lam"])
    assert a["iters"][0] == c["iters"][0]
