"""The KKT step around the solve (Sec. II-A, Eq. (schur) and the zeta blocks)
on the GPU against the CPU oracle.

Tolerances: gamma and (dx, du) are a few small FP64 matrix-vector products
per knot with the FP64 Q_k^-1, R_k^-1 of the build; the oracle forms the same
products from its own Cholesky inverses, so both agree to ~1e-12 relative to
the largest entry (1e-10 is asserted).  End to end, the solve stops at a
relative residual tol, so dz carries an error of about kappa_2(S) * tol
against the dense KKT solution.
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


def mixed_batch(seed):
    """Ragged shapes incl. N = 1, nu = 0, nx = 1 and nx = 64 (the largest state
    size); nx = 6, 14, 26 with nu <= nx / 2 run the staged kernels (among them
    N = 1, nu = 0, and horizons that span several of their strips of 64, 32
    and 8 knots, with ragged ends), the other shapes the generic ones."""
    rng = np.random.default_rng(seed)
    shapes = [(1, 6, 3), (2, 4, 2), (17, 14, 7), (33, 26, 13), (9, 36, 12), (5, 1, 0), (12, 5, 0),
              (3, 64, 16), (40, 6, 3), (64, 14, 1), (1, 26, 13), (4, 14, 0), (7, 26, 2), (5, 26, 20),
              (70, 6, 2), (131, 6, 3)]
    probs = [inputs.draw_problem(rng, N, nx, nu, "wishart", 1e4) for N, nx, nu in shapes]
    return inputs.pack(probs)


def vectors(b, seed):
    rng = np.random.default_rng(seed)
    nv = int(b.off_v[-1])
    off_u = np.zeros(b.P + 1, dtype=np.int64)
    off_u[1:] = np.cumsum(b.N.astype(np.int64) * b.nu.astype(np.int64))
    return rng.standard_normal(nv), rng.standard_normal(int(off_u[-1])), rng.standard_normal(nv), off_u


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
def test_kkt_rhs_and_recovery_match_the_oracle(prec):
    """gamma from (q, r, c) and (dx, du) from a given lambda, knot by knot,
    against the oracle's KKT functions on every problem of a ragged batch;
    the storage precision of the solve does not touch these FP64 products."""
    from paper_2309_06427_amd import solver
    b = mixed_batch(81)
    q, r, c, off_u = vectors(b, 82)
    lam = np.random.default_rng(83).standard_normal(int(b.off_v[-1]))
    with solver.DeviceBatch(b) as db:
        assert np.array_equal(db.solver.off_u, off_u)
        db.build("sym", prec)
        assert (db.status.cpu().numpy() == 0).all()
        dq, dr, dc = dev(q), dev(r), dev(c)
        db.kkt_rhs(dq, dr, dc)
        db.lam.copy_(dev(lam))
        dx, du = db.kkt_recover(dq, dr)
        torch.cuda.synchronize()
        g, dx, du = db.gamma.cpu().numpy(), dx.cpu().numpy(), du.cpu().numpy()
    for i in range(b.P):
        p = b.problem(i)
        N, nx, nu = p["N"], p["nx"], p["nu"]
        sv, su = slice(b.off_v[i], b.off_v[i + 1]), slice(off_u[i], off_u[i + 1])
        st, g_ref = oracle.kkt_rhs(p["A"], p["B"], p["Q"], p["R"], q[sv], r[su], c[sv])
        assert st == oracle.OK
        assert np.abs(g[sv] - g_ref).max() <= 1e-10 * np.abs(g_ref).max(), i
        st, dx_ref, du_ref = oracle.kkt_recover(p["A"], p["B"], p["Q"], p["R"], q[sv], r[su], lam[sv])
        assert st == oracle.OK
        assert np.abs(dx[sv] - dx_ref).max() <= 1e-10 * np.abs(dx_ref).max(), i
        if nu:
            assert np.abs(du[su] - du_ref).max() <= 1e-10 * max(np.abs(du_ref).max(), 1e-300), i
            assert not du[su][(N - 1) * nu:].any(), i


def test_kkt_step_end_to_end_solves_the_dense_kkt_system():
    """gamma -> solve -> recovery on the GPU reproduces the dense KKT solution
    [G C^T; C 0]^-1 [g; c] (lambda* = -lambda) to the solve's tolerance."""
    from paper_2309_06427_amd import solver
    from tests.test_oracle_extensions import kkt_dense
    rng = np.random.default_rng(91)
    shapes = [(1, 6, 3), (7, 4, 2), (20, 6, 3), (12, 14, 7), (9, 5, 0)]
    b = inputs.pack([inputs.draw_problem(rng, N, nx, nu, "wishart", 1e4) for N, nx, nu in shapes])
    q, r, c, off_u = vectors(b, 92)
    tol = 1e-10
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp64")
        dq, dr = dev(q), dev(r)
        db.kkt_rhs(dq, dr, dev(c))
        db.solve(tol)
        out = db.results()
        dx, du = db.kkt_recover(dq, dr)
        torch.cuda.synchronize()
        dx, du = dx.cpu().numpy(), du.cpu().numpy()
    assert ((out["status"] & ~16) == 0).all(), out["status"]
    for i in range(b.P):
        p = b.problem(i)
        sv, su = slice(b.off_v[i], b.off_v[i + 1]), slice(off_u[i], off_u[i + 1])
        _, lam_star, dx_d, du_d, _, _ = kkt_dense(p, q[sv], r[su], c[sv])
        assert np.abs(out["lam"][sv] + lam_star).max() <= 1e-5 * np.abs(lam_star).max(), i
        assert np.abs(dx[sv] - dx_d).max() <= 1e-5 * np.abs(dx_d).max(), i
        if p["nu"]:
            assert np.abs(du[su] - du_d).max() <= 1e-5 * np.abs(du_d).max(), i


def test_kkt_calls_need_a_build_of_their_own():
    """Before any build, and after a build from ready S blocks (no Q^-1, R^-1),
    the KKT calls are refused with SSP_ERR_STATE and write nothing."""
    from paper_2309_06427_amd import solver
    b = mixed_batch(95)
    q, r, c, _ = vectors(b, 96)
    with solver.DeviceBatch(b) as db:
        dq, dr, dc = dev(q), dev(r), dev(c)
        before = db.gamma.clone()
        with pytest.raises(RuntimeError, match="ssp_kkt_rhs"):
            db.kkt_rhs(dq, dr, dc)
        with pytest.raises(RuntimeError, match="ssp_kkt_recover"):
            db.kkt_recover(dq, dr)
        torch.cuda.synchronize()
        assert torch.equal(before, db.gamma)
        db.build("sym", "fp64")
        db.kkt_rhs(dq, dr, dc)
        torch.cuda.synchronize()
        D, L = np.zeros(int(b.off_nn[-1])), np.zeros(int(b.off_nn[-1]))
        for i in range(b.P):
            p = b.problem(i)
            _, Di, Li, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
            D[b.off_nn[i]:b.off_nn[i + 1]], L[b.off_nn[i]:b.off_nn[i + 1]] = Di.ravel(), Li.ravel()
        db.solver.build_from_blocks("sym", "fp64", dev(D), dev(L), db.status)
        with pytest.raises(RuntimeError, match="ssp_kkt_rhs"):
            db.kkt_rhs(dq, dr, dc)


@pytest.mark.parametrize("kind,prec", [("mixed", "fp64"), ("mixed", "fp32_refine64"), ("scaled", "fp32_refine64")])
def test_build_without_stored_inverses(kind, prec):
    """With ssp_set_keep_inverses(b, 0) the build stores the same S and the
    same preconditioner blocks, bit for bit, and
    the KKT calls are refused until a build that keeps Q^-1, R^-1; after one,
    gamma matches the oracle again."""
    from paper_2309_06427_amd import solver
    # "scaled": state sizes 14 and 26 with nu = nx / 2 only, whose default
    # build is the scaled basis (compared through export(3))
    b = mixed_batch(97) if kind == "mixed" else inputs.batch(12, seed=99, N_range=(1, 40), nx_choices=(14, 26))
    which = (0, 1) if kind == "mixed" else (0, 1, 3)
    q, r, c, off_u = vectors(b, 98)
    with solver.DeviceBatch(b) as db:
        dq, dr, dc = dev(q), dev(r), dev(c)
        db.build("sym", prec)
        keep = [db.export(w) for w in which]
        db.solver.set_keep_inverses(False)
        db.build("sym", prec)
        lean = [db.export(w) for w in which]
        for (d0, o0), (d1, o1) in zip(keep, lean):
            assert np.array_equal(d0, d1) and np.array_equal(o0, o1)
        assert (db.results()["status"] == 0).all()
        with pytest.raises(RuntimeError, match="ssp_kkt_rhs"):
            db.kkt_rhs(dq, dr, dc)
        with pytest.raises(RuntimeError, match="ssp_kkt_recover"):
            db.kkt_recover(dq, dr)
        db.solver.set_keep_inverses(True)
        db.build("sym", prec)
        db.kkt_rhs(dq, dr, dc)
        g = db.gamma.cpu().numpy()
    for i in range(b.P):
        p = b.problem(i)
        sv, su = slice(b.off_v[i], b.off_v[i + 1]), slice(off_u[i], off_u[i + 1])
        _, g_ref = oracle.kkt_rhs(p["A"], p["B"], p["Q"], p["R"], q[sv], r[su], c[sv])
        assert np.abs(g[sv] - g_ref).max() <= 1e-10 * np.abs(g_ref).max(), i
