"""Parity at the benchmark's full size and launch configuration.

The whole ragged batch (4096 problems, N up to 256, nx in {6, 14, 26}, 585 849
knots) is built and solved on the GPU exactly as the benchmark times it: the
scaled persistent solve with the mapping the autotuner picks for it (256
threads, 48 336 B of LDS), symmetric stair, FP32 storage with FP64 refinement
to a relative residual of 1e-6.  The oracle cannot solve all of it in a test,
so a sample of problems is checked one by one: the longest problem of every
state size plus a seeded random draw.

Bars (per sampled problem):
  * the true FP64 relative residual of the GPU's lambda, recomputed by the
    oracle from its own S, is <= tol, and equals the residual the GPU reports
    to 1e-3 tol;
  * ||lam - lam*|| / ||lam*|| <= kappa_2(S) tol against the oracle's direct
    (block-Cholesky) solution, kappa_2(S) from S's extreme eigenvalues;
  * iteration counts within 25 % + 3 of the oracle's own PCG (textbook form in
    the original basis, so not step for step the same).
Over the whole batch: every status is OK (no block-Jacobi takeover) and every
reported residual is <= tol.

The same batch and precision also run every other preconditioner (scalar
Jacobi in the fused solve; block-Jacobi, additive stair and the degree-3
Neumann polynomial in the scaled solve), as the benchmark's comparison does,
with the same per-problem bars against the oracle's direct solution; and the
KKT step around the solve (right-hand side from seeded q, r, c, then the
recovery from the GPU's lambda), whose FP64 products must match the oracle's
KKT functions to 1e-10 of the largest entry on the sampled problems, which
cover every state size and so every KKT kernel class.
"""
import numpy as np
import pytest

import oracle
from paper_2309_06427_amd import inputs
from tests import dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-6
MAPPING = (256, 48336)


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_06427_amd import solver
    b = inputs.make("batch4096_ragged")
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp32_refine64")
        db.solver.set_scaled_mapping(*MAPPING)
        db.solve(TOL)
        out = db.results()
        kern = db.solver.solve_kernel()[0]
        mapping = db.solver.scaled_mapping()
    return b, out, kern, mapping


def sample(b):
    idx = set(int(i) for i in np.random.default_rng(1234).choice(b.P, 40, replace=False))
    for nx in np.unique(b.nx):
        cls = np.flatnonzero(b.nx == nx)
        idx.add(int(cls[np.argmax(b.N[cls])]))
    return sorted(idx)


def test_whole_batch_converges_in_the_bench_configuration(full):
    b, out, kern, mapping = full
    assert kern == 4 and mapping[:2] == MAPPING
    assert b.P == 4096 and int(b.N.sum()) == 585849 and b.N.max() == 256
    assert (out["status"] == 0).all(), np.unique(out["status"], return_counts=True)
    assert out["relres"].max() <= TOL


def test_sampled_problems_match_the_oracle(full):
    b, out, _, _ = full
    ids = sample(b)
    ref = oracle.solve_batch(inputs.pack([b.problem(i) for i in ids]), "sym", "fp32_refine64", tol=TOL,
                             tau_min=min(1e-6, 0.5 * TOL))
    for j, i in enumerate(ids):
        p = b.problem(i)
        lam = out["lam"][b.off_v[i]:b.off_v[i + 1]]
        st, D, L, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        assert st == oracle.OK
        rr = oracle.relres(D, L, p["gamma"], lam)
        assert rr <= TOL * 1.0001, (i, rr)
        assert abs(rr - out["relres"][i]) <= 1e-3 * TOL, (i, rr, out["relres"][i])
        st, lam_star = oracle.direct(D, L, p["gamma"])
        assert st == oracle.OK
        kap = dense.kappa(D, L)
        err = np.linalg.norm(lam - lam_star) / np.linalg.norm(lam_star)
        assert err <= kap * TOL, (i, err, kap)
        it, it_ref = float(out["iters"][i]), float(ref["iters"][j])
        assert abs(it - it_ref) <= 0.25 * it_ref + 3, (i, it, it_ref)


@pytest.fixture(scope="module")
def refs(full):
    """The oracle's S blocks, direct solution and kappa_2(S) of each sampled problem."""
    b = full[0]
    out = {}
    for i in sample(b):
        p = b.problem(i)
        st, D, L, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        assert st == oracle.OK
        st, lam_star = oracle.direct(D, L, p["gamma"])
        assert st == oracle.OK
        out[i] = (D, L, lam_star, dense.kappa(D, L))
    return out


@pytest.mark.parametrize("pc", ["jacobi", "bj", "add", "poly3"])
def test_every_preconditioner_at_full_size(full, refs, pc):
    from paper_2309_06427_amd import solver
    b = full[0]
    with solver.DeviceBatch(b) as db:
        db.build(pc, "fp32_refine64")
        db.solve(TOL)
        out = db.results()
        kern = db.solver.solve_kernel()[0]
    assert kern == (2 if pc == "jacobi" else 4), kern
    assert ((out["status"] & ~16) == 0).all(), np.unique(out["status"], return_counts=True)
    assert out["relres"].max() <= TOL
    for i, (D, L, lam_star, kap) in refs.items():
        p = b.problem(i)
        lam = out["lam"][b.off_v[i]:b.off_v[i + 1]]
        rr = oracle.relres(D, L, p["gamma"], lam)
        assert rr <= TOL * 1.0001, (pc, i, rr)
        err = np.linalg.norm(lam - lam_star) / np.linalg.norm(lam_star)
        assert err <= kap * TOL, (pc, i, err, kap)


def test_kkt_step_at_full_size(full):
    from paper_2309_06427_amd import solver
    b = full[0]
    rng = np.random.default_rng(77)
    off_u = np.concatenate([[0], np.cumsum(b.N.astype(np.int64) * b.nu)])
    nv = int(b.off_v[-1])
    q, c, r = rng.standard_normal(nv), rng.standard_normal(nv), rng.standard_normal(int(off_u[-1]))
    dev = lambda x: torch.from_numpy(x).cuda()
    with solver.DeviceBatch(b) as db:
        assert np.array_equal(db.solver.off_u, off_u)
        db.build("sym", "fp32_refine64")
        db.kkt_rhs(dev(q), dev(r), dev(c))
        torch.cuda.synchronize()
        g = db.gamma.cpu().numpy()
        db.solve(TOL)
        lam = db.results()["lam"]
        dx, du = db.kkt_recover(dev(q), dev(r))
        torch.cuda.synchronize()
        dx, du = dx.cpu().numpy(), du.cpu().numpy()
    ids = sample(b)
    assert set(int(x) for x in b.nx[ids]) == {6, 14, 26}
    for i in ids:
        p = b.problem(i)
        sv, su = slice(b.off_v[i], b.off_v[i + 1]), slice(off_u[i], off_u[i + 1])
        st, g_ref = oracle.kkt_rhs(p["A"], p["B"], p["Q"], p["R"], q[sv], r[su], c[sv])
        assert st == oracle.OK
        assert np.abs(g[sv] - g_ref).max() <= 1e-10 * np.abs(g_ref).max(), i
        st, dx_ref, du_ref = oracle.kkt_recover(p["A"], p["B"], p["Q"], p["R"], q[sv], r[su], lam[sv])
        assert st == oracle.OK
        assert np.abs(dx[sv] - dx_ref).max() <= 1e-10 * np.abs(dx_ref).max(), i
        assert np.abs(du[su] - du_ref).max() <= 1e-10 * np.abs(du_ref).max(), i
