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
