"""Problems whose six PCG recurrence vectors the scaled solve keeps in LDS
(short horizons at small state sizes) against the oracle, beside problems of
the same state size whose vectors stream through HBM.

At the bench's mapping (256 threads, 48 336 B) and FP32 storage with the
symmetric stair, nx = 6 keeps every horizon up to 273 knots in LDS and
nx = 14 up to 92 (ssp_scaled_onchip_horizon).  The batch straddles the
nx = 14 limit (N = 91, 92, 93) and holds both kinds at each size.  Bars, per
problem: status OK, reported relative residual <= tol and equal to the
oracle's recomputation to 1e-3 tol, and ||lam - lam*|| / ||lam*|| <=
kappa_2(S) tol against the oracle's direct solution; for every preconditioner
of the scaled solve (block-Jacobi, whose horizon is longer, the stairs and the
degree-3 Neumann polynomial, whose horizon is shorter).
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
SHAPES = [(14, 32), (14, 91), (14, 92), (14, 93), (14, 150), (14, 256), (6, 32), (6, 200), (6, 256), (14, 60),
          (6, 1), (14, 1), (14, 2)]


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(4321)
    probs = [inputs.draw_problem(rng, N, nx, nx // 2, "wishart", 1e4) for nx, N in SHAPES]
    b = inputs.pack(probs)
    refs = []
    for i in range(b.P):
        p = b.problem(i)
        st, D, L, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        assert st == oracle.OK
        st, lam_star = oracle.direct(D, L, p["gamma"])
        assert st == oracle.OK
        refs.append((D, L, lam_star, dense.kappa(D, L)))
    return b, refs


@pytest.mark.parametrize("pc", ["sym", "add", "bj", "poly3"])
def test_vectors_in_lds_match_the_oracle(batch, pc):
    from paper_2309_06427_amd import solver
    b, refs = batch
    hor = {nx: solver.scaled_onchip_horizon(nx, pc, "fp32_refine64", *MAPPING) for nx in (6, 14)}
    if pc == "sym":
        assert hor == {6: 273, 14: 92}
    kinds = {(int(nx), int(N) <= hor[int(nx)]) for nx, N in zip(b.nx, b.N)}
    assert {(14, True), (14, False), (6, True)} <= kinds, kinds
    with solver.DeviceBatch(b) as db:
        db.build(pc, "fp32_refine64")
        db.solver.set_scaled_mapping(*MAPPING)
        db.solve(TOL)
        out = db.results()
        assert db.solver.solve_kernel()[0] == 4
        assert db.solver.scaled_mapping()[:2] == MAPPING
    assert ((out["status"] & ~16) == 0).all(), out["status"]
    for i, (D, L, lam_star, kap) in enumerate(refs):
        p = b.problem(i)
        lam = out["lam"][b.off_v[i]:b.off_v[i + 1]]
        rr = oracle.relres(D, L, p["gamma"], lam)
        assert rr <= TOL * 1.0001, (pc, i, rr)
        assert abs(rr - out["relres"][i]) <= 1e-3 * TOL, (pc, i, rr, out["relres"][i])
        err = np.linalg.norm(lam - lam_star) / np.linalg.norm(lam_star)
        assert err <= kap * TOL, (pc, i, err, kap)
