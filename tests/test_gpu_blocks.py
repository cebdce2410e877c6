"""GPU parity of the build from given blocks (``ssp_build_from_blocks``) against
the CPU oracle's preconditioner of the same S, on SPD block-tridiagonal
matrices that do not come from dynamics (seeded, ``inputs.block_batch``).

Tolerances are those of the assembled build (FP64: stored blocks within 1e-12
of the oracle's, relative to the problem's largest entry; solves: FP64 to
1e-9 with ||lam - lam*|| / ||lam*|| <= kappa_2(S) * tol against the oracle's
direct solve, FP32 storage with FP64 refinement to 1e-6 likewise).
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


# ragged sizes: single-block problems, odd and even horizons, compiled and
# generic state sizes
NS = [1, 2, 7, 33, 64, 5, 40, 17, 90, 3]
NXS = [3, 6, 14, 26, 6, 36, 14, 5, 26, 9]


def _batch(seed, margin=0.5):
    return inputs.block_batch(NS, NXS, seed, margin)


def _dev(b, pc, prec):
    from paper_2309_06427_amd import solver
    db = solver.DeviceBlockBatch(b)
    db.build(pc, prec)
    return db


def _blocks(b, flat, i):
    n, x = int(b.N[i]), int(b.nx[i])
    return flat[b.off_nn[i]:b.off_nn[i + 1]].reshape(n, x, x)


def _seg(b, v, i):
    return v[b.off_v[i]:b.off_v[i + 1]]


@pytest.mark.parametrize("pc", ["bj", "add", "sym"])
def test_blocks_build_fp64_matches_oracle(pc):
    b = _batch(1)
    db = _dev(b, pc, "fp64")
    st = db.results()["status"]
    assert (st == 0).all(), st
    Sd, So = db.export(0)
    Pd, Po = db.export(1)
    for i in range(b.P):
        q = b.problem(i)
        ost, Di, M = oracle.precond(q["D"], q["L"], pc)
        assert ost == oracle.OK
        L = q["L"].copy()
        L[0] = 0.0
        for got, want in ((_blocks(b, Sd, i), q["D"]), (_blocks(b, So, i), L), (_blocks(b, Pd, i), Di),
                          (_blocks(b, Po, i), M)):
            scale = max(np.abs(want).max(), 1e-300)
            assert np.abs(got - want).max() <= 1e-12 * scale, i


def test_blocks_build_fp32_storage_keeps_S_to_fp64():
    """FP32 storage keeps S as hi + lo pairs (the refinement residual's S) and
    D^-1 in FP32."""
    b = _batch(2)
    db = _dev(b, "sym", "fp32_refine64")
    Sd, So = db.export(0)
    Pd, _ = db.export(1)
    for i in range(b.P):
        q = b.problem(i)
        _, Di, _ = oracle.precond(q["D"], q["L"], "sym")
        L = q["L"].copy()
        L[0] = 0.0
        for got, want, tol in ((_blocks(b, Sd, i), q["D"], 1e-14), (_blocks(b, So, i), L, 1e-14),
                               (_blocks(b, Pd, i), Di, 2e-7)):
            assert np.abs(got - want).max() <= tol * np.abs(want).max(), i


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("pc", ["bj", "add", "sym"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32_refine64", 1e-6)])
def test_blocks_solve_matches_direct_solution(pc, prec, tol, kernel):
    """Fused kernel (0) and the explicit-block kernel (1, stair blocks built on
    demand from the stored D^-1 and L) on S given by blocks."""
    b = _batch(3)
    db = _dev(b, pc, prec)
    if kernel:
        db.solver.set_mapping(128, 0, kernel)
    db.solve(tol)
    out = db.results()
    assert (out["status"] == 0).all(), out["status"]
    assert out["relres"].max() <= tol * 1.0001
    for i in range(b.P):
        q = b.problem(i)
        _, x = oracle.direct(q["D"], q["L"], q["gamma"])
        from tests import dense
        ev = np.linalg.eigvalsh(dense.assemble(q["D"], q["L"]))
        err = np.linalg.norm(_seg(b, out["lam"], i) - x) / np.linalg.norm(x)
        assert err <= ev[-1] / ev[0] * tol * 1.01, i


def test_blocks_fp64_iterations_match_oracle_pcg():
    """Same recurrences on the same S: FP64 iteration counts within 1 of the oracle's."""
    b = _batch(4)
    db = _dev(b, "sym", "fp64")
    db.solve(1e-8)
    out = db.results()
    for i in range(b.P):
        q = b.problem(i)
        _, Di, M = oracle.precond(q["D"], q["L"], "sym")
        st, lam, it = oracle.pcg(q["D"], q["L"], Di, M, q["gamma"], tol=1e-8)
        assert st == oracle.OK
        assert abs(int(out["iters"][i]) - it) <= 1, i
        err = np.linalg.norm(_seg(b, out["lam"], i) - lam) / np.linalg.norm(lam)
        assert err <= 1e-10, i


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
def test_blocks_indefinite_diagonal_block_is_not_spd(prec):
    """A D_k with a negative eigenvalue marks its problem NOT_SPD (as the oracle
    does) and leaves the other problems untouched."""
    b = _batch(5)
    bad = 3
    q = b.problem(bad)
    k = q["N"] // 2
    q["D"][k] -= 2.0 * np.linalg.eigvalsh(q["D"][k]).max() * np.eye(q["nx"])  # writes into b.D
    assert oracle.precond(q["D"], q["L"], "sym")[0] == oracle.NOT_SPD
    db = _dev(b, "sym", prec)
    db.solve(1e-6)
    out = db.results()
    assert out["status"][bad] == oracle.NOT_SPD
    others = np.arange(b.P) != bad
    assert (out["status"][others] == 0).all()
    assert out["relres"][others].max() <= 1e-6 * 1.0001


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32_refine64", 1e-6)])
def test_blocks_single_long_problem_cooperative(prec, tol):
    """One long problem built from blocks runs the cooperative solve (several
    workgroups) and matches the oracle's direct solution."""
    b = inputs.block_batch([160], [14], 9)
    db = _dev(b, "sym", prec)
    db.solve(tol)
    out = db.results()
    assert db.solver.solve_kernel()[0] == 3
    assert out["status"][0] == 0
    assert out["relres"][0] <= tol * 1.0001
    q = b.problem(0)
    _, x = oracle.direct(q["D"], q["L"], q["gamma"])
    from tests import dense
    ev = np.linalg.eigvalsh(dense.assemble(q["D"], q["L"]))
    err = np.linalg.norm(out["lam"] - x) / np.linalg.norm(x)
    assert err <= ev[-1] / ev[0] * tol * 1.01
