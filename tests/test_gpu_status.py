"""Statuses across repeated solves without a rebuild: only a build failure
(NOT_SPD) makes a solve skip a problem; an earlier solve's iteration limit or
fallback flags do not."""
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


@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_second_solve_after_maxiter_runs_again(kernel):
    from paper_2309_06427_amd import solver
    b = inputs.batch(6, 31, N_range=(8, 40), nx_choices=(6, 14))
    ref = oracle.solve_batch(b, "sym", "fp64", 1e-9)
    with solver.DeviceBatch(b) as db:
        if kernel:
            db.solver.set_mapping(128, 0, kernel)
        db.build("sym", "fp64")
        db.solve(1e-9, max_iter=1)
        first = db.results()
        assert ((first["status"] & 7) == 2).all(), first["status"]
        db.solve(1e-9)  # same status array, no rebuild
        second = db.results()
    assert (second["status"] == 0).all(), second["status"]
    assert np.all(np.abs(second["iters"] - ref["iters"]) <= 1)
    assert np.abs(second["lam"] - ref["lam"]).max() <= 1e-7 * np.abs(ref["lam"]).max()


def test_not_spd_build_is_still_skipped_on_a_second_solve():
    from paper_2309_06427_amd import solver
    b = inputs.batch(4, 32, N_range=(8, 20), nx_choices=(6,))
    Q = b.Q.copy()
    Q[b.off_nn[2]:b.off_nn[2] + 36] = -np.eye(6).ravel()  # problem 2, knot 0: indefinite
    b.Q = Q
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp32_refine64")
        for _ in range(2):
            db.solve(1e-6)
            out = db.results()
            assert out["status"][2] == 1 and np.isnan(out["relres"][2]) and out["iters"][2] == 0
            assert not out["lam"][b.off_v[2]:b.off_v[3]].any()
            assert (out["status"][[0, 1, 3]] & ~16 == 0).all()
