"""The allocation-free solve entry point (ssp_solve_noalloc) against ssp_solve.

Both run the same kernels on the same inputs; only the solve workspace
differs (the library's fixed per-device array instead of the handle's
buffers), so every output (lambda, iterations, residuals, statuses, outer
steps) must agree bit for bit.  Two calls in a row reuse the array, the
second on a smaller batch, and each solver path (scaled persistent, fused
per-class, explicit blocks) runs through it.
"""
import numpy as np
import pytest

from paper_2309_06427_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("lam", "iters", "relres", "status", "outer")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def both(b, pc, prec, tol, kernel=0, lam0=None, warm_first=False):
    """(ssp_solve results, ssp_solve_noalloc results, solve kernel) on one handle."""
    from paper_2309_06427_amd import solver
    with solver.DeviceBatch(b) as db:
        if kernel:
            db.solver.set_mapping(256, 0, kernel)
        out = {}
        order = ("noalloc", "plain") if warm_first else ("plain", "noalloc")
        for which in order:
            db.build(pc, prec)
            db.lam.fill_(np.nan)
            db.iters.fill_(-1)
            db.relres.fill_(-1.0)
            l0 = None if lam0 is None else torch.from_numpy(lam0).cuda()
            db.solve(tol, lam0=l0, fallback=lam0 is not None, noalloc=which == "noalloc")
            out[which] = db.results()
            out[which + "_kernel"] = db.solver.solve_kernel()[0]
    return out


def assert_same(out):
    assert out["plain_kernel"] == out["noalloc_kernel"]
    for k in KEYS:
        a, b = out["plain"][k], out["noalloc"][k]
        assert np.array_equal(a, b, equal_nan=True), k


def test_two_calls_in_a_row_the_second_smaller_scaled_path():
    big = inputs.batch(40, seed=201, N_range=(16, 120), nx_choices=(6, 14, 26, 36))
    small = inputs.batch(6, seed=202, N_range=(2, 30), nx_choices=(6, 14))
    o1 = both(big, "sym", "fp32_refine64", 1e-6)
    assert o1["plain_kernel"] == 4
    assert ((o1["plain"]["status"] & ~16) == 0).all()
    assert_same(o1)
    o2 = both(small, "poly2", "fp64", 1e-9)
    assert o2["plain_kernel"] == 4
    assert ((o2["plain"]["status"] & ~16) == 0).all()
    assert_same(o2)


def test_noalloc_first_on_a_fresh_handle_then_plain():
    """The allocation-free call as the first solve of a handle (with a warm
    start and its fallback), then ssp_solve: the same results."""
    b = inputs.batch(12, seed=203, N_range=(8, 60), nx_choices=(6, 14, 26))
    lam0 = np.random.default_rng(5).standard_normal(int(b.off_v[-1]))
    o = both(b, "sym", "fp32_refine64", 1e-6, lam0=lam0, warm_first=True)
    assert_same(o)


def test_fused_path_and_explicit_path():
    """State sizes outside the compiled classes take the fused per-class
    kernel; the explicit-block kernel first needs its blocks allocated by a
    plain solve, and refuses the allocation-free call before that."""
    from paper_2309_06427_amd import solver
    from paper_2309_06427_amd._lib import SspError
    b = inputs.batch(10, seed=204, N_range=(4, 50), nx_choices=(5, 9))
    o = both(b, "sym", "fp64", 1e-9)
    assert o["plain_kernel"] == 2
    assert (o["plain"]["status"] == 0).all()
    assert_same(o)
    with solver.DeviceBatch(b) as db:
        db.solver.set_mapping(256, 0, 1)
        db.build("sym", "fp64")
        with pytest.raises(SspError, match="ssp_solve_noalloc"):
            db.solve(1e-9, noalloc=True)
    o = both(b, "sym", "fp64", 1e-9, kernel=1)
    assert o["plain_kernel"] == 1
    assert_same(o)


def test_rejects_a_batch_beyond_the_fixed_workspace():
    """72 bytes per lambda entry under FP64 storage: a horizon of 30000 knots
    of state size 36 (1.08 M entries) exceeds the 64 MiB array; the check
    comes before anything is launched."""
    from paper_2309_06427_amd import solver
    from paper_2309_06427_amd._lib import SspError
    s = solver.BatchSolver(np.array([30000], np.int32), np.array([36], np.int32), np.array([12], np.int32))
    try:
        z = torch.zeros(30000 * 36, dtype=torch.float64, device="cuda")
        i32 = torch.zeros(1, dtype=torch.int32, device="cuda")
        f64 = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(SspError, match="bytes of solve workspace"):
            s.solve_noalloc(1e-6, 0, z, z, 0, i32, f64, i32)
    finally:
        s.close()
