"""The scaled solve (one persistent grid over the batch, PCG in the basis
W S W^T = I + Oh with W_k = C_k^-1, D_k = C_k C_k^T) against the CPU oracle.

Tolerances
  * W_k and Oh_k (FP64 storage): W_k^T W_k = D_k^-1 and Oh_k = W_k L_k W_{k-1}^T
    to 1e-10 relative; the preconditioners they apply, assembled densely, equal
    the oracle's Phi^-1 to 1e-9 (FP64) / 2e-4 (FP32 storage rounding).
  * Solves: true FP64 relative residual <= tol on every problem (the
    library's own check, recomputed here by the oracle from the returned
    lambda) and ||lam - lam*|| / ||lam*|| <= kappa_2(S) * tol against the
    oracle's direct solve; iteration counts within 25 % + 3 of the oracle's
    (the scaled solve stops on its recurrence residual in the scaled basis).
"""
import numpy as np
import pytest

import oracle
from paper_2309_06427_amd import inputs
from tests import dense

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CLASSES = (6, 14, 26, 36)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def scaled_tau(tol):
    """The scaled solve's floor on the inner tolerance under refinement: the
    first inner solve aims at theta tol (theta = 1/2), never above 1e-6."""
    return min(1e-6, 0.5 * tol)


def seg(b, v, i):
    return v[b.off_v[i]:b.off_v[i + 1]]


def exact(b):
    out = []
    for i in range(b.P):
        p = b.problem(i)
        st, D, L, Di, M = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        assert st == 0
        S = dense.assemble(D, L) if D.shape[0] * D.shape[1] <= 1200 else None
        out.append(dict(D=D, L=L, Di=Di, lam=oracle.direct(D, L, p["gamma"])[1],
                        kappa=np.linalg.cond(S) if S is not None else None))
    return out


def run(b, pc, prec, tol, kernel=0, lam0=None, fallback=False):
    from paper_2309_06427_amd import solver
    with solver.DeviceBatch(b) as db:
        if kernel:
            db.solver.set_mapping(256, 0, kernel)
        db.build(pc, prec)
        l0 = None if lam0 is None else torch.from_numpy(lam0).cuda()
        db.solve(tol, lam0=l0, fallback=fallback)
        out = db.results()
        out["kernel"] = db.solver.solve_kernel()[0]
    return out


@pytest.mark.parametrize("pc", ["bj", "add", "sym", "poly2", "poly3"])
@pytest.mark.parametrize("prec,tol", [("fp32_refine64", 1e-6), ("fp64", 1e-9)])
def test_scaled_solve_matches_oracle(pc, prec, tol):
    b = inputs.batch(20, seed=71, N_range=(1, 70), nx_choices=CLASSES)
    ex = exact(b)
    out = run(b, pc, prec, tol, kernel=4)
    assert out["kernel"] == 4
    assert ((out["status"] & ~16) == 0).all(), out["status"]
    ref = oracle.solve_batch(b, pc, prec, tol=tol, tau_min=scaled_tau(tol))
    assert ((ref["status"] & ~16) == 0).all()
    for i in range(b.P):
        p = b.problem(i)
        lam = seg(b, out["lam"], i)
        rr = oracle.relres(ex[i]["D"], ex[i]["L"], p["gamma"], lam)
        assert rr <= tol * 1.0001, (i, rr)
        assert abs(rr - out["relres"][i]) <= 1e-3 * tol + 1e-12 * rr, (i, rr, out["relres"][i])
        kap = ex[i]["kappa"] if ex[i]["kappa"] is not None else 1e6
        err = np.linalg.norm(lam - ex[i]["lam"]) / np.linalg.norm(ex[i]["lam"])
        assert err <= kap * tol, (i, err, kap)
    it, it_ref = out["iters"].astype(float), ref["iters"].astype(float)
    assert np.all(np.abs(it - it_ref) <= 0.25 * it_ref + 3), (it, it_ref)


def test_preconditioner_ordering_on_the_gpu():
    """Degree 3 < symmetric stair < additive stair < block-Jacobi in mean iterations."""
    b = inputs.batch(24, seed=72, N_range=(32, 120), nx_choices=(6, 14, 26))
    means = {pc: run(b, pc, "fp32_refine64", 1e-6)["iters"].mean() for pc in ("bj", "add", "sym", "poly3")}
    assert means["poly3"] < means["sym"] < means["add"] < means["bj"], means


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-11), ("fp32_refine64", 2e-6)])
def test_scaled_basis_blocks(prec, rtol):
    """Exported W_k, Oh_k: W_k lower triangular with W_k^T W_k = D_k^-1, Oh_k =
    W_k L_k W_{k-1}^T; W^T (I - Oh) W and W^T (I - Oh/2) W are the oracle's
    symmetric and additive stair preconditioners (Sec. IV, Sec. III), and the
    D^-1 exported after the scaled build (formed as W^T W) is the oracle's."""
    from paper_2309_06427_amd import solver
    b = inputs.batch(8, seed=73, N_range=(2, 12), nx_choices=CLASSES)
    n = int(b.off_nn[-1])
    with solver.DeviceBatch(b) as db:
        db.solver.set_mapping(256, 0, 4)
        db.build("sym", prec)
        Zf = torch.empty(n, dtype=torch.float64, device="cuda")
        Of = torch.empty(n, dtype=torch.float64, device="cuda")
        db.solver.export(3, Zf, Of)
        Df = torch.empty(n, dtype=torch.float64, device="cuda")
        Mf = torch.empty(n, dtype=torch.float64, device="cuda")
        db.solver.export(1, Df, Mf)
        torch.cuda.synchronize()
        Zf, Of, Df, Mf = Zf.cpu().numpy(), Of.cpu().numpy(), Df.cpu().numpy(), Mf.cpu().numpy()
    for i in range(b.P):
        p = b.problem(i)
        N, nx = int(b.N[i]), int(b.nx[i])
        Z = Zf[b.off_nn[i]:b.off_nn[i + 1]].reshape(N, nx, nx)
        Oh = Of[b.off_nn[i]:b.off_nn[i + 1]].reshape(N, nx, nx)
        _, D, L, Di, Msym = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        _, _, _, _, Madd = oracle.build(p["A"], p["B"], p["Q"], p["R"], "add")
        assert not np.triu(Z, 1).any()
        Dig = Df[b.off_nn[i]:b.off_nn[i + 1]].reshape(N, nx, nx)
        Mg = Mf[b.off_nn[i]:b.off_nn[i + 1]].reshape(N, nx, nx)
        assert np.abs(Dig - Di).max() <= rtol * 100 * np.abs(Di).max()
        assert np.abs(Mg - Msym).max() <= rtol * 100 * max(np.abs(Msym).max(), 1e-30)
        for k in range(N):
            scale = np.abs(Di[k]).max()
            assert np.abs(Z[k].T @ Z[k] - Di[k]).max() <= rtol * 10 * scale, (i, k)
        assert not Oh[0].any()
        for k in range(1, N):
            want = Z[k] @ L[k] @ Z[k - 1].T
            assert np.abs(Oh[k] - want).max() <= rtol * 10 * max(np.abs(want).max(), 1e-30), (i, k)
        Zd = np.zeros((N * nx, N * nx))
        for k in range(N):
            Zd[k * nx:(k + 1) * nx, k * nx:(k + 1) * nx] = Z[k]
        Od = dense.assemble(np.zeros_like(Oh), Oh)
        for c, M in ((1.0, Msym), (0.5, Madd)):
            got = Zd.T @ (np.eye(N * nx) - c * Od) @ Zd
            want = dense.assemble(Di, M)
            assert np.abs(got - want).max() <= rtol * 100 * np.abs(want).max(), (i, c)


def test_scaled_graph_replays_bit_exact():
    """The persistent grid's queue is reset by a fill kernel inside the
    captured step, so every replay gives the eager results bit for bit (the
    problem -> workgroup assignment varies, each problem's arithmetic does not)."""
    from paper_2309_06427_amd import solver
    b = inputs.batch(48, 74, N_range=(8, 90), nx_choices=(6, 14, 26))
    with solver.DeviceBatch(b) as db:

        def step():
            db.build("sym", "fp32_refine64")
            db.solve(1e-6)

        step()
        ref = db.results()
        assert db.solver.solve_kernel()[0] == 4
        assert (ref["status"] == 0).all()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        for rep in range(3):
            db.build("bj", "fp32_refine64")
            db.solve(1e-6)
            assert (db.results()["status"] == 0).all()
            g.replay()
            out = db.results()
            for k in ("lam", "iters", "relres", "status", "outer"):
                assert np.array_equal(out[k], ref[k]), (rep, k)
        del g


def test_scaled_statuses_and_warm_start():
    """NOT_SPD problems are skipped; a warm start worse than zero (and the
    zero start itself, a tie) falls back like the oracle; a second solve
    without rebuild after an iteration limit runs again."""
    from paper_2309_06427_amd import solver
    b = inputs.batch(6, 75, N_range=(8, 40), nx_choices=(6, 14))
    rng = np.random.default_rng(3)
    lam0 = 1e3 * rng.standard_normal(b.gamma.shape[0])
    lam0[:b.off_v[1]] = 0.0
    ref = oracle.solve_batch(b, "sym", "fp32_refine64", 1e-6, lam0=lam0, fallback=True, tau_min=scaled_tau(1e-6))
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp32_refine64")
        db.solve(1e-6, lam0=torch.from_numpy(lam0).cuda(), fallback=True)
        out = db.results()
        assert db.solver.solve_kernel()[0] == 4
        assert np.array_equal(out["status"] & ~16, ref["status"] & ~16), (out["status"], ref["status"])
        db.solve(1e-6, max_iter=1)
        lim = db.results()
        assert ((lim["status"] & 7) == 2).all()
        db.solve(1e-6)
        again = db.results()
        assert ((again["status"] & ~16) == 0).all() and again["relres"].max() <= 1e-6


def test_scaled_not_spd_problem_is_skipped():
    from paper_2309_06427_amd import solver
    b = inputs.batch(4, 76, N_range=(8, 20), nx_choices=(6,))
    Q = b.Q.copy()
    Q[b.off_nn[2]:b.off_nn[2] + 36] = -np.eye(6).ravel()
    b.Q = Q
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp32_refine64")
        for _ in range(2):
            db.solve(1e-6)
            out = db.results()
            assert db.solver.solve_kernel()[0] == 4
            assert out["status"][2] == 1 and np.isnan(out["relres"][2]) and out["iters"][2] == 0
            assert (out["status"][[0, 1, 3]] & ~16 == 0).all()


def test_scalar_jacobi_runs_the_classic_kernel_and_matches_oracle():
    b = inputs.batch(10, seed=77, N_range=(4, 50), nx_choices=(5, 6, 14))
    ref = oracle.solve_batch(b, "jacobi", "fp64", tol=1e-9)
    out = run(b, "jacobi", "fp64", 1e-9)
    assert out["kernel"] in (1, 2)
    assert (out["status"] == 0).all()
    assert np.all(np.abs(out["iters"] - ref["iters"]) <= 1)
    assert np.abs(out["lam"] - ref["lam"]).max() <= 1e-7 * np.abs(ref["lam"]).max()
    out32 = run(b, "jacobi", "fp32_refine64", 1e-6)
    assert ((out32["status"] & ~16) == 0).all() and out32["relres"].max() <= 1e-6


def test_fp64_accumulation_option_reports_both_errors():
    """Inner products summed in FP32 (default) and in FP64 (the option): both
    reach tol with errors within kappa_2(S) tol on ill-conditioned problems;
    the option changes the iterates (it takes effect) and turning it off
    again restores the default results bit for bit.  Prints both errors."""
    from paper_2309_06427_amd import solver
    b = inputs.make("batch1024_n128_nx26_cond1e6", P=16)
    exact, kap = [], []
    for i in range(b.P):
        p = b.problem(i)
        _, D, L, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        exact.append(oracle.direct(D, L, p["gamma"])[1])
        kap.append(dense.kappa(D, L))
    res = {}
    with solver.DeviceBatch(b) as db:
        db.build("sym", "fp32_refine64")
        for name, on in (("fp32_sums", False), ("fp64_sums", True), ("fp32_again", False)):
            db.solver.set_reduction_fp64(on)
            db.solve(1e-6)
            out = db.results()
            assert db.solver.solve_kernel()[0] == 4
            err = np.array([np.linalg.norm(seg(b, out["lam"], i) - exact[i]) / np.linalg.norm(exact[i])
                            for i in range(b.P)])
            res[name] = (out, err)
            print(f"{name}: iters {out['iters'].mean():.2f} outer {out['outer'].mean():.2f} "
                  f"max relres {out['relres'].max():.2e} median err {np.median(err):.2e} max err {err.max():.2e}")
            assert ((out["status"] & ~16) == 0).all() and out["relres"].max() <= 1e-6
            assert np.all(err <= np.array(kap) * 1e-6)
    assert not np.array_equal(res["fp32_sums"][0]["lam"], res["fp64_sums"][0]["lam"])
    for k in ("lam", "iters", "relres", "status"):
        assert np.array_equal(res["fp32_sums"][0][k], res["fp32_again"][0][k])


def test_autotune_cache_reuses_the_choice(tmp_path):
    """The first autotune times candidates and stores its choice under the
    batch's key; a second batch of the same kind (new handle, same state
    sizes and size buckets) takes the stored mapping without timing, and its
    solve is valid."""
    import json
    from paper_2309_06427_amd import solver
    path = str(tmp_path / "tune.json")
    b1 = inputs.batch(40, seed=81, N_range=(20, 100), nx_choices=(6, 14, 26))
    b2 = inputs.batch(40, seed=82, N_range=(20, 100), nx_choices=(6, 14, 26))
    with solver.DeviceBatch(b1) as d1, solver.DeviceBatch(b2) as d2:
        d1.build("sym", "fp32_refine64")
        d1.autotune(1e-6, cache=path)
        t1, l1, _, ms1 = d1.solver.scaled_mapping()
        assert ms1 > 0  # timed here
        data = json.load(open(path))
        assert list(data) == [d1.tune_key()] and data[d1.tune_key()] == {"kind": "scaled", "threads": t1, "lds": l1}
        d2.build("sym", "fp32_refine64")
        assert d2.tune_key() == d1.tune_key()
        d2.autotune(1e-6, cache=path)
        t2, l2, _, ms2 = d2.solver.scaled_mapping()
        assert (t2, l2) == (t1, l1) and ms2 == 0.0  # taken from the cache, not timed
        out = d2.results()
        assert ((out["status"] & ~16) == 0).all() and out["relres"].max() <= 1e-6
        assert json.load(open(path)) == data
