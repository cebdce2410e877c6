"""GPU parity of the learned warm start (network kernels through the C ABI)
against the FP64 reference oracle.mlp, and what the trained network gains.

Tolerances (FP32 matrix-core products against FP64):
  * GEMM: max |C - C_ref| <= 2e-6 * K * max|A| * max|B| (FP32 accumulation of
    K products).
  * Forward, loss, gradient: relative error (norm of the difference over the
    norm of the reference) <= 2e-4; the inputs are standardised FP32 values
    of unit size and every sum has at most a few thousand terms.
  * Scaling statistics: relative 1e-5.
  * Adam: relative 1e-5 against the oracle's update from the same gradient.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2309_06427_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 64, 16), (70, 130, 37), (200, 26, 1378), (5, 300, 64)])
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_matches_numpy(M, N, K, ta, tb):
    from paper_2309_06427_amd import _lib
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((M, N), np.nan, dtype=torch.float32, device="cuda")
    L = _lib.load()
    _lib.check(L.ssp_gemm_f32(M, N, K, dA.data_ptr(), A.shape[1], ta, dB.data_ptr(), B.shape[1], tb,
                              dC.data_ptr(), N, torch.cuda.current_stream().cuda_stream), "gemm")
    C = dC.cpu().numpy()
    bound = 2e-6 * K * np.abs(A).max() * np.abs(B).max()
    assert np.isfinite(C).all()
    assert np.abs(C - ref).max() <= bound


def _pool(nx, P, seed, N_range=(3, 40), prec="fp64"):
    """Device batch of one nx, the oracle's blocks and exact solutions."""
    from paper_2309_06427_amd import solver
    b = inputs.batch(P, seed, N_range=N_range, nx_choices=(nx,))
    db = solver.DeviceBatch(b)
    db.build("sym", prec)
    probs = []
    for p in range(P):
        pr = b.problem(p)
        st, D, L, Di, M = oracle.build(pr["A"], pr["B"], pr["Q"], pr["R"], "sym")
        st, lam = oracle.direct(D, L, pr["gamma"])
        probs.append((D, L, pr["gamma"], lam))
    lam_star = np.concatenate([p[3] for p in probs])
    return b, db, probs, torch.from_numpy(lam_star).cuda()


def _net(nx, H, seed):
    from paper_2309_06427_amd.warmstart import WarmStartNet
    net = WarmStartNet(nx, H)
    theta = inputs.mlp_init(nx, H, seed) + 0.05 * np.random.default_rng(seed).standard_normal(
        mlp.n_params(nx, H))
    theta = theta.astype(np.float32)
    net.set_params(theta)
    return net, theta.astype(np.float64)


@pytest.mark.parametrize("nx,H", [(6, 128), (14, 32), (3, 16)])
def test_scaling_statistics_match_numpy(nx, H):
    b, db, probs, lam_star = _pool(nx, 5, 11)
    net, _ = _net(nx, H, 1)
    net.fit_scaling(db, lam_star)
    mu, isd, ys = net.get_scaling()
    X = np.concatenate([mlp.features(D, L, g) for (D, L, g, _) in probs])
    mu_ref, isd_ref = mlp.feature_stats(X)
    assert rel(mu, mu_ref) < 1e-5
    assert rel(isd, isd_ref) < 1e-5
    lam = lam_star.cpu().numpy()
    assert abs(ys - np.sqrt(np.mean(lam * lam))) <= 1e-5 * np.sqrt(np.mean(lam * lam))


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
@pytest.mark.parametrize("nx,H", [(6, 128), (14, 32), (26, 128), (5, 32)])
def test_forward_matches_oracle(nx, H, prec):
    """The first layer gathers its inputs through a table of offsets; nx = 5
    (nx^2 odd) and H = 32 (a partial hidden tile) check its edges."""
    b, db, probs, lam_star = _pool(nx, 4, 12, prec=prec)
    net, theta = _net(nx, H, 2)
    net.fit_scaling(db, lam_star)
    mu, isd, ys = net.get_scaling()
    out = torch.full_like(db.gamma, np.nan)
    net.predict(db, out)
    got = out.cpu().numpy()
    X = np.concatenate([mlp.features(D, L, g) for (D, L, g, _) in probs])
    ref, _ = mlp.forward(theta, X, mu.astype(np.float64), isd.astype(np.float64), ys, nx, H)
    assert np.isfinite(got).all()
    assert rel(got, ref.ravel()) < 2e-4


def test_predict_only_touches_its_state_size():
    from paper_2309_06427_amd import solver
    b = inputs.batch(6, 13, N_range=(3, 20), nx_choices=(6, 14))
    db = solver.DeviceBatch(b)
    db.build("sym", "fp32_refine64")
    net, _ = _net(6, 32, 3)
    out = torch.full_like(db.gamma, 7.0)
    net.predict(db, out)
    got = out.cpu().numpy()
    for p in range(b.P):
        s = got[b.off_v[p]:b.off_v[p + 1]]
        if b.nx[p] == 6:
            assert np.all(s != 7.0)
        else:
            assert np.all(s == 7.0)


@pytest.mark.parametrize("nx,H", [(6, 128), (14, 32)])
def test_loss_and_gradient_match_oracle(nx, H):
    b, db, probs, lam_star = _pool(nx, 6, 14)
    net, theta = _net(nx, H, 4)
    net.fit_scaling(db, lam_star)
    mu, isd, ys = net.get_scaling()
    p0, p1 = 1, 5
    loss = net.loss_grad(db, p0, p1, lam_star)
    g = net.get_grad()
    ref_loss, ref_g = mlp.loss_and_grad(theta, probs[p0:p1], mu.astype(np.float64), isd.astype(np.float64),
                                        ys, nx, H)
    assert abs(float(loss) - ref_loss) <= 2e-4 * ref_loss
    assert rel(g, ref_g) < 2e-4
    # bitwise reproducible
    net.loss_grad(db, p0, p1, lam_star)
    assert np.array_equal(net.get_grad(), g)


def test_adam_matches_oracle():
    b, db, probs, lam_star = _pool(6, 3, 15)
    net, theta = _net(6, 32, 5)
    net.fit_scaling(db, lam_star)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = net.get_params().astype(np.float64)
    for t in (1, 2, 3):
        net.loss_grad(db, 0, 3, lam_star)
        g = net.get_grad().astype(np.float64)
        net.adam(1e-3)
        th, m, v = mlp.adam_step(th, g, m, v, t, 1e-3)
        assert rel(net.get_params(), th) < 1e-5


def test_training_lowers_loss_and_warm_start_saves_iterations():
    from paper_2309_06427_amd import solver
    from paper_2309_06427_amd.warmstart import WarmStartNet, training_pool
    nx = 6
    db, lam_star = training_pool(nx, 192, seed=21)
    net = WarmStartNet(nx, 64)
    net.set_params(inputs.mlp_init(nx, 64, seed=0).astype(np.float32))
    net.fit_scaling(db, lam_star)
    hist = net.train(db, lam_star, epochs=12, problems_per_step=8, lr=2e-3, lr_final=2e-4, seed=0)
    assert hist[-1] < 0.5 * hist[0]
    # held-out problems: zero start vs learned start, FP32 with FP64 refinement to 1e-6
    test = inputs.batch(48, 40, nx_choices=(nx,))
    tb = solver.DeviceBatch(test)
    tb.build("sym", "fp32_refine64")
    tb.solve(1e-6)
    zero = tb.results()
    net.predict(tb)
    tb.solve(1e-6, warm_in_place=True, fallback=True)
    warm = tb.results()
    assert (zero["status"] == 0).all()
    assert ((warm["status"] & ~8) == 0).all()
    assert warm["relres"].max() <= 1e-6 and zero["relres"].max() <= 1e-6
    assert warm["iters"].mean() < zero["iters"].mean()


def test_fallback_restarts_from_zero_like_the_oracle():
    from paper_2309_06427_amd import solver
    b = inputs.batch(6, 16, N_range=(5, 30), nx_choices=(6, 14))
    rng = np.random.default_rng(0)
    lam0 = 1e3 * rng.standard_normal(b.gamma.shape[0])  # far worse than zero
    # problem 0: a zero start, whose residual is exactly gamma; the tie is not
    # "below ||gamma||", so it falls back too (both norms summed in one order)
    lam0[: b.off_v[1]] = 0.0
    ref0 = oracle.solve_batch(b, "sym", "fp64", 1e-8)
    ref = oracle.solve_batch(b, "sym", "fp64", 1e-8, lam0=lam0, fallback=True)
    assert (ref["status"] == 8).all()
    db = solver.DeviceBatch(b)
    db.build("sym", "fp64")
    db.solve(1e-8)
    gz = db.results()
    db.solve(1e-8, lam0=torch.from_numpy(lam0).cuda(), fallback=True)
    gw = db.results()
    assert np.array_equal(gw["status"], ref["status"])
    # the restart scales by ||gamma|| from the norm pass instead of the residual sweep's
    # sum (a different summation order), so the iterates agree to rounding
    assert np.array_equal(gw["iters"], gz["iters"])
    assert np.abs(gw["lam"] - gz["lam"]).max() <= 1e-12 * np.abs(gz["lam"]).max()
    assert np.all(np.abs(gw["iters"] - ref0["iters"]) <= 1)


def test_checkpoint_resume_is_bit_exact(tmp_path):
    """Training stopped after one epoch, checkpointed (weights, standardisation,
    Adam moments and step count) and resumed in a new network handle for the
    second epoch gives the uninterrupted two-epoch run bit for bit."""
    from paper_2309_06427_amd.warmstart import WarmStartNet, training_pool
    nx, H = 6, 32
    db, lam_star = training_pool(nx, 24, seed=23)
    kw = dict(epochs=2, problems_per_step=4, lr=2e-3, lr_final=2e-4, seed=5)
    theta0 = inputs.mlp_init(nx, H, seed=2).astype(np.float32)

    full = WarmStartNet(nx, H)
    full.set_params(theta0)
    full.fit_scaling(db, lam_star)
    hist_full = full.train(db, lam_star, **kw)
    th_full, st_full = full.get_params(), full.get_state()

    part = WarmStartNet(nx, H)
    part.set_params(theta0)
    part.fit_scaling(db, lam_star)
    hist_1 = part.train(db, lam_star, end_epoch=1, **kw)
    path = str(tmp_path / "ckpt.npz")
    part.checkpoint(path, epoch=1)
    part.close()
    resumed, ep = WarmStartNet.resume(path)
    assert ep == 1
    hist_2 = resumed.train(db, lam_star, start_epoch=ep, **kw)
    th_res, st_res = resumed.get_params(), resumed.get_state()
    assert np.array_equal(np.concatenate([hist_1, hist_2]), hist_full)
    assert np.array_equal(th_res, th_full)
    assert np.array_equal(st_res[0], st_full[0]) and np.array_equal(st_res[1], st_full[1])
    assert st_res[2] == st_full[2] == 2 * 6
    for n in (full, resumed):
        n.close()
    db.close()


def test_training_labels_match_the_oracle():
    """The training pool's labels (the library's FP64 PCG to 1e-10) against the
    oracle's direct solution on 256 systems: within kappa_2(S) * 1e-10."""
    from tests import dense
    from paper_2309_06427_amd.warmstart import training_pool
    nx = 14
    db, lam_star = training_pool(nx, 256, seed=31)
    lab = lam_star.cpu().numpy()
    b = db.batch
    for i in range(b.P):
        p = b.problem(i)
        st, D, L, _, _ = oracle.build(p["A"], p["B"], p["Q"], p["R"], "sym")
        assert st == oracle.OK
        st, ref = oracle.direct(D, L, p["gamma"])
        err = np.linalg.norm(lab[b.off_v[i]:b.off_v[i + 1]] - ref) / np.linalg.norm(ref)
        assert err <= dense.kappa(D, L) * 1e-10, (i, err)
    db.close()
