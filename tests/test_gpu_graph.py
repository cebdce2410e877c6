"""The whole step (FP64 assembly + batched solve, optionally the learned warm
start) captured into one HIP graph replays to the eager result, bit for bit,
every time, with eager work of the program between the replays."""
import numpy as np
import pytest

from paper_2309_06427_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _capture(fn):
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        fn()
    return g


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
def test_graph_replays_match_eager(prec):
    from paper_2309_06427_amd import solver
    b = inputs.batch(40, 31, N_range=(8, 60), nx_choices=(6, 14, 26, 5))
    db = solver.DeviceBatch(b)

    def step():
        db.build("sym", prec)
        db.solve(1e-6)

    step()
    ref = db.results()
    assert (ref["status"] == 0).all()
    g = _capture(step)
    for rep in range(3):
        # eager work of the program between replays: another preconditioner
        db.build("bj", prec)
        db.solve(1e-6)
        other = db.results()
        assert (other["status"] == 0).all()
        g.replay()
        out = db.results()
        for k in ("lam", "iters", "relres", "status", "outer"):
            assert np.array_equal(out[k], ref[k]), (rep, k)


def test_graph_with_warm_start_matches_eager():
    from paper_2309_06427_amd import solver
    from paper_2309_06427_amd.warmstart import WarmStartNet
    b = inputs.batch(24, 32, N_range=(8, 60), nx_choices=(6, 14))
    db = solver.DeviceBatch(b)
    nets = []
    for nx in (6, 14):
        n = WarmStartNet(nx, 32)
        n.set_params((0.05 * np.random.default_rng(nx).standard_normal(n.n_params)).astype(np.float32))
        nets.append(n)

    def step():
        db.build("sym", "fp32_refine64")
        db.lam.zero_()
        for n in nets:
            n.predict(db)
        db.solve(1e-6, warm_in_place=True, fallback=True)

    step()
    ref = db.results()
    assert ((ref["status"] & ~8) == 0).all()
    g = _capture(step)
    for rep in range(3):
        db.build("sym", "fp32_refine64")
        db.solve(1e-6)
        db.results()
        g.replay()
        out = db.results()
        for k in ("lam", "iters", "relres", "status", "outer"):
            assert np.array_equal(out[k], ref[k]), (rep, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine64"])
def test_graph_replays_cooperative_solve(prec):
    """A single long problem (the cooperative kernel: tagged cross-workgroup
    records and a tag counter that carries across launches) replays from a
    graph to the eager bits, with eager solves of the same batch between."""
    from paper_2309_06427_amd import solver
    b = inputs.pack([inputs.draw_problem(np.random.default_rng(21), 300, 26, 13)])
    db = solver.DeviceBatch(b)

    def step():
        db.build("sym", prec)
        db.solve(1e-6)

    step()
    ref = db.results()
    assert db.solver.solve_kernel()[0] == 3 and ref["status"][0] & ~16 == 0
    g = _capture(step)
    for rep in range(3):
        db.build("add", prec)
        db.solve(1e-6)
        assert db.results()["status"][0] & ~16 == 0
        db.lam.fill_(5.0)
        g.replay()
        out = db.results()
        for k in ("lam", "iters", "relres", "status", "outer"):
            assert np.array_equal(out[k], ref[k]), (rep, k)
