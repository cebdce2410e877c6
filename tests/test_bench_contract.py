"""bench.py's command-line contract: one JSON line with the agreed keys, and a
clear refusal of more than one GPU.  bench.main() runs in this process (no
child process is started from a process that may hold the GPU)."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = {"metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
        "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"}


def _run(monkeypatch, *argv):
    if ROOT not in sys.path:
        monkeypatch.syspath_prepend(ROOT)
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", *argv])
    return bench.main()


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    assert _run(monkeypatch, "--gpus", "2") == 2
    out = capsys.readouterr()
    assert "one GPU" in out.err
    assert out.out.strip() == ""


@pytest.mark.gpu
def test_one_json_line_with_the_contract_keys(monkeypatch, capsys):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc = _run(monkeypatch, "--workload", "single_n50_nx14", "--steps", "3", "--warmup", "1", "--no-compare",
              "--warm", "zero", "--cpu-sample", "1")
    assert rc == 0
    lines = [l for l in capsys.readouterr().out.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    assert KEYS <= set(d)
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert d["config"]["workload"] == "single_n50_nx14"
    roof = d["roofline"]
    assert {"bound", "achieved", "peak", "unit", "frac", "traffic"} <= set(roof)
    assert 0 < roof["frac"] < 1
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1


def test_kkt_bytes_count_each_block_and_vector_once(monkeypatch):
    """Three knots, nx = 2, nu = 1, counted by hand: Q^-1 on 3 knots (12
    elements), A, B, R^-1 on the 2 knots with a successor (2 x (4 + 2 + 1));
    right-hand side q, c, gamma (18) and r of 2 knots; recovery q, lambda, dx
    (18), r of 2 knots and du (3)."""
    if ROOT not in sys.path:
        monkeypatch.syspath_prepend(ROOT)
    import numpy as np
    import bench
    from paper_2309_06427_amd import inputs
    b = inputs.pack([inputs.draw_problem(np.random.default_rng(0), 3, 2, 1)])
    rhs, rec = bench.kkt_bytes(b)
    assert rhs.tolist() == [8.0 * (12 + 14 + 18 + 2)]
    assert rec.tolist() == [8.0 * (12 + 14 + 18 + 2 + 3)]


def test_scaled_bytes_by_hand_and_on_chip_vectors(monkeypatch):
    """One problem, N = 3 knots, nx = 2, FP32 storage, 5 inner iterations in
    one outer step from a zero start, counted by hand:
      blocks: Oh on N - 1 = 2 knots per pass, 6 passes (5 + the initial one),
              4 * 4 * 2 * 6 = 192 B; W twice, 2 * 4 * 3 * 4 = 96 B; no FP64
              residual sweep (zero start): 288 B;
      vectors, per row (6 rows): 12 * 4 * 5 update-pass bytes, 8 + 4 * 4 for
              the initial pass, 40 + 4 for the transforms, 16 once: 324 B per
              row, 1944 B.
    With the vectors in LDS only the FP64 parts remain: 8 + 40 + 16 = 64 B per
    row; the block bytes do not change."""
    if ROOT not in sys.path:
        monkeypatch.syspath_prepend(ROOT)
    import numpy as np
    import bench
    from paper_2309_06427_amd import inputs
    b = inputs.pack([inputs.draw_problem(np.random.default_rng(0), 3, 2, 1)])
    it, st = np.array([5]), np.array([1])
    blk, vec = bench.scaled_bytes(b, it, st, "fp32_refine64")
    assert blk.tolist() == [288.0] and vec.tolist() == [6 * 324.0]
    blk2, vec2 = bench.scaled_bytes(b, it, st, "fp32_refine64", np.array([True]))
    assert blk2.tolist() == [288.0] and vec2.tolist() == [6 * 64.0]
    _, vec3 = bench.scaled_bytes(b, it, st, "fp32_refine64", np.array([False]))
    assert vec3.tolist() == vec.tolist()


@pytest.mark.gpu
def test_compare_and_kkt_timings_are_reported(monkeypatch, capsys):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rc = _run(monkeypatch, "--workload", "single_n50_nx14", "--steps", "2", "--warmup", "1", "--warm", "zero",
              "--no-cpu-baseline", "--no-graph")
    assert rc == 0
    d = json.loads([l for l in capsys.readouterr().out.splitlines() if l.strip()][0])
    cmp = d["detail"]["compare"]
    assert set(cmp) == {"jacobi", "bj", "add", "sym", "poly3"}
    for pc, c in cmp.items():
        assert c["solve_ms"] > 0 and c["build_ms"] > 0 and c["solve_algorithmic_bytes"] > 0, pc
        assert 0 < c["solve_frac"] < 1, pc
    kkt = d["detail"]["kkt"]
    assert kkt["rhs_ms"] > 0 and kkt["recover_ms"] > 0
    assert 0 < kkt["rhs_frac"] < 1 and 0 < kkt["recover_frac"] < 1
    assert d["valid"]
