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
