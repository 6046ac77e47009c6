"""bench.py paths that run without a GPU: the one-GPU refusal and the oracle's
host timing line (the same routine that fills the benchmark's cpu_baseline)."""
import json

import bench


def _last_json(capsys):
    out = capsys.readouterr().out.strip().splitlines()
    return json.loads(out[-1])


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    d = _last_json(capsys)
    assert d["n_gpus"] == 2 and "one GPU" in d["error"]


def test_host_oracle_timing_line(capsys):
    # one plan of the paper-scale case run to its own stop, here a cap of three
    # accepted steps, with one BLAS thread
    assert bench.main(["--cpu-only", "--cpu-threads", "1", "--cpu-plans", "1",
                       "--iters", "3"]) == 0
    d = _last_json(capsys)
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "plans/s"
    assert cb["cores"] == 1
    assert cb["value"] > 0.0
    assert abs(d["s_per_plan"] * cb["value"] - 1.0) < 1e-12
    assert "at most 3 steps; 3 accepted steps in all" in cb["sample"]
    assert cb["host_cpu"]
