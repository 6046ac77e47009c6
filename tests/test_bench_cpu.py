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


def test_kernel_source_hash_ignores_comments_only(tmp_path):
    # The traffic figure stays valid across comment edits of the kernel
    # source, and is dropped for any change of its code.
    import bench
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    b.write_text("// a note\nint f(int x) {\n\n  return x + 1;  // another note\n}\n")
    c.write_text("int f(int x) {\n  return x + 2;  // one\n}\n")
    assert bench.kernel_source_hash(str(a)) == bench.kernel_source_hash(str(b))
    assert bench.kernel_source_hash(str(a)) != bench.kernel_source_hash(str(c))
