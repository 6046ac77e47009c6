"""The oracle's pins fail under every planted mistake of tests/planted.py.

Each mistake rewrites one passage of the oracle (in a private copy loaded by
the pytest plugin, in a subprocess) and the three pin suites run against it;
the run must end with at least one failed test.  This is what makes the pins
evidence: a pin suite that passes a wrong oracle proves nothing.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import planted  # noqa: E402

PIN_SUITES = ["tests/test_oracle_pins.py", "tests/test_oracle_lbfgs_pins.py",
              "tests/test_mlp_oracle_pins.py"]


@pytest.mark.parametrize("name", sorted(planted.MISTAKES))
def test_planted_passage_exists_once(name):
    fname, src = planted.planted_source(name)
    with open(os.path.join(ROOT, "oracle", fname)) as fh:
        assert fh.read() != src


def _run(name):
    env = dict(os.environ, GMCO_PLANT=name, PYTHONPATH=HERE + os.pathsep + os.environ.get("PYTHONPATH", ""),
               OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-p", "planted", "-p", "no:cacheprovider",
                        "-x", "-q", "-m", "not gpu", *PIN_SUITES], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED ")]
    return name, r.returncode, failed, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin():
    names = sorted(planted.MISTAKES)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 2)) as ex:
        results = list(ex.map(_run, names))
    missed = [(n, rc, out) for n, rc, failed, out in results if rc != 1 or not failed]
    for n, rc, failed, _ in results:
        print(f"{n}: caught by {failed[0] if failed else '-'}")
    assert not missed, "\n\n".join(f"{n} (exit {rc}):\n{out}" for n, rc, out in missed)
