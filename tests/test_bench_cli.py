"""Host checks of the benchmark's command line (no GPU work)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    # The engine runs on one GPU; any other count exits with a JSON message
    # before torch or the library is touched.
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                       env={**os.environ, **env}, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("argv", [["--workload", "table1", "--apps", "no-such-app"],
                                  ["--workload", "mnist512", "--apps", "MNIST-512c"]])
def test_bench_rejects_bad_app_filter(argv):
    # --apps names Table I applications and only applies to that workload;
    # a bad value is an argument error, raised before any GPU work.
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--apps" in r.stderr
