"""bench.py's command-line contract on the host: a request for more than one
GPU (by flag or by a launcher's WORLD_SIZE) ends with exit status 2 and a
message, before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,world", [(["--gpus", "2"], "1"), (["--gpus", "8"], "1"), ([], "4")])
def test_multi_gpu_request_exits(argv, world):
    env = dict(os.environ, WORLD_SIZE=world)
    out = subprocess.run([sys.executable, "bench.py", *argv], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 2, out.stderr
    assert "one GPU only" in out.stderr
    assert out.stdout == ""


def test_help_lists_workloads():
    out = subprocess.run([sys.executable, "bench.py", "--help"], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0
    for w in ("square", "batched", "serving", "precision", "copy", "algorithms"):
        assert w in out.stdout
