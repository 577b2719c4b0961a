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


def _load_bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_null_unless_taken_on_current_kernel(tmp_path, monkeypatch):
    # The HBM-traffic figure is reported only when the committed counter
    # summary was taken on the current GEMM sources and the same workload.
    import json
    b = _load_bench()
    wl = "fp64 n=8192 winograd depth 3 (Kronecker-fused)"
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.traffic_for(wl) is None                                   # no file
    f.write_text(json.dumps({"kernel_sha": b.kernel_sha(), "workload": wl, "hbm_bytes_per_launch": 123}))
    assert b.traffic_for(wl) == 123
    assert b.traffic_for("fp64 n=8192 winograd depth 2 (Kronecker-fused)") is None  # other workload
    f.write_text(json.dumps({"kernel_sha": "0" * 16, "workload": wl, "hbm_bytes_per_launch": 123}))
    assert b.traffic_for(wl) is None                                   # stale kernel
    f.write_text("not json")
    assert b.traffic_for(wl) is None


def test_kernel_sha_covers_the_gemm_sources():
    b = _load_bench()
    names = sorted(os.path.basename(p) for p in b.KERNEL_SRCS)
    assert names == ["gemm_common.h", "gemm_tile.h", "kernels_gemm.hip"]
    assert all(os.path.exists(p) for p in b.KERNEL_SRCS)
