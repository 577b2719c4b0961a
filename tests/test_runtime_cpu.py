"""The binding and PyTorch share one HIP runtime in the process, whatever the
import order (PyTorch for ROCm ships its own copy of the runtime; a second
copy next to it breaks streams and events)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytest.importorskip("torch")
if not os.path.exists(os.path.join(ROOT, "paper_2312_12732_amd", "libmf.so")):
    pytest.skip("libmf.so not built", allow_module_level=True)

PROBE = """
import sys
{first}
{second}
maps = open('/proc/self/maps').read()
libs = sorted({{l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}})
print(len(libs))
"""


@pytest.mark.parametrize("order", [("from paper_2312_12732_amd import mf", "import torch"),
                                   ("import torch", "from paper_2312_12732_amd import mf")])
def test_one_hip_runtime(order):
    code = PROBE.format(first=order[0], second=order[1])
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
