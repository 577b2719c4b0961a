"""The persistent batched kernel, checked on the CPU in its compiled form.

A loop of workgroup tasks whose ticket is fetched by one lane can compile
into a loop that lane leaves alone: the other lanes of its wave keep passing
the barriers of the loop body on a stale task while it waits to reconverge,
and the launch never ends (what the first persistent form did on the device).
These tests compile the batched kernels for gfx950 with the library's own
flags and check the assembly for that shape (tests/isa_check.py): no loop that
contains a barrier may mask off exiting lanes, and no barrier may sit inside
a lane-masked region.  A planted kernel with the fault's shape (the ticket
fetch and the completion count in separate one-lane regions on either side
of the back edge) must be flagged, and the same loop with one region must
not."""
import os
import shutil
import subprocess

import pytest

import isa_check as ic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_12732_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-O3", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-x", "hip", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S"]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")


def compile_asm(src_path, tmp_path):
    out = os.path.join(tmp_path, os.path.basename(src_path) + ".s")
    r = subprocess.run([HIPCC, *FLAGS, "-o", out, src_path], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    with open(out) as f:
        return f.read()


@pytest.fixture(scope="module")
def batch_asm(tmp_path_factory):
    return compile_asm(os.path.join(CSRC, "kernels_batch.hip"), str(tmp_path_factory.mktemp("isa")))


@pytest.mark.parametrize("fragment", ["batch_persistentId", "batch_persistentIf", "batch_gemm_phaseId",
                                      "batch_gemm_phaseIf", "batch_combine_phaseId", "batch_combine_phaseIf"])
def test_batch_kernel_barriers_are_wave_uniform(batch_asm, fragment):
    syms = ic.kernel_symbols(batch_asm, fragment)
    assert len(syms) == 1, syms
    lines = ic.function_lines(batch_asm, syms[0])
    assert ic.loops_with_divergent_barriers(lines) == []
    assert ic.barriers_in_masked_regions(lines) == 0


def test_persistent_kernel_has_its_barriers(batch_asm):
    """The check is not vacuous: the persistent loop has barriers and loops."""
    lines = ic.function_lines(batch_asm, ic.kernel_symbols(batch_asm, "batch_persistentId")[0])
    assert sum(ln.strip().startswith("s_barrier") for ln in lines) >= 3
    assert any("Loop Header" in ln for ln in lines)


SPLIT = r"""
#include <hip/hip_runtime.h>
__global__ void __launch_bounds__(512) ticket_loop(int* ctr, const int* tasks, int ntasks, float* out) {
  __shared__ int s_task;
  __shared__ float buf[512];
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(ctr, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= ntasks) return;
    buf[threadIdx.x] = tasks[t] * 2.0f;
    __syncthreads();
    out[t * 512 + threadIdx.x] = buf[(threadIdx.x + 1) & 511];
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(ctr + 1, 1);
  }
}
"""

ONE_REGION = r"""
#include <hip/hip_runtime.h>
__global__ void __launch_bounds__(512) ticket_loop(int* ctr, const int* tasks, int ntasks, float* out) {
  __shared__ int s_task;
  __shared__ float buf[512];
  int prev = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      if (prev) atomicAdd(ctr + 1, 1);
      s_task = atomicAdd(ctr, 1);
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= ntasks) break;
    buf[threadIdx.x] = tasks[t] * 2.0f;
    __syncthreads();
    out[t * 512 + threadIdx.x] = buf[(threadIdx.x + 1) & 511];
    __syncthreads();
    prev = 1;
  }
}
"""


@pytest.mark.parametrize("source,flagged", [(SPLIT, True), (ONE_REGION, False)])
def test_checker_on_planted_ticket_loops(tmp_path, source, flagged):
    src = tmp_path / "loop.hip"
    src.write_text(source)
    asm = compile_asm(str(src), str(tmp_path))
    lines = ic.function_lines(asm, ic.kernel_symbols(asm, "ticket_loop")[0])
    assert bool(ic.loops_with_divergent_barriers(lines)) == flagged
