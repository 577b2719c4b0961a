"""GPU parity of the batched form: many products of different sizes,
algorithms and depths, run as one launch per phase over all instances,
against the CPU oracle and against standalone products."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def plan(sizes, dtype):
    s = mf.mf_algo_builtin("winograd")
    s2 = mf.mf_algo_compose(s, s)
    p = mf.mf_algo_builtin("strassen")
    choices = [(None, 0), (s, 1), (s, 2), (s2, 1), (p, 1)]
    algos, depths = [], []
    for i in range(len(sizes)):
        a, d = choices[i % len(choices)]
        algos.append(a)
        depths.append(d)
    return mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), dtype)


def run(batch, As, Bs, tdtype, workspace=None):
    dA = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", tdtype) for a in As]
    dB = [torch.from_numpy(np.ascontiguousarray(b)).to("cuda:0", tdtype) for b in Bs]
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(batch, dA, dB, dC, workspace=workspace)
    torch.cuda.synchronize()
    assert not batch.aborted()
    return [c.cpu().numpy().astype(np.float64) for c in dC]


SIZES = mi.batch_sizes(20, 30) + [100, 300, 513, 64, 1]


def test_batch_matches_standalone_for_classical():
    sizes = [256, 640, 1024]
    b = mf.mf_batch_create(sizes, [None] * 3, [0] * 3, [0] * 3, mf.MF_F64)
    As = [mi.uniform(n, 1 + i) for i, n in enumerate(sizes)]
    Bs = [mi.uniform(n, 11 + i) for i, n in enumerate(sizes)]
    Cs = run(b, As, Bs, torch.float64)
    for A, B, C in zip(As, Bs, Cs):
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        dC = torch.empty_like(dA)
        mf.mf_classical_mm(dA, dB, dC)
        torch.cuda.synchronize()
        assert np.array_equal(C, dC.cpu().numpy())


def test_tiny_fast_batch():
    """Two instances with dependencies (pre-additions, then GEMM tiles)."""
    s = mf.mf_algo_builtin("winograd")
    sizes = [256, 384]
    b = mf.mf_batch_create(sizes, [s, s], [1, 1], [0, 0], mf.MF_F64)
    As = [mi.int_uniform(n, 900 + i).astype(np.float64) for i, n in enumerate(sizes)]
    Bs = [mi.int_uniform(n, 950 + i).astype(np.float64) for i, n in enumerate(sizes)]
    for A, B, C in zip(As, Bs, run(b, As, Bs, torch.float64)):
        assert np.array_equal(C, A @ B)


def test_batch_fp64_int_exact():
    b = plan(SIZES, mf.MF_F64)
    As = [mi.int_uniform(n, 100 + i).astype(np.float64) for i, n in enumerate(SIZES)]
    Bs = [mi.int_uniform(n, 200 + i).astype(np.float64) for i, n in enumerate(SIZES)]
    Cs = run(b, As, Bs, torch.float64)
    for A, B, C in zip(As, Bs, Cs):
        assert np.array_equal(C, A @ B)


def test_batch_fp64_uniform_and_deterministic():
    b = plan(SIZES, mf.MF_F64)
    As = [mi.uniform(n, 300 + i) for i, n in enumerate(SIZES)]
    Bs = [mi.uniform(n, 400 + i) for i, n in enumerate(SIZES)]
    C1 = run(b, As, Bs, torch.float64)
    ws = torch.empty(max(1, b.workspace_bytes() // 8), dtype=torch.float64, device="cuda:0")
    C2 = run(b, As, Bs, torch.float64, workspace=ws)
    for A, B, c1, c2 in zip(As, Bs, C1, C2):
        assert np.array_equal(c1, c2)
        assert om.rel_fro_error(c1, om.classical_mm(A, B)) < 1e-11


def test_batch_fp32():
    b = plan(SIZES, mf.MF_F32)
    As = [mi.int_uniform(n, 500 + i).astype(np.float32) for i, n in enumerate(SIZES)]
    Bs = [mi.int_uniform(n, 600 + i).astype(np.float32) for i, n in enumerate(SIZES)]
    Cs = run(b, As, Bs, torch.float32)
    for A, B, C in zip(As, Bs, Cs):
        assert np.array_equal(C, A.astype(np.float64) @ B.astype(np.float64))
    As = [mi.uniform(n, 700 + i).astype(np.float32) for i, n in enumerate(SIZES)]
    Bs = [mi.uniform(n, 800 + i).astype(np.float32) for i, n in enumerate(SIZES)]
    Cs = run(b, As, Bs, torch.float32)
    for A, B, C in zip(As, Bs, Cs):
        ref = om.classical_mm(A.astype(np.float64), B.astype(np.float64))
        assert om.rel_fro_error(C, ref) < 2e-5


def test_batch_rejects_mismatched_inputs():
    b = plan([256, 512], mf.MF_F64)
    A = torch.zeros(256, 256, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        mf.mf_batch_run(b, [A, A], [A, A], [torch.empty_like(A), torch.empty_like(A)])


def test_batch_bitwise_equals_standalone_fast():
    """Every instance runs the plan of the standalone call with the same
    arguments: results agree bit for bit on uniform inputs."""
    s = mf.mf_algo_builtin("winograd")
    s2 = mf.mf_algo_compose(s, s)
    sizes = [1024, 700, 1536, 512, 1000]
    algos = [s, s, s2, s, s]
    depths = [2, 1, 1, 3, 2]
    for code, tdt in ((mf.MF_F64, torch.float64), (mf.MF_F32, torch.float32)):
        b = mf.mf_batch_create(sizes, algos, depths, [0] * len(sizes), code)
        As = [mi.uniform(n, 1000 + i) for i, n in enumerate(sizes)]
        Bs = [mi.uniform(n, 1100 + i) for i, n in enumerate(sizes)]
        Cs = run(b, As, Bs, tdt)
        for A, B, C, al, d in zip(As, Bs, Cs, algos, depths):
            dA = torch.from_numpy(A).to("cuda:0", tdt)
            dB = torch.from_numpy(B).to("cuda:0", tdt)
            dC = torch.empty_like(dA)
            mf.mf_fastmm(al, d, 0, dA, dB, dC)
            torch.cuda.synchronize()
            assert np.array_equal(C, dC.cpu().numpy().astype(np.float64))
