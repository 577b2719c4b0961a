"""GPU parity of the fused-operand schedule (MF_SCHED_FUSED: pre-additions in
the GEMM's operand load, post-additions in its epilogue) through the C ABI:
integer inputs bit-exact against the oracle at ragged and tile-aligned sizes,
FP64 within 1e-11 at n = 8192 on sampled rows, bitwise equal to the stored
schedule for algorithms whose coefficients are all +-1 (the operand sums and
the epilogue sums take the same operations in the same order), and with
alpha/beta, rectangular operands and leading dimensions through mf_gemm."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om
from oracle import rect as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

FUSED = None


def fused():
    return mf.MF_SCHED_FUSED


def dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)


def lib_algo(name):
    if name == "w444":
        w = mf.mf_algo_builtin("winograd")
        return mf.mf_algo_compose(w, w)
    if name == "rebased":
        X, Y, Z = mi.unimodular(2, 7), mi.unimodular(2, 8), mi.unimodular(2, 9)
        return mf.mf_algo_rebase(mf.mf_algo_builtin("strassen"), X, Y, Z)
    return mf.mf_algo_builtin(name)


def run(algo, A, B, schedule, dt=torch.float64):
    dA, dB = dev(A, dt), dev(B, dt)
    dC = torch.full_like(dA, float("nan"))
    mf.mf_fastmm(algo, 1, 0, dA, dB, dC, leaf=schedule)
    torch.cuda.synchronize()
    return dC


@pytest.mark.parametrize("name", ["strassen", "winograd", "strassen1969", "rebased", "w444"])
@pytest.mark.parametrize("n", [1000, 1001, 2048])
def test_fused_int_exact(name, n):
    print(f"fused int {name} n={n}", flush=True)
    a = lib_algo(name)
    A = mi.int_uniform(n, 60 + n % 7)
    B = mi.int_uniform(n, 70 + n % 5)
    got = run(a, A.astype(np.float64), B.astype(np.float64), fused()).cpu().numpy()
    assert np.array_equal(got, om.classical_mm(A, B).astype(np.float64))


@pytest.mark.parametrize("name", ["strassen", "winograd", "strassen1969"])
@pytest.mark.parametrize("n", [1024, 1001])
def test_fused_bitwise_equals_stored_schedule(name, n):
    a = lib_algo(name)
    A = mi.uniform(n, 80)
    B = mi.uniform(n, 81)
    f = run(a, A, B, fused())
    s = run(a, A, B, 0)
    assert torch.equal(f, s)


def test_fused_fp64_full_size_sampled():
    n = 8192
    print(f"fused winograd fp64 n={n}", flush=True)
    A = mi.uniform(n, 10)
    B = mi.uniform(n, 11)
    got = run(lib_algo("winograd"), A, B, fused())
    rows = np.sort(np.random.default_rng(3).choice(n, size=48, replace=False))
    err = om.rel_fro_error(got[torch.from_numpy(rows).cuda()].cpu().numpy(), om.rows_reference(A, B, rows))
    assert err < 1e-11


def test_fused_fp32():
    n = 1536
    A = mi.uniform(n, 12).astype(np.float32)
    B = mi.uniform(n, 13).astype(np.float32)
    got = run(lib_algo("winograd"), A, B, fused(), torch.float32).cpu().numpy().astype(np.float64)
    err = om.rel_fro_error(got, om.classical_mm(A.astype(np.float64), B.astype(np.float64)))
    assert err < 2e-5


def test_fused_gemm_rect_alpha_beta_and_ld():
    """<2,2,3;11> fused on rectangular column windows, alpha = 2, beta = -1."""
    s = mf.mf_algo_builtin("strassen")
    hk = mf.mf_algo_concat(s, mf.mf_algo_classical(2, 2, 1), "n")
    M, K, N = 700, 520, 990
    big_a = mi.int_uniform_rect(M, K + 11, 1)
    big_b = mi.int_uniform_rect(K, N + 6, 2)
    C0 = mi.int_uniform_rect(M, N, 3)
    dA, dB, dC = dev(big_a.astype(np.float64)), dev(big_b.astype(np.float64)), dev(C0.astype(np.float64))
    mf.mf_gemm(hk, 1, 0, dA[:, 11:], dB[:, :N], dC, 2.0, -1.0, schedule=fused())
    torch.cuda.synchronize()
    want = 2 * om.classical_mm(big_a[:, 11:], big_b[:, :N]) - C0
    assert np.array_equal(dC.cpu().numpy(), want.astype(np.float64))
    U, V, W = hk.uvw()
    ohk = orc.make(2, 2, 3, U, V, W)
    assert orc.brent_violations(ohk) == 0


def test_fused_rejects_deeper_and_bf16():
    w = mf.mf_algo_builtin("winograd")
    A = torch.zeros(1024, 1024, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mf.MFError) as e:
        mf.mf_fastmm(w, 2, 0, A, A.clone(), torch.empty_like(A), leaf=fused())
    assert e.value.status == mf.MF_ERR_UNSUPPORTED
    A32 = A.float()
    with pytest.raises(mf.MFError) as e:
        mf.mf_fastmm(w, 1, 0, A32, A32.clone(), torch.empty_like(A32), leaf=fused() | mf.MF_LEAF_BF16)
    assert e.value.status == mf.MF_ERR_UNSUPPORTED
