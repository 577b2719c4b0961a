"""GPU parity of classical products over rows that are not 16-byte aligned
(odd n in FP64, n not a multiple of 4 in FP32, odd leading dimensions, or
operand bases 8 bytes past an aligned address), which copy both operands
into aligned workspace blocks before the GEMM from n = 192 on: integer
inputs bit-exact against the CPU oracle, standalone, through mf_gemm with
alpha / beta and one-sided odd strides, and as batch instances in both
batch forms; sizes on either side of the threshold."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)


@pytest.mark.parametrize("n,dt", [(191, torch.float64), (193, torch.float64), (1037, torch.float64),
                                  (2049, torch.float64), (258, torch.float32), (1037, torch.float32)])
def test_classical_copy_int_exact(n, dt):
    print(f"classical unaligned n={n} {dt}", flush=True)
    A = mi.int_uniform(n, 10 + n)
    B = mi.int_uniform(n, 20 + n)
    dA, dB = dev(A.astype(np.float64), dt), dev(B.astype(np.float64), dt)
    dC = torch.full_like(dA, float("nan"))
    mf.mf_classical_mm(dA, dB, dC)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), om.classical_mm(A, B).astype(np.float64))


@pytest.mark.parametrize("M,N,K,pad_a,pad_b", [(700, 500, 400, 1, 0), (300, 600, 500, 0, 1),
                                               (600, 700, 300, 3, 5), (200, 1000, 250, 1, 1)])
def test_gemm_odd_strides_alpha_beta_int_exact(M, N, K, pad_a, pad_b):
    """Views with odd leading dimensions (column slices of wider matrices) on
    either or both sides; C = 2 A B - C0."""
    print(f"gemm odd strides {M}x{N}x{K} lda+{pad_a} ldb+{pad_b}", flush=True)
    A = mi.int_uniform_rect(M, K, 31 + M)
    B = mi.int_uniform_rect(K, N, 41 + N)
    C0 = mi.int_uniform_rect(M, N, 51 + K)
    Aw = torch.zeros(M, K + pad_a, dtype=torch.float64, device="cuda:0")
    Bw = torch.zeros(K, N + pad_b, dtype=torch.float64, device="cuda:0")
    Aw[:, :K] = dev(A.astype(np.float64), torch.float64)
    Bw[:, :N] = dev(B.astype(np.float64), torch.float64)
    dC = dev(C0.astype(np.float64), torch.float64)
    mf.mf_gemm(None, 0, 0, Aw[:, :K], Bw[:, :N], dC, 2.0, -1.0)
    torch.cuda.synchronize()
    want = 2 * om.classical_mm(A, B) - C0
    assert np.array_equal(dC.cpu().numpy(), want.astype(np.float64))


@pytest.mark.parametrize("form", [mf.MF_BATCH_PHASES, mf.MF_BATCH_PERSISTENT])
def test_batch_classical_copies_int_exact(form):
    """Classical batch instances of odd n (copies) beside aligned and
    below-threshold ones, each equal to the oracle."""
    sizes = [385, 1037, 256, 129, 193, 640]
    print(f"batch form {form} sizes {sizes}", flush=True)
    b = mf.mf_batch_create(sizes, [None] * len(sizes), [0] * len(sizes), [0] * len(sizes), mf.MF_F64, form)
    As = [mi.int_uniform(n, 60 + i) for i, n in enumerate(sizes)]
    Bs = [mi.int_uniform(n, 70 + i) for i, n in enumerate(sizes)]
    dA = [dev(a.astype(np.float64), torch.float64) for a in As]
    dB = [dev(x.astype(np.float64), torch.float64) for x in Bs]
    dC = [torch.full_like(a, float("nan")) for a in dA]
    mf.mf_batch_run(b, dA, dB, dC)
    torch.cuda.synchronize()
    assert not b.aborted()
    for A, B, C in zip(As, Bs, dC):
        assert np.array_equal(C.cpu().numpy(), om.classical_mm(A, B).astype(np.float64))


def offset_view(x, dt, ld):
    """x as a view with leading dimension ld whose base lies 8 bytes past
    the (256-byte aligned) start of its allocation."""
    rows, cols = x.shape
    shift = 8 // torch.tensor([], dtype=dt).element_size()
    buf = torch.zeros(rows * ld + shift, dtype=dt, device="cuda:0")
    v = buf[shift:].view(rows, ld)[:, :cols]
    v.copy_(dev(x.astype(np.float64), dt))
    assert v.data_ptr() % 16 == 8
    return v


@pytest.mark.parametrize("n,dt", [(1024, torch.float64), (640, torch.float32)])
def test_offset_bases_int_exact(n, dt):
    """Square operands at bases 8 bytes off alignment (rows aligned): the
    classical product and Winograd depth 1 copy them first; mf_gemm takes a
    rectangular offset view of A."""
    print(f"offset bases n={n} {dt}", flush=True)
    A = mi.int_uniform(n, 80 + n)
    B = mi.int_uniform(n, 90 + n)
    want = om.classical_mm(A, B).astype(np.float64)
    dA, dB = offset_view(A, dt, n), dev(B.astype(np.float64), dt)
    for run in (lambda C: mf.mf_classical_mm(dA, dB, C),
                lambda C: mf.mf_fastmm(mf.mf_algo_builtin("winograd"), 1, 0, dA, dB, C)):
        dC = torch.full((n, n), float("nan"), dtype=dt, device="cuda:0")
        run(dC)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.float64), want)
    M, K, N = 500, 600, 700
    Ar = mi.int_uniform_rect(M, K, 81)
    Br = mi.int_uniform_rect(K, N, 82)
    dC = torch.full((M, N), float("nan"), dtype=dt, device="cuda:0")
    mf.mf_gemm(None, 0, 0, offset_view(Ar, dt, K + 8), offset_view(Br, dt, N), dC)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.float64), om.classical_mm(Ar, Br).astype(np.float64))
