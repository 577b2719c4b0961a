"""The allocation-free entry point (mf_fastmm_noalloc) against mf_fastmm,
through the C ABI: same plan, so the results must be bitwise equal, on two
calls in a row (the second smaller, so the scratch array holds the first
call's descriptors and workspace when it starts), plus the integer product
against the oracle and the rejection of a request beyond the scratch limit."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

SCRATCH = 256 << 20


def dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)


def both(algo, depth, A, B, dt=torch.float64):
    """C from mf_fastmm and from mf_fastmm_noalloc on the same operands."""
    dA, dB = dev(A, dt), dev(B, dt)
    ref = torch.full_like(dA, float("nan"))
    got = torch.full_like(dA, float("nan"))
    mf.mf_fastmm(algo, depth, 0, dA, dB, ref)
    mf.mf_fastmm_noalloc(algo, depth, 0, dA, dB, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("name,depth,sizes", [("winograd", 2, (1000, 600)), ("strassen", 1, (1024, 257))])
def test_noalloc_equals_fastmm_twice(name, depth, sizes):
    algo = mf.mf_algo_builtin(name)
    for k, n in enumerate(sizes):
        print(f"noalloc {name} depth {depth} n={n} call {k}", flush=True)
        assert mf.mf_workspace_bytes(algo, depth, 0, n) < SCRATCH
        A = mi.uniform(n, 50 + k)
        B = mi.uniform(n, 60 + k)
        ref, got = both(algo, depth, A, B)
        assert np.array_equal(ref, got), f"n={n}: results differ from mf_fastmm"
        err = om.rel_fro_error(got, om.classical_mm(A, B))
        assert err < 1e-11


def test_noalloc_int_exact_and_fp32():
    algo = mf.mf_algo_builtin("winograd")
    comp = mf.mf_algo_compose(algo, algo)
    for n, seed in ((777, 3), (513, 5)):
        print(f"noalloc <4,4,4;49> int n={n}", flush=True)
        A = mi.int_uniform(n, seed)
        B = mi.int_uniform(n, seed + 1)
        ref, got = both(comp, 1, A.astype(np.float64), B.astype(np.float64))
        assert np.array_equal(got, om.classical_mm(A, B).astype(np.float64))
        assert np.array_equal(ref, got)
    for n in (900, 300):
        print(f"noalloc fp32 winograd depth 2 n={n}", flush=True)
        A = mi.uniform(n, 7).astype(np.float32)
        B = mi.uniform(n, 8).astype(np.float32)
        ref, got = both(algo, 2, A, B, torch.float32)
        assert np.array_equal(ref, got)


def test_noalloc_rejects_beyond_limit():
    algo = mf.mf_algo_builtin("winograd")
    n = 4096
    assert mf.mf_workspace_bytes(algo, 1, 0, n) > SCRATCH
    A = torch.zeros(n, n, dtype=torch.float64, device="cuda:0")
    B = torch.zeros_like(A)
    C = torch.zeros_like(A)
    with pytest.raises(mf.MFError) as ei:
        mf.mf_fastmm_noalloc(algo, 1, 0, A, B, C)
    assert ei.value.status == mf.MF_ERR_SHAPE
    assert "scratch" in str(ei.value)
    # the array still serves a request that fits afterwards
    Ai = mi.int_uniform(512, 11)
    Bi = mi.int_uniform(512, 12)
    ref, got = both(algo, 1, Ai.astype(np.float64), Bi.astype(np.float64))
    assert np.array_equal(got, om.classical_mm(Ai, Bi).astype(np.float64))


def test_noalloc_reads_unaligned_rows_in_place_when_copies_do_not_fit():
    """Odd n: mf_fastmm copies both operands into aligned blocks, which at
    n = 4097 (FP64) need more than the scratch array; the allocation-free call
    then reads the rows in place (same K steps over the same zero padding),
    bitwise equal to mf_fastmm.  A smaller odd call after it copies again."""
    w = mf.mf_algo_builtin("winograd")
    n = 4097
    assert mf.mf_workspace_bytes(w, 0, 0, n) > SCRATCH
    print(f"noalloc classical unaligned n={n} (read in place)", flush=True)
    Ai = mi.int_uniform(n, 21)
    Bi = mi.int_uniform(n, 22)
    ref, got = both(w, 0, Ai.astype(np.float64), Bi.astype(np.float64))
    assert np.array_equal(ref, got)
    rows = [0, 1, 2048, n - 1]
    assert np.array_equal(got[rows], om.rows_reference(Ai, Bi, rows))
    ref, got = both(w, 0, mi.uniform(n, 23), mi.uniform(n, 24))
    assert np.array_equal(ref, got)
    m = 1037
    assert 0 < mf.mf_workspace_bytes(w, 0, 0, m) < SCRATCH
    print(f"noalloc classical unaligned n={m} (copies)", flush=True)
    ref, got = both(w, 0, mi.uniform(m, 25), mi.uniform(m, 26))
    assert np.array_equal(ref, got)


def test_noalloc_offset_bases_equal_fastmm():
    """Operand bases 8 bytes off alignment: the allocation-free call copies
    them as mf_fastmm does (the copies fit the array), bitwise equal."""
    w = mf.mf_algo_builtin("winograd")
    n = 768
    print(f"noalloc offset bases n={n}", flush=True)
    buf_a = torch.zeros(n * n + 1, dtype=torch.float64, device="cuda:0")
    buf_b = torch.zeros(n * n + 1, dtype=torch.float64, device="cuda:0")
    dA, dB = buf_a[1:].view(n, n), buf_b[1:].view(n, n)
    dA.copy_(dev(mi.uniform(n, 27)))
    dB.copy_(dev(mi.uniform(n, 28)))
    assert dA.data_ptr() % 16 == 8
    for depth in (0, 1):
        ref = torch.full_like(dA, float("nan"))
        got = torch.full_like(dA, float("nan"))
        mf.mf_fastmm(w, depth, 0, dA, dB, ref)
        mf.mf_fastmm_noalloc(w, depth, 0, dA, dB, got)
        torch.cuda.synchronize()
        assert torch.equal(ref, got)
