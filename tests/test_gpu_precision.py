"""GPU parity of the precision form: FP32 storage and additions, leaves in
FP32, BF16 (FP32 accumulation) or split-BF16x3, through the C ABI.

Reference: the FP64 CPU oracle applied to the FP32-rounded inputs, so input
rounding is excluded from the measured error.

Exactness pin: on integer inputs in [-8, 8] every intermediate of the
algorithm is an integer small enough to be exact in the leaf precision
(|T|, |S| <= 16 * 8 = 128 <= 256 at depth <= 2 is exact in BF16's 8-bit
significand; products and sums stay below 2^24, exact in FP32), so every mode
must match the integer product bit for bit.  At depth 3 |T| reaches 512,
which BF16 rounds but the split form represents exactly (hi + lo).

Tolerances (normwise, ||C_hat - C||_F / ||C||_F, n <= 1024), per depth d:
tol = e0 * 2.5^d * 3.  e0 is the depth-0 error of the leaf arithmetic on
uniform[-1,1] inputs at this size: FP32 leaves 4e-7 (FP32 accumulation over
K = 1024 terms, about sqrt(K) u with u = 2^-24), BF16 leaves 2e-3 (each
operand rounded to 8 significant bits, u = 2^-9, so about 2u per product),
split-BF16x3 4e-6 (hi + lo carry 16 bits; the dropped lo*lo term and the FP32
accumulation dominate).  2.5 is the growth per Strassen level of the normwise
error on these inputs (the CPU emulation of FP32 leaves gives 2.4, BF16 2.6,
BF16x3 2.6 per level at n = 1024-2048), and 3 the margin.  Scaled inputs
(rows and columns times log-uniform factors in [1e-4, 1e4]) keep the
normwise error relative to ||C|| at the same level; their componentwise
error max |C_hat - C| / (|A| |B|) is small for the classical product and
large for any fast level (the fast method is not componentwise stable)."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

LEAVES = {"f32": mf.MF_LEAF_F32, "bf16": mf.MF_LEAF_BF16, "bf16x3": mf.MF_LEAF_BF16X3}
E0 = {"f32": 4e-7, "bf16": 2e-3, "bf16x3": 4e-6}


def tol(leaf, depth):
    return E0[leaf] * 2.5 ** depth * 3


def dev32(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


def run(algo, depth, A, B, leaf):
    dA, dB = dev32(A), dev32(B)
    dC = torch.full_like(dA, float("nan"))
    if algo is None:
        mf.mf_classical_mm(dA, dB, dC) if leaf == mf.MF_LEAF_NATIVE else mf.mf_fastmm(
            mf.mf_algo_builtin("strassen"), 0, 0, dA, dB, dC, leaf=leaf)
    else:
        mf.mf_fastmm(algo, depth, 0, dA, dB, dC, leaf=leaf)
    torch.cuda.synchronize()
    return dC.cpu().numpy().astype(np.float64)


def ref64(A, B):
    return om.classical_mm(A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("leaf", list(LEAVES))
@pytest.mark.parametrize("depth", [0, 1, 2])
@pytest.mark.parametrize("n", [256, 300])
def test_int_exact(leaf, depth, n):
    A = mi.int_uniform(n, 3).astype(np.float64)
    B = mi.int_uniform(n, 4).astype(np.float64)
    got = run(mf.mf_algo_builtin("strassen"), depth, A, B, LEAVES[leaf])
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("leaf", ["f32", "bf16x3"])
def test_int_exact_depth3(leaf):
    A = mi.int_uniform(512, 5).astype(np.float64)
    B = mi.int_uniform(512, 6).astype(np.float64)
    got = run(mf.mf_algo_builtin("winograd"), 3, A, B, LEAVES[leaf])
    assert np.array_equal(got, A @ B)


def test_native_fp32_storage_is_f32_leaf():
    A = mi.uniform(512, 1)
    B = mi.uniform(512, 2)
    s = mf.mf_algo_builtin("strassen")
    assert np.array_equal(run(s, 1, A, B, mf.MF_LEAF_NATIVE), run(s, 1, A, B, mf.MF_LEAF_F32))


def test_fp32_classical():
    A = mi.uniform(1024, 1)
    B = mi.uniform(1024, 2)
    err = om.rel_fro_error(run(None, 0, A, B, mf.MF_LEAF_NATIVE), ref64(A, B))
    assert err < 2e-6


@pytest.mark.parametrize("leaf", list(LEAVES))
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
def test_uniform_error(leaf, depth):
    n = 1024
    A = mi.uniform(n, 20)
    B = mi.uniform(n, 21)
    err = om.rel_fro_error(run(mf.mf_algo_builtin("winograd"), depth, A, B, LEAVES[leaf]), ref64(A, B))
    assert err < tol(leaf, depth), err


def test_bf16x3_recovers_accuracy():
    n = 1024
    A = mi.uniform(n, 20)
    B = mi.uniform(n, 21)
    s = mf.mf_algo_builtin("strassen")
    e1 = om.rel_fro_error(run(s, 1, A, B, LEAVES["bf16"]), ref64(A, B))
    e3 = om.rel_fro_error(run(s, 1, A, B, LEAVES["bf16x3"]), ref64(A, B))
    assert e3 < e1 / 50


@pytest.mark.parametrize("leaf", list(LEAVES))
def test_scaled_inputs_normwise(leaf):
    # rows and columns scaled by log-uniform factors in [1e-4, 1e4]: the
    # normwise error relative to ||C|| stays within the uniform-input bound
    n = 512
    A = mi.scaled(n, 22, 23, 24).astype(np.float32).astype(np.float64)
    B = mi.scaled(n, 25, 26, 27).astype(np.float32).astype(np.float64)
    ref = ref64(A, B)
    got = run(mf.mf_algo_builtin("strassen"), 2, A, B, LEAVES[leaf])
    assert om.rel_fro_error(got, ref) < tol(leaf, 2)


def test_scaled_inputs_componentwise():
    """The componentwise error on scaled inputs: small for the classical
    product (FP32 leaves), many orders larger once one fast level mixes
    blocks of different scales."""
    n = 512
    A = mi.scaled(n, 22, 23, 24).astype(np.float32).astype(np.float64)
    B = mi.scaled(n, 25, 26, 27).astype(np.float32).astype(np.float64)
    ref = ref64(A, B)
    c0 = om.componentwise_error(run(None, 0, A, B, mf.MF_LEAF_F32), ref, A, B)
    c1 = om.componentwise_error(run(mf.mf_algo_builtin("strassen"), 1, A, B, mf.MF_LEAF_F32), ref, A, B)
    assert c0 < 1e-5
    assert c1 > 1e3 * c0


def test_precision_determinism():
    A = dev32(mi.uniform(512, 1))
    B = dev32(mi.uniform(512, 2))
    s = mf.mf_algo_builtin("winograd")
    for leaf in LEAVES.values():
        C1 = torch.empty_like(A)
        C2 = torch.empty_like(A)
        mf.mf_fastmm(s, 2, 0, A, B, C1, leaf=leaf)
        mf.mf_fastmm(s, 2, 0, A, B, C2, leaf=leaf)
        torch.cuda.synchronize()
        assert torch.equal(C1, C2)


@pytest.mark.parametrize("leaf", ["bf16", "bf16x3"])
@pytest.mark.parametrize("n,depth", [(4000, 0), (4001, 1), (3000, 2)])
def test_bf16_staging_large_ragged(leaf, n, depth):
    """BF16 leaf operands are staged (A row-major, B transposed, zero padding)
    before the GEMM: ragged sizes over many staging tiles, integer inputs
    (exact in BF16 and in the FP32 sums) compared exactly on sampled rows and
    columns, first and last included."""
    A = mi.int_uniform(n, 90).astype(np.float64)
    B = mi.int_uniform(n, 91).astype(np.float64)
    got = run(mf.mf_algo_builtin("winograd") if depth else None, depth, A, B, LEAVES[leaf])
    rows = np.unique(np.concatenate([np.random.default_rng(n).choice(n, size=24, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([np.random.default_rng(n + 1).choice(n, size=24, replace=False), [0, n - 1]]))
    assert np.array_equal(got[rows], om.rows_reference(A, B, rows))
    assert np.array_equal(got[:, cols], A @ B[:, cols])


@pytest.mark.parametrize("leaf", ["bf16", "bf16x3"])
@pytest.mark.parametrize("name,n", [("444", 300), ("444", 301), ("classical3", 299), ("winograd", 301)])
def test_bf16_staging_sets_int_exact(leaf, name, n):
    """BF16 leaves fuse the last pre-addition level into the staging: one
    staging set per block of the level above, 16 inputs for <4,4,4;49>
    (Winograd composed with itself), 9 for the <3,3,3;27> classical control,
    4 for Winograd.  Ragged sizes put quarters partly or wholly in the virtual
    padding; odd n makes the caller's rows unaligned (element-wise loads).
    Integer inputs in [-2, 2] keep every staged operand (|T| <= 16 * 2) exact in
    BF16 and every sum below 2^24, so the result must be the integer product."""
    A = mi.int_uniform(n, 92, -2, 2).astype(np.float64)
    B = mi.int_uniform(n, 93, -2, 2).astype(np.float64)
    w = mf.mf_algo_builtin("winograd")
    algo = mf.mf_algo_compose(w, w) if name == "444" else mf.mf_algo_builtin(name)
    got = run(algo, 1, A, B, LEAVES[leaf])
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("leaf", ["bf16", "bf16x3"])
def test_bf16_fused_depth2_uniform_error(leaf):
    """Kronecker-fused depth 2 (one level of <4,4,4;49>) with BF16 leaves
    matches the level-by-level depth 2 within the leaf tolerance, and both stay
    within it against the FP64 oracle."""
    n = 512
    A = mi.uniform(n, 94).astype(np.float32).astype(np.float64)
    B = mi.uniform(n, 95).astype(np.float32).astype(np.float64)
    w = mf.mf_algo_builtin("winograd")
    ref = ref64(A, B)
    fused = run(mf.mf_algo_compose(w, w), 1, A, B, LEAVES[leaf])
    level = run(w, 2, A, B, LEAVES[leaf])
    assert om.rel_fro_error(fused, ref) < tol(leaf, 2)
    assert om.rel_fro_error(level, ref) < tol(leaf, 2)
