"""CPU-only checks of the C-ABI library: it loads, exports every declared
symbol, builds the same algorithms as the oracle (host algebra only) and
rejects invalid requests before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(mf_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared_symbols()
    assert "mf_fastmm" in names and "mf_classical_mm" in names and "mf_algo_from_uvw" in names
    for n in names:
        assert hasattr(mf.lib, n), n
    assert set(names) == set(mf.EXPORTED)


def oracle_table(t):
    U, V, W, conv = mi.as_float_tables(t)
    return oa.canonical(t["n0"], U, V, W, conv)


def same(alg_handle, o):
    U, V, W = alg_handle.uvw()
    return np.array_equal(U, o.U) and np.array_equal(V, o.V) and np.array_equal(W, o.W)


@pytest.mark.parametrize("name,table", [("strassen", mi.STRASSEN_PAPER), ("winograd", mi.WINOGRAD),
                                        ("strassen1969", mi.STRASSEN_1969)])
def test_builtins_match_published_tables(name, table):
    assert same(mf.mf_algo_builtin(name), oracle_table(table))


@pytest.mark.parametrize("p", [2, 3])
def test_builtin_classical(p):
    assert same(mf.mf_algo_builtin(f"classical{p}"), oa.classical_algo(p))


def test_from_uvw_deepmind_convention():
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    a = mf.mf_algo_from_uvw(2, U, V, W, conv)
    assert same(a, oracle_table(mi.STRASSEN_PAPER))
    assert a.info() == {"n0": 2, "R": 7, "nnz_u": 14, "nnz_v": 14, "nnz_w": 12}


def test_from_uvw_rejects_wrong_convention_and_flips():
    U, V, W, _ = mi.as_float_tables(mi.STRASSEN_PAPER)
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_from_uvw(2, U, V, W, mf.MF_W_ROWMAJOR_C)
    assert e.value.status == mf.MF_ERR_BRENT
    U2 = U.copy()
    U2[1, 3] = -1
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_from_uvw(2, U2, V, W, mf.MF_W_DEEPMIND_CT)
    assert e.value.status == mf.MF_ERR_BRENT


def test_from_uvw_argument_errors():
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    for bad in (0, 9):
        with pytest.raises(mf.MFError):
            mf.mf_algo_from_uvw(bad, U, V, W, conv)
    with pytest.raises(mf.MFError):
        mf.mf_algo_from_uvw(2, U, V, W, 7)
    Un = U.copy()
    Un[0, 0] = np.nan
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_from_uvw(2, Un, V, W, conv)
    assert e.value.status == mf.MF_ERR_ARG


def test_compose_matches_oracle():
    s = mf.mf_algo_builtin("winograd")
    o = oracle_table(mi.WINOGRAD)
    assert same(mf.mf_algo_compose(s, s), oa.power(o, 2))
    c3 = mf.mf_algo_builtin("classical3")
    # split factor 6 > 8 is rejected; 2 x 3 = 6 is allowed
    assert same(mf.mf_algo_compose(s, c3), oa.compose(o, oa.classical_algo(3)))
    s2 = mf.mf_algo_compose(s, s)
    assert same(mf.mf_algo_compose(s2, s), oa.power(o, 3))
    with pytest.raises(mf.MFError):
        mf.mf_algo_compose(s2, s2)  # split factor 16


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_rebase_matches_oracle(seed):
    X, Y, Z = (mi.unimodular(2, seed * 10 + t) for t in range(3))
    s = mf.mf_algo_builtin("strassen")
    o = oracle_table(mi.STRASSEN_PAPER)
    assert same(mf.mf_algo_rebase(s, X, Y, Z), oa.rebase(o, X, Y, Z))


def test_rebase_rejects_singular():
    s = mf.mf_algo_builtin("strassen")
    I = np.eye(2, dtype=np.int64)
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_rebase(s, 2 * I, I, I)
    assert e.value.status == mf.MF_ERR_ARG


def expected_ws(n, depth, mat_u, mat_v, R=7, p=2, min_wg=1 << 62):
    """Closed form of the executor's workspace (elements of 8 bytes):
    level l of the pre-additions materialises mat_u + mat_v children of each
    of the R^(l-1) parents, each of size (n'/p^l)^2 (n' = p^d * m, m = n/p^d
    rounded up to 16, the leaf step of FP64 / FP32 leaves); when the
    ceil(m/128)^2 tile positions times
    R^lo groups first reach min_wg workgroups at lo outer levels (a
    standalone product takes every level: lo = d), every group keeps a result
    block of size (m p^(d-lo))^2 and every post-addition parent below the
    top one a block p times larger."""
    size, d = n, 0
    while d < depth and size > 128 and R ** (d + 1) <= 1 << 16:
        size, d = -(-size // p), d + 1
    depth = d
    P = p ** depth
    m = 16 * -(-(-(-n // P)) // 16)
    npad = P * m
    elems = 0
    for lev in range(1, depth + 1):
        s = npad // p ** lev
        elems += (mat_u + mat_v) * R ** (lev - 1) * s * s
    pos = (-(-m // 128)) ** 2
    lo = 0
    while lo < depth and pos * R ** lo < min_wg:
        lo += 1
    if lo:
        mo = m * p ** (depth - lo)
        elems += R ** lo * mo * mo
        csz = mo
        for lev in range(lo, 1, -1):
            csz *= p
            elems += R ** (lev - 1) * csz * csz
    return 8 * elems


def test_workspace_bytes_closed_form():
    s = mf.mf_algo_builtin("strassen")
    # depth 1: 4 materialised T and 4 materialised S of (n/2)^2 doubles, and the
    # 7 stored products of (n/2)^2
    assert mf.mf_workspace_bytes(s, 1, 0, 8192) == 8 * (8 + 7) * 4096 ** 2 == expected_ws(8192, 1, 4, 4)
    # depth 2: level 1 (4 + 4 blocks of (n/2)^2), level 2 (7 x (4 + 4) blocks of
    # (n/4)^2), the 49 products of (n/4)^2 and 7 level-1 parents of (n/2)^2
    assert mf.mf_workspace_bytes(s, 2, 0, 8192) == 8 * (8 * 4096 ** 2 + 56 * 2048 ** 2 + 49 * 2048 ** 2
                                                         + 7 * 4096 ** 2)
    assert mf.mf_workspace_bytes(s, 2, 0, 8192) == expected_ws(8192, 2, 4, 4)
    # depth 3: 343 products of (n/8)^2, 49 level-2 parents of (n/4)^2 and 7 level-1 parents of (n/2)^2
    assert mf.mf_workspace_bytes(s, 3, 0, 8192) == 8 * (8 * 4096 ** 2 + 56 * 2048 ** 2 + 392 * 1024 ** 2
                                                         + 343 * 1024 ** 2 + 49 * 2048 ** 2 + 7 * 4096 ** 2)
    assert mf.mf_workspace_bytes(s, 3, 0, 8192) == expected_ws(8192, 3, 4, 4)
    # ragged: n = 1000, leaf size rounded up to 16 (500 -> 512)
    assert mf.mf_workspace_bytes(s, 1, 0, 1000) == expected_ws(1000, 1, 4, 4)
    assert mf.mf_workspace_bytes(s, 2, 0, 1000) == expected_ws(1000, 2, 4, 4)
    # classical (depth 0 or cutoff >= n) needs no workspace
    assert mf.mf_workspace_bytes(s, 0, 0, 8192) == 0
    assert mf.mf_workspace_bytes(s, 2, 8192, 8192) == 0
    # classical <3,3,3;27>: every column is a single block, no pre-addition;
    # 484 tile positions < 1024, so each product is its own group
    c3 = mf.mf_workspace_bytes(mf.mf_algo_builtin("classical3"), 1, 0, 8192)
    assert c3 == expected_ws(8192, 1, 0, 0, R=27, p=3) == 27 * 2736 ** 2 * 8
    # Winograd: also 4 materialised columns in U and in V
    w = mf.mf_algo_builtin("winograd")
    assert mf.mf_workspace_bytes(w, 1, 0, 4096) == expected_ws(4096, 1, 4, 4)
    assert mf.mf_workspace_bytes(w, 3, 0, 4096) == expected_ws(4096, 3, 4, 4)
    # Strassen 1969: 5 materialised columns in U and in V
    s69 = mf.mf_algo_builtin("strassen1969")
    assert mf.mf_workspace_bytes(s69, 2, 0, 8192) == expected_ws(8192, 2, 5, 5)
    # FP32 storage halves every byte count
    assert mf.mf_workspace_bytes(s, 2, 0, 8192, mf.MF_F32) * 2 == expected_ws(8192, 2, 4, 4)


def test_workspace_bytes_paper_size_24012():
    # The paper's largest size (Section 3.2): 24012^2 doubles ~ 4.6 GB per
    # matrix.  This executor materialises 4 + 4 blocks and stores the 7
    # products at depth 1.
    s = mf.mf_algo_builtin("strassen")
    m = 16 * -(-12006 // 16)
    assert m == 12016
    assert mf.mf_workspace_bytes(s, 1, 0, 24012) == 8 * (8 + 7) * m * m


def _call_fastmm(algo, depth, cutoff, A, B, C, n, dtype):
    return mf.lib.mf_fastmm(algo.handle if algo else None, depth, cutoff, ctypes.c_void_p(A), ctypes.c_void_p(B),
                            ctypes.c_void_p(C), n, dtype, None)


def test_fastmm_argument_validation_without_device():
    s = mf.mf_algo_builtin("strassen")
    A, B, C = 0x100000, 0x200000, 0x300000
    n = 16
    assert _call_fastmm(None, 1, 0, A, B, C, n, mf.MF_F64) == mf.MF_ERR_ARG
    assert _call_fastmm(s, -1, 0, A, B, C, n, mf.MF_F64) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, -1, A, B, C, n, mf.MF_F64) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, 0, A, B, C, -1, mf.MF_F64) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, 0, A, B, C, n, 7) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, 0, A, B, C, n, mf.MF_F64 | (9 << 8)) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, 0, A, B, C, n, mf.MF_F64 | mf.MF_LEAF_BF16) == mf.MF_ERR_UNSUPPORTED
    assert _call_fastmm(s, 1, 0, 0, B, C, n, mf.MF_F64) == mf.MF_ERR_ARG
    assert _call_fastmm(s, 1, 0, A, B, A + 8, n, mf.MF_F64) == mf.MF_ERR_ARG      # C overlaps A
    assert _call_fastmm(s, 1, 0, A, B, B - 8, n, mf.MF_F64) == mf.MF_ERR_ARG      # C overlaps B
    assert _call_fastmm(s, 1, 0, A + 4, B, C, n, mf.MF_F64) == mf.MF_ERR_ARG      # misaligned
    assert _call_fastmm(s, 1, 0, A, B, C, (1 << 20) + 1, mf.MF_F64) == mf.MF_ERR_SHAPE
    assert "overlap" in mf.mf_last_error() or mf.mf_last_error() != ""
    # n == 0 is a no-op and needs no pointers
    assert _call_fastmm(s, 1, 0, 0, 0, 0, 0, mf.MF_F64) == mf.MF_OK
    assert mf.lib.mf_classical_mm(None, None, None, 0, mf.MF_F64, None) == mf.MF_OK


def test_fastmm_ws_validation_without_device():
    # The caller's workspace is checked for size, alignment and overlap with
    # A, B and C before anything is enqueued (the addresses are never read).
    s = mf.mf_algo_builtin("strassen")
    n = 256
    need = mf.mf_workspace_bytes(s, 1, 0, n)
    mat = n * n * 8
    A, B, C, W = 0x1000000, 0x2000000, 0x3000000, 0x4000000

    def call(ws, nbytes):
        return mf.lib.mf_fastmm_ws(s.handle, 1, 0, ctypes.c_void_p(A), ctypes.c_void_p(B), ctypes.c_void_p(C), n,
                                   mf.MF_F64, ctypes.c_void_p(ws), nbytes, None)

    assert call(0, need) == mf.MF_ERR_ARG                     # NULL workspace
    assert call(W, need - 1) == mf.MF_ERR_SHAPE               # too small
    assert call(W + 128, need) == mf.MF_ERR_ARG               # not 256-byte aligned
    assert call(A + mat - 256, need) == mf.MF_ERR_ARG         # starts inside A
    assert "overlaps" in mf.mf_last_error()
    assert call(B - need + 256, need) == mf.MF_ERR_ARG        # ends inside B
    assert call(C - 256 * 1024, need + 256 * 1024) == mf.MF_ERR_ARG  # covers C


def test_unsupported_algorithm_shape_is_reported():
    # split factor 5 (25 inputs per block combination) has no compiled kernel
    c5 = oa.classical_algo(5)
    a = mf.mf_algo_from_uvw(5, c5.U, c5.V, c5.W, mf.MF_W_ROWMAJOR_C)
    with pytest.raises(mf.MFError) as e:
        mf.mf_workspace_bytes(a, 1, 0, 1000)
    assert e.value.status == mf.MF_ERR_UNSUPPORTED
    assert mf.mf_workspace_bytes(a, 0, 0, 1000) == 0  # classical still works


def test_deep_recursion_plans():
    s = mf.mf_algo_builtin("strassen")
    assert mf.mf_workspace_bytes(s, 4, 0, 8192) == expected_ws(8192, 4, 4, 4)
    # depth beyond what the size allows stops once a level reaches the tile
    assert mf.mf_workspace_bytes(s, 10, 0, 256) == expected_ws(256, 1, 4, 4) == 8 * (8 + 7) * 128 ** 2
    assert mf.mf_workspace_bytes(s, 10, 0, 4096) == expected_ws(4096, 5, 4, 4)


def _tune(nsizes, n, dtype, algos, max_depth, work=1e9, copies=4, reps=1):
    k = max(1, nsizes)
    n_arr = (ctypes.c_int64 * k)(*(list(n) + [1] * (k - len(n))))
    a_arr = (ctypes.c_void_p * max(1, len(algos)))(*[a.handle.value if a else None for a in algos])
    choice = (ctypes.c_int * k)()
    ms = (ctypes.c_double * (k * (1 + len(algos) * max(0, max_depth)) + 1))()
    return mf.lib.mf_autotune_batch(nsizes, n_arr, dtype, a_arr, len(algos), max_depth, work, copies, reps, None,
                                    choice, ms)


def test_autotune_argument_validation_without_device():
    s = mf.mf_algo_builtin("winograd")
    assert _tune(0, [256], mf.MF_F64, [s], 2) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64 | mf.MF_LEAF_BF16, [s], 2) == mf.MF_ERR_UNSUPPORTED
    assert _tune(1, [256], 7, [s], 2) == mf.MF_ERR_UNSUPPORTED
    assert _tune(1, [0], mf.MF_F64, [s], 2) == mf.MF_ERR_SHAPE
    assert _tune(1, [(1 << 16) + 1], mf.MF_F64, [s], 2) == mf.MF_ERR_SHAPE
    assert _tune(1, [256], mf.MF_F64, [s], -1) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64, [s], 9) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64, [None], 2) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64, [s], 2, work=0.0) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64, [s], 2, copies=0) == mf.MF_ERR_ARG
    assert _tune(1, [256], mf.MF_F64, [s], 2, reps=0) == mf.MF_ERR_ARG


def test_plan_query_closed_forms():
    """Algorithmic bytes and flops of the plan against closed forms (Winograd
    form: 4 materialised T and 4 materialised S per level)."""
    w = mf.mf_algo_builtin("winograd")
    n = 8192
    for d in (1, 2, 3):
        q = mf.mf_plan_query(w, d, 0, n)
        assert q["levels"] == d and q["products"] == 7 ** d and q["leaf_m"] == n >> d
        assert q["gemm_flops"] == 7 ** d * 2.0 * (n >> d) ** 3
        # level l, per operand: its 7^l blocks of size n / 2^l are read once and
        # the 4 materialised children of each are written
        pre = sum(2 * 8 * 7 ** lv * ((n >> lv) ** 2 + 4 * (n >> (lv + 1)) ** 2) for lv in range(d))
        assert q["pre_bytes"] == pre
        assert q["ws_bytes"] == mf.mf_workspace_bytes(w, d, 0, n)
        # outer post-additions: level l reads R children and writes p^2 quarters of 7^l parents
        lo = q["levels_outer"]
        post = sum(8 * 7 ** lv * (7 + 4) * (n >> (lv + 1)) ** 2 for lv in range(lo))
        assert q["post_bytes"] == post
    c = mf.mf_plan_query(None, 0, 0, 1000)
    assert c["levels"] == 0 and c["products"] == 1 and c["leaf_m"] == 1008 and c["pre_bytes"] == 0
    # virtual padding: the inputs count only their valid elements (n = 1000: quarters of 500 x 500), while a
    # materialised child is a whole 512 x 512 workspace block, zeros included, as the leaf GEMM reads it
    q = mf.mf_plan_query(w, 1, 0, 1000)
    assert q["leaf_m"] == 512 and q["pre_bytes"] == 2 * 8 * (1000 * 1000 + 4 * 512 * 512)
    # padded leaves: leaf sizes in steps of 16 (FP64 / FP32 leaves) or whole
    # 128 tiles (BF16 leaves); executed work over whole 128 tiles in rows and
    # columns, the valid inner size (rounded up to 16) in K for FP64 / FP32
    # leaves, the padded K for BF16 ones
    q = mf.mf_plan_query(None, 0, 0, 1040)
    assert q["leaf_m"] == 1040 and q["gemm_flops"] == 2.0 * 1152 * 1152 * 1040
    q = mf.mf_plan_query(None, 0, 0, 1037)
    assert q["leaf_m"] == 1040 and q["gemm_flops"] == 2.0 * 1152 * 1152 * 1040
    q = mf.mf_plan_query(None, 0, 0, 1040, mf.MF_F32 | mf.MF_LEAF_BF16)
    assert q["leaf_m"] == 1152 and q["gemm_flops"] == 2.0 * 1152 ** 3
    # Winograd depth 1 at n = 1040: leaf 528, blocks split at 528, so A12 and A22
    # have 512 valid columns and B21 and B22 512 valid rows.  M1 = A12 B21,
    # M2 = (..) B22 and M3 = A22 (..) run K = 512; M0 = A11 B11 and the three
    # products of two materialised (whole 528 x 528) blocks run K = 528, each
    # over 5 x 5 tiles.
    q = mf.mf_plan_query(w, 1, 0, 1040)
    assert q["leaf_m"] == 528 and q["gemm_flops"] == 2.0 * 640 * 640 * (4 * 528 + 3 * 512)


def test_workspace_bytes_bf16_staging():
    """BF16 leaves stage every leaf operand once as BF16 planes (2 planes for
    split-BF16x3): A operands and transposed B operands, m x m each, placed
    after the FP32 workspace (256-byte aligned).  The last pre-addition level
    is fused into the staging, so its sums take no FP32 workspace: Strassen at
    depth 1 keeps only the 7 stored products (the FP32 leaves also hold the 4
    + 4 materialised operand sums)."""
    s = mf.mf_algo_builtin("strassen")
    m2 = 4096 ** 2
    assert mf.mf_workspace_bytes(s, 1, 0, 8192, mf.MF_F32) == (8 + 7) * m2 * 4
    for leaf, planes in ((mf.MF_LEAF_BF16, 1), (mf.MF_LEAF_BF16X3, 2)):
        assert mf.mf_workspace_bytes(s, 1, 0, 8192, mf.MF_F32 | leaf) == 7 * m2 * 4 + 2 * 7 * planes * m2 * 2
        # depth 2: the 8 level-1 sums (4096^2) are stored, level 2 is fused; 49 stored products (2048^2) and
        # the 7 level-1 results of the post-addition (4096^2)
        assert mf.mf_workspace_bytes(s, 2, 0, 8192, mf.MF_F32 | leaf) == \
            (8 * m2 + 49 * m2 // 4 + 7 * m2) * 4 + 2 * 49 * planes * (m2 // 4) * 2
        # classical: one product, a 1000 x 1000 problem in a 1024 leaf
        assert mf.mf_workspace_bytes(s, 0, 0, 1000, mf.MF_F32 | leaf) == 2 * planes * 1024 ** 2 * 2
    assert mf.mf_workspace_bytes(s, 0, 0, 1000, mf.MF_F32 | mf.MF_LEAF_F32) == 0


def test_kron3_plan_closed_form():
    """Depth 3 Kronecker-fused (<8,8,8;343>, three factors of Winograd) is one
    level: 343 products of n/8, pre-addition bytes 2 * 8 * (n^2 + (7^3 - 3^3) m^2)
    (every quarter of A and B read once, the 316 non-aliased operands written
    once), post-addition 8 * (343 m^2 + n^2), workspace (2 * 316 + 343) m^2 * 8."""
    w = mf.mf_algo_builtin("winograd")
    c8 = mf.mf_algo_compose(mf.mf_algo_compose(w, w), w)
    n, m = 8192, 1024
    q = mf.mf_plan_query(c8, 1, 0, n, mf.MF_F64)
    assert q["levels"] == 1 and q["products"] == 343 and q["leaf_m"] == m
    assert q["pre_stages"] == 1 and q["post_stages"] == 1
    assert q["pre_bytes"] == 2 * 8 * (n * n + 316 * m * m)
    assert q["post_bytes"] == 8 * (343 * m * m + n * n)
    assert mf.mf_workspace_bytes(c8, 1, 0, n) == (2 * 316 + 343) * m * m * 8
    assert mf.mf_workspace_bytes(c8, 1, 0, 4096, mf.MF_F32) == (2 * 316 + 343) * 512 * 512 * 4


@pytest.mark.parametrize("n", [1000, 1001, 1024, 8000])
def test_kron3_plan_closed_form_ragged(n):
    """Sizes that 8 x the 16 leaf step does not divide: the leaf is padded to
    m = 16 * ceil(ceil(n / 8) / 16).  Input views exclude the virtual padding,
    so the quarters of A and B still total n^2 elements read; workspace blocks
    are written whole (m^2 each, zeros in the padding); C is written over its
    n^2 valid elements."""
    w = mf.mf_algo_builtin("winograd")
    c8 = mf.mf_algo_compose(mf.mf_algo_compose(w, w), w)
    m = 16 * -(-(-(-n // 8)) // 16)
    for dtype, eb in ((mf.MF_F64, 8), (mf.MF_F32, 4)):
        # rows of A and B not 16-byte aligned (n = 1001): the 27 aliased
        # operands per side are copied too, so all 343 are stored
        stored = 343 if (n * eb) % 16 else 316
        q = mf.mf_plan_query(c8, 1, 0, n, dtype)
        assert q["leaf_m"] == m and q["products"] == 343
        assert q["pre_bytes"] == 2 * eb * (n * n + stored * m * m)
        assert q["post_bytes"] == eb * (343 * m * m + n * n)
        assert mf.mf_workspace_bytes(c8, 1, 0, n, dtype) == (2 * stored + 343) * m * m * eb


def test_unaligned_rows_copy_aliased_views_at_the_first_level():
    """Rows of A and B that are not 16-byte aligned (odd n in FP64, n not a
    multiple of 4 in FP32): the first level copies its aliased quarters into
    workspace blocks (Winograd: 3 per side besides the 4 combinations), so
    every leaf operand has aligned rows; deeper levels and aligned requests
    alias as before."""
    w = mf.mf_algo_builtin("winograd")
    m = 512  # ceil(1001 / 2) = 501 rounded up to 16
    q = mf.mf_plan_query(w, 1, 0, 1001)  # 8008-byte rows
    assert q["leaf_m"] == m and q["pre_bytes"] == 2 * 8 * (1001 * 1001 + 7 * m * m)
    assert mf.mf_workspace_bytes(w, 1, 0, 1001) == 8 * (7 + 7 + 7) * m * m
    q = mf.mf_plan_query(w, 1, 0, 1002)  # 8016-byte rows: aligned
    assert q["pre_bytes"] == 2 * 8 * (1002 * 1002 + 4 * m * m)
    assert mf.mf_workspace_bytes(w, 1, 0, 1002) == 8 * (4 + 4 + 7) * m * m
    q = mf.mf_plan_query(w, 1, 0, 1002, mf.MF_F32)  # 4008-byte rows: not aligned in FP32
    assert q["pre_bytes"] == 2 * 4 * (1002 * 1002 + 7 * m * m)
    # depth 2: level 2 splits workspace blocks only, so it aliases as before
    q1 = mf.mf_plan_query(w, 2, 0, 2001)
    q0 = mf.mf_plan_query(w, 2, 0, 2002)
    m2 = 16 * -(-(-(-2001 // 4)) // 16)
    assert q1["leaf_m"] == q0["leaf_m"] == m2
    # three more first-level blocks per side; the second level is unchanged
    assert (mf.mf_workspace_bytes(w, 2, 0, 2001) - mf.mf_workspace_bytes(w, 2, 0, 2002)
            == 8 * 2 * 3 * (2 * m2) ** 2)


def test_classical_copies_unaligned_rows_past_the_threshold():
    """A classical product over rows that are not 16-byte aligned copies both
    operands once into square blocks of n rounded up to 16 (one pre-addition
    stage of one-term combinations: the valid n x n read, the whole block
    written), from n = 192 on; aligned rows and smaller sizes copy nothing."""
    cases = [  # (n, dtype, copied)
        (1037, mf.MF_F64, True), (1040, mf.MF_F64, False), (193, mf.MF_F64, True), (191, mf.MF_F64, False),
        (129, mf.MF_F64, False), (1038, mf.MF_F32, True), (1036, mf.MF_F32, False), (1037, mf.MF_F32, True),
    ]
    w = mf.mf_algo_builtin("winograd")
    for n, dtype, copied in cases:
        eb = 8 if dtype == mf.MF_F64 else 4
        b = 16 * -(-n // 16)
        q = mf.mf_plan_query(None, 0, 0, n, dtype)
        assert q["levels"] == 0 and q["products"] == 1, (n, dtype)
        assert q["pre_stages"] == (1 if copied else 0), (n, dtype)
        assert q["pre_bytes"] == (2 * eb * (n * n + b * b) if copied else 0), (n, dtype)
        assert q["ws_bytes"] == mf.mf_workspace_bytes(w, 0, 0, n, dtype) == (2 * eb * b * b if copied else 0)
        # the copies hold zeros past the views, so the product runs the padded K in whole steps
        assert q["gemm_flops"] == 2.0 * (128 * -(-n // 128)) ** 2 * b, (n, dtype)


@pytest.mark.parametrize("table", ["WINOGRAD", "STRASSEN_PAPER", "STRASSEN_1969"])
def test_kron3_stored_operands_match_oracle_aliases(table):
    """The library stores every operand of <8,8,8;343> except the aliased
    ones (a single nonzero coefficient: a block view whose coefficient goes
    into the epilogue), so its pre-addition writes are (343 - aliased) m^2 per
    side.  Both sides build the cube from the same printed factor table; the
    aliased count comes from the oracle's own composition."""
    U, V, W, conv = mi.as_float_tables(getattr(mi, table))
    f = mf.mf_algo_from_uvw(2, U, V, W, conv)
    c8 = mf.mf_algo_compose(mf.mf_algo_compose(f, f), f)
    cube = oa.power(oa.canonical(2, U, V, W, conv), 3)
    aliased_u = len(oa.single_coefficient_columns(cube.U))
    aliased_v = len(oa.single_coefficient_columns(cube.V))
    assert (aliased_u, aliased_v) == ((8, 8) if table == "STRASSEN_1969" else (27, 27))
    stored = (343 - aliased_u) + (343 - aliased_v)
    n, m = 4096, 512
    q = mf.mf_plan_query(c8, 1, 0, n, mf.MF_F64)
    assert q["pre_bytes"] == 8 * (2 * n * n + stored * m * m)


def test_kron3_unsupported_forms():
    """<8,8,8;343> is not staged for BF16 leaves (at most 16 inputs per staging
    set): the plan reports MF_ERR_UNSUPPORTED instead of running."""
    w = mf.mf_algo_builtin("winograd")
    c8 = mf.mf_algo_compose(mf.mf_algo_compose(w, w), w)
    for leaf in (mf.MF_LEAF_BF16, mf.MF_LEAF_BF16X3):
        with pytest.raises(Exception) as ei:
            mf.mf_workspace_bytes(c8, 1, 0, 4096, mf.MF_F32 | leaf)
        assert "UNSUPPORTED" in str(ei.value)


def test_composition_is_associative():
    """(F1 x F2) x F3 and F1 x (F2 x F3) are the same <8,8,8;343> algorithm (the
    block re-indexing of the Kronecker construction is mixed-radix), and it
    satisfies the Brent equations (checked when the library builds it)."""
    w = mf.mf_algo_builtin("winograd")
    s = mf.mf_algo_builtin("strassen")
    left = mf.mf_algo_compose(mf.mf_algo_compose(w, s), w)
    right = mf.mf_algo_compose(w, mf.mf_algo_compose(s, w))
    for x, y in zip(left.uvw(), right.uvw()):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    U, V, W = left.uvw()[:3]
    again = mf.mf_algo_from_uvw(8, np.asarray(U), np.asarray(V), np.asarray(W))
    assert again.info()["R"] == 343


# ------------------------------------------------- split factors 2 and 3
# <6,6,6;189>: the paper's Strassen composed with the classical <3,3,3;27>
# in either order (Section 2: factor 6 = 2 x 3 or 3 x 2, and the order changes
# the temporary space and the error).  No kernel combines 36 blocks into 189
# products and back, so the planner runs the composition as its two factors,
# one level each, outer factor first.

def test_mixed_factor_composition_brent_and_shape():
    s = mf.mf_algo_builtin("strassen")
    c3 = mf.mf_algo_builtin("classical3")
    for outer, inner in ((s, c3), (c3, s)):
        a = mf.mf_algo_compose(outer, inner)
        assert a.info()["n0"] == 6 and a.info()["R"] == 189
        q = mf.mf_plan_query(a, 1, 0, 2048)
        assert q["levels"] == 2 and q["products"] == 189
        # leaf: ceil(2048 / 6) = 342 rounded up to the leaf step of 16
        assert q["leaf_m"] == 352


def test_mixed_factor_workspace_by_order():
    """Workspace of the two orders at n = 2048 (m = 352, n' = 6 m), in m^2
    elements: Strassen first materialises 4 + 4 blocks of (3m)^2 at level 1
    (the classical level aliases every block), stores 189 products and 7
    level-1 parents of (3m)^2: 72 + 189 + 63 = 324.  Classical first aliases
    level 1 and materialises 27 x (4 + 4) blocks of m^2 at level 2, stores 189
    products and 27 parents of (2m)^2: 216 + 189 + 108 = 513."""
    s = mf.mf_algo_builtin("strassen")
    c3 = mf.mf_algo_builtin("classical3")
    m = 352
    assert mf.mf_workspace_bytes(mf.mf_algo_compose(s, c3), 1, 0, 2048) == 8 * 324 * m * m
    assert mf.mf_workspace_bytes(mf.mf_algo_compose(c3, s), 1, 0, 2048) == 8 * 513 * m * m


def test_mixed_factor_matches_oracle_composition():
    s = mf.mf_algo_builtin("strassen")
    c3 = mf.mf_algo_builtin("classical3")
    o_s = oracle_table(mi.STRASSEN_PAPER)
    o_c3 = oa.classical_algo(3)
    for (outer, inner), (o_out, o_in) in (((s, c3), (o_s, o_c3)), ((c3, s), (o_c3, o_s))):
        assert same(mf.mf_algo_compose(outer, inner), oa.compose(o_out, o_in))


def test_batch_form_argument_checked_on_host():
    """The persistent form takes only the narrow combinations, and an unknown
    form is rejected; both at planning time, without a device."""
    w = mf.mf_algo_builtin("winograd")
    w2 = mf.mf_algo_compose(w, w)
    b = mf.mf_batch_create([256, 512], [w, w], [1, 2], [0, 0], mf.MF_F64, form=mf.MF_BATCH_PERSISTENT)
    assert b.workspace_bytes() > 0
    with pytest.raises(mf.MFError) as ei:
        mf.mf_batch_create([1024], [w2], [1], [0], mf.MF_F64, form=mf.MF_BATCH_PERSISTENT)
    assert ei.value.status == mf.MF_ERR_UNSUPPORTED
    # the phase form takes the wide <4,4,4;49> post-addition
    mf.mf_batch_create([1024], [w2], [1], [0], mf.MF_F64)
    with pytest.raises(mf.MFError) as ei:
        mf.mf_batch_create([256], [w], [1], [0], mf.MF_F64, form=7)
    assert ei.value.status == mf.MF_ERR_ARG


def test_noalloc_rejects_beyond_scratch_on_host():
    """A request whose workspace exceeds the fixed scratch array is rejected
    before anything touches a device (pointers are never dereferenced)."""
    w = mf.mf_algo_builtin("winograd")
    n = 4096
    assert mf.mf_workspace_bytes(w, 1, 0, n) > (256 << 20)
    A, B, C = 1 << 20, 2 << 40, 3 << 40
    st = mf.lib.mf_fastmm_noalloc(w.handle, 1, 0, ctypes.c_void_p(A), ctypes.c_void_p(B), ctypes.c_void_p(C), n,
                                  mf.MF_F64, None)
    assert st == mf.MF_ERR_SHAPE
    assert "scratch" in mf.lib.mf_last_error().decode()
