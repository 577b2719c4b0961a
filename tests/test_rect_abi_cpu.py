"""CPU-only checks of the rectangular part of the C ABI: the library's own
algebra (classical <m0,k0,n0>, direct sums, Kronecker products, Brent check)
against the oracle coefficient by coefficient, the planner's level rule for
rectangular shapes, and mf_gemm's argument checks (all before any device
use)."""
import ctypes

import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import rect as orc

mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def ostrassen():
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    return orc.from_square(oa.canonical(2, U, V, W, conv))


def same(h, o):
    U, V, W = h.uvw()
    return (h.shape() == (o.m0, o.k0, o.n0, o.R) and np.array_equal(U, o.U) and np.array_equal(V, o.V)
            and np.array_equal(W, o.W))


def lib_pieces():
    s = mf.mf_algo_builtin("strassen")
    hk = mf.mf_algo_concat(s, mf.mf_algo_classical(2, 2, 1), "n")          # <2,2,3;11>
    r233 = mf.mf_algo_concat(hk, mf.mf_algo_classical(2, 1, 3), "k")       # <2,3,3;17>
    r322 = mf.mf_algo_concat(s, mf.mf_algo_classical(1, 2, 2), "m")        # <3,2,2;11>
    return s, hk, r233, r322


def oracle_pieces():
    s = ostrassen()
    hk = orc.concat(s, orc.classical(2, 2, 1), "n")
    r233 = orc.concat(hk, orc.classical(2, 1, 3), "k")
    r322 = orc.concat(s, orc.classical(1, 2, 2), "m")
    return s, hk, r233, r322


@pytest.mark.parametrize("shape", [(2, 3, 2), (1, 2, 3), (3, 3, 1), (2, 2, 2)])
def test_classical_matches_oracle(shape):
    assert same(mf.mf_algo_classical(*shape), orc.classical(*shape))


def test_direct_sums_and_products_match_oracle():
    lib, ora = lib_pieces(), oracle_pieces()
    for h, o in zip(lib[1:], ora[1:]):
        assert same(h, o)
    assert same(mf.mf_algo_compose(lib[2], lib[3]), orc.compose(ora[2], ora[3]))
    assert same(mf.mf_algo_compose(lib[3], lib[2]), orc.compose(ora[3], ora[2]))
    assert mf.mf_algo_compose(lib[2], lib[3]).shape() == (6, 6, 6, 187)


def test_brent_check_rejects_planted_change():
    o = oracle_pieces()[1]
    U = o.U.astype(np.float64)
    mf.mf_algo_from_uvw_rect(2, 2, 3, U, o.V, o.W)
    U[3, 9] += 1
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_from_uvw_rect(2, 2, 3, U, o.V, o.W)
    assert e.value.status == mf.MF_ERR_BRENT


def test_concat_shape_mismatch_and_rebase_rejected():
    s = mf.mf_algo_builtin("strassen")
    with pytest.raises(mf.MFError):
        mf.mf_algo_concat(s, mf.mf_algo_classical(1, 2, 2), "n")  # rows differ
    hk = mf.mf_algo_concat(s, mf.mf_algo_classical(2, 2, 1), "n")
    I = np.eye(2, dtype=np.int64)
    with pytest.raises(mf.MFError) as e:
        mf.mf_algo_rebase(hk, I, I, I)
    assert e.value.status == mf.MF_ERR_UNSUPPORTED


def test_rectangular_algorithm_on_square_plan_levels():
    _, hk, r233, r322 = lib_pieces()
    # <2,2,3;11> on n = 1000: 1000 -> 500 / 500 / 334 -> 250 / 250 / 112; the
    # next level would cut N below the 128 leaf tile
    assert mf.mf_plan_query(hk, 3, 0, 1000)["levels"] == 2
    six = mf.mf_algo_compose(r233, r322)
    q = mf.mf_plan_query(six, 1, 0, 1536)
    assert q["levels"] == 2 and q["products"] == 187  # runs as its two factors


def gemm_status(**kw):
    a = dict(algo=None, depth=0, cutoff=0, M=256, N=256, K=256, alpha=1.0, A=1 << 20, lda=256, B=1 << 30,
             ldb=256, beta=0.0, C=1 << 40, ldc=256, dtype=mf.MF_F64)
    a.update(kw)
    st = mf.lib.mf_gemm(a["algo"], a["depth"], a["cutoff"], a["M"], a["N"], a["K"], a["alpha"],
                        ctypes.c_void_p(a["A"]), a["lda"], ctypes.c_void_p(a["B"]), a["ldb"], a["beta"],
                        ctypes.c_void_p(a["C"]), a["ldc"], a["dtype"], None)
    return st, mf.lib.mf_last_error().decode()


def test_gemm_argument_checks_before_device_use():
    assert gemm_status(M=0)[0] == mf.MF_OK
    assert gemm_status(N=0)[0] == mf.MF_OK
    assert gemm_status(K=0)[0] == mf.MF_ERR_SHAPE
    assert gemm_status(lda=100)[0] == mf.MF_ERR_ARG
    assert gemm_status(ldc=100)[0] == mf.MF_ERR_ARG
    assert gemm_status(C=(1 << 20) + 8)[0] == mf.MF_ERR_ARG  # C overlaps A
    assert gemm_status(depth=1)[0] == mf.MF_ERR_ARG          # no algorithm
    assert gemm_status(dtype=mf.MF_F32 | mf.MF_LEAF_BF16)[0] == mf.MF_ERR_UNSUPPORTED
    assert gemm_status(alpha=float("nan"))[0] == mf.MF_ERR_ARG
    assert gemm_status(A=(1 << 20) + 4)[0] == mf.MF_ERR_ARG  # misaligned
    # operand tiles are addressed with 32-bit byte offsets: lda, ldb <= 2^21
    assert gemm_status(lda=(1 << 21) + 1)[0] == mf.MF_ERR_SHAPE
    assert gemm_status(ldb=(1 << 21) + 1)[0] == mf.MF_ERR_SHAPE
