"""GPU parity of the FP64 path against the CPU oracle, through the C ABI.

Integer-valued inputs must give bit-exact results (every intermediate is an
integer below 2^53); uniform[-1,1] inputs must stay within the normwise
relative error bound 1e-11 (depth <= 3, n <= 8192)."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")

FP64_TOL = 1e-11


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def run_fast(algo, depth, cutoff, A, B):
    dA, dB = dev(A), dev(B)
    dC = torch.full_like(dA, float("nan"))
    mf.mf_fastmm(algo, depth, cutoff, dA, dB, dC)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def run_classical(A, B):
    dA, dB = dev(A), dev(B)
    dC = torch.full_like(dA, float("nan"))
    mf.mf_classical_mm(dA, dB, dC)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def oracle_algo(name):
    table = {"strassen": mi.STRASSEN_PAPER, "winograd": mi.WINOGRAD, "strassen1969": mi.STRASSEN_1969}[name]
    U, V, W, conv = mi.as_float_tables(table)
    return oa.canonical(2, U, V, W, conv)


@pytest.fixture(scope="module", autouse=True)
def _announce():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


# ------------------------------------------------------------------ classical

@pytest.mark.parametrize("n", [1, 2, 64, 127, 128, 129, 256, 300, 1000])
def test_classical_int_exact(n):
    A = mi.int_uniform(n, 3)
    B = mi.int_uniform(n, 4)
    got = run_classical(A.astype(np.float64), B.astype(np.float64))
    assert np.array_equal(got, om.classical_mm(A, B).astype(np.float64))


@pytest.mark.parametrize("n", [256, 1024, 1536])
def test_classical_fp64_close(n):
    A = mi.uniform(n, 1)
    B = mi.uniform(n, 2)
    err = om.rel_fro_error(run_classical(A, B), om.classical_mm(A, B))
    assert err < 1e-14


# ------------------------------------------------------- fast, bit-exact ints

def levels_taken(algo, depth, n):
    return mf.mf_plan_query(algo, depth, 0, n)["levels"]


# levels the planner takes: a level needs the current size above the 128 leaf
# tile, so n = 256 takes one level at any depth, n = 300 two (300 -> 150 -> 75)
# and n >= 1024 all three
EXPECTED_LEVELS = {256: 1, 300: 2, 1024: 3, 1025: 3, 1500: 3}


@pytest.mark.parametrize("name", ["strassen", "winograd", "strassen1969"])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("n", [256, 300, 1024, 1025, 1500])
def test_fast_int_exact(name, depth, n):
    A = mi.int_uniform(n, 3)
    B = mi.int_uniform(n, 4)
    algo = mf.mf_algo_builtin(name)
    assert levels_taken(algo, depth, n) == min(depth, EXPECTED_LEVELS[n])
    got = run_fast(algo, depth, 0, A.astype(np.float64), B.astype(np.float64))
    want = om.classical_mm(A, B)
    # the oracle's own fast executor reaches the same integers
    if n <= 300:
        assert np.array_equal(om.fast_mm(A, B, oracle_algo(name), depth), want)
    assert np.array_equal(got, want.astype(np.float64))


def test_paper_config_n256_depth1():
    """n = 256, Strassen as printed in the paper, one level."""
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    algo = mf.mf_algo_from_uvw(2, U, V, W, conv)
    Ai = mi.int_uniform(256, 3)
    Bi = mi.int_uniform(256, 4)
    got = run_fast(algo, 1, 0, Ai.astype(np.float64), Bi.astype(np.float64))
    assert np.array_equal(got, om.fast_mm(Ai, Bi, oracle_algo("strassen"), 1).astype(np.float64))
    A = mi.uniform(256, 1)
    B = mi.uniform(256, 2)
    err = om.rel_fro_error(run_fast(algo, 1, 0, A, B), om.classical_mm(A, B))
    assert err < FP64_TOL


@pytest.mark.parametrize("seed", [7, 8])
def test_rebased_int_exact(seed):
    X, Y, Z = (mi.unimodular(2, seed * 10 + t) for t in range(3))
    algo = mf.mf_algo_rebase(mf.mf_algo_builtin("strassen"), X, Y, Z)
    A = mi.int_uniform(512, 5)
    B = mi.int_uniform(512, 6)
    for depth in (1, 2):
        got = run_fast(algo, depth, 0, A.astype(np.float64), B.astype(np.float64))
        assert np.array_equal(got, (A @ B).astype(np.float64))


def test_classical_333_control_exact():
    algo = mf.mf_algo_builtin("classical3")
    for n in (384, 500):
        A = mi.int_uniform(n, 7)
        B = mi.int_uniform(n, 8)
        got = run_fast(algo, 1, 0, A.astype(np.float64), B.astype(np.float64))
        assert np.array_equal(got, (A @ B).astype(np.float64))


def test_composed_444_49_matches_depth2():
    """<4,4,4;49> = Strassen-Winograd composed with itself, run as one level
    of split factor 4, and the same algorithm as two levels: identical
    integers, FP64 results within the bound (their summation orders differ:
    one 16-input combination versus two levels of 4-input combinations)."""
    s = mf.mf_algo_builtin("winograd")
    s2 = mf.mf_algo_compose(s, s)
    assert s2.info()["R"] == 49 and s2.info()["n0"] == 4
    Ai = mi.int_uniform(1024, 11).astype(np.float64)
    Bi = mi.int_uniform(1024, 12).astype(np.float64)
    assert np.array_equal(run_fast(s2, 1, 0, Ai, Bi), Ai @ Bi)
    assert np.array_equal(run_fast(s, 2, 0, Ai, Bi), Ai @ Bi)
    A = mi.uniform(1024, 11)
    B = mi.uniform(1024, 12)
    ref = om.classical_mm(A, B)
    assert om.rel_fro_error(run_fast(s2, 1, 0, A, B), ref) < FP64_TOL
    assert om.rel_fro_error(run_fast(s, 2, 0, A, B), ref) < FP64_TOL


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 129, 255])
def test_tiny_sizes_take_at_most_one_level_and_stay_exact(n):
    """Requests for depth 1-3 at sizes up to 255: n <= 128 runs the classical
    GEMM (no level is taken), 129 and 255 one level; all exact."""
    A = mi.int_uniform(n, 13)
    B = mi.int_uniform(n, 14)
    algo = mf.mf_algo_builtin("strassen")
    for depth in (1, 2, 3):
        assert levels_taken(algo, depth, n) == (0 if n <= 128 else 1)
        got = run_fast(algo, depth, 0, A.astype(np.float64), B.astype(np.float64))
        assert np.array_equal(got, (A @ B).astype(np.float64)), (n, depth)


@pytest.mark.parametrize("n", [1025, 1500, 2047])
def test_three_levels_on_ragged_sizes_exact(n):
    """Depth 3 really taken (three levels of virtual padding) at ragged n."""
    A = mi.int_uniform(n, 15)
    B = mi.int_uniform(n, 16)
    for name in ("strassen", "winograd"):
        algo = mf.mf_algo_builtin(name)
        assert levels_taken(algo, 3, n) == 3
        got = run_fast(algo, 3, 0, A.astype(np.float64), B.astype(np.float64))
        assert np.array_equal(got, (A @ B).astype(np.float64)), (name, n)


def test_cutoff_selects_levels():
    s = mf.mf_algo_builtin("strassen")
    A = mi.uniform(512, 1)
    B = mi.uniform(512, 2)
    # cutoff >= n: classical; it must equal the library's classical GEMM bitwise
    assert np.array_equal(run_fast(s, 3, 512, A, B), run_classical(A, B))
    # cutoff 256 with depth 3: one level only, equal to depth 1
    assert np.array_equal(run_fast(s, 3, 256, A, B), run_fast(s, 1, 0, A, B))


# ------------------------------------------------------------ FP64 accuracy

@pytest.mark.parametrize("name", ["strassen", "winograd"])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_fast_fp64_error_1024(name, depth):
    A = mi.uniform(1024, 10)
    B = mi.uniform(1024, 11)
    err = om.rel_fro_error(run_fast(mf.mf_algo_builtin(name), depth, 0, A, B), om.classical_mm(A, B))
    assert err < FP64_TOL


def test_determinism_and_workspace_variant():
    s = mf.mf_algo_builtin("strassen")
    A = dev(mi.uniform(1024, 21))
    B = dev(mi.uniform(1024, 22))
    C1 = torch.empty_like(A)
    C2 = torch.empty_like(A)
    C3 = torch.empty_like(A)
    mf.mf_fastmm(s, 2, 0, A, B, C1)
    mf.mf_fastmm(s, 2, 0, A, B, C2)
    nbytes = mf.mf_workspace_bytes(s, 2, 0, 1024)
    ws = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    mf.mf_fastmm_ws(s, 2, 0, A, B, C3, ws)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2) and torch.equal(C1, C3)


def test_workspace_too_small_rejected():
    s = mf.mf_algo_builtin("strassen")
    A = dev(mi.uniform(256, 1))
    B = dev(mi.uniform(256, 2))
    C = torch.empty_like(A)
    ws = torch.empty(16, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mf.MFError) as e:
        mf.mf_fastmm_ws(s, 1, 0, A, B, C, ws)
    assert e.value.status == mf.MF_ERR_SHAPE


# --------------------------------------------- full size, sampled rows

@pytest.mark.parametrize("n,name,depth", [(4096, "winograd", 1), (4096, "winograd", 3), (8192, "strassen", 1),
                                          (8192, "strassen", 2), (8192, "winograd", 3)])
def test_full_size_sampled_rows(n, name, depth):
    A = mi.uniform(n, 10)
    B = mi.uniform(n, 11)
    got = run_fast(mf.mf_algo_builtin(name), depth, 0, A, B)
    rows = np.sort(np.random.default_rng(5).choice(n, size=48, replace=False))
    ref = om.rows_reference(A, B, rows)
    err = om.rel_fro_error(got[rows], ref)
    assert err < FP64_TOL, err
    assert np.isfinite(got).all()


def test_bench_configuration_sampled():
    """The benchmarked configuration itself: n = 8192 FP64, Strassen-Winograd
    depth 2 run Kronecker-fused (one level of <4,4,4;49>), on the benchmark's
    inputs (uniform, seeds 10 and 11), and on integer inputs exactly; rows
    sampled, first and last included, and the same for the level-by-level
    schedule, whose result must agree within the bound."""
    n = 8192
    w = mf.mf_algo_builtin("winograd")
    fused = mf.mf_algo_compose(w, w)
    A = mi.uniform(n, 10)
    B = mi.uniform(n, 11)
    rows = np.unique(np.concatenate([np.random.default_rng(6).choice(n, size=40, replace=False), [0, n - 1]]))
    ref = om.rows_reference(A, B, rows)
    got_f = run_fast(fused, 1, 0, A, B)
    got_l = run_fast(w, 2, 0, A, B)
    assert om.rel_fro_error(got_f[rows], ref) < FP64_TOL
    assert om.rel_fro_error(got_l[rows], ref) < FP64_TOL
    assert om.rel_fro_error(got_f, got_l) < FP64_TOL
    Ai = mi.int_uniform(n, 12).astype(np.float64)
    Bi = mi.int_uniform(n, 13).astype(np.float64)
    assert np.array_equal(run_fast(fused, 1, 0, Ai, Bi)[rows], om.rows_reference(Ai, Bi, rows))


def test_bench_default_depth3_sampled():
    """The benchmark's default: n = 8192 FP64, Strassen-Winograd depth 3 run
    Kronecker-fused (one level of <8,8,8;343>), on the benchmark's inputs
    (uniform, seeds 10 and 11) within the bound on sampled rows, first and
    last included; agreeing with the level-by-level depth 3 within the bound;
    exact on integer inputs ([-8, 8]: |T| <= 512, every sum below 2^53)."""
    n = 8192
    w = mf.mf_algo_builtin("winograd")
    c888 = mf.mf_algo_compose(mf.mf_algo_compose(w, w), w)
    A = mi.uniform(n, 10)
    B = mi.uniform(n, 11)
    rows = np.unique(np.concatenate([np.random.default_rng(8).choice(n, size=40, replace=False), [0, n - 1]]))
    ref = om.rows_reference(A, B, rows)
    got_f = run_fast(c888, 1, 0, A, B)
    got_l = run_fast(w, 3, 0, A, B)
    assert om.rel_fro_error(got_f[rows], ref) < FP64_TOL
    assert om.rel_fro_error(got_f, got_l) < FP64_TOL
    Ai = mi.int_uniform(n, 14).astype(np.float64)
    Bi = mi.int_uniform(n, 15).astype(np.float64)
    assert np.array_equal(run_fast(c888, 1, 0, Ai, Bi)[rows], om.rows_reference(Ai, Bi, rows))


# ------------------------------------------------------------- large leaves
# Full-size exactness of the GEMM on large leaves: classical n = 4000, 4001
# (masked edge tiles: valid extent 4000 / 4001 inside a 4096 leaf), 4096 and
# 6144 (interior), and depth-1 products at 6144 and 8192; every sampled row and
# column, including the first and the last, is compared exactly.
@pytest.mark.parametrize("n", [4000, 4001, 4096, 6144])
def test_large_tile_classical_int_exact_rows(n):
    A = mi.int_uniform(n, 60).astype(np.float64)
    B = mi.int_uniform(n, 61).astype(np.float64)
    got = run_classical(A, B)
    rows = np.sort(np.random.default_rng(n).choice(n, size=40, replace=False))
    rows = np.unique(np.concatenate([rows, [0, n - 1]]))
    assert np.array_equal(got[rows], om.rows_reference(A, B, rows))
    cols = np.unique(np.concatenate([np.random.default_rng(n + 1).choice(n, size=40, replace=False), [0, n - 1]]))
    assert np.array_equal(got[:, cols], A @ B[:, cols])


@pytest.mark.parametrize("n", [6144, 8192])
def test_large_tile_fast_depth1_int_exact_rows(n):
    A = mi.int_uniform(n, 62).astype(np.float64)
    B = mi.int_uniform(n, 63).astype(np.float64)
    got = run_fast(mf.mf_algo_builtin("winograd"), 1, 0, A, B)
    rows = np.unique(np.concatenate([np.random.default_rng(n).choice(n, size=32, replace=False), [0, n - 1]]))
    assert np.array_equal(got[rows], om.rows_reference(A, B, rows))


def test_largest_configuration_sampled():
    """n = 16384 (the largest size of the workloads): Strassen-Winograd depth
    1 and depth 2 Kronecker-fused, sampled rows against the oracle within the
    bound, and integer inputs exactly."""
    n = 16384
    w = mf.mf_algo_builtin("winograd")
    A = mi.uniform(n, 20)
    B = mi.uniform(n, 21)
    rows = np.unique(np.concatenate([np.random.default_rng(7).choice(n, size=24, replace=False), [0, n - 1]]))
    ref = om.rows_reference(A, B, rows)
    for algo, depth in ((w, 1), (mf.mf_algo_compose(w, w), 1)):
        got = run_fast(algo, depth, 0, A, B)
        assert om.rel_fro_error(got[rows], ref) < FP64_TOL
    Ai = mi.int_uniform(n, 22).astype(np.float64)
    Bi = mi.int_uniform(n, 23).astype(np.float64)
    got = run_fast(w, 2, 0, Ai, Bi)
    assert np.array_equal(got[rows], om.rows_reference(Ai, Bi, rows))


# ------------------------------------------ Kronecker-fused depth 3 (<8,8,8;343>)

def kron3(name):
    if name == "mixed":  # Winograd x Strassen x Winograd: the factors differ
        w, s = mf.mf_algo_builtin("winograd"), mf.mf_algo_builtin("strassen")
        return mf.mf_algo_compose(mf.mf_algo_compose(w, s), w)
    a = mf.mf_algo_builtin(name)
    return mf.mf_algo_compose(mf.mf_algo_compose(a, a), a)


@pytest.mark.parametrize("name", ["winograd", "strassen", "strassen1969", "mixed"])
@pytest.mark.parametrize("n", [1000, 1001, 1024])
def test_kron3_int_exact(name, n):
    """Depth 3 as one level of <8,8,8;343> (the three-factor Kronecker
    composition), whose pre- and post-additions run factor by factor: 64
    quarter blocks in, 343 products; 343 products in, 64 blocks out.  n = 1000
    puts part of the 8 x 8 split in the virtual padding.  Integer inputs keep
    every intermediate below 2^53 (|T| <= 64 * 8, |P| <= 128 * 512^2, sums of
    343 such), so the result is the exact product.  n = 1001 also makes the
    caller's rows unaligned (element-wise loads and stores).  Strassen's 1969
    form has 2 aliased operands per side and factor instead of 3, so its cube
    stores 335 operands per side instead of 316."""
    A = mi.int_uniform(n, 96)
    B = mi.int_uniform(n, 97)
    got = run_fast(kron3(name), 1, 0, A.astype(np.float64), B.astype(np.float64))
    assert np.array_equal(got, om.classical_mm(A, B).astype(np.float64))


def test_kron3_uniform_error_and_determinism():
    """uniform[-1,1]: within the FP64 bound against the oracle, equal to the
    level-by-level depth 3 within the same bound, and bitwise reproducible."""
    n = 1024
    A = mi.uniform(n, 98)
    B = mi.uniform(n, 99)
    ref = om.classical_mm(A, B)
    w = mf.mf_algo_builtin("winograd")
    fused = run_fast(kron3("winograd"), 1, 0, A, B)
    level = run_fast(w, 3, 0, A, B)
    assert om.rel_fro_error(fused, ref) < FP64_TOL
    assert om.rel_fro_error(level, ref) < FP64_TOL
    assert np.array_equal(fused, run_fast(kron3("winograd"), 1, 0, A, B))


@pytest.mark.parametrize("n", [1000, 1024])
def test_kron3_fp32_storage(n):
    """FP32 storage and leaves through the same factor-by-factor kernels (two
    elements per thread), whole and ragged."""
    A = mi.uniform(n, 100).astype(np.float32)
    B = mi.uniform(n, 101).astype(np.float32)
    dA, dB = torch.from_numpy(A).to("cuda:0"), torch.from_numpy(B).to("cuda:0")
    dC = torch.full_like(dA, float("nan"))
    mf.mf_fastmm(kron3("winograd"), 1, 0, dA, dB, dC)
    torch.cuda.synchronize()
    ref = om.classical_mm(A.astype(np.float64), B.astype(np.float64))
    assert om.rel_fro_error(dC.cpu().numpy().astype(np.float64), ref) < 2e-5


# ------------------------------------------- split factors 2 and 3 (<6,6,6;189>)

@pytest.mark.parametrize("order", ["strassen_then_classical3", "classical3_then_strassen"])
@pytest.mark.parametrize("n", [300, 1000, 2048])
def test_mixed_split_factors_int_exact(order, n):
    """The paper's Strassen composed with the classical <3,3,3;27> in either
    order (split factor 6 = 2 x 3 or 3 x 2), run as two levels: exact on
    integers; at n = 300 also equal to the oracle's composed algorithm."""
    s = mf.mf_algo_builtin("strassen")
    c3 = mf.mf_algo_builtin("classical3")
    algo = mf.mf_algo_compose(s, c3) if order.startswith("strassen") else mf.mf_algo_compose(c3, s)
    assert mf.mf_plan_query(algo, 1, 0, n)["levels"] == 2
    A = mi.int_uniform(n, 17)
    B = mi.int_uniform(n, 18)
    want = om.classical_mm(A, B)
    if n == 300:
        o_s, o_c3 = oracle_algo("strassen"), oa.classical_algo(3)
        o_alg = oa.compose(o_s, o_c3) if order.startswith("strassen") else oa.compose(o_c3, o_s)
        assert np.array_equal(om.fast_mm(A, B, o_alg, 1), want)
    got = run_fast(algo, 1, 0, A.astype(np.float64), B.astype(np.float64))
    assert np.array_equal(got, want.astype(np.float64))


def test_mixed_split_factors_fp64_error_by_order():
    """Both orders within the FP64 bound at n = 2048; their errors differ
    (different summation order), as the paper notes for 2 x 3 against 3 x 2."""
    s = mf.mf_algo_builtin("strassen")
    c3 = mf.mf_algo_builtin("classical3")
    A = mi.uniform(2048, 10)
    B = mi.uniform(2048, 11)
    ref = om.classical_mm(A, B)
    errs = {}
    for name, algo in (("2x3", mf.mf_algo_compose(s, c3)), ("3x2", mf.mf_algo_compose(c3, s))):
        errs[name] = om.rel_fro_error(run_fast(algo, 1, 0, A, B), ref)
        assert errs[name] < FP64_TOL
    print(f"<6,6,6;189> n=2048 rel err: 2x3 {errs['2x3']:.3e}, 3x2 {errs['3x2']:.3e}", flush=True)
    assert errs["2x3"] != errs["3x2"]
