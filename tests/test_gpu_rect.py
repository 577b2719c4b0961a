"""GPU parity of rectangular products and of C = alpha A B + beta C through
the C ABI (mf_gemm), against the rectangular CPU oracle: integer inputs
bit-exact, uniform inputs within the FP64 bound 1e-11 (FP32 2e-5).  Covers
rectangular algorithms built by direct sums and Kronecker products (the
6 x 6 x 6 algorithm from non-square pieces in both factor orders), square
algorithms on rectangular operands, leading dimensions larger than the rows,
ragged sizes, and the scaling paths (GEMM epilogue, post-addition kernels,
the wide and the Kronecker-factored post-additions)."""
import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om
from oracle import rect as orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mf = pytest.importorskip("paper_2312_12732_amd.mf", reason="libmf.so not built")


def lib_algos():
    s = mf.mf_algo_builtin("strassen")
    w = mf.mf_algo_builtin("winograd")
    hk = mf.mf_algo_concat(s, mf.mf_algo_classical(2, 2, 1), "n")        # <2,2,3;11>
    r232 = mf.mf_algo_concat(s, mf.mf_algo_classical(2, 1, 2), "k")      # <2,3,2;11>
    r233 = mf.mf_algo_concat(hk, mf.mf_algo_classical(2, 1, 3), "k")     # <2,3,3;17>
    r322 = mf.mf_algo_concat(s, mf.mf_algo_classical(1, 2, 2), "m")      # <3,2,2;11>
    return {"strassen": s, "winograd": w, "hk223": hk, "r232": r232, "r233": r233, "r322": r322,
            "six_233_322": mf.mf_algo_compose(r233, r322), "six_322_233": mf.mf_algo_compose(r322, r233),
            "c223": mf.mf_algo_classical(2, 2, 3), "w444": mf.mf_algo_compose(w, w),
            "w888": mf.mf_algo_compose(mf.mf_algo_compose(w, w), w)}


def oracle_algos():
    def sq(t):
        U, V, W, conv = mi.as_float_tables(t)
        return orc.from_square(oa.canonical(2, U, V, W, conv))
    s, w = sq(mi.STRASSEN_PAPER), sq(mi.WINOGRAD)
    hk = orc.concat(s, orc.classical(2, 2, 1), "n")
    r233 = orc.concat(hk, orc.classical(2, 1, 3), "k")
    r322 = orc.concat(s, orc.classical(1, 2, 2), "m")
    return {"strassen": s, "winograd": w, "hk223": hk, "r232": orc.concat(s, orc.classical(2, 1, 2), "k"),
            "r233": r233, "r322": r322, "six_233_322": orc.compose(r233, r322),
            "six_322_233": orc.compose(r322, r233), "c223": orc.classical(2, 2, 3),
            "w444": orc.compose(w, w), "w888": orc.compose(orc.compose(w, w), w)}


LIB = None


def algo(name):
    global LIB
    if LIB is None:
        LIB = lib_algos()
    return LIB[name]


def dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0", dt)


def run_gemm(name, depth, A, B, C0=None, alpha=1.0, beta=0.0, dt=torch.float64):
    M, K = A.shape
    N = B.shape[1]
    dA, dB = dev(A, dt), dev(B, dt)
    dC = dev(C0, dt) if C0 is not None else torch.full((M, N), float("nan"), dtype=dt, device="cuda:0")
    mf.mf_gemm(algo(name) if name else None, depth, 0, dA, dB, dC, alpha, beta)
    torch.cuda.synchronize()
    return dC.cpu().numpy().astype(np.float64)


INT_CASES = [  # algorithm, depth, M, K, N
    ("hk223", 1, 512, 384, 768), ("hk223", 2, 1000, 700, 1500), ("r322", 2, 1536, 1024, 1024),
    ("r232", 1, 640, 900, 640), ("r233", 1, 700, 1000, 999), ("c223", 1, 300, 260, 390),
    ("six_233_322", 1, 1536, 1536, 1536), ("six_322_233", 1, 1536, 1536, 1536),
    ("winograd", 2, 1000, 600, 1300), ("strassen", 1, 257, 1000, 129), ("w444", 1, 1024, 768, 1280),
]


@pytest.mark.parametrize("name,depth,M,K,N", INT_CASES)
def test_rect_int_exact(name, depth, M, K, N):
    print(f"rect int {name} depth {depth} {M}x{K}x{N}", flush=True)
    A = mi.int_uniform_rect(M, K, 100 + M)
    B = mi.int_uniform_rect(K, N, 200 + N)
    got = run_gemm(name, depth, A.astype(np.float64), B.astype(np.float64))
    want = orc.fast_gemm(A, B, oracle_algos()[name], depth)
    assert np.array_equal(want, om.classical_mm(A, B))
    assert np.array_equal(got, want.astype(np.float64))


@pytest.mark.parametrize("name,depth,M,K,N", [("hk223", 2, 1024, 1024, 1536), ("six_233_322", 1, 3072, 3072, 3072),
                                              ("six_322_233", 1, 3072, 3072, 3072), ("winograd", 3, 2048, 1536, 2560)])
def test_rect_fp64_close(name, depth, M, K, N):
    print(f"rect fp64 {name} depth {depth} {M}x{K}x{N}", flush=True)
    A = mi.uniform_rect(M, K, 1)
    B = mi.uniform_rect(K, N, 2)
    err = om.rel_fro_error(run_gemm(name, depth, A, B), om.classical_mm(A, B))
    assert err < 1e-11


def test_rect_fp32_close():
    A = mi.uniform_rect(1100, 800, 3).astype(np.float32)
    B = mi.uniform_rect(800, 1300, 4).astype(np.float32)
    got = run_gemm("hk223", 2, A, B, dt=torch.float32)
    err = om.rel_fro_error(got, om.classical_mm(A.astype(np.float64), B.astype(np.float64)))
    assert err < 2e-5


@pytest.mark.parametrize("name,depth", [(None, 0), ("winograd", 1), ("hk223", 2), ("w444", 1), ("w888", 1)])
def test_alpha_beta_int_exact(name, depth):
    """alpha = 2, beta = -3 on integers: exact; every path that writes C (the
    classical epilogue, the 7- and 11-input post-additions, the wide 49-input
    one and the Kronecker-factored one)."""
    print(f"alpha/beta {name} depth {depth}", flush=True)
    M, K, N = (1024, 1024, 1024) if name in ("w444", "w888") else (600, 500, 700)
    A = mi.int_uniform_rect(M, K, 11)
    B = mi.int_uniform_rect(K, N, 12)
    C0 = mi.int_uniform_rect(M, N, 13)
    got = run_gemm(name, depth, A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64), 2.0, -3.0)
    want = 2 * om.classical_mm(A, B) - 3 * C0
    assert np.array_equal(got, want.astype(np.float64))


# A tile past a view's last row (column) is computed as the tile that ends at
# the view's edge when the views are at least one tile wide, the inner size is
# a whole number of K steps and the outputs end inside that tile; it writes only
# the rows (columns) it owns.  With beta = 1 an element written twice, or not at
# all, breaks the exact result.
EDGE_CASES = [  # algorithm, depth, M, K, N, dtype
    (None, 0, 200, 208, 336, "f64"),     # rows and columns move
    (None, 0, 200, 208, 335, "f64"),     # odd N: B rows not 16-byte aligned, columns stay masked
    (None, 0, 320, 320, 320, "f64"),     # square, both move
    (None, 0, 1000, 1008, 1111, "f64"),  # rows move, odd N stays masked
    (None, 0, 100, 96, 260, "f64"),      # fewer rows than a tile: masked; columns move
    (None, 0, 192, 320, 448, "f32"),     # FP32: both move
    (None, 0, 700, 200, 129, "f32"),     # K = 200 not a whole number of K steps: masked
    ("winograd", 1, 400, 416, 464, "f64"),  # stored products of padded views: masked
    ("hk223", 1, 520, 416, 780, "f64"),     # rectangular algorithm, products into C
]


@pytest.mark.parametrize("name,depth,M,K,N,dt", EDGE_CASES)
def test_edge_tiles_int_exact(name, depth, M, K, N, dt):
    print(f"edge tiles {name} depth {depth} {M}x{K}x{N} {dt}", flush=True)
    A = mi.int_uniform_rect(M, K, 51 + M)
    B = mi.int_uniform_rect(K, N, 52 + N)
    C0 = mi.int_uniform_rect(M, N, 53)
    tdt = torch.float64 if dt == "f64" else torch.float32
    got = run_gemm(name, depth, A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64), 1.0, 1.0, dt=tdt)
    want = om.classical_mm(A, B) + C0
    assert np.array_equal(got, want.astype(np.float64))


def test_random_shapes_int_exact():
    """Seeded sweep over shapes that mix every tile case: sizes below and above
    one tile, odd and even (rows of A, B and C aligned to 16 bytes or not),
    inner sizes that are or are not whole K steps, classical and one or two
    levels of Winograd and of a rectangular algorithm, FP64 and FP32, beta = 1
    so that an element written twice or not at all breaks the exact result."""
    rng = np.random.default_rng(2024)
    for case in range(24):
        M, K, N = (int(x) for x in rng.integers(60, 700, size=3))
        name, depth = [(None, 0), ("winograd", 1), ("winograd", 2), ("hk223", 1)][case % 4]
        tdt = torch.float64 if case % 3 else torch.float32
        print(f"random shape {case}: {name} depth {depth} {M}x{K}x{N} {tdt}", flush=True)
        A = mi.int_uniform_rect(M, K, 300 + case)
        B = mi.int_uniform_rect(K, N, 400 + case)
        C0 = mi.int_uniform_rect(M, N, 500 + case)
        got = run_gemm(name, depth, A.astype(np.float64), B.astype(np.float64), C0.astype(np.float64), 1.0, 1.0,
                       dt=tdt)
        assert np.array_equal(got, (om.classical_mm(A, B) + C0).astype(np.float64)), (case, name, depth, M, K, N)


@pytest.mark.parametrize("name,depth", [(None, 0), ("winograd", 2), ("six_233_322", 1)])
def test_beta_zero_does_not_read_c(name, depth):
    M, K, N = (1536, 1536, 1536) if name == "six_233_322" else (700, 300, 500)
    A = mi.int_uniform_rect(M, K, 21)
    B = mi.int_uniform_rect(K, N, 22)
    got = run_gemm(name, depth, A.astype(np.float64), B.astype(np.float64), None, 3.0, 0.0)  # C holds NaN
    assert np.array_equal(got, (3 * om.classical_mm(A, B)).astype(np.float64))


def test_alpha_beta_fp64_close():
    A = mi.uniform_rect(900, 1100, 31)
    B = mi.uniform_rect(1100, 700, 32)
    C0 = mi.uniform_rect(900, 700, 33)
    got = run_gemm("hk223", 1, A, B, C0, 0.75, 1.5)
    want = orc.fast_gemm(A, B, oracle_algos()["hk223"], 1, alpha=0.75, beta=1.5, C=C0)
    assert om.rel_fro_error(got, want) < 1e-11


def test_leading_dimensions_larger_than_rows():
    """Operands and result as column windows of wider matrices: the columns
    outside the windows are left untouched."""
    M, K, N = 520, 700, 900
    big_a = mi.int_uniform_rect(M, K + 37, 41)
    big_b = mi.int_uniform_rect(K, N + 64, 42)
    big_c = mi.int_uniform_rect(M, N + 9, 43)
    dA, dB, dC = dev(big_a.astype(np.float64)), dev(big_b.astype(np.float64)), dev(big_c.astype(np.float64))
    mf.mf_gemm(algo("hk223"), 2, 0, dA[:, 5:5 + K], dB[:, 64:], dC[:, 9:], 1.0, 1.0)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    want = big_c.copy()
    want[:, 9:] += om.classical_mm(big_a[:, 5:5 + K], big_b[:, 64:])
    assert np.array_equal(got, want.astype(np.float64))


def test_gemm_equals_fastmm_on_square():
    """Same square request through both entry points: the same plan, the
    same bits."""
    n = 1024
    A = mi.uniform(n, 51)
    B = mi.uniform(n, 52)
    dA, dB = dev(A), dev(B)
    c1 = torch.empty_like(dA)
    c2 = torch.empty_like(dA)
    mf.mf_fastmm(algo("winograd"), 2, 0, dA, dB, c1)
    mf.mf_gemm(algo("winograd"), 2, 0, dA, dB, c2)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)


def test_factor_order_workspace_and_error():
    """The two orders of the 6 x 6 x 6 algorithm from non-square pieces (the
    order effect of Section 2): both exact on integers (above), both within
    the FP64 bound here; their workspace differs."""
    n = 3072
    w1 = mf.mf_workspace_bytes(algo("six_233_322"), 1, 0, n)
    w2 = mf.mf_workspace_bytes(algo("six_322_233"), 1, 0, n)
    assert w1 > 0 and w2 > 0 and w1 != w2
