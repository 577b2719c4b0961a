"""Pins for the rectangular oracle (oracle/rect.py): Brent equations written
as brute force, the textbook product, direct sums and Kronecker products that
must stay correct, brute-force products on tiny inputs, closed forms of
C = alpha A B + beta C, and planted mistakes that must be caught."""
import itertools

import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om
from oracle import rect as orc


def strassen():
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    return orc.from_square(oa.canonical(2, U, V, W, conv))


def winograd():
    U, V, W, conv = mi.as_float_tables(mi.WINOGRAD)
    return orc.from_square(oa.canonical(2, U, V, W, conv))


def hk223():
    """<2,2,3;11>: Strassen on the first two block columns, the textbook
    product on the third."""
    return orc.concat(strassen(), orc.classical(2, 2, 1), "n")


def r233():
    """<2,3,3;17> = <2,2,3;11> (+)_k <2,1,3;6>."""
    return orc.concat(hk223(), orc.classical(2, 1, 3), "k")


def r322():
    """<3,2,2;11> = Strassen (+)_m <1,2,2;4>."""
    return orc.concat(strassen(), orc.classical(1, 2, 2), "m")


def brent_by_definition(a):
    """The Brent equations evaluated on random integer block matrices: the
    algorithm applied to scalar blocks must give the product exactly."""
    g = np.random.default_rng(7)
    for _ in range(5):
        A = g.integers(-5, 6, size=(a.m0, a.k0))
        B = g.integers(-5, 6, size=(a.k0, a.n0))
        T = [sum(a.U[i * a.k0 + k, r] * A[i, k] for i in range(a.m0) for k in range(a.k0)) for r in range(a.R)]
        S = [sum(a.V[k * a.n0 + j, r] * B[k, j] for k in range(a.k0) for j in range(a.n0)) for r in range(a.R)]
        C = [[sum(a.W[i * a.n0 + j, r] * T[r] * S[r] for r in range(a.R)) for j in range(a.n0)]
             for i in range(a.m0)]
        if C != (A @ B).tolist():
            return False
    return True


def brute(A, B):
    return [[sum(int(A[i][t]) * int(B[t][j]) for t in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (2, 3, 2), (3, 2, 4), (1, 3, 2), (3, 3, 3)])
def test_classical_rect_satisfies_brent(shape):
    a = orc.classical(*shape)
    assert a.R == shape[0] * shape[1] * shape[2]
    assert orc.brent_violations(a) == 0
    assert brent_by_definition(a)


def test_every_single_coefficient_change_of_classical_232_is_caught():
    a = orc.classical(2, 3, 2)
    caught = 0
    for which in "UVW":
        X = getattr(a, which)
        for row, col in itertools.product(range(X.shape[0]), range(X.shape[1])):
            Y = X.copy()
            Y[row, col] += 1
            b = orc.RectAlgo(a.m0, a.k0, a.n0, a.R, *(Y if w == which else getattr(a, w) for w in "UVW"))
            caught += orc.brent_violations(b) > 0
    assert caught == a.U.size + a.V.size + a.W.size


def test_square_algorithms_as_rectangular():
    for a in (strassen(), winograd()):
        assert orc.brent_violations(a) == 0
        assert brent_by_definition(a)


@pytest.mark.parametrize("make,shape,R", [(hk223, (2, 2, 3), 11), (r322, (3, 2, 2), 11),
                                          (lambda: orc.concat(strassen(), orc.classical(2, 1, 2), "k"), (2, 3, 2), 11),
                                          (r233, (2, 3, 3), 17)])
def test_direct_sums_are_correct_algorithms(make, shape, R):
    a = make()
    assert (a.m0, a.k0, a.n0, a.R) == (*shape, R)
    assert orc.brent_violations(a) == 0
    assert brent_by_definition(a)


def test_direct_sum_in_the_wrong_place_is_caught():
    """Strassen's products put after the textbook ones but the blocks left in
    place: the sum along n no longer matches its own coefficient layout."""
    a = hk223()
    V = a.V.copy()
    V[:, [0, 7]] = V[:, [7, 0]]  # swap a Strassen and a textbook B operand
    assert orc.brent_violations(orc.RectAlgo(2, 2, 3, 11, a.U, V, a.W)) > 0


def test_six_by_six_from_non_square_pieces():
    """<2,3,3;17> (x) <3,2,2;11> = <6,6,6;187>: a square 6 x 6 x 6 algorithm
    from non-square factors, fewer products than Strassen (x) classical 3 (189)."""
    a = orc.compose(r233(), r322())
    assert (a.m0, a.k0, a.n0, a.R) == (6, 6, 6, 187)
    assert orc.brent_violations(a) == 0
    b = orc.compose(r322(), r233())
    assert (b.m0, b.k0, b.n0, b.R) == (6, 6, 6, 187)
    assert orc.brent_violations(b) == 0
    assert not np.array_equal(a.U, b.U)  # the order of the factors gives a different algorithm


def test_compose_agrees_with_square_compose():
    U, V, W, conv = mi.as_float_tables(mi.WINOGRAD)
    w = oa.canonical(2, U, V, W, conv)
    sq = oa.compose(w, w)
    rc = orc.compose(orc.from_square(w), orc.from_square(w))
    assert np.array_equal(sq.U, rc.U) and np.array_equal(sq.V, rc.V) and np.array_equal(sq.W, rc.W)


def test_plain_kron_without_reindexing_fails_brent():
    a, b = hk223(), r322()
    c = orc.compose(a, b)
    raw = orc.RectAlgo(c.m0, c.k0, c.n0, c.R, np.kron(a.U, b.U), np.kron(a.V, b.V), np.kron(a.W, b.W))
    assert orc.brent_violations(raw) > 0


@pytest.mark.parametrize("alg,M,K,N,depth", [(hk223, 4, 4, 6, 1), (hk223, 8, 4, 9, 2), (r322, 6, 4, 4, 1),
                                             (r233, 5, 7, 3, 1), (strassen, 3, 5, 7, 2)])
def test_fast_gemm_matches_brute_force_tiny(alg, M, K, N, depth):
    a = alg()
    A = mi.int_uniform_rect(M, K, 10 + M)
    B = mi.int_uniform_rect(K, N, 20 + N)
    got = orc.fast_gemm(A, B, a, depth)
    assert got.tolist() == brute(A, B)


@pytest.mark.parametrize("alg,M,K,N,depth", [(hk223, 37, 50, 23, 2), (r322, 64, 40, 80, 2),
                                             (lambda: orc.compose(r233(), r322()), 60, 66, 72, 1),
                                             (lambda: orc.compose(r322(), r233()), 61, 67, 73, 1)])
def test_fast_gemm_int_exact(alg, M, K, N, depth):
    a = alg()
    A = mi.int_uniform_rect(M, K, 30 + M)
    B = mi.int_uniform_rect(K, N, 40 + N)
    assert np.array_equal(orc.fast_gemm(A, B, a, depth), om.classical_mm(A, B))


def test_composition_equals_recursion_on_ints():
    a = hk223()
    A = mi.int_uniform_rect(40, 16, 5)
    B = mi.int_uniform_rect(16, 36, 6)
    assert np.array_equal(orc.fast_gemm(A, B, orc.compose(a, a), 1), orc.fast_gemm(A, B, a, 2))


def test_alpha_beta_closed_forms():
    a = hk223()
    M, K, N = 9, 6, 12
    A = mi.int_uniform_rect(M, K, 1)
    B = mi.int_uniform_rect(K, N, 2)
    C = mi.int_uniform_rect(M, N, 3)
    AB = np.array(brute(A, B))
    assert np.array_equal(orc.fast_gemm(A, B, a, 1, alpha=0, beta=5, C=C), 5 * C)
    assert np.array_equal(orc.fast_gemm(A, B, a, 1, alpha=3, beta=0), 3 * AB)
    assert np.array_equal(orc.fast_gemm(A, B, a, 1, alpha=2, beta=-3, C=C), 2 * AB - 3 * C)
    eye = np.eye(M, dtype=np.int64)
    Bsq = mi.int_uniform_rect(M, N, 4)
    assert np.array_equal(orc.fast_gemm(eye, Bsq, a, 1, alpha=-1, beta=1, C=C), C - Bsq)
    # beta = 0 ignores C, even when it holds NaN
    Cf = np.full((M, N), np.nan)
    out = orc.fast_gemm(A.astype(np.float64), B.astype(np.float64), a, 1, alpha=1.0, beta=0.0, C=Cf)
    assert np.array_equal(out, AB.astype(np.float64))


def test_levels_taken_rule():
    a = hk223()  # splits 2, 2, 3
    assert orc.levels_taken(100, 100, 100, a, 3, 0) == 3
    assert orc.levels_taken(100, 100, 100, a, 3, 30) == 2   # 100 -> 50 -> 25: 25 <= 30 stops
    assert orc.levels_taken(100, 100, 9, a, 3, 4) == 1      # N: 9 -> 3, 3 <= 4 stops
    assert orc.levels_taken(8, 8, 8, orc.classical(1, 1, 1), 3, 0) == 0  # no split


def test_float_error_small_and_nonzero():
    a = hk223()
    A = mi.uniform_rect(120, 96, 1)
    B = mi.uniform_rect(96, 150, 2)
    got = orc.fast_gemm(A, B, a, 2)
    err = om.rel_fro_error(got, om.classical_mm(A, B))
    assert 0 < err < 1e-14
