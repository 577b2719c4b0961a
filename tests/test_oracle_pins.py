"""Pins for the CPU oracle: each test checks the oracle against something other
than itself (the paper's printed example, the Brent equations written as
brute force, the textbook product, closed forms, planted mistakes)."""
import itertools
import os
import re

import numpy as np
import pytest

import mf_inputs as mi
from oracle import algebra as oa
from oracle import matmul as om

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_strassen():
    U, V, W, conv = mi.as_float_tables(mi.STRASSEN_PAPER)
    return oa.canonical(2, U, V, W, conv)


def table_algo(t):
    U, V, W, conv = mi.as_float_tables(t)
    return oa.canonical(t["n0"], U, V, W, conv)


ALL_BASE = {"strassen_paper": paper_strassen, "winograd": lambda: table_algo(mi.WINOGRAD),
            "strassen_1969": lambda: table_algo(mi.STRASSEN_1969)}


# ---------------------------------------------------------------- classical

def brute_force_mm(A, B):
    """Triple loop over Python ints/floats: the definition of Section 2."""
    n, k = len(A), len(A[0])
    m = len(B[0])
    return [[sum(A[i][t] * B[t][j] for t in range(k)) for j in range(m)] for i in range(n)]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_classical_matches_brute_force_on_ints(n):
    A = mi.int_uniform(n, 100 + n)
    B = mi.int_uniform(n, 200 + n)
    got = om.classical_mm(A, B)
    want = brute_force_mm(A.tolist(), B.tolist())
    assert got.tolist() == want


def test_classical_float_close_to_exact_sum():
    import math
    A = mi.uniform(9, 5)
    B = mi.uniform(9, 6)
    got = om.classical_mm(A, B)
    for i in range(9):
        for j in range(9):
            exact = math.fsum(A[i, t] * B[t, j] for t in range(9))
            assert abs(got[i, j] - exact) <= 1e-15 * 9


def test_classical_closed_forms():
    n = 12
    I = np.eye(n, dtype=np.int64)
    A = mi.int_uniform(n, 7)
    assert np.array_equal(om.classical_mm(A, I), A)
    assert np.array_equal(om.classical_mm(I, A), A)
    # permutation: (P A)[i] = A[perm[i]]
    perm = np.random.default_rng(3).permutation(n)
    P = np.zeros((n, n), dtype=np.int64)
    P[np.arange(n), perm] = 1
    assert np.array_equal(om.classical_mm(P, A), A[perm])
    # rank one: (u v^T)(x y^T) = (v . x) u y^T ; a transposed operand breaks it
    g = np.random.default_rng(4)
    u, v, x, y = (g.integers(-5, 6, size=n) for _ in range(4))
    got = om.classical_mm(np.outer(u, v), np.outer(x, y))
    assert np.array_equal(got, int(v @ x) * np.outer(u, y))


def test_classical_int_exact_path_matches_integer_loop():
    """Integer operands within the 2^53 bound go through float64 BLAS; the
    result equals numpy's integer loop (a separate implementation of the
    definition) on ragged rectangular shapes and at a moderate size."""
    g = np.random.default_rng(11)
    for m, k, n in ((1, 1, 1), (3, 5, 2), (17, 64, 33), (200, 301, 150)):
        A = g.integers(-8, 9, size=(m, k))
        B = g.integers(-8, 9, size=(k, n))
        assert om.exact_in_float64(A, B)
        got = om.classical_mm(A, B)
        assert got.dtype == np.int64
        assert np.array_equal(got, np.matmul(A, B))


def test_classical_int_beyond_the_float64_bound_stays_exact():
    """Entries 2^27 + 1: one product (2^54 + 2^28 + 1) already has no float64
    representation, so the float path would round; the oracle must take the
    integer loop and match Python's big integers."""
    v = 2 ** 27 + 1
    A = np.array([[v, v], [v, -v]], dtype=np.int64)
    B = np.array([[v, 1], [v, v]], dtype=np.int64)
    assert not om.exact_in_float64(A, B)
    want = brute_force_mm(A.tolist(), B.tolist())
    assert om.classical_mm(A, B).tolist() == want
    # planted mistake: the float path on the same operands is wrong
    wrong = np.matmul(A.astype(np.float64), B.astype(np.float64)).astype(np.int64)
    assert wrong.tolist() != want
    # rows_reference takes the same exact path
    assert om.rows_reference(A, B, [1]).tolist() == [[float(x) for x in want[1]]]


def test_exact_in_float64_bound_is_tight():
    # K max|A| max|B| = 2^53 - 2^26 passes, 2^53 does not
    A = np.full((1, 1), 2 ** 26, dtype=np.int64)
    assert om.exact_in_float64(A, np.full((1, 1), 2 ** 27 - 1, dtype=np.int64))
    assert not om.exact_in_float64(A, np.full((1, 1), 2 ** 27, dtype=np.int64))
    assert not om.exact_in_float64(np.ones((1, 1)), np.ones((1, 1)))  # floats never take the integer path


# -------------------------------------------------------- worked example

def _parse_terms(s):
    out = {}
    for tok in s.split():
        c, blk = tok.split(":")
        out[blk] = int(c)
    return out


def test_paper_worked_example():
    alg = paper_strassen()
    lines = [ln for ln in open(os.path.join(GOLDEN, "paper_strassen_worked_example.txt"))
             if ln.strip() and not ln.startswith("#")]
    for ln in lines:
        lhs, rhs = [x.strip() for x in ln.split("=", 1)]
        if lhs.startswith("C"):
            c = int(lhs[1:])
            prods = sorted(int(t.strip()[1:]) for t in rhs.split("+"))
            nz = [r for r in range(alg.R) if alg.W[c, r] != 0]
            assert nz == prods and all(alg.W[c, r] == 1 for r in prods), ln
        else:
            r = int(lhs[1:])
            m = re.match(r"\((.*)\) \* \((.*)\)", rhs)
            ta, tb = _parse_terms(m.group(1)), _parse_terms(m.group(2))
            got_a = {f"A{k}": int(alg.U[k, r]) for k in range(4) if alg.U[k, r]}
            got_b = {f"B{k}": int(alg.V[k, r]) for k in range(4) if alg.V[k, r]}
            assert got_a == ta and got_b == tb, ln


def test_paper_example_numerically():
    # 2x2 scalar blocks: C0 = A0 B0 + A1 B2 and C3 = A2 B1 + A3 B3
    alg = paper_strassen()
    A = np.array([[2, 3], [5, 7]], dtype=np.int64)
    B = np.array([[11, 13], [17, 19]], dtype=np.int64)
    C = om.fast_mm(A, B, alg, depth=1)
    assert C[0, 0] == 2 * 11 + 3 * 17
    assert C[1, 1] == 5 * 13 + 7 * 19


def test_classical_graph_print_matches_classical_algo():
    alg = oa.classical_algo(2)
    lines = [ln.strip() for ln in open(os.path.join(GOLDEN, "classical_2x2_graph.txt"))
             if ln.strip() and not ln.startswith("#")]
    for ln in lines:
        c = int(re.match(r"CDP\[(\d+)\]", ln).group(1))
        pairs = sorted((int(a), int(b)) for a, b in re.findall(r"ADP\[(\d+)\]\) \* \(BDP\[(\d+)\]", ln))
        got = sorted((int(np.flatnonzero(alg.U[:, r])[0]), int(np.flatnonzero(alg.V[:, r])[0]))
                     for r in range(alg.R) if alg.W[c, r])
        assert got == pairs


# ------------------------------------------------------------------ Brent

def brent_by_definition(alg, A, B):
    """Evaluate the algorithm on symbolic-free integer scalars (p x p, 1x1
    blocks) and compare with the product; used as an independent check of
    ``brent_violations`` on random integer matrices."""
    p = alg.p
    a = A.reshape(-1)
    b = B.reshape(-1)
    c = np.zeros(p * p, dtype=np.int64)
    for r in range(alg.R):
        c += alg.W[:, r] * int(alg.U[:, r] @ a) * int(alg.V[:, r] @ b)
    return c.reshape(p, p)


@pytest.mark.parametrize("name", list(ALL_BASE))
def test_brent_holds_for_base_algorithms(name):
    alg = ALL_BASE[name]()
    assert alg.R == 7
    assert oa.brent_violations(alg) == 0
    for s in range(5):
        A = mi.int_uniform(2, 10 + s)
        B = mi.int_uniform(2, 20 + s)
        assert np.array_equal(brent_by_definition(alg, A, B), A @ B)


def test_printed_labels_are_needed():
    # Reading the printed c^t rows as C0, C1, C2, C3 in order breaks the algorithm.
    U, V, W, _ = mi.as_float_tables(mi.STRASSEN_PAPER)
    wrong = oa.canonical(2, U, V, W, 0)
    assert oa.brent_violations(wrong) > 0
    A = mi.int_uniform(2, 1)
    B = mi.int_uniform(2, 2)
    assert not np.array_equal(brent_by_definition(wrong, A, B), A @ B)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_classical_algo_brent(p):
    alg = oa.classical_algo(p)
    assert alg.R == p ** 3
    assert oa.brent_violations(alg) == 0


@pytest.mark.parametrize("which,idx", list(itertools.product("UVW", range(28))))
def test_every_single_coefficient_flip_is_caught(which, idx):
    # planted mistake: change one coefficient of Strassen by +1 (a sign or a
    # dropped term); the Brent check and the integer product must both see it.
    alg = paper_strassen()
    k, r = divmod(idx, 7)
    M = {"U": alg.U.copy(), "V": alg.V.copy(), "W": alg.W.copy()}
    M[which][k, r] += 1
    bad = oa.Algo(2, 7, M["U"], M["V"], M["W"])
    assert oa.brent_violations(bad) > 0
    A = mi.int_uniform(8, 31)
    B = mi.int_uniform(8, 32)
    assert not np.array_equal(om.fast_mm(A, B, bad, depth=1), A @ B)


# ---------------------------------------------------------- composition

def test_compose_product_counts():
    s = paper_strassen()
    assert oa.power(s, 2).R == 49 and oa.power(s, 2).p == 4
    assert oa.power(s, 3).R == 343 and oa.power(s, 3).p == 8
    c3 = oa.classical_algo(3)
    assert oa.compose(s, c3).R == 7 * 27 and oa.compose(s, c3).p == 6


@pytest.mark.parametrize("name", list(ALL_BASE))
def test_compose_brent(name):
    alg = ALL_BASE[name]()
    assert oa.brent_violations(oa.power(alg, 2)) == 0
    assert oa.brent_violations(oa.compose(alg, oa.classical_algo(3))) == 0
    assert oa.brent_violations(oa.compose(oa.classical_algo(3), alg)) == 0


def test_compose_nnz_and_aliases():
    s2 = oa.power(paper_strassen(), 2)
    assert (np.count_nonzero(s2.U), np.count_nonzero(s2.V), np.count_nonzero(s2.W)) == (196, 196, 144)
    assert len(oa.single_coefficient_columns(s2.U)) == 9
    assert len(oa.single_coefficient_columns(s2.V)) == 9


@pytest.mark.parametrize("name", list(ALL_BASE))
def test_cube_brent_and_counts(name):
    # <8,8,8;343> = F (x) F (x) F: the 64^3 Brent equations hold exactly, and
    # nonzeros and single-coefficient (aliased) columns multiply factor by
    # factor, since a composed coefficient is the product of one coefficient
    # from each factor.
    f = ALL_BASE[name]()
    c = oa.power(f, 3)
    assert (c.p, c.R) == (8, 343)
    assert oa.brent_violations(c) == 0
    for X, Xf in ((c.U, f.U), (c.V, f.V), (c.W, f.W)):
        assert np.count_nonzero(X) == np.count_nonzero(Xf) ** 3
    assert len(oa.single_coefficient_columns(c.U)) == len(oa.single_coefficient_columns(f.U)) ** 3
    assert len(oa.single_coefficient_columns(c.V)) == len(oa.single_coefficient_columns(f.V)) ** 3


@pytest.mark.parametrize("n", [64, 100])
def test_cube_equals_three_levels_on_ints(n):
    w = ALL_BASE["winograd"]()
    A = mi.int_uniform(n, 43)
    B = mi.int_uniform(n, 44)
    fused = om.fast_mm(A, B, oa.power(w, 3), depth=1)
    assert np.array_equal(fused, om.fast_mm(A, B, w, depth=3))
    assert np.array_equal(fused, A @ B)


def test_raw_kron_without_reindexing_fails():
    # Plain np.kron of the factor matrices uses the nested row order; the
    # composition needs the row-major re-indexing.
    s = paper_strassen()
    raw = oa.Algo(4, 49, np.kron(s.U, s.U), np.kron(s.V, s.V), np.kron(s.W, s.W))
    assert oa.brent_violations(raw) > 0


def test_power_equals_recursion_on_ints():
    s = ALL_BASE["winograd"]()
    A = mi.int_uniform(32, 41)
    B = mi.int_uniform(32, 42)
    two_levels = om.fast_mm(A, B, s, depth=2)
    fused = om.fast_mm(A, B, oa.power(s, 2), depth=1)
    assert np.array_equal(two_levels, fused)
    assert np.array_equal(fused, A @ B)


# -------------------------------------------------------------- re-basis

@pytest.mark.parametrize("seed", [7, 8, 9, 10])
def test_rebase_brent_and_exact(seed):
    s = paper_strassen()
    X, Y, Z = (mi.unimodular(2, seed * 10 + t) for t in range(3))
    for M in (X, Y, Z):
        assert abs(round(np.linalg.det(M))) == 1
    rb = oa.rebase(s, X, Y, Z)
    assert oa.brent_violations(rb) == 0
    A = mi.int_uniform(16, seed)
    B = mi.int_uniform(16, seed + 1)
    assert np.array_equal(om.fast_mm(A, B, rb, depth=2), A @ B)


def test_rebase_identity_is_noop():
    s = paper_strassen()
    I = np.eye(2, dtype=np.int64)
    rb = oa.rebase(s, I, I, I)
    assert np.array_equal(rb.U, s.U) and np.array_equal(rb.V, s.V) and np.array_equal(rb.W, s.W)


def test_rebase_swap_permutes_blocks():
    # X = swap: A' = X A has its block rows exchanged; U'_r = X^T U_r swaps
    # the rows of each coefficient matrix accordingly.
    s = paper_strassen()
    X = np.array([[0, 1], [1, 0]], dtype=np.int64)
    I = np.eye(2, dtype=np.int64)
    rb = oa.rebase(s, X, I, I)
    for r in range(7):
        assert np.array_equal(rb.U[:, r].reshape(2, 2), s.U[:, r].reshape(2, 2)[[1, 0]])
        assert np.array_equal(rb.W[:, r].reshape(2, 2), s.W[:, r].reshape(2, 2)[[1, 0]])
    assert oa.brent_violations(rb) == 0


def test_rebase_rejects_non_unimodular():
    s = paper_strassen()
    I = np.eye(2, dtype=np.int64)
    with pytest.raises(ValueError):
        oa.rebase(s, 2 * I, I, I)


# ------------------------------------------------------ fast vs classical

@pytest.mark.parametrize("name", list(ALL_BASE))
@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 256])
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
def test_fast_equals_classical_on_ints(name, n, depth):
    alg = ALL_BASE[name]()
    A = mi.int_uniform(n, 3)
    B = mi.int_uniform(n, 4)
    assert np.array_equal(om.fast_mm(A, B, alg, depth=depth), om.classical_mm(A, B))


@pytest.mark.parametrize("n", [5, 13, 100, 129])
def test_fast_ragged_sizes_pad_and_crop(n):
    alg = paper_strassen()
    A = mi.int_uniform(n, 5)
    B = mi.int_uniform(n, 6)
    for depth in (1, 2, 3):
        assert np.array_equal(om.fast_mm(A, B, alg, depth=depth), A @ B)


def test_classical_algo_through_executor_is_textbook():
    c3 = oa.classical_algo(3)
    A = mi.int_uniform(27, 8)
    B = mi.int_uniform(27, 9)
    assert np.array_equal(om.fast_mm(A, B, c3, depth=2), A @ B)


def test_cutoff_levels():
    assert om.levels_taken(256, 2, 3, 0) == 3
    assert om.levels_taken(256, 2, 3, 64) == 2      # 256 > 64, 128 > 64, 64 stops
    assert om.levels_taken(256, 2, 3, 256) == 0
    assert om.levels_taken(100, 2, 3, 30) == 2      # 100 -> 50 -> 25
    assert om.levels_taken(8, 3, 2, 0) == 2


def test_dropped_term_in_executor_is_caught(monkeypatch):
    # planted mistake in the oracle: skip the last coefficient of every
    # combination; the integer comparison against the classical product fails.
    orig = om._combine

    def bad_combine(coeffs, blocks, m, dtype):
        c = np.array(coeffs).copy()
        nz = np.flatnonzero(c)
        if len(nz) > 1:
            c[nz[-1]] = 0
        return orig(c, blocks, m, dtype)

    monkeypatch.setattr(om, "_combine", bad_combine)
    A = mi.int_uniform(8, 1)
    B = mi.int_uniform(8, 2)
    assert not np.array_equal(om.fast_mm(A, B, paper_strassen(), depth=1), A @ B)


def test_transposed_block_indexing_is_caught(monkeypatch):
    # planted mistake: column-major block numbering instead of row-major.
    def bad_block(X, k, p, m):
        j, i = divmod(k, p)
        return X[i * m:(i + 1) * m, j * m:(j + 1) * m]

    monkeypatch.setattr(om, "_block", bad_block)
    A = mi.int_uniform(8, 1)
    B = mi.int_uniform(8, 2)
    assert not np.array_equal(om.fast_mm(A, B, paper_strassen(), depth=1), A @ B)


# --------------------------------------------------------- floating point

@pytest.mark.parametrize("depth", [1, 2, 3])
def test_fp64_error_small_and_grows_with_depth(depth):
    # Within the normwise bound (a small multiple of the unit roundoff times
    # a polynomial in n); the fp64 bar of the build is 1e-11.
    n = 512
    A = mi.uniform(n, 1)
    B = mi.uniform(n, 2)
    ref = om.classical_mm(A, B)
    err = om.rel_fro_error(om.fast_mm(A, B, paper_strassen(), depth=depth), ref)
    assert err < 1e-13
    assert err > 0.0


def test_error_metrics_closed_form():
    C = np.ones((4, 4))
    assert om.rel_fro_error(C * (1 + 1e-3), C) == pytest.approx(1e-3)
    A = np.eye(4)
    assert om.componentwise_error(C + 0.5, C, np.ones((4, 4)), A) == pytest.approx(0.5)
    assert om.max_scaled_error(C + 0.25, C, 2 * np.ones((4, 4)), A) == pytest.approx(0.125)


# ----------------------------------------------------- sampled definition rows
# rows_reference is the checker of every full-size parity test: row i of the
# definition C_ij = sum_k A_ik B_kj (Section 2) for sampled i only.

@pytest.mark.parametrize("n", [1, 4, 7, 13])
def test_rows_reference_matches_brute_force_rows(n):
    A = mi.int_uniform(n, 300 + n)
    B = mi.int_uniform(n, 400 + n)
    rows = sorted(set(np.random.default_rng(n).integers(0, n, size=max(1, n // 2)).tolist()))
    got = om.rows_reference(A, B, rows)
    full = brute_force_mm(A.tolist(), B.tolist())
    assert got.shape == (len(rows), n)
    for a, i in enumerate(rows):
        assert got[a].tolist() == [float(x) for x in full[i]]


def test_rows_reference_float_rows_close_to_exact_sum():
    import math
    n = 11
    A = mi.uniform(n, 31)
    B = mi.uniform(n, 32)
    rows = [0, 5, 10]
    got = om.rows_reference(A, B, rows)
    for a, i in enumerate(rows):
        for j in range(n):
            exact = math.fsum(A[i, t] * B[t, j] for t in range(n))
            assert abs(got[a, j] - exact) <= 1e-15 * n


def test_rows_reference_closed_forms():
    n = 16
    A = mi.int_uniform(n, 41)
    rows = [2, 3, 11]
    # identity on the right: the sampled rows of A themselves
    assert np.array_equal(om.rows_reference(A, np.eye(n, dtype=np.int64), rows), A[rows].astype(np.float64))
    # permutation on the right moves columns: (A P)[i, perm[j]] = A[i, j]
    perm = np.random.default_rng(6).permutation(n)
    P = np.zeros((n, n), dtype=np.int64)
    P[np.arange(n), perm] = 1
    got = om.rows_reference(A, P, rows)
    assert np.array_equal(got[:, perm], A[rows].astype(np.float64))
    # rank one: rows of (u v^T)(x y^T) are (v . x) u_i y^T
    g = np.random.default_rng(7)
    u, v, x, y = (g.integers(-5, 6, size=n) for _ in range(4))
    got = om.rows_reference(np.outer(u, v), np.outer(x, y), rows)
    assert np.array_equal(got, (int(v @ x) * np.outer(u, y))[rows].astype(np.float64))


def test_rows_reference_planted_mistakes_are_caught():
    """A transposed B, shifted rows or a transposed A all change the rows."""
    n = 9
    A = mi.int_uniform(n, 51)
    B = mi.int_uniform(n, 52)
    rows = [1, 4, 8]
    want = np.array([[sum(int(A[i, t]) * int(B[t, j]) for t in range(n)) for j in range(n)] for i in rows],
                    dtype=np.float64)
    assert np.array_equal(om.rows_reference(A, B, rows), want)
    assert not np.array_equal(om.rows_reference(A, B.T.copy(), rows), want)
    assert not np.array_equal(om.rows_reference(A, B, [r - 1 for r in rows]), want)
    assert not np.array_equal(om.rows_reference(A.T.copy(), B, rows), want)


def test_flop_count_and_unit_roundoff_closed_forms():
    # the classical product of two n x n matrices takes n^3 multiplications and n^2 (n - 1) additions;
    # effective GFLOP/s counts 2 n^3 (Section 2's definition, one multiply-add per term)
    for n in (1, 2, 3, 10, 8192):
        assert om.flops(n) == 2.0 * n * n * n
    # unit roundoff of IEEE double: 1 + u rounds back to 1 (ties to even), 1 + 2u does not
    u = om.unit_roundoff()
    assert 1.0 + u == 1.0 and 1.0 + 2 * u > 1.0
    assert om.unit_roundoff(24) == float(np.finfo(np.float32).eps) / 2
    # transpose_index is an involution that swaps the 2-d block index
    for p in (2, 3, 4):
        for t in range(p * p):
            assert oa.transpose_index(oa.transpose_index(t, p), p) == t
            assert oa.transpose_index(t, p) == (t % p) * p + t // p
