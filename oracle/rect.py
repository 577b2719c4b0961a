"""Oracle: rectangular bilinear algorithms <m0,k0,n0;R> and the scaled
product C = alpha A B + beta C.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module;
only the tests do.

Section 2 of the paper partitions the operands by split factors and writes a
fast algorithm as three coefficient matrices acting on the blocks; it works
with square splits for simplicity and notes that products of other shapes
(the 6 x 6 x 6 problem from non-square pieces) are built the same way, by
Kronecker products of the factor matrices.  Section 3 (Matrix Flow) states the
operation as C = alpha A B.  Here, for an M x K operand A split into m0 x k0
blocks A_(i,k) (row index i k0 + k), a K x N operand B split into k0 x n0
blocks B_(k,j) (index k n0 + j) and C split into m0 x n0 blocks C_(i,j)
(index i n0 + j):

    T_r = sum U[(i,k), r] A_(i,k),   S_r = sum V[(k,j), r] B_(k,j),
    P_r = T_r S_r,                   C_(i,j) = sum_r W[(i,j), r] P_r.

The algorithm is correct exactly when the Brent equations hold:
sum_r U[(i,k),r] V[(k',j),r] W[(i',j'),r] = [i = i'] [k = k'] [j = j'].

New algorithms come from two exact constructions: the Kronecker product
(apply one algorithm, then another to each product) and the direct sum along
one dimension (split C, K or the rows of A in two and run one algorithm on
each part), which is how a rectangular fast algorithm is obtained from
Strassen's <2,2,2;7> and textbook pieces, e.g. <2,2,3;11> = <2,2,2;7> (+)_n
<2,2,1;2 x 2>.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .algebra import Algo, _int_matrix
from .matmul import classical_mm


@dataclass(frozen=True)
class RectAlgo:
    """<m0,k0,n0;R>: U is (m0 k0) x R, V (k0 n0) x R, W (m0 n0) x R, int64."""
    m0: int
    k0: int
    n0: int
    R: int
    U: np.ndarray
    V: np.ndarray
    W: np.ndarray


def make(m0: int, k0: int, n0: int, U, V, W) -> RectAlgo:
    U, V, W = _int_matrix(U), _int_matrix(V), _int_matrix(W)
    R = U.shape[1]
    if U.shape != (m0 * k0, R) or V.shape != (k0 * n0, R) or W.shape != (m0 * n0, R):
        raise ValueError("U, V, W shapes do not match <m0,k0,n0;R>")
    return RectAlgo(m0, k0, n0, R, U, V, W)


def from_square(a: Algo) -> RectAlgo:
    """A canonical square <p,p,p;R> algorithm as a rectangular one."""
    return RectAlgo(a.p, a.p, a.p, a.R, a.U, a.V, a.W)


def brent_violations(a: RectAlgo) -> int:
    """Failing Brent equations over all (m0 k0)(k0 n0)(m0 n0) index triples,
    evaluated exactly in int64."""
    t = np.einsum("ar,br,cr->abc", a.U, a.V, a.W)
    want = np.zeros_like(t)
    for i in range(a.m0):
        for k in range(a.k0):
            for j in range(a.n0):
                want[i * a.k0 + k, k * a.n0 + j, i * a.n0 + j] = 1
    return int(np.count_nonzero(t != want))


def classical(m0: int, k0: int, n0: int) -> RectAlgo:
    """The textbook partitioned product: one product A_(i,k) B_(k,j) per
    (i, j, k) in that loop order, added into C_(i,j); R = m0 k0 n0."""
    R = m0 * k0 * n0
    U = np.zeros((m0 * k0, R), dtype=np.int64)
    V = np.zeros((k0 * n0, R), dtype=np.int64)
    W = np.zeros((m0 * n0, R), dtype=np.int64)
    r = 0
    for i in range(m0):
        for j in range(n0):
            for k in range(k0):
                U[i * k0 + k, r] = 1
                V[k * n0 + j, r] = 1
                W[i * n0 + j, r] = 1
                r += 1
    return RectAlgo(m0, k0, n0, R, U, V, W)


def compose(outer: RectAlgo, inner: RectAlgo) -> RectAlgo:
    """Apply ``outer`` first and ``inner`` to each of its products: the
    algorithm of shape <m1 m2, k1 k2, n1 n2; R1 R2>.  A block (I, J) of a
    finer grid with I = i1 r2 + i2, J = j1 c2 + j2 (r2 x c2 the inner grid of
    that operand) is inner block (i2, j2) of outer block (i1, j1); its
    coefficient for product r1 R2 + r2 is the product of the two factors'
    coefficients."""
    def kron_rows(X1, X2, r1, c1, r2, c2):
        cols = c1 * c2
        out = np.zeros((r1 * r2 * cols, X1.shape[1] * X2.shape[1]), dtype=np.int64)
        for i1 in range(r1):
            for j1 in range(c1):
                for i2 in range(r2):
                    for j2 in range(c2):
                        row = (i1 * r2 + i2) * cols + (j1 * c2 + j2)
                        out[row] = np.kron(X1[i1 * c1 + j1], X2[i2 * c2 + j2])
        return out

    o, i = outer, inner
    return RectAlgo(o.m0 * i.m0, o.k0 * i.k0, o.n0 * i.n0, o.R * i.R,
                    kron_rows(o.U, i.U, o.m0, o.k0, i.m0, i.k0),
                    kron_rows(o.V, i.V, o.k0, o.n0, i.k0, i.n0),
                    kron_rows(o.W, i.W, o.m0, o.n0, i.m0, i.n0))


def concat(a: RectAlgo, b: RectAlgo, axis: str) -> RectAlgo:
    """Direct sum along one dimension; the products of ``a`` come first.

    axis 'n': C = [A Ba | A Bb] (columns of B and C split n0a + n0b);
    axis 'm': C = [Aa B ; Ab B] (rows of A and C split m0a + m0b);
    axis 'k': C = Aa Ba + Ab Bb (columns of A and rows of B split k0a + k0b).
    """
    R = a.R + b.R

    def place(rows, cols, blocks):
        # blocks: list of (X, row0, col0, nrows, ncols, r0): X's block (x, y)
        # goes to block (row0 + x, col0 + y) of a rows x cols grid, product r0 + r
        out = np.zeros((rows * cols, R), dtype=np.int64)
        for X, row0, col0, nr, nc, r0 in blocks:
            for x in range(nr):
                for y in range(nc):
                    out[(row0 + x) * cols + col0 + y, r0:r0 + X.shape[1]] = X[x * nc + y]
        return out

    if axis == "n":
        if (a.m0, a.k0) != (b.m0, b.k0):
            raise ValueError("shapes do not concatenate along n")
        m0, k0, n0 = a.m0, a.k0, a.n0 + b.n0
        U = place(m0, k0, [(a.U, 0, 0, m0, k0, 0), (b.U, 0, 0, m0, k0, a.R)])
        V = place(k0, n0, [(a.V, 0, 0, k0, a.n0, 0), (b.V, 0, a.n0, k0, b.n0, a.R)])
        W = place(m0, n0, [(a.W, 0, 0, m0, a.n0, 0), (b.W, 0, a.n0, m0, b.n0, a.R)])
    elif axis == "m":
        if (a.k0, a.n0) != (b.k0, b.n0):
            raise ValueError("shapes do not concatenate along m")
        m0, k0, n0 = a.m0 + b.m0, a.k0, a.n0
        U = place(m0, k0, [(a.U, 0, 0, a.m0, k0, 0), (b.U, a.m0, 0, b.m0, k0, a.R)])
        V = place(k0, n0, [(a.V, 0, 0, k0, n0, 0), (b.V, 0, 0, k0, n0, a.R)])
        W = place(m0, n0, [(a.W, 0, 0, a.m0, n0, 0), (b.W, a.m0, 0, b.m0, n0, a.R)])
    elif axis == "k":
        if (a.m0, a.n0) != (b.m0, b.n0):
            raise ValueError("shapes do not concatenate along k")
        m0, k0, n0 = a.m0, a.k0 + b.k0, a.n0
        U = place(m0, k0, [(a.U, 0, 0, m0, a.k0, 0), (b.U, 0, a.k0, m0, b.k0, a.R)])
        V = place(k0, n0, [(a.V, 0, 0, a.k0, n0, 0), (b.V, a.k0, 0, b.k0, n0, a.R)])
        W = place(m0, n0, [(a.W, 0, 0, m0, n0, 0), (b.W, 0, 0, m0, n0, a.R)])
    else:
        raise ValueError("axis must be 'm', 'k' or 'n'")
    return RectAlgo(m0, k0, n0, R, U, V, W)


def levels_taken(M: int, K: int, N: int, a: RectAlgo, depth: int, cutoff: int) -> int:
    """Levels taken: one more while levels remain and every dimension that
    the algorithm splits (split factor > 1) still exceeds the cutoff."""
    d = 0
    sizes = [M, K, N]
    splits = [a.m0, a.k0, a.n0]
    while d < depth and all(s > cutoff for s, q in zip(sizes, splits) if q > 1) and max(splits) > 1:
        sizes = [-(-s // q) for s, q in zip(sizes, splits)]
        d += 1
    return d


def _blocks(X: np.ndarray, rows: int, cols: int):
    br, bc = X.shape[0] // rows, X.shape[1] // cols
    return [X[x * br:(x + 1) * br, y * bc:(y + 1) * bc] for x in range(rows) for y in range(cols)]


def _combine(coeffs, blocks, dtype):
    out = np.zeros(blocks[0].shape, dtype=dtype)
    for c, X in zip(coeffs, blocks):
        if c != 0:
            out += dtype.type(c) * X if c != 1 else X
    return out


def _fast_divisible(A, B, a: RectAlgo, d: int):
    if d == 0:
        return classical_mm(A, B)
    dtype = np.result_type(A.dtype, B.dtype)
    Ab = _blocks(A, a.m0, a.k0)
    Bb = _blocks(B, a.k0, a.n0)
    C = np.zeros((A.shape[0], B.shape[1]), dtype=dtype)
    Cb = _blocks(C, a.m0, a.n0)
    for r in range(a.R):
        P = _fast_divisible(_combine(a.U[:, r], Ab, dtype), _combine(a.V[:, r], Bb, dtype), a, d - 1)
        for c in range(a.m0 * a.n0):
            w = a.W[c, r]
            if w != 0:
                Cb[c] += dtype.type(w) * P if w != 1 else P
    return C


def fast_gemm(A: np.ndarray, B: np.ndarray, a: RectAlgo, depth: int, cutoff: int = 0,
              alpha=1, beta=0, C=None) -> np.ndarray:
    """alpha (A B) + beta C with A B formed by ``depth`` levels of ``a``
    (recursion as in equation "strassen", products in index order).  Sizes
    that the splits do not divide are zero-padded at the top and the result
    cropped; beta = 0 ignores C (which may then be None)."""
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("inner dimensions differ")
    d = levels_taken(M, K, N, a, depth, cutoff)
    dtype = np.result_type(A.dtype, B.dtype)
    qm, qk, qn = a.m0 ** d, a.k0 ** d, a.n0 ** d
    Mp, Kp, Np = qm * -(-M // qm), qk * -(-K // qk), qn * -(-N // qn)
    Ap = np.zeros((Mp, Kp), dtype=dtype)
    Bp = np.zeros((Kp, Np), dtype=dtype)
    Ap[:M, :K] = A
    Bp[:K, :N] = B
    P = _fast_divisible(Ap, Bp, a, d)[:M, :N]
    out = P if alpha == 1 else dtype.type(alpha) * P
    if beta != 0:
        out = out + dtype.type(beta) * np.asarray(C, dtype=dtype)
    return out
