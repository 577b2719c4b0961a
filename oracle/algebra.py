"""Oracle: algebra of bilinear fast matrix-multiplication algorithms.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

An algorithm <p,p,p;R> is three integer (or rational) matrices U, V, W of
shape p^2 x R.  Section 2 of the paper (equation "strassen") defines how they
act on a product C = A B partitioned by the split factor p into blocks with a
single row-major index (A_k, k = i*p + j, the partition equations of
Section 2):

    T_r = sum_k U[k, r] A_k,   S_r = sum_l V[l, r] B_l,   P_r = T_r S_r,
    C_c = sum_r W[c, r] P_r.

Canonical form used here: row c of W is the coefficient row of C_c (C indexed
row-major).  The paper prints Strassen's c^t with its rows labelled
C_0, C_2, C_1, C_3, i.e. the printed row t gives the coefficients of the C
block whose 2-d index is the transpose of t's; ``canonical`` undoes that.

Every routine is written for clarity, in exact integer arithmetic (Python ints
or int64), and pinned by the not-gpu tests against the paper's worked
example, brute-force Brent equations, the textbook product and planted
mistakes.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np


@dataclass(frozen=True)
class Algo:
    """A canonical <p,p,p;R> algorithm: U, V, W are p^2 x R int64 arrays."""
    p: int
    R: int
    U: np.ndarray
    V: np.ndarray
    W: np.ndarray


def _int_matrix(x) -> np.ndarray:
    a = np.asarray(x)
    if a.dtype.kind == "f":
        if not np.all(a == np.round(a)):
            raise ValueError("oracle algebra handles integer coefficients only")
        a = np.round(a)
    return a.astype(np.int64)


def transpose_index(t: int, p: int) -> int:
    """Row-major block index of the transpose of block t in a p x p grid."""
    return (t % p) * p + (t // p)


def canonical(n0: int, U, V, W, w_convention: int) -> Algo:
    """Bring (U, V, W) to the canonical form.

    w_convention 0: row c of W already belongs to C_c (row-major C).
    w_convention 1: DeepMind-style c^t as printed in Section 2; printed row t
    belongs to the C block with the transposed 2-d index, which is how the
    paper's labels C_0, C_2, C_1, C_3 arise for p = 2.
    """
    U = _int_matrix(U)
    V = _int_matrix(V)
    W = _int_matrix(W)
    p2 = n0 * n0
    if U.shape[0] != p2 or V.shape != U.shape or W.shape != U.shape:
        raise ValueError("U, V, W must all be n0^2 x R")
    if w_convention == 1:
        Wc = np.zeros_like(W)
        for t in range(p2):
            Wc[transpose_index(t, n0)] = W[t]
        W = Wc
    elif w_convention != 0:
        raise ValueError("unknown W convention")
    return Algo(n0, U.shape[1], U, V, W)


def brent_violations(alg: Algo) -> int:
    """Count the Brent equations that fail.

    The algorithm computes C = A B for every A, B exactly when, for all block
    indices a = (i, k), b = (k2, j), c = (i2, j2),

        sum_r U[a, r] V[b, r] W[c, r] = [k == k2] [i == i2] [j == j2].

    The left side is evaluated exactly (int64, no overflow at these sizes) for
    all p^6 triples.
    """
    p = alg.p
    p2 = p * p
    t = np.einsum("ar,br,cr->abc", alg.U, alg.V, alg.W)
    want = np.zeros((p2, p2, p2), dtype=np.int64)
    for i in range(p):
        for k in range(p):
            for j in range(p):
                want[i * p + k, k * p + j, i * p + j] = 1
    return int(np.count_nonzero(t != want))


def classical_algo(p: int) -> Algo:
    """The textbook partitioned product (equation "recursion" of Section 2)
    written as an algorithm: one product per (i, k, j) with
    C_{i p + j} += A_{i p + k} B_{k p + j}; R = p^3."""
    R = p ** 3
    U = np.zeros((p * p, R), dtype=np.int64)
    V = np.zeros((p * p, R), dtype=np.int64)
    W = np.zeros((p * p, R), dtype=np.int64)
    r = 0
    for i in range(p):
        for j in range(p):
            for k in range(p):
                U[i * p + k, r] = 1
                V[k * p + j, r] = 1
                W[i * p + j, r] = 1
                r += 1
    return Algo(p, R, U, V, W)


def compose(outer: Algo, inner: Algo) -> Algo:
    """Algorithm of split factor p1*p2 obtained by applying ``outer`` first and
    ``inner`` to each of its products (the Kronecker construction of
    Section 2, left factor = first split).

    Block (I, J) of the p1*p2 grid is block (i2, j2) inside block (i1, j1) of
    the outer grid, with I = i1*p2 + i2 and J = j1*p2 + j2.  Its coefficient
    for product r = r1*R2 + r2 is the outer coefficient of (i1, j1) times the
    inner coefficient of (i2, j2).  This is the Kronecker product of the
    factor matrices with the rows re-indexed from the nested order to the
    row-major order of the finer grid.
    """
    p1, p2 = outer.p, inner.p
    p = p1 * p2
    R = outer.R * inner.R

    def kron_rows(X1, X2):
        out = np.zeros((p * p, R), dtype=np.int64)
        for i1 in range(p1):
            for j1 in range(p1):
                for i2 in range(p2):
                    for j2 in range(p2):
                        row = (i1 * p2 + i2) * p + (j1 * p2 + j2)
                        out[row] = np.kron(X1[i1 * p1 + j1], X2[i2 * p2 + j2])
        return out

    return Algo(p, R, kron_rows(outer.U, inner.U), kron_rows(outer.V, inner.V),
                kron_rows(outer.W, inner.W))


def power(alg: Algo, d: int) -> Algo:
    """``alg`` composed with itself d times (d >= 1): the one-level algorithm
    of split factor p^d that equals d levels of recursion."""
    out = alg
    for _ in range(d - 1):
        out = compose(out, alg)
    return out


def _int_inverse(M: np.ndarray) -> np.ndarray:
    """Exact inverse of a unimodular integer matrix (Gauss-Jordan over the
    rationals); raises if M is not invertible over the integers."""
    n = M.shape[0]
    a = [[Fraction(int(M[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        piv = next((r for r in range(c, n) if a[r][c] != 0), None)
        if piv is None:
            raise ValueError("singular matrix")
        a[c], a[piv] = a[piv], a[c]
        f = a[c][c]
        a[c] = [x / f for x in a[c]]
        for r in range(n):
            if r != c and a[r][c] != 0:
                g = a[r][c]
                a[r] = [x - g * y for x, y in zip(a[r], a[c])]
    inv = np.array([[a[i][n + j] for j in range(n)] for i in range(n)], dtype=object)
    if any(x.denominator != 1 for x in inv.flat):
        raise ValueError("inverse is not integer: matrix is not unimodular")
    return np.array([[int(x) for x in row] for row in inv], dtype=np.int64)


def rebase(alg: Algo, X, Y, Z) -> Algo:
    """Transform an algorithm by invertible p x p integer matrices X, Y, Z.

    Apply ``alg`` to A' = X A Y^-1 and B' = Y B Z^-1; the product is
    X (A B) Z^-1, so A B = X^-1 (A' B') Z.  Writing column r of U as a p x p
    matrix U_r (T_r = <U_r, A>, the Frobenius inner product), this gives the
    algorithm
        U'_r = X^T U_r Y^-T,  V'_r = Y^T V_r Z^-T,  W'_r = X^-1 W_r Z,
    which again computes C = A B.  Unimodular X, Y, Z keep it integer.
    """
    p = alg.p
    X = _int_matrix(X)
    Y = _int_matrix(Y)
    Z = _int_matrix(Z)
    Xi, Yi, Zi = _int_inverse(X), _int_inverse(Y), _int_inverse(Z)
    U2 = np.zeros_like(alg.U)
    V2 = np.zeros_like(alg.V)
    W2 = np.zeros_like(alg.W)
    for r in range(alg.R):
        Ur = alg.U[:, r].reshape(p, p)
        Vr = alg.V[:, r].reshape(p, p)
        Wr = alg.W[:, r].reshape(p, p)
        U2[:, r] = (X.T @ Ur @ Yi.T).reshape(-1)
        V2[:, r] = (Y.T @ Vr @ Zi.T).reshape(-1)
        W2[:, r] = (Xi @ Wr @ Z).reshape(-1)
    return Algo(p, alg.R, U2, V2, W2)


def single_coefficient_columns(X: np.ndarray) -> list:
    """Columns with exactly one non-zero coefficient: the combined operand is
    a (scaled) view of one block and need not be formed."""
    return [r for r in range(X.shape[1]) if np.count_nonzero(X[:, r]) == 1]
