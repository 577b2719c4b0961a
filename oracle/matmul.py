"""Oracle: classical and fast matrix products on the CPU.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

* ``classical_mm``  the plain definition C_ij = sum_k A_ik B_kj (Section 2),
  computed by numpy's matmul: OpenBLAS for float64; for integer operands
  exactly, by OpenBLAS on the values as float64 when K max|A| max|B| < 2^53
  (then every product and partial sum is an integer below 2^53, which float64
  holds exactly, so no sum rounds in any order) and by numpy's integer loop
  otherwise.
* ``fast_mm``       the recursive fast algorithm of equation "strassen"
  (Section 2): form T_r and S_r from the coefficient columns, multiply
  recursively, and distribute P_r into the C blocks, product by product in
  index order (the sequential evaluation of the instruction list described
  in Section 3).
* error metrics used by every accuracy report.

Readings of what the paper leaves open (depth and cutoff are not defined
there; sizes that the split factor does not divide are avoided there):
recursion continues while levels remain and the current size exceeds the
cutoff; a size that p^d does not divide is padded with zero rows and columns
at the top level and the result is cropped.
"""
from __future__ import annotations

import math

import numpy as np

from .algebra import Algo


def _int_bound(X: np.ndarray) -> int:
    """max |x| over an integer array, as a Python int (0 if empty)."""
    return max(abs(int(X.max())), abs(int(X.min()))) if X.size else 0


def exact_in_float64(A: np.ndarray, B: np.ndarray) -> bool:
    """Integer operands whose products and partial sums of A B all stay below
    2^53 in magnitude (K max|A| max|B| < 2^53)."""
    if not (np.issubdtype(A.dtype, np.integer) and np.issubdtype(B.dtype, np.integer)):
        return False
    return A.shape[1] * _int_bound(A) * _int_bound(B) < 2 ** 53


def classical_mm(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B by definition (library matmul in the element type given;
    integer operands exactly, see the module docstring)."""
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shape mismatch")
    if exact_in_float64(A, B):
        C = np.matmul(A.astype(np.float64), B.astype(np.float64))
        return C.astype(np.result_type(A.dtype, B.dtype))
    return np.matmul(A, B)


def _block(X: np.ndarray, k: int, p: int, m: int) -> np.ndarray:
    """Block k of the p x p row-major partition of X (block size m)."""
    i, j = divmod(k, p)
    return X[i * m:(i + 1) * m, j * m:(j + 1) * m]


def _combine(coeffs: np.ndarray, blocks, m: int, dtype) -> np.ndarray:
    """sum_k coeffs[k] * blocks[k], over non-zero coefficients in k order."""
    out = np.zeros((m, m), dtype=dtype)
    for k, c in enumerate(coeffs):
        if c != 0:
            out += dtype.type(c) * blocks[k] if c != 1 else blocks[k]
    return out


def fast_mm_divisible(A: np.ndarray, B: np.ndarray, alg: Algo, depth: int, cutoff: int) -> np.ndarray:
    """Recursive fast product; requires p^levels | n for the levels taken."""
    n = A.shape[0]
    if depth <= 0 or n <= cutoff:
        return classical_mm(A, B)
    p = alg.p
    if n % p:
        raise ValueError("size not divisible by the split factor")
    m = n // p
    dtype = np.result_type(A.dtype, B.dtype)
    Ab = [_block(A, k, p, m) for k in range(p * p)]
    Bb = [_block(B, k, p, m) for k in range(p * p)]
    C = np.zeros((n, n), dtype=dtype)
    Cb = [_block(C, k, p, m) for k in range(p * p)]
    for r in range(alg.R):
        T = _combine(alg.U[:, r], Ab, m, dtype)
        S = _combine(alg.V[:, r], Bb, m, dtype)
        P = fast_mm_divisible(T, S, alg, depth - 1, cutoff)
        for c in range(p * p):
            w = alg.W[c, r]
            if w != 0:
                Cb[c] += dtype.type(w) * P if w != 1 else P
    return C


def levels_taken(n: int, p: int, depth: int, cutoff: int) -> int:
    """Number of recursion levels taken for an n x n product: a level is
    taken while levels remain and the current (padded) size exceeds the
    cutoff."""
    d = 0
    size = n
    while d < depth and size > cutoff:
        size = -(-size // p)
        d += 1
    return d


def fast_mm(A: np.ndarray, B: np.ndarray, alg: Algo, depth: int, cutoff: int = 0) -> np.ndarray:
    """C = A B by ``depth`` levels of ``alg``.  A size that p^levels does not
    divide is zero-padded at the top level and the result cropped."""
    n = A.shape[0]
    if A.shape != (n, n) or B.shape != (n, n):
        raise ValueError("square operands of equal size expected")
    d = levels_taken(n, alg.p, depth, cutoff)
    if d == 0:
        return classical_mm(A, B)
    q = alg.p ** d
    npad = q * (-(-n // q))
    if npad == n:
        return fast_mm_divisible(A, B, alg, d, cutoff)
    dtype = np.result_type(A.dtype, B.dtype)
    Ap = np.zeros((npad, npad), dtype=dtype)
    Bp = np.zeros((npad, npad), dtype=dtype)
    Ap[:n, :n] = A
    Bp[:n, :n] = B
    # The padded size is a multiple of p^d and every level above the last
    # still exceeds the cutoff, so exactly d levels are taken on it.
    return fast_mm_divisible(Ap, Bp, alg, d, cutoff)[:n, :n]


def rel_fro_error(C_hat: np.ndarray, C_ref: np.ndarray) -> float:
    """Normwise relative error ||C_hat - C_ref||_F / ||C_ref||_F in float64."""
    d = np.asarray(C_hat, dtype=np.float64) - np.asarray(C_ref, dtype=np.float64)
    den = np.linalg.norm(np.asarray(C_ref, dtype=np.float64))
    return float(np.linalg.norm(d) / den) if den > 0 else float(np.linalg.norm(d))


def max_scaled_error(C_hat, C_ref, A, B) -> float:
    """max |C_hat - C_ref| / (max|A| max|B|)  (a normwise max-entry metric)."""
    d = np.abs(np.asarray(C_hat, np.float64) - np.asarray(C_ref, np.float64)).max()
    return float(d / (np.abs(A).max() * np.abs(B).max()))


def componentwise_error(C_hat, C_ref, A, B) -> float:
    """max_ij |C_hat - C_ref|_ij / (|A| |B|)_ij  (componentwise metric)."""
    den = classical_mm(np.abs(np.asarray(A, np.float64)), np.abs(np.asarray(B, np.float64)))
    d = np.abs(np.asarray(C_hat, np.float64) - np.asarray(C_ref, np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, d / den, 0.0)
    return float(q.max())


def rows_reference(A: np.ndarray, B: np.ndarray, rows) -> np.ndarray:
    """Exact-definition rows C[i, :] = A[i, :] B for sampled i, returned as
    float64 (integer operands: the exact integer rows of classical_mm)."""
    A = np.asarray(A)
    B = np.asarray(B)
    if np.issubdtype(A.dtype, np.integer) and np.issubdtype(B.dtype, np.integer):
        return classical_mm(A[rows], B).astype(np.float64)
    return np.matmul(np.asarray(A, np.float64)[rows], np.asarray(B, np.float64))


def flops(n: int) -> float:
    """Classical operation count 2 n^3 used for effective GFLOP/s."""
    return 2.0 * float(n) ** 3


def unit_roundoff(bits: int = 53) -> float:
    return math.ldexp(1.0, -bits)
