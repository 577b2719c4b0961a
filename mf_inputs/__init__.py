"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds *data only*: seeded random generators and fast-algorithm
coefficient tables in the raw form in which they are published.  It contains
none of the method's arithmetic (no canonicalisation, no Brent check, no
Kronecker composition, no products); each side does that with its own code.

Workload recipes (all generated in float64 on the host with numpy's PCG64):

* ``uniform(n, seed)``            A[i, j] ~ U[-1, 1]
* ``int_uniform(n, seed)``        A[i, j] ~ U{-8, ..., 8} (int64)
* ``scaled(n, seed)``             D1 * A0 * D2 with A0 ~ U[-1, 1] and D1, D2
                                  diagonal with entries log-uniform in
                                  [1e-4, 1e4] (rows and columns scaled)
* ``batch_sizes(count, seed)``    n_i = 64 * round(exp(U(ln 128, ln 2048)) / 64)
* ``serving_requests(...)``       Poisson arrivals, n log-uniform in
                                  [256, 8192], dtype 70 % fp32 / 30 % fp64
* ``unimodular(p, seed)``         a random integer p x p matrix with
                                  determinant +-1 (product of elementary
                                  shears with +-1 multipliers and an optional
                                  row swap), used to re-base an algorithm
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Fast-algorithm tables, as published.
# ---------------------------------------------------------------------------

# Strassen's <2,2,2;7> exactly as printed in Section 2 of the paper (the
# DeepMind-style factor matrices a, b and c^t).  Rows of ``a`` are A_0..A_3,
# rows of ``b`` are B_0..B_3, columns are the products 0..6.  The rows of
# ``ct`` are printed with the labels C_0, C_2, C_1, C_3 (in that order).
STRASSEN_PAPER = {
    "n0": 2,
    "R": 7,
    "a": [
        [0, 1, 1, 0, 1, 1, 0],
        [0, 0, -1, 1, 0, 0, 0],
        [1, 1, 1, 0, 1, 0, 0],
        [-1, -1, -1, 0, 0, 0, 1],
    ],
    "b": [
        [0, 0, 0, 0, 1, 1, 0],
        [1, 1, 0, 0, 1, 0, 1],
        [0, 1, 1, 1, 1, 0, 0],
        [0, 1, 1, 0, 1, 0, 1],
    ],
    "ct": [
        [0, 0, 0, 1, 0, 1, 0],
        [0, -1, 0, 0, 1, -1, -1],
        [-1, 1, -1, -1, 0, 0, 0],
        [1, 0, 0, 0, 0, 0, 1],
    ],
    "ct_row_labels": [0, 2, 1, 3],
}

# Winograd's variant of Strassen (seven products, fifteen additions when the
# partial sums are shared), written as plain coefficient matrices.  Blocks
# 0..3 are (11, 12, 21, 22); the rows of ``c`` index C row-major.
#   M0 = A11 B11                      M1 = A12 B21
#   M2 = (A11 + A12 - A21 - A22) B22  M3 = A22 (B11 - B12 - B21 + B22)
#   M4 = (A21 + A22)(B12 - B11)       M5 = (A21 + A22 - A11)(B11 - B12 + B22)
#   M6 = (A11 - A21)(B22 - B12)
#   C11 = M0 + M1                     C12 = M0 + M2 + M4 + M5
#   C21 = M0 - M3 + M5 + M6           C22 = M0 + M4 + M5 + M6
WINOGRAD = {
    "n0": 2,
    "R": 7,
    "a": [
        [1, 0, 1, 0, 0, -1, 1],
        [0, 1, 1, 0, 0, 0, 0],
        [0, 0, -1, 0, 1, 1, -1],
        [0, 0, -1, 1, 1, 1, 0],
    ],
    "b": [
        [1, 0, 0, 1, -1, 1, 0],
        [0, 0, 0, -1, 1, -1, -1],
        [0, 1, 0, -1, 0, 0, 0],
        [0, 0, 1, 1, 0, 1, 1],
    ],
    "c": [
        [1, 1, 0, 0, 0, 0, 0],
        [1, 0, 1, 0, 1, 1, 0],
        [1, 0, 0, -1, 0, 1, 1],
        [1, 0, 0, 0, 1, 1, 1],
    ],
}

# Strassen's original 1969 form, blocks 0..3 = (11, 12, 21, 22), C row-major.
#   M0 = (A11 + A22)(B11 + B22)  M1 = (A21 + A22) B11   M2 = A11 (B12 - B22)
#   M3 = A22 (B21 - B11)         M4 = (A11 + A12) B22   M5 = (A21 - A11)(B11 + B12)
#   M6 = (A12 - A22)(B21 + B22)
#   C11 = M0 + M3 - M4 + M6   C12 = M2 + M4   C21 = M1 + M3   C22 = M0 - M1 + M2 + M5
STRASSEN_1969 = {
    "n0": 2,
    "R": 7,
    "a": [
        [1, 0, 1, 0, 1, -1, 0],
        [0, 0, 0, 0, 1, 0, 1],
        [0, 1, 0, 0, 0, 1, 0],
        [1, 1, 0, 1, 0, 0, -1],
    ],
    "b": [
        [1, 1, 0, -1, 0, 1, 0],
        [0, 0, 1, 0, 0, 1, 0],
        [0, 0, 0, 1, 0, 0, 1],
        [1, 0, -1, 0, 1, 0, 1],
    ],
    "c": [
        [1, 0, 0, 1, -1, 0, 1],
        [0, 0, 1, 0, 1, 0, 0],
        [0, 1, 0, 1, 0, 0, 0],
        [1, -1, 1, 0, 0, 1, 0],
    ],
}


def as_float_tables(table):
    """Return (U, V, W, w_convention) as float64 arrays for a table above.

    ``w_convention`` is 1 for the paper's printed c^t (its rows are handed over
    in the printed order) and 0 for tables whose ``c`` rows index C row-major.
    No arithmetic is applied: the rows are passed exactly as written.
    """
    U = np.asarray(table["a"], dtype=np.float64)
    V = np.asarray(table["b"], dtype=np.float64)
    if "ct" in table:
        return U, V, np.asarray(table["ct"], dtype=np.float64), 1
    return U, V, np.asarray(table["c"], dtype=np.float64), 0


# ---------------------------------------------------------------------------
# Seeded generators.
# ---------------------------------------------------------------------------

def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n x n matrix with entries i.i.d. uniform in [-1, 1]."""
    a = rng(seed).uniform(-1.0, 1.0, size=(n, n))
    return a.astype(dtype)


def int_uniform(n: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """n x n int64 matrix with entries i.i.d. uniform in {lo, ..., hi}."""
    return rng(seed).integers(lo, hi + 1, size=(n, n), dtype=np.int64)


def uniform_rect(rows: int, cols: int, seed: int, dtype=np.float64) -> np.ndarray:
    """rows x cols matrix with entries i.i.d. uniform in [-1, 1]."""
    return rng(seed).uniform(-1.0, 1.0, size=(rows, cols)).astype(dtype)


def int_uniform_rect(rows: int, cols: int, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """rows x cols int64 matrix with entries i.i.d. uniform in {lo, ..., hi}."""
    return rng(seed).integers(lo, hi + 1, size=(rows, cols), dtype=np.int64)


def log_uniform_diag(n: int, seed: int, lo: float = 1e-4, hi: float = 1e4) -> np.ndarray:
    """Vector of n scale factors, log-uniform in [lo, hi]."""
    return np.exp(rng(seed).uniform(math.log(lo), math.log(hi), size=n))


def scaled(n: int, seed_a: int, seed_rows: int, seed_cols: int) -> np.ndarray:
    """D1 * A0 * D2: a uniform[-1,1] matrix with rows and columns scaled by
    independent log-uniform factors in [1e-4, 1e4]."""
    a0 = uniform(n, seed_a)
    d1 = log_uniform_diag(n, seed_rows)
    d2 = log_uniform_diag(n, seed_cols)
    return (d1[:, None] * a0) * d2[None, :]


def batch_sizes(count: int = 512, seed: int = 30, lo: int = 128, hi: int = 2048,
                multiple: int = 64) -> list:
    """Sizes log-uniform in [lo, hi], rounded to a multiple of ``multiple``."""
    x = np.exp(rng(seed).uniform(math.log(lo), math.log(hi), size=count))
    return [int(max(lo, min(hi, multiple * round(v / multiple)))) for v in x]


def serving_requests(count: int, seed: int = 40, lo: int = 256, hi: int = 8192,
                     fp32_share: float = 0.7):
    """List of (n, dtype_name) pairs: n log-uniform in [lo, hi] (rounded to an
    integer), dtype 'f32' with probability ``fp32_share`` else 'f64'."""
    g = rng(seed)
    ns = np.exp(g.uniform(math.log(lo), math.log(hi), size=count))
    ds = g.uniform(0.0, 1.0, size=count)
    return [(int(round(v)), "f32" if d < fp32_share else "f64") for v, d in zip(ns, ds)]


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    gaps = rng(seed).exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


def unimodular(p: int, seed: int, shears: int = 3) -> np.ndarray:
    """Random p x p int64 matrix with determinant +-1: a product of ``shears``
    elementary matrices I + s * e_i e_j^T (i != j, s in {-1, +1}), optionally
    followed by a swap of two rows."""
    g = rng(seed)
    m = np.eye(p, dtype=np.int64)
    for _ in range(shears):
        i, j = g.choice(p, size=2, replace=False)
        e = np.eye(p, dtype=np.int64)
        e[i, j] = 1 if g.integers(0, 2) else -1
        m = e @ m
    if p > 1 and g.integers(0, 2):
        i, j = g.choice(p, size=2, replace=False)
        m[[i, j]] = m[[j, i]]
    return m


# SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), used as a
# counter-based generator: element i = 2u - 1, u = top 53 bits of
# mix(seed + (i + 1) * GAMMA) times 2^-53.
_SPLITMIX_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def counter_uniform(count: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Counter-based uniform[-1, 1) values (the serving runtime's operands)."""
    return counter_uniform_at(np.arange(count, dtype=np.uint64), seed, dtype)


def counter_uniform_at(index: np.ndarray, seed: int, dtype=np.float64) -> np.ndarray:
    """Elements `index` (0-based) of counter_uniform(..., seed): element e is
    the SplitMix64 output for counter e + 1, so any subset (say some rows of
    a matrix) can be drawn without the rest.  Works in place on two integer
    arrays (fresh large arrays are slow to fault in on some hosts)."""
    z = np.array(index, dtype=np.uint64)
    t = np.empty_like(z)
    with np.errstate(over="ignore"):
        z += np.uint64(1)
        z *= _SPLITMIX_GAMMA
        z += np.uint64(seed)
        np.right_shift(z, np.uint64(30), out=t)
        z ^= t
        z *= np.uint64(0xBF58476D1CE4E5B9)
        np.right_shift(z, np.uint64(27), out=t)
        z ^= t
        z *= np.uint64(0x94D049BB133111EB)
        np.right_shift(z, np.uint64(31), out=t)
        z ^= t
        np.right_shift(z, np.uint64(11), out=z)
    del t
    u = z.astype(np.float64)
    del z
    u *= 2.0 ** -53
    u *= 2.0
    u -= 1.0
    return u.astype(dtype, copy=False)
