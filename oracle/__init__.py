"""CPU oracle for the fast bilinear matrix product.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct implementation
used by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark to judge the HIP path.  The product library never imports, links
or calls anything in this package, and this package shares no code with it.

Parity status: every function here is pinned by not-gpu tests against facts
fixed by the paper or by mathematics (the paper's worked example, Brent
equations, the textbook product, brute force on tiny inputs, closed forms,
planted mistakes).  That includes ``rows_reference``, the sampled-row form of
the definition that checks every full-size product: it is pinned row by row
against a brute-force triple loop, exact sums, closed forms (identity,
permutation, rank one) and planted mistakes (a transposed operand, shifted
rows).  The exact integer product (float64 BLAS below the 2^53 bound, the
integer loop above it) is pinned against the integer loop, Python's big
integers and a planted case where the float path would round.  The
rectangular module (``rect``: <m0,k0,n0;R> algorithms, direct sums, Kronecker
products and C = alpha A B + beta C) is pinned the same way in
tests/test_oracle_rect_pins.py.  No function is parity-unpinned.
"""
from .algebra import (Algo, brent_violations, canonical, classical_algo, compose, power,  # noqa: F401
                      rebase, single_coefficient_columns, transpose_index)
from .matmul import (classical_mm, componentwise_error, fast_mm, fast_mm_divisible,  # noqa: F401
                     flops, levels_taken, max_scaled_error, rel_fro_error, rows_reference)
from . import rect  # noqa: F401,E402
