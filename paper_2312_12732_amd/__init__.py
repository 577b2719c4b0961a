"""mf: fast bilinear matrix multiplication (Strassen-like algorithms given by
their factor matrices U, V, W) on AMD Instinct MI355X.

The compute path is the C-ABI library ``libmf.so`` (include/mf.h) built from
``csrc/`` for gfx950; ``mf`` is its thin Python binding.
"""
