"""lpx: transformation-record code variants of the batched dense contraction
out[k,e,i] = sum_j D[k][i][j] u[e][j] (and dense GEMM) for MI355X (gfx950).

The compute path is the C-ABI library ``liblpx.so`` (hand-written HIP
kernels); ``paper_1405_7470_amd.lpx`` is its thin ctypes binding.  Importing
this package loads nothing; ``inputs`` holds the seeded synthetic-data
generators.
"""
__all__ = ["inputs", "lpx"]
