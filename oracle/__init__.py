"""CPU oracle for y = A x and the conversions it needs -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct statement of what the GPU library computes, written from
Bergmans, Meerbergen and Vandebril, "Algorithms for Parallel Shared-Memory Sparse Matrix-Vector
Multiplication on Unstructured Matrices" (arXiv 2502.19284).  Only tests/, the smoke check and
the benchmark's CPU-baseline leg may import it.  The GPU library neither imports nor links it,
and the two share no code; both take inputs from the separate `synth` generators.

Modules:
  spmv      canonical triplets, CRS, Algorithm 1 (plain and accurate), triplet SpMV
  curves    Hilbert and Z-Morton orders inside a block
  mergepath merge path walk, split points, band-wise merge SpMV
  formats   decoders and structural checks of converted CRS and CSBH arrays
  measure   block-size rule, break-even count, row-scaled error

Parity pins live in tests/test_oracle_*.py.  The generators' statistics are "parity unpinned"
(the paper prints no numbers for them); only sanity ranges are checked.
"""
from . import curves, formats, measure, mergepath, spmv  # noqa: F401
from ._clib import build  # noqa: F401
