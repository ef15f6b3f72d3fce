"""spx -- sparse matrix-vector multiplication y = A x on AMD MI355X (gfx950).

A from-scratch HIP implementation of the formats and load-balancing strategies studied by
Bergmans, Meerbergen and Vandebril (arXiv 2502.19284): row-split CRS, merge-path CRS and
compressed sparse blocks in Hilbert (CSBH) or Z-Morton (CSB) order, the row-partitioned hybrids
BCOHC / BCOHCH, and compressed sparse blocks over frequency-ranked columns (CSBR), with conversion
from triplets by device radix sort; products with several right-hand sides; batches of many
matrices; and a serving loop over resident matrices.  The C ABI is include/spx.h and include/spx_serve.h; this package is its thin Python
binding.
"""
from .spx import (ARRAYS, FORMATS, LIB_PATH, PLANS, Batch, Matrix, Server,  # noqa: F401
                  SpxError, break_even,
                  convert,
                  header_functions, load, probe_gather, profile_collect, profile_enable,
                  use_torch_allocator, version)
