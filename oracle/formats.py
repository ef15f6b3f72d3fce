"""Oracle decoders and structural checks for converted formats.  Test infrastructure only.

A conversion is correct when decoding the converted arrays gives back exactly the canonical
triplets (same coordinates, bit-identical values) and the format's ordering rules hold.

CRS (Section 2): row_ptr[m+1] non-decreasing from 0 to nnz; columns ascend inside a row.
CSB (Section 3.1) and CSB with Hilbert order inside blocks, CSBH (Section 4.1): beta x beta blocks;
blk_ptr has
one entry per block in row-wise block order plus a final nnz; inside a block each entry's local
row and column are packed into one 32-bit word, row in the upper 16 bits; entries of a block
follow the Hilbert order of their local (row, col).
"""
import numpy as np

from .curves import hilbert_index_array, zmorton_index


def decode_crs(row_ptr):
    """Row index of every stored entry of a CRS matrix."""
    row_ptr = np.asarray(row_ptr, np.int64)
    return np.repeat(np.arange(len(row_ptr) - 1, dtype=np.int64), np.diff(row_ptr))


def check_crs(m, n, row_ptr, col, val, canon_row, canon_col, canon_val):
    """Raise AssertionError unless the CRS arrays equal the canonical triplets exactly."""
    row_ptr = np.asarray(row_ptr, np.int64)
    assert row_ptr.shape == (m + 1,), "row_ptr length"
    assert row_ptr[0] == 0 and row_ptr[-1] == len(col) == len(val), "row_ptr ends"
    assert np.all(np.diff(row_ptr) >= 0), "row_ptr not monotone"
    rows = decode_crs(row_ptr)
    assert len(rows) == len(canon_row), "entry count"
    assert np.array_equal(rows, np.asarray(canon_row, np.int64)), "row indices"
    assert np.array_equal(np.asarray(col, np.int64), np.asarray(canon_col, np.int64)), "columns"
    a = np.asarray(val, np.float64).view(np.int64)
    b = np.asarray(canon_val, np.float64).view(np.int64)
    assert np.array_equal(a, b), "values differ bitwise"


def beta_blocks(m, n, log2_beta):
    beta = 1 << log2_beta
    return (m + beta - 1) // beta, (n + beta - 1) // beta


def decode_csbh(m, n, log2_beta, blk_ptr, packed, val):
    """Decode CSBH arrays to triplets in storage order: (row, col, val, block, local_r, local_c)."""
    nbr, nbc = beta_blocks(m, n, log2_beta)
    blk_ptr = np.asarray(blk_ptr, np.int64)
    assert blk_ptr.shape == (nbr * nbc + 1,), "blk_ptr length"
    blk = np.repeat(np.arange(nbr * nbc, dtype=np.int64), np.diff(blk_ptr))
    p = np.asarray(packed, np.uint32).astype(np.int64)
    lr = p >> 16
    lc = p & 0xFFFF
    row = (blk // nbc) * (1 << log2_beta) + lr
    col = (blk % nbc) * (1 << log2_beta) + lc
    return row, col, np.asarray(val, np.float64), blk, lr, lc


def check_csbh(m, n, log2_beta, blk_ptr, packed, val, canon_row, canon_col, canon_val):
    """CSB with Hilbert order inside blocks (Section 4.1)."""
    check_csb(m, n, log2_beta, blk_ptr, packed, val, canon_row, canon_col, canon_val, "hilbert")


def check_csb(m, n, log2_beta, blk_ptr, packed, val, canon_row, canon_col, canon_val,
              order="zmorton"):
    """Raise AssertionError unless the CSB arrays hold exactly the canonical triplets, blocks are
    in row-wise order, and entries inside each block follow the block order ('hilbert' or
    'zmorton', Section 3.1) strictly."""
    blk_ptr = np.asarray(blk_ptr, np.int64)
    assert blk_ptr[0] == 0 and blk_ptr[-1] == len(packed) == len(val), "blk_ptr ends"
    assert np.all(np.diff(blk_ptr) >= 0), "blk_ptr not monotone"
    row, col, v, blk, lr, lc = decode_csbh(m, n, log2_beta, blk_ptr, packed, val)
    beta = 1 << log2_beta
    assert np.all(lr < beta) and np.all(lc < beta), "local index >= beta"
    assert np.all(row < m) and np.all(col < n), "entry outside the matrix"
    if order == "hilbert":
        h = hilbert_index_array(log2_beta, lr, lc)
    else:
        h = np.array([zmorton_index(log2_beta, a, b) for a, b in zip(lr, lc)], dtype=np.int64)
    same = blk[1:] == blk[:-1]
    assert np.all(h[1:][same] > h[:-1][same]), "not strictly increasing %s order in a block" % order
    # compare as multisets keyed by (row, col); coordinates are unique after summing repeats
    order = np.lexsort((col, row))
    assert np.array_equal(row[order], np.asarray(canon_row, np.int64)), "rows"
    assert np.array_equal(col[order], np.asarray(canon_col, np.int64)), "cols"
    a = v[order].view(np.int64)
    b = np.asarray(canon_val, np.float64).view(np.int64)
    assert np.array_equal(a, b), "values differ bitwise"


# ---------------------------------------------------------------- CSB over ranked rows and columns
#
# CSBR keeps the block idea of Section 3.1 (a block row's slice of y stays on chip, and a block
# reads only a range of x) with rows and columns renumbered; both are pure reorderings of the
# stored entries:
#   * rows are ranked by decreasing number of raw triplets, ties by increasing row; only rows with
#     at least one triplet get a rank (the others have y = 0);
#   * block rows (panels) are 2^pb consecutive row ranks;
#   * columns are ranked by decreasing number of raw triplets; among columns with equal counts,
#     by increasing first panel (the least panel among its triplets), then increasing last panel
#     (the greatest), then increasing column; only columns with at least one triplet get a rank;
#   * a block is (panel, 2^rb consecutive column ranks); blocks are stored panel by panel, segment
#     by segment; inside a block the entries are ordered by column rank, then row rank, and each
#     packs (column rank mod 2^rb) << pb | (row rank mod 2^pb).
# The product is the same y = A x; only the summation order differs.

CSBR_PB = 14
CSBR_RB = 18


def csbr_row_order(m, raw_rows):
    """Row of each row rank: decreasing raw triplet count, ties by increasing row index."""
    cnt = np.bincount(np.asarray(raw_rows, np.int64), minlength=m)[:m]
    r = np.flatnonzero(cnt > 0)
    return r[np.lexsort((r, -cnt[r]))].astype(np.int64)


def csbr_col_order(m, n, raw_rows, raw_cols, pb=CSBR_PB):
    """Column of each column rank: decreasing raw triplet count, then increasing first panel,
    increasing last panel and increasing column index (panel of row r = its row rank >> pb)."""
    rows = np.asarray(raw_rows, np.int64)
    cols = np.asarray(raw_cols, np.int64)
    ranked = csbr_row_order(m, rows)
    row_rank = np.zeros(m, np.int64)
    row_rank[ranked] = np.arange(len(ranked))
    cnt = np.bincount(cols, minlength=n)[:n]
    first = np.full(n, np.iinfo(np.int64).max, np.int64)
    last = np.full(n, -1, np.int64)
    np.minimum.at(first, cols, row_rank[rows] >> pb)
    np.maximum.at(last, cols, row_rank[rows] >> pb)
    c = np.flatnonzero(cnt > 0)
    return c[np.lexsort((c, last[c], first[c], -cnt[c]))].astype(np.int64)


def decode_csbr(row_order, blk_ptr, packed, col_order, pb=CSBR_PB, rb=CSBR_RB):
    """Triplet coordinates in storage order: (row, col, panel, column rank, row rank)."""
    blk_ptr = np.asarray(blk_ptr, np.int64)
    row_order = np.asarray(row_order, np.int64)
    npan = max(1, -(-len(row_order) // (1 << pb)))
    nblk = len(blk_ptr) - 1
    assert nblk % npan == 0, "blk_ptr length is not panels x segments + 1"
    nseg = nblk // npan
    blk = np.repeat(np.arange(nblk, dtype=np.int64), np.diff(blk_ptr))
    panel, seg = blk // nseg, blk % nseg
    p = np.asarray(packed, np.int64) & 0xFFFFFFFF
    crank = (seg << rb) + (p >> pb)
    rrank = (panel << pb) + (p & ((1 << pb) - 1))
    col_order = np.asarray(col_order, np.int64)
    assert np.all(crank < len(col_order)), "column rank beyond the ranked columns"
    assert np.all(rrank < len(row_order)), "row rank beyond the ranked rows"
    return row_order[rrank], col_order[crank], panel, crank, rrank


def check_csbr(m, n, raw_rows, raw_cols, blk_ptr, packed, val, col_order, row_order, canon_row,
               canon_col, canon_val, pb=CSBR_PB, rb=CSBR_RB):
    """Raise AssertionError unless the CSBR arrays hold exactly the canonical triplets in the
    format's storage order: both rankings, the segment count, (panel, column rank, row rank)
    strictly increasing along storage, and bit-identical values."""
    want_rows = csbr_row_order(m, raw_rows)
    assert np.array_equal(np.asarray(row_order, np.int64), want_rows), "row ranking"
    want_cols = csbr_col_order(m, n, raw_rows, raw_cols, pb)
    assert np.array_equal(np.asarray(col_order, np.int64), want_cols), "column ranking"
    nr = len(want_cols)
    rbits = max(rb, (max(nr, 1) - 1).bit_length())
    npan = max(1, -(-len(want_rows) // (1 << pb)))
    blk_ptr = np.asarray(blk_ptr, np.int64)
    assert len(blk_ptr) == npan * (1 << (rbits - rb)) + 1, "segments per panel"
    assert blk_ptr[0] == 0 and blk_ptr[-1] == len(packed) == len(val), "blk_ptr ends"
    assert np.all(np.diff(blk_ptr) >= 0), "blk_ptr not monotone"
    row, col, panel, crank, rrank = decode_csbr(want_rows, blk_ptr, packed, want_cols, pb, rb)
    key = [(int(a), int(b), int(c)) for a, b, c in zip(panel, crank, rrank)]
    assert all(key[i] < key[i + 1] for i in range(len(key) - 1)), \
        "not in (panel, column rank, row rank) order"
    order = np.lexsort((col, row))
    assert np.array_equal(row[order], np.asarray(canon_row, np.int64)), "rows"
    assert np.array_equal(col[order], np.asarray(canon_col, np.int64)), "cols"
    a = np.asarray(val, np.float64)[order].view(np.int64)
    b = np.asarray(canon_val, np.float64).view(np.int64)
    assert np.array_equal(a, b), "values differ bitwise"
