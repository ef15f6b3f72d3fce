"""Oracle for the BCOHC and BCOHCH formats (Section 3.2 and its hybrid variants): static row
partitions with about equal entry counts, blocks of beta x beta in Hilbert order inside each
partition, and inside every block the entries either row by row (BCOHC, compressed triplets) or in
Hilbert order over the partition's entries (BCOHCH).  Test infrastructure.

Readings where the paper is silent (its workers are CPU threads):
  * a partition is a range of whole rows; row r starts a partition when r is 0, when r is a
    multiple of WINDOW rows (so that a partition's output rows fit one on-chip window), or when
    the number of raw triplets in rows before r and before r - 1 fall in different multiples of
    target = max(2^16, ceil(E / 2048));
  * the block grid is the CSB grid (block row r >> k, block column c >> k), its Hilbert order is
    the curve of level K2 = ceil(log2(max(block rows, block columns))) with x = block column,
    y = block row (the orientation of the paper's figure);
  * BCOHCH sorts a partition's entries by the Hilbert index of level K2 + k of (row, col); that
    index's leading 2*K2 bits are the block's Hilbert index, so blocks stay in Hilbert order.
"""
import numpy as np

from . import curves

WINDOW = 8192


def ceil_log2(v):
    v = int(v)
    return 0 if v <= 1 else (v - 1).bit_length()


def target(E):
    return max(1 << 16, -(-int(E) // 2048))


def partition_starts(m, raw_rows, E):
    """First row of every partition, followed by m."""
    cnt = np.bincount(np.asarray(raw_rows, np.int64), minlength=m)[:m] if m > 0 else np.zeros(0)
    cum = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    t = target(E)
    r = np.arange(m, dtype=np.int64)
    start = (r == 0) | (r % WINDOW == 0)
    start[1:] |= (cum[1:m] // t) != (cum[0:m - 1] // t)
    return np.concatenate([np.flatnonzero(start), [m]]).astype(np.int64)


def order(m, n, k, rows, cols, starts, hilbert_entries):
    """Storage order of canonical triplets (rows, cols): returns the permutation and, per entry,
    its partition, block row and block column."""
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    part = np.searchsorted(starts, rows, side="right") - 1
    br, bc = rows >> k, cols >> k
    nbr = max(1, -(-m // (1 << k)))
    nbc = max(1, -(-n // (1 << k)))
    K2 = ceil_log2(max(nbr, nbc))
    if hilbert_entries:
        h = curves.hilbert_index_array(K2 + k, rows, cols)
        perm = np.lexsort((h, part))
    else:
        hb = curves.hilbert_index_array(K2, br, bc)
        perm = np.lexsort((cols, rows, hb, part))
    return perm, part, br, bc


def decode(k, blk_ptr, blk_coord, packed, values):
    """Triplets in storage order from the block table (start pointers, (br << 16) | bc) and the
    packed local indices ((lr << 16) | lc)."""
    blk_ptr = np.asarray(blk_ptr, np.int64)
    coord = np.asarray(blk_coord, np.int64) & 0xFFFFFFFF
    cntb = np.diff(blk_ptr)
    br = np.repeat(coord >> 16, cntb)
    bc = np.repeat(coord & 0xFFFF, cntb)
    p = np.asarray(packed, np.int64) & 0xFFFFFFFF
    return (br << k) + (p >> 16), (bc << k) + (p & 0xFFFF), np.asarray(values, np.float64)


def check_bcoh(m, n, k, raw_rows, E, part_row, part_blk, blk_ptr, blk_coord, packed, values,
               crow, ccol, cval, hilbert_entries):
    """Structural and exact check of converted arrays against canonical triplets (crow, ccol,
    cval): partitions, block table, storage order and values bit for bit."""
    starts = partition_starts(m, raw_rows, E)
    assert np.array_equal(np.asarray(part_row, np.int64), starts), "partition rows"
    blk_ptr = np.asarray(blk_ptr, np.int64)
    nb = len(blk_ptr) - 1
    assert blk_ptr[0] == 0 and blk_ptr[-1] == len(cval) and np.all(np.diff(blk_ptr) > 0)
    rows, cols, vals = decode(k, blk_ptr, blk_coord, packed, values)
    perm, part, br, bc = order(m, n, k, crow, ccol, starts, hilbert_entries)
    assert np.array_equal(rows, np.asarray(crow, np.int64)[perm]), "rows in storage order"
    assert np.array_equal(cols, np.asarray(ccol, np.int64)[perm]), "columns in storage order"
    assert np.array_equal(vals.view(np.int64), np.asarray(cval, np.float64)[perm].view(np.int64))
    # blocks: maximal runs of one (partition, block row, block column)
    bpart = part[perm][blk_ptr[:-1]] if nb else np.zeros(0, np.int64)
    key = np.stack([part[perm], br[perm], bc[perm]], axis=1)
    if len(key):
        new = np.concatenate([[True], np.any(key[1:] != key[:-1], axis=1)])
        assert np.array_equal(np.flatnonzero(new), blk_ptr[:-1]), "block starts"
    part_blk = np.asarray(part_blk, np.int64)
    P = len(starts) - 1
    assert len(part_blk) == P + 1 and part_blk[-1] == nb
    want = np.searchsorted(bpart, np.arange(P + 1), side="left")
    assert np.array_equal(part_blk, want), "first block of each partition"
