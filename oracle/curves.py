"""Oracle for the space-filling orders inside a block.  Test infrastructure only.

Hilbert order (Sections 3.2 and 4.1, fig:Hilbert) and Z-Morton order (Section 3.1, fig:ZMorton)
on a 2^k x 2^k block, for a cell at local (row r, column c).

Hilbert: the curve of side 2^k is built recursively from four copies of the curve of side
2^(k-1), with orientation changes per quadrant.  Writing x = column and y = row, the four copies
are visited in the order
    q=0: lower-left  quadrant (x < h, y < h), copy transposed: (x, y) -> (y, x)
    q=1: quadrant x < h, y >= h, copy shifted by (0, h)
    q=2: quadrant x >= h, y >= h, copy shifted by (h, h)
    q=3: quadrant x >= h, y < h, copy reflected through the anti-diagonal (x, y) -> (h-1-y, h-1-x)
         and shifted by (h, 0)
with h = 2^(k-1) (rows grow downwards, so "y < h" is the top half of the drawn block).  The
index of a cell is q * h^2 plus the index of the untransformed cell inside that copy.  This is
the classical construction (Hilbert 1891); the figure's 2x2, 4x4 and 8x8 orders pin it.

Z-Morton: quadrants top-left, top-right, bottom-left, bottom-right, recursively.
"""
import numpy as np


def hilbert_index(k, r, c):
    """Hilbert index of local cell (r, c) in a 2^k x 2^k block (scalar, recursive)."""
    x, y = int(c), int(r)
    d = 0
    while k > 0:
        h = 1 << (k - 1)
        if x < h and y < h:
            q, x, y = 0, y, x
        elif x < h:
            q, y = 1, y - h
        elif y >= h:
            q, x, y = 2, x - h, y - h
        else:
            q, x, y = 3, h - 1 - y, h - 1 - (x - h)
        d += q * h * h
        k -= 1
    return d


def hilbert_index_array(k, r, c):
    """Vectorised hilbert_index over arrays r, c (same recursion, all cells at once)."""
    x = np.asarray(c, np.int64).copy()
    y = np.asarray(r, np.int64).copy()
    d = np.zeros(x.shape, np.int64)
    while k > 0:
        h = 1 << (k - 1)
        q0 = (x < h) & (y < h)
        q1 = (x < h) & (y >= h)
        q2 = (x >= h) & (y >= h)
        q3 = (x >= h) & (y < h)
        nx = np.where(q0, y, np.where(q1, x, np.where(q2, x - h, h - 1 - y)))
        ny = np.where(q0, x, np.where(q1, y - h, np.where(q2, y - h, h - 1 - (x - h))))
        d += np.where(q0, 0, np.where(q1, 1, np.where(q2, 2, 3))) * (h * h)
        x, y = nx, ny
        k -= 1
    return d


def hilbert_order(k):
    """Cells (row, col) of a 2^k block in Hilbert visiting order (brute force inversion)."""
    side = 1 << k
    cells = [(r, c) for r in range(side) for c in range(side)]
    return sorted(cells, key=lambda rc: hilbert_index(k, rc[0], rc[1]))


def zmorton_index(k, r, c):
    """Z-Morton index of local cell (r, c): quadrant TL, TR, BL, BR recursively."""
    r, c = int(r), int(c)
    d = 0
    while k > 0:
        h = 1 << (k - 1)
        q = 2 * (r >= h) + (c >= h)
        d += q * h * h
        r, c = r % h, c % h
        k -= 1
    return d


def zmorton_index_array(k, r, c):
    """zmorton_index over arrays: the same quadrant descent (TL, TR, BL, BR, Section 3.1), level by
    level from the top, applied to every cell at once."""
    r = np.asarray(r, np.int64).copy()
    c = np.asarray(c, np.int64).copy()
    d = np.zeros(r.shape, np.int64)
    while k > 0:
        h = 1 << (k - 1)
        q = 2 * (r >= h) + (c >= h)
        d += q * h * h
        r %= h
        c %= h
        k -= 1
    return d


def zmorton_order(k):
    side = 1 << k
    cells = [(r, c) for r in range(side) for c in range(side)]
    return sorted(cells, key=lambda rc: zmorton_index(k, rc[0], rc[1]))
