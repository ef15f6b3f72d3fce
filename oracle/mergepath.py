"""Oracle for the merge path (Section 3.3, fig:SPMV-MergePath).  Test infrastructure only.

Two sorted lists A and B are merged by walking from (0, 0): at each step the smaller of A[i] and
B[j] is consumed; on a tie A is consumed first (the figure takes A=3 before B=3 and A=5 before
B=5).  Thread t of p starts on diagonal t*items, the point of the path with i + j equal to it.

For CRS SpMV, A = row_ptr[1..m] (row ends) and B = 0, 1, ..., nnz-1 (entry indices): consuming
entry k adds data[k]*x[col_ind[k]] to a running value, consuming row end i writes the running
value to y[i] and resets it; a band's unfinished running value is carried out with its row and
added into y afterwards, in band order.
"""
import numpy as np


def walk(A, B):
    """Full merge path: list of (i, j) after 0, 1, ..., len(A)+len(B) steps, and the merged
    sequence as (list_name, value) pairs."""
    i = j = 0
    path = [(0, 0)]
    merged = []
    while i < len(A) or j < len(B):
        if j >= len(B) or (i < len(A) and A[i] <= B[j]):
            merged.append(("A", A[i]))
            i += 1
        else:
            merged.append(("B", B[j]))
            j += 1
        path.append((i, j))
    return path, merged


def splits(A, B, items):
    """Start points of bands of `items` diagonals (last point is the end of the path)."""
    path, _ = walk(A, B)
    total = len(A) + len(B)
    diags = list(range(0, total, items)) + [total]
    return [path[d] for d in diags]


def is_path_point(A, B, i, j):
    """True when (i, j) lies on the merge path: every consumed item precedes every unconsumed one
    under the tie rule, i.e. A[i-1] <= B[j] and B[j-1] < A[i] (missing neighbours ignored)."""
    if i < 0 or j < 0 or i > len(A) or j > len(B):
        return False
    if i > 0 and j < len(B) and not (A[i - 1] <= B[j]):
        return False
    if j > 0 and i < len(A) and not (B[j - 1] < A[i]):
        return False
    return True


def spmv_bands(row_ptr, col_ind, data, x, items):
    """Merge-based CRS SpMV run band by band, sequentially, exactly as described.

    Returns (y, carries) with carries = [(row, value)] per band (row = m when nothing is
    carried).  y already includes the carries, added in band order.
    """
    row_ptr = np.asarray(row_ptr, np.int64)
    m = len(row_ptr) - 1
    nnz = int(row_ptr[-1])
    A = row_ptr[1:]
    total = m + nnz
    y = np.zeros(m, np.float64)
    carries = []
    for d0 in range(0, max(total, 1), items):
        d1 = min(d0 + items, total)
        i, j = _search(A, nnz, d0)
        temp = 0.0
        for _ in range(d1 - d0):
            if j >= nnz or (i < m and A[i] <= j):
                y[i] = temp
                temp = 0.0
                i += 1
            else:
                temp = temp + float(data[j]) * float(x[col_ind[j]])
                j += 1
        carries.append((i, temp) if i < m else (m, 0.0))
    for r, v in carries:
        if r < m:
            y[r] = y[r] + v
    return y, carries


def _search(A, nnz, d):
    # walk-equivalent point on diagonal d for A = row ends, B = 0..nnz-1 (linear scan; small inputs)
    i = j = 0
    while i + j < d:
        if j >= nnz or (i < len(A) and A[i] <= j):
            i += 1
        else:
            j += 1
    return i, j
