"""Oracle for conversion and y = A x: canonical triplets, CRS, Algorithm 1.  Test infrastructure.

Definitions followed (Bergmans, Meerbergen, Vandebril, arXiv 2502.19284):
  * triplet format and its SpMV equation (Section 2);
  * CRS: entries in row-wise order, row_ptr with m+1 entries (Section 2);
  * Algorithm 1 (CRS SpMV): y = 0, then y[i] += data[k] * x[col_ind[k]] in increasing k.
Readings where the paper is silent: columns ascend inside a row; repeated coordinates are summed
in increasing original index; explicit zeros are kept; y is overwritten.
"""
import numpy as np

from ._clib import lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def canonical_coo(m, n, row, col, val, sum_duplicates=True):
    """Canonical triplets: stable sort by (row, col); each run of equal coordinates summed.

    Returns (row, col, val, perm) where perm is the stable sorting permutation of the input.
    Raises ValueError on an index outside [0, m) x [0, n).
    """
    row = _i32(row)
    col = _i32(col)
    val = _f64(val)
    E = row.shape[0]
    if E and (row.min() < 0 or row.max() >= m or col.min() < 0 or col.max() >= n):
        raise ValueError("index out of range")
    order = np.lexsort((col, row)).astype(np.int64)  # lexsort is a stable sort
    r = row[order]
    c = col[order]
    if not sum_duplicates:
        return r, c, val[order], order
    head = np.ones(E, dtype=bool)
    if E > 1:
        head[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    starts = np.flatnonzero(head).astype(np.int64)
    run_start = np.append(starts, np.int64(E)).astype(np.int64)
    out = np.empty(starts.shape[0], np.float64)
    if starts.shape[0]:
        lib().ref_sum_runs(starts.shape[0], run_start, order, val, out)
    return r[starts], c[starts], out, order


def crs_from_canonical(m, row, col, val):
    """CRS arrays from canonical triplets: row_ptr by counting entries per row (m+1 entries)."""
    counts = np.bincount(_i32(row), minlength=m).astype(np.int64) if len(row) else np.zeros(m, np.int64)
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, _i32(col), _f64(val)


def crs(m, n, row, col, val, sum_duplicates=True):
    """Triplets -> canonical CRS (row_ptr int64[m+1], col_ind int32, data float64)."""
    r, c, v, _ = canonical_coo(m, n, row, col, val, sum_duplicates)
    return crs_from_canonical(m, r, c, v)


def alg1(row_ptr, col_ind, data, x):
    """Algorithm 1 exactly as printed (plain double arithmetic, sequential)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    m = row_ptr.shape[0] - 1
    y = np.empty(m, np.float64)
    lib().ref_alg1(m, row_ptr, _i32(col_ind), _f64(data), _f64(x), y)
    return y


def parcrs(row_ptr, col_ind, data, x, chunk=512):
    """ParCRS (Section 5.1): Algorithm 1 with rows shared among OpenMP threads in dynamic chunks;
    every row is summed in the same order, so the result equals alg1 bit for bit.  Returns
    (y, threads used)."""
    m = len(row_ptr) - 1
    y = np.empty(m)
    used = lib().ref_parcrs(m, np.ascontiguousarray(row_ptr, np.int64), _i32(col_ind),
                            _f64(data), _f64(x), y, int(chunk))
    return y, used


def alg1_accurate(row_ptr, col_ind, data, x):
    """Algorithm 1 plus the accurate reference: returns (y_plain, y_ref, scale).

    y_ref sums each row's products with exact product errors and Neumaier compensation;
    scale[i] = sum |a_ik| |x_k|.  Used as the comparison point of the row-scaled error.
    """
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    m = row_ptr.shape[0] - 1
    yp = np.empty(m, np.float64)
    yr = np.empty(m, np.float64)
    s = np.empty(m, np.float64)
    lib().ref_alg1_accurate(m, row_ptr, _i32(col_ind), _f64(data), _f64(x), yp, yr, s)
    return yp, yr, s


def triplet_spmv(m, row, col, val, x):
    """Triplet SpMV (Section 2 equation), in the given entry order."""
    y = np.empty(m, np.float64)
    row = _i32(row)
    lib().ref_triplet_spmv(row.shape[0], row, _i32(col), _f64(val), _f64(x), m, y)
    return y


def reference(m, n, row, col, val, x, sum_duplicates=True):
    """Full oracle from raw triplets: returns dict(row_ptr, col, val, y_plain, y_ref, scale)."""
    rp, c, v = crs(m, n, row, col, val, sum_duplicates)
    yp, yr, s = alg1_accurate(rp, c, v, x)
    return dict(row_ptr=rp, col=c, val=v, y_plain=yp, y_ref=yr, scale=s)


def rows_reference(m, n, row, col, val, x, rows):
    """Oracle restricted to a set of rows (for full-size checks on sampled outputs).

    Selects the raw triplets of the given rows, canonicalises them and applies Algorithm 1.
    Returns (rows_sorted, y_plain, y_ref, scale) for those rows.
    """
    rows = np.unique(np.asarray(rows, np.int64))
    mask = np.zeros(m, dtype=bool)
    mask[rows] = True
    sel = np.flatnonzero(mask[np.asarray(row)])
    rr = np.asarray(row)[sel]
    # renumber the sampled rows 0..len(rows)-1, keeping their order
    local = np.searchsorted(rows, rr).astype(np.int32)
    yp, yr, s = alg1_accurate(*crs(len(rows), n, local, np.asarray(col)[sel],
                                   np.asarray(val)[sel]), x)
    return rows, yp, yr, s


def spmm(row_ptr, col_ind, data, X):
    """Products with several right-hand sides: column c of the result is Algorithm 1 applied to
    column c of X (n x k), so Y = A X column by column.  Returns (Y_plain, Y_ref, S), each m x k:
    the plain sums, the accurate reference and the scale |A| |X| of alg1_accurate."""
    X = np.asarray(X, np.float64)
    m = len(row_ptr) - 1
    k = X.shape[1]
    Y = np.empty((m, k))
    R = np.empty((m, k))
    S = np.empty((m, k))
    for c in range(k):
        Y[:, c], R[:, c], S[:, c] = alg1_accurate(row_ptr, col_ind, data, np.ascontiguousarray(X[:, c]))
    return Y, R, S
