"""GPU parity of the product with k right-hand sides (Y = A X) against the CPU oracle, through the
C ABI, in both operand layouts and every stored value type.

Bar: integer-valued inputs are bit-exact; FP64 float inputs within row-scaled error 1e-12 per
element of Y; FP32 / bfloat16 stored values within the worst-case FP32 dot-product bound of
oracle.precision.dot_error_bound against the oracle on the rounded inputs.
"""
import ctypes
import sys

import numpy as np
import pytest

import synth
from oracle import measure, precision, spmv

pytestmark = pytest.mark.gpu
CRS = ["rowsplit", "merge"]
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def spx():
    import torch

    from ._lib import ensure_built
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    import paper_2502_19284_amd as spx
    spx.use_torch_allocator(True)
    return spx


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _xdev(X, vt, layout, pad=0):
    """X (n x k numpy) as a device tensor of the product's type in the given layout; pad adds
    unused rows (column-major) or columns (row-major) to the leading dimension."""
    import torch
    dt = torch.float64 if vt == "f64" else torch.float32
    n, k = X.shape
    if layout == "col":
        buf = torch.zeros((k, n + pad), dtype=dt, device="cuda")
        buf[:, :n] = _dev(X.T, dt)
        return buf[:, :n].t()
    buf = torch.zeros((n, k + pad), dtype=dt, device="cuda")
    buf[:, :k] = _dev(X, dt)
    return buf[:, :k]


def _convert(spx, fmt, vt, m, n, row, col, val, **kw):
    import torch
    return spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                       (m, n), fmt, value_type=vt, **kw)


def _check(vt, m, n, row, col, val, X, Y, kind, what):
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    rp, _, _ = spmv.crs_from_canonical(m, cr, cc, cv)
    if vt == "f64":
        Yp, Yr, S = spmv.spmm(rp, cc, cv, X)
        if kind == "int":
            assert measure.equal_ignoring_zero_sign(Y, Yp), what
        else:
            err = measure.scaled_error(Y.ravel(), Yr.ravel(), S.ravel())
            assert err.max(initial=0.0) <= TOL, "%s: max scaled error %.3g" % (what, err.max())
        return
    rv = precision.round_f32(cv) if vt == "f32" else precision.round_bf16(cv)
    Yp, Yr, S = spmv.spmm(rp, cc, rv, precision.round_f32(X))
    if kind == "int":
        assert measure.equal_ignoring_zero_sign(Y, Yp), what
        return
    lens = (np.diff(rp) + 2)[:, None] * np.ones((1, X.shape[1]), np.int64)
    err = measure.scaled_error(Y.ravel(), Yr.ravel(), S.ravel())
    assert np.all(err <= precision.dot_error_bound(lens.ravel(), 0.0) + 1e-300), what


def _product(spx, A, X, vt, layout, pad=0):
    import torch
    Xd = _xdev(X, vt, layout, pad)
    Y = A.spmm(Xd)
    torch.cuda.synchronize()
    return Y.double().cpu().numpy()


@pytest.fixture(scope="module")
def rmat14():
    row, col = synth.rmat(14, 16, seed=0)
    return (1 << 14), (1 << 14), row, col


def _xmat(n, k, seed, kind):
    return np.stack([synth.xvec(n, seed=seed * 1000 + c, kind=kind) for c in range(k)], axis=1)


@pytest.mark.parametrize("fmt", CRS)
@pytest.mark.parametrize("vt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("kind", ["int", "float"])
@pytest.mark.parametrize("layout,k", [("col", 1), ("col", 5), ("col", 32), ("row", 3),
                                      ("row", 32)])
def test_spmm_rmat14(spx, rmat14, fmt, vt, kind, layout, k):
    m, n, row, col = rmat14
    val = synth.values(len(row), seed=0, kind=kind)
    X = _xmat(n, k, 1, kind)
    say("spmm rmat14", fmt, vt, kind, layout, k)
    A = _convert(spx, fmt, vt, m, n, row, col, val)
    Y = _product(spx, A, X, vt, layout)
    _check(vt, m, n, row, col, val, X, Y, kind, "rmat14 %s %s %s %s k=%d" % (fmt, vt, kind, layout, k))


@pytest.mark.parametrize("fmt", CRS)
@pytest.mark.parametrize("vt", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["col", "row"])
def test_spmm_chunks_and_padding(spx, fmt, vt, layout):
    # k beyond one 64-column chunk, leading dimensions larger than the minimum
    rng = np.random.default_rng(3)
    m, n, E = 3001, 2003, 40_000
    row, col = rng.integers(0, m, E).astype(np.int32), rng.integers(0, n, E).astype(np.int32)
    for kind in ("int", "float"):
        val = synth.values(E, seed=4, kind=kind)
        for k in (64, 65, 130):
            X = _xmat(n, k, 2, kind)
            say("spmm chunks", fmt, vt, layout, kind, k)
            A = _convert(spx, fmt, vt, m, n, row, col, val)
            Y = _product(spx, A, X, vt, layout, pad=7)
            _check(vt, m, n, row, col, val, X, Y, kind, "chunks k=%d" % k)
            A.close()


@pytest.mark.parametrize("fmt", CRS)
@pytest.mark.parametrize("vt", ["f64", "f32", "bf16"])
def test_spmm_long_rows_and_hot_columns(spx, fmt, vt):
    # rows spanning many tiles and groups, empty rows, and the compact hot-row copy
    rng = np.random.default_rng(5)
    m, n = 4001, 6007
    row = np.concatenate([rng.integers(0, m // 2, 60_000), np.full(40_000, 7),
                          np.full(9000, 3000), np.full(3, m - 1)])
    col = rng.integers(0, n, len(row))
    p = rng.permutation(len(row))
    row, col = row[p].astype(np.int32), col[p].astype(np.int32)
    for kind in ("int", "float"):
        val = synth.values(len(row), seed=9, kind=kind)
        for k, layout in ((8, "col"), (32, "row"), (2, "col")):
            X = _xmat(n, k, 3, kind)
            say("spmm long rows", fmt, vt, kind, k, layout)
            A = _convert(spx, fmt, vt, m, n, row, col, val, hot_columns=500)
            Y = _product(spx, A, X, vt, layout)
            _check(vt, m, n, row, col, val, X, Y, kind, "long rows k=%d" % k)
            A.close()


@pytest.mark.parametrize("fmt", CRS)
def test_spmm_degenerate_shapes(spx, fmt):
    rng = np.random.default_rng(8)
    cases = [
        (5, 4, np.zeros(0, np.int32), np.zeros(0, np.int32)),          # no entries: Y = 0
        (1, 5000, np.zeros(9000, np.int32), rng.integers(0, 5000, 9000).astype(np.int32)),
        (5000, 1, rng.integers(0, 5000, 9000).astype(np.int32), np.zeros(9000, np.int32)),
        (0, 7, np.zeros(0, np.int32), np.zeros(0, np.int32)),           # no rows
    ]
    for m, n, row, col in cases:
        val = synth.values(len(row), seed=2, kind="int")
        for k in (1, 4):
            X = _xmat(n, k, 4, "int")
            A = _convert(spx, fmt, "f64", m, n, row, col, val)
            Y = _product(spx, A, X, "f64", "col")
            assert Y.shape == (m, k)
            _check("f64", m, n, row, col, val, X, Y, "int", "degenerate %dx%d k=%d" % (m, n, k))
            if m > 0 and len(row) == 0:
                assert np.all(Y == 0) and not np.any(np.signbit(Y))
            A.close()


def test_spmm_errors(spx, rmat14):
    import torch
    m, n, row, col = rmat14
    val = synth.values(len(row), seed=0)
    A = _convert(spx, "merge", "f64", m, n, row, col, val)
    L = spx.load()
    X = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    Y = torch.zeros((4, m), dtype=torch.float64, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    assert L.spx_spmm(A.handle, 0, P(X), n, P(Y), m, 0, None) == -1        # k < 1
    assert L.spx_spmm(A.handle, 4, P(X), n - 1, P(Y), m, 0, None) == -1    # ldx < n
    assert L.spx_spmm(A.handle, 4, P(X), n, P(Y), m - 1, 0, None) == -1    # ldy < m
    assert L.spx_spmm(A.handle, 4, P(X), 3, P(Y), 4, 1, None) == -1        # row-major ldx < k
    assert L.spx_spmm(A.handle, 4, P(X), n, P(Y), m, 2, None) == -1        # unknown layout
    assert L.spx_spmm(A.handle, 4, None, n, P(Y), m, 0, None) == -1        # NULL X
    inside = ctypes.c_void_p(X.data_ptr() + 8 * n)                         # Y inside X's span
    assert L.spx_spmm(A.handle, 2, P(X), n, inside, n, 0, None) == -4
    assert L.spx_spmm(None, 4, P(X), n, P(Y), m, 0, None) == -1
    with pytest.raises(TypeError):
        A.spmm(torch.zeros((n, 2), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        A.spmm(torch.zeros((n + 1, 2), dtype=torch.float64, device="cuda"))
    B = _convert(spx, "csbh", "f64", m, n, row, col, val)
    assert L.spx_spmm(B.handle, 4, P(X), n, P(Y), m, 0, None) == -7
    with pytest.raises(spx.SpxError):
        B.spmm(torch.zeros((n, 2), dtype=torch.float64, device="cuda"))
    # the failed calls wrote nothing
    assert torch.count_nonzero(Y).item() == 0


def test_spmm_repeated_calls_reuse_scratch(spx, rmat14):
    # growing k, shrinking k and switching layouts on one handle give the same results as fresh
    # handles (scratch is grown and reused)
    m, n, row, col = rmat14
    val = synth.values(len(row), seed=0, kind="int")
    A = _convert(spx, "rowsplit", "f32", m, n, row, col, val)
    for k, layout in ((2, "col"), (40, "col"), (3, "row"), (70, "col"), (1, "row")):
        X = _xmat(n, k, 5, "int")
        Y = _product(spx, A, X, "f32", layout)
        _check("f32", m, n, row, col, val, X, Y, "int", "reuse k=%d %s" % (k, layout))
