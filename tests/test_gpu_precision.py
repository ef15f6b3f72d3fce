"""GPU parity of the reduced-precision forms (FP32 / bfloat16 stored values, FP32 x and y) of
every format: the CRS formats (FP32 sums inside a tile or row block) and the block formats
(FP32 products, FP64 sums).

Bar: integer-valued inputs are bit-exact (every value, product and partial sum is an integer
below 2^24); float inputs stay within the worst-case FP32 dot-product bound of
oracle.precision.dot_error_bound per row; stored values equal the oracle's rounding bit for bit.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import bcoh, formats, measure, precision, spmv

pytestmark = pytest.mark.gpu
CRS = ["rowsplit", "merge"]
BLOCK = ["csbh", "csb", "bcohc", "bcohch", "csbr"]  # FP32 products, FP64 sums
FMTS = CRS + BLOCK
UVAL = {"f32": precision.U32, "bf16": precision.UBF16}


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


def _run(spx, fmt, vt, m, n, row, col, val, x, **kw):
    import torch
    d = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=t)
    A = spx.convert(d(row, torch.int32), d(col, torch.int32), d(val, torch.float64), (m, n), fmt,
                    value_type=vt, **kw)
    y = A.spmv(d(x, torch.float32)).double().cpu().numpy()
    return A, y


def _check(A, vt, m, n, row, col, val, x, y, kind):
    # oracle on the same inputs rounded as the product sees them: values after repeats are
    # summed, rounded once; x rounded to FP32
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    rv = precision.round_f32(cv) if vt == "f32" else precision.round_bf16(cv)
    xr = precision.round_f32(x)
    rp, _, _ = spmv.crs_from_canonical(m, cr, cc, cv)
    yp, yr, s = spmv.alg1_accurate(rp, cc, rv, xr)
    if kind == "int":
        assert measure.equal_ignoring_zero_sign(y, yp), "integer inputs must be bit-exact"
    else:
        # error against the exact product of the rounded inputs is bounded by FP32 arithmetic;
        # against the unrounded FP64 oracle the input roundings add u_value + u32
        lens = np.diff(rp) + 2  # k products and sums, plus the final FP32 rounding of y
        err = measure.scaled_error(y, yr, s)
        assert np.all(err <= precision.dot_error_bound(lens, 0.0) + 1e-300)
        _, y64, s64 = spmv.alg1_accurate(rp, cc, cv, x)
        e64 = measure.scaled_error(y, y64, s64)
        assert np.all(e64 <= precision.dot_error_bound(lens, UVAL[vt]))
        say("  %s vs FP64 oracle: max %.3g median %.3g" % (vt, e64.max(), np.median(e64)))
    # stored values are the oracle's rounding, bit for bit (CSBR: taken to canonical order through
    # its decoded coordinates)
    got = A.export("values").cpu()
    if A.format in BLOCK:  # storage order -> canonical order through the decoded coordinates
        packed = A.export("packed").cpu().numpy().view(np.uint32)
        bp = A.export("blk_ptr").cpu().numpy()
        if A.format == "csbr":
            r, c, _, _, _ = formats.decode_csbr(A.export("row_order").cpu().numpy(), bp, packed,
                                                A.export("col_order").cpu().numpy())
        elif A.format in ("csbh", "csb"):
            r, c, _, _, _, _ = formats.decode_csbh(m, n, A.log2_beta, bp, packed,
                                                   np.zeros(len(packed)))
        else:
            r, c, _ = bcoh.decode(A.log2_beta, bp,
                                  A.export("blk_coord").cpu().numpy().view(np.uint32), packed,
                                  np.zeros(len(packed)))
        got = got[__import__("torch").from_numpy(np.lexsort((c, r)))]
    if vt == "f32":
        assert np.array_equal(got.numpy().astype(np.float64), rv)
    else:
        bits = got.view(dtype=__import__("torch").int16).numpy().view(np.uint16)
        assert np.array_equal(bits, precision.bf16_bits(cv))


@pytest.fixture(scope="module")
def rmat14():
    row, col = synth.rmat(14, 16, seed=0)
    return (1 << 14), (1 << 14), row, col


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["int", "float"])
def test_precision_rmat14(spx, rmat14, fmt, vt, kind):
    m, n, row, col = rmat14
    val = synth.values(len(row), seed=0, kind=kind)
    x = synth.xvec(n, seed=0, kind=kind)
    say("precision", fmt, vt, kind)
    A, y = _run(spx, fmt, vt, m, n, row, col, val, x)
    assert A.value_type == {"f32": 1, "bf16": 2}[vt]
    _check(A, vt, m, n, row, col, val, x, y, kind)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("vt", ["f32", "bf16"])
def test_precision_long_rows_and_hot_columns(spx, fmt, vt):
    # rows longer than a tile / row block / chunk (FP64 across tiles and for long rows), with the
    # hot-column copy forced on (CRS); CSBR with panels split into many units (FP64 partials)
    rng = np.random.default_rng(5)
    m, n = 4001, 6007
    row = np.concatenate([rng.integers(0, m, 80_000), np.full(40_000, 7), np.full(5000, 3000)])
    col = np.concatenate([rng.integers(0, n, 80_000), rng.integers(0, n, 45_000)])
    p = rng.permutation(len(row))
    row, col = row[p].astype(np.int32), col[p].astype(np.int32)
    for kind in ("int", "float"):
        val = synth.values(len(row), seed=9, kind=kind)
        x = synth.xvec(n, seed=9, kind=kind)
        kw = (dict(hot_columns=500) if fmt in CRS else
              dict(tile_items=3000) if fmt in ("csbr", "csbh", "csb") else {})
        A, y = _run(spx, fmt, vt, m, n, row, col, val, x, **kw)
        _check(A, vt, m, n, row, col, val, x, y, kind)


def test_precision_entry_points_reject_mismatch(spx, rmat14):
    import torch
    m, n, row, col = rmat14
    val = synth.values(len(row), seed=0)
    d = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=t)
    A = spx.convert(d(row, torch.int32), d(col, torch.int32), d(val, torch.float64), (m, n),
                    "merge", value_type="f32")
    with pytest.raises(TypeError):
        A.spmv(torch.zeros(n, dtype=torch.float64, device="cuda"))
    # the C entry point for FP64 products refuses a reduced-precision handle
    L = spx.load()
    import ctypes
    xb = torch.zeros(n, dtype=torch.float64, device="cuda")
    yb = torch.zeros(m, dtype=torch.float64, device="cuda")
    st = L.spx_spmv(A.handle, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(yb.data_ptr()), None)
    assert st == -7
    B = spx.convert(d(row, torch.int32), d(col, torch.int32), d(val, torch.float64), (m, n),
                    "csbh", value_type="bf16")
    st = L.spx_spmv(B.handle, ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(yb.data_ptr()), None)
    assert st == -7


@pytest.mark.parametrize("vt", ["f32", "bf16"])
def test_stored_value_rounding_edges(spx, vt):
    # the device's rounding of stored values against the oracle's on edge values: bfloat16
    # subnormals (spacing 2^-133) and their ties, the smallest normal, values that overflow to
    # the infinity, exact ties in the normal range, signed zeros
    import torch
    vals = np.array([2.0 ** -134, 3 * 2.0 ** -135, 1.5 * 2.0 ** -133, 2.5 * 2.0 ** -133,
                     2.0 ** -126, (1 - 2.0 ** -9) * 2.0 ** -126, 1e-40, -1e-40, 1e-45,
                     (2 - 2.0 ** -7) * 2.0 ** 127, (2 - 2.0 ** -8) * 2.0 ** 127, -3.4e38, 1e300,
                     1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, 257.0, -0.0, 0.0, 1e-320, 0.1, -7.0])
    rng = np.random.default_rng(21)
    vals = np.concatenate([vals, np.ldexp(rng.uniform(-1, 1, 2000), rng.integers(-140, 128,
                                                                               2000))])
    n = len(vals)
    row = np.arange(n, dtype=np.int32)  # one entry per row: canonical order = input order
    col = np.zeros(n, dtype=np.int32)
    d = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=t)
    A = spx.convert(d(row, torch.int32), d(col, torch.int32), d(vals, torch.float64), (n, 1),
                    "rowsplit", value_type=vt)
    got = A.export("values").cpu()
    if vt == "f32":
        want = np.asarray(vals, np.float64).astype(np.float32).view(np.uint32)
        assert np.array_equal(got.numpy().view(np.uint32), want)
    else:
        bits = got.view(dtype=torch.int16).numpy().view(np.uint16)
        want = precision.bf16_bits(vals)
        bad = np.flatnonzero(bits != want)
        assert len(bad) == 0, [(vals[i], hex(bits[i]), hex(want[i])) for i in bad[:5]]
    A.close()
