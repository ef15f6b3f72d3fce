"""GPU parity: every format's conversion and product against the CPU oracle, through the C ABI.

Bar: bit-exact for integer work (conversion arrays, partitions, integer-valued products);
row-scaled error |y - y_ref| / sum_k |a_ik x_k| <= 1e-12 for floating-point products, where
y_ref is the oracle's compensated Algorithm 1.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import bcoh, formats, measure, mergepath, spmv

pytestmark = pytest.mark.gpu
FMTS = ["rowsplit", "merge", "csbh", "csb", "bcohc", "bcohch", "csbr"]
BCOH = ("bcohc", "bcohch")
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


def _run(spx, fmt, m, n, row, col, val, x, **kw):
    import torch
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), fmt, **kw)
    y = A.spmv(_dev(x, torch.float64))
    torch.cuda.synchronize()
    return A, y.cpu().numpy()


def _check_float(y, ref, what):
    err = measure.scaled_error(y, ref["y_ref"], ref["scale"])
    worst = float(err.max()) if len(err) else 0.0
    assert worst <= TOL, "%s: max scaled error %.3g at row %d" % (what, worst, int(err.argmax()))
    return worst


def _check_int(y, ref, what):
    assert measure.equal_ignoring_zero_sign(y, ref["y_plain"]), what


def _check_structure(A, m, n, row, col, val):
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    if A.format in BCOH:
        parts = A.export("parts").cpu().numpy()
        P = A.parts
        bcoh.check_bcoh(m, n, A.log2_beta, row, len(row), parts[:P + 1], parts[P + 1:],
                        A.export("blk_ptr").cpu().numpy(),
                        A.export("blk_coord").cpu().numpy().view(np.uint32),
                        A.export("packed").cpu().numpy().view(np.uint32),
                        A.export("values").cpu().numpy(), cr, cc, cv, A.format == "bcohch")
    elif A.format == "csbr":
        formats.check_csbr(m, n, row, col, A.export("blk_ptr").cpu().numpy(),
                           A.export("packed").cpu().numpy().view(np.uint32),
                           A.export("values").cpu().numpy(), A.export("col_order").cpu().numpy(),
                           A.export("row_order").cpu().numpy(), cr, cc, cv)
    elif A.format in ("csbh", "csb"):
        formats.check_csb(m, n, A.log2_beta, A.export("blk_ptr").cpu().numpy(),
                          A.export("packed").cpu().numpy().view(np.uint32),
                          A.export("values").cpu().numpy(), cr, cc, cv,
                          "hilbert" if A.format == "csbh" else "zmorton")
    else:
        formats.check_crs(m, n, A.export("row_ptr").cpu().numpy(),
                          A.export("col_ind").cpu().numpy(), A.export("values").cpu().numpy(),
                          cr, cc, cv)
    assert A.nnz == len(cr)


# ---------------------------------------------------------------- hand-made edge cases


def _cases():
    cases = {}
    n = 37
    idx = np.arange(n, dtype=np.int32)
    cases["identity"] = (n, n, idx, idx, np.ones(n))
    cases["diagonal"] = (n, n, idx, idx, synth.values(n, seed=3))
    cases["empty_nnz0"] = (9, 5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    cases["one_by_one"] = (1, 1, np.array([0], np.int32), np.array([0], np.int32), np.array([2.5]))
    # m != n, one dense row among empty ones (the almost-dense-row case)
    cases["dense_row"] = (7, 5000, np.full(5000, 4, np.int32), np.arange(5000, dtype=np.int32),
                          synth.values(5000, seed=4))
    # heavy repeats of a few coordinates, in scrambled order
    rng = np.random.default_rng(5)
    r = rng.integers(0, 3, 4000).astype(np.int32)
    c = rng.integers(0, 3, 4000).astype(np.int32)
    cases["repeats"] = (3, 3, r, c, synth.values(4000, seed=5))
    # explicit zeros and entries whose products are -0
    cases["zeros"] = (4, 4, np.array([0, 1, 1, 3], np.int32), np.array([1, 1, 2, 3], np.int32),
                      np.array([0.0, -0.0, 0.0, 1.0]))
    # a single entry in the last row and column
    cases["corner"] = (1000, 999, np.array([999], np.int32), np.array([998], np.int32),
                       np.array([-1.5]))
    # more than 4096 repeats of two coordinates among other entries, scrambled: the sort's
    # segments of equal keys that stay larger than one workgroup's share after the last digit
    rng = np.random.default_rng(11)
    r = np.concatenate([np.full(9000, 5), np.full(6000, 999), rng.integers(0, 1000, 30000)])
    c = np.concatenate([np.full(9000, 7), np.zeros(6000), rng.integers(0, 1000, 30000)])
    perm = rng.permutation(len(r))
    cases["long_repeats"] = (1000, 1000, r[perm].astype(np.int32), c[perm].astype(np.int32),
                             synth.values(len(r), seed=11))
    # one row of 20000 entries among 40000 scattered ones in a 70000 x 70000 matrix: split
    # levels over row digits, then over column digits inside the long row
    r = np.concatenate([np.full(20000, 3), rng.integers(0, 70000, 40000)])
    c = np.concatenate([rng.integers(0, 70000, 20000), rng.integers(0, 70000, 40000)])
    perm = rng.permutation(len(r))
    cases["deep_split"] = (70000, 70000, r[perm].astype(np.int32), c[perm].astype(np.int32),
                           synth.values(len(r), seed=12))
    # a large shape whose high row and column bits the entries never use (the CRS sort's first
    # digit, chosen from the shape, is constant), and more than 4096 copies of one coordinate
    cases["narrow_entries"] = (1 << 20, 1 << 20, rng.integers(0, 200, 9000).astype(np.int32),
                               rng.integers(0, 300, 9000).astype(np.int32),
                               synth.values(9000, seed=13))
    cases["all_equal_large"] = (40, 50, np.full(7000, 17, np.int32), np.full(7000, 33, np.int32),
                                synth.values(7000, seed=14))
    # sizes around one workgroup's share of the sort (4096 keys sorted whole in LDS; one more
    # splits by the top digit first), with repeats
    for E in (4096, 4097, 8193):
        cases["size_%d" % E] = (3000, 2000, rng.integers(0, 3000, E).astype(np.int32),
                                rng.integers(0, 2000, E).astype(np.int32),
                                synth.values(E, seed=E))
    return cases


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("case", sorted(_cases()))
def test_handmade(spx, fmt, case):
    m, n, row, col, val = _cases()[case]
    say("handmade", case, fmt, m, n, len(row))
    x = synth.xvec(n, seed=7)
    x[::5] = -x[::5]
    ref = spmv.reference(m, n, row, col, val, x)
    A, y = _run(spx, fmt, m, n, row, col, val, x)
    _check_float(y, ref, case)
    _check_structure(A, m, n, row, col, val)
    # empty rows are +0 exactly
    empty = np.diff(ref["row_ptr"]) == 0
    assert np.all(y[empty] == 0.0) and not np.any(np.signbit(y[empty]))


# ---------------------------------------------------------------- R-MAT scale 14 (float and integer)


@pytest.fixture(scope="module")
def rmat14():
    m = n = 1 << 14
    row, col = synth.rmat(14, 16, seed=0)
    out = {}
    for kind in ("float", "int"):
        val = synth.values(len(row), seed=0, kind=kind)
        x = synth.xvec(n, seed=0, kind=kind)
        out[kind] = (val, x, spmv.reference(m, n, row, col, val, x))
    return m, n, row, col, out


@pytest.mark.parametrize("fmt", FMTS)
def test_rmat14_float(spx, rmat14, fmt):
    m, n, row, col, d = rmat14
    val, x, ref = d["float"]
    say("rmat14 float", fmt)
    A, y = _run(spx, fmt, m, n, row, col, val, x)
    worst = _check_float(y, ref, "rmat14 " + fmt)
    say("  max scaled error %.3g, parts %d" % (worst, A.parts))
    _check_structure(A, m, n, row, col, val)


@pytest.mark.parametrize("fmt", FMTS)
def test_rmat14_int_bit_exact(spx, rmat14, fmt):
    m, n, row, col, d = rmat14
    val, x, ref = d["int"]
    say("rmat14 int", fmt)
    A, y = _run(spx, fmt, m, n, row, col, val, x)
    _check_int(y, ref, "rmat14 int " + fmt)
    _check_structure(A, m, n, row, col, val)


def test_merge_tile_starts_match_oracle(spx, rmat14):
    import torch
    m, n, row, col, d = rmat14
    val, x, ref = d["int"]
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), "merge")
    coords = A.export("parts").cpu().numpy().reshape(-1, 2)
    tile = 2048
    rp = ref["row_ptr"]
    want = mergepath.splits(list(rp[1:]), list(range(int(rp[-1]))), tile)
    assert [tuple(c) for c in coords.tolist()] == [tuple(w) for w in want]


# ---------------------------------------------------------------- ragged sizes, long rows, many tiles


def _ragged_matrix(seed, m, n, E, long_rows=()):
    rng = np.random.default_rng(seed)
    row = rng.integers(0, m, E).astype(np.int32)
    col = rng.integers(0, n, E).astype(np.int32)
    parts_r = [row]
    parts_c = [col]
    for r, length in long_rows:
        parts_r.append(np.full(length, r, np.int32))
        parts_c.append(rng.integers(0, n, length).astype(np.int32))
    row = np.concatenate(parts_r)
    col = np.concatenate(parts_c)
    p = rng.permutation(len(row))
    return row[p], col[p]


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("kind", ["float", "int"])
def test_ragged_long_rows(spx, fmt, kind):
    # rows far longer than a row block, a merge tile and a row-split chunk, beside short rows,
    # with sizes that are not multiples of any tile
    m, n = 5003, 7777
    row, col = _ragged_matrix(11, m, n, 150_001,
                              long_rows=[(0, 30_000), (2500, 1500), (5002, 20_000), (17, 9000)])
    val = synth.values(len(row), seed=12, kind=kind)
    x = synth.xvec(n, seed=13, kind=kind)
    say("ragged", fmt, kind, len(row))
    ref = spmv.reference(m, n, row, col, val, x)
    A, y = _run(spx, fmt, m, n, row, col, val, x)
    if kind == "int":
        _check_int(y, ref, "ragged int " + fmt)
    else:
        _check_float(y, ref, "ragged " + fmt)
    _check_structure(A, m, n, row, col, val)


@pytest.mark.parametrize("log2_beta,unit", [(1, 0), (4, 64), (6, 1000), (9, 5000), (13, 0)])
@pytest.mark.parametrize("fmt", ["csbh", "csb"])
def test_csbh_block_sizes_and_split_rows(spx, log2_beta, unit, fmt):
    # small units force block rows to be split into several units with partial slices
    m, n = 3001, 4099
    row, col = _ragged_matrix(21, m, n, 60_000, long_rows=[(100, 12_000)])
    val = synth.values(len(row), seed=22, kind="int")
    x = synth.xvec(n, seed=23, kind="int")
    say(fmt, "beta", log2_beta, "unit", unit)
    ref = spmv.reference(m, n, row, col, val, x)
    A, y = _run(spx, fmt, m, n, row, col, val, x, log2_beta=log2_beta, tile_items=unit)
    assert A.log2_beta == log2_beta
    _check_int(y, ref, "%s int beta %d" % (fmt, log2_beta))
    _check_structure(A, m, n, row, col, val)


@pytest.mark.parametrize("fmt", ["csbr", "bcohc"])
def test_bucketed_count_many_buckets(spx, fmt):
    # rows and columns of CSBR just under the 2^26 limit of the bucketed counts: 4096 buckets of
    # 2^14 indices (the whole range of the scatter's bucket scan); BCOHC, whose key holds the
    # partition (at most 8192 rows each) and the Hilbert index, fits 64 bits up to 2^25 rows
    # (2048 buckets).  Few triplets per bucket, most buckets of a sub-tile empty, heavy rows in
    # the first and the last bucket and a heavy column
    rng = np.random.default_rng(71)
    m = (1 << 26) - 3 if fmt == "csbr" else (1 << 25) - 3
    n = m if fmt == "csbr" else 4096
    E = 400_000
    row = rng.integers(0, m, E)
    col = rng.integers(0, n, E)
    row[:20_000] = 5
    row[20_000:30_000] = m - 1
    col[30_000:40_000] = n - 2
    perm = rng.permutation(E)
    row, col = row[perm].astype(np.int32), col[perm].astype(np.int32)
    val = synth.values(E, seed=72, kind="int")
    x = synth.xvec(n, seed=73, kind="int")
    ref = spmv.reference(m, n, row, col, val, x)
    say("bucketed count, 4096 buckets", fmt)
    A, y = _run(spx, fmt, m, n, row, col, val, x)
    _check_int(y, ref, "%s with 4096 buckets" % fmt)
    if fmt == "csbr":
        _check_structure(A, m, n, row, col, val)


@pytest.mark.parametrize("unit", [0, 700, 5000, 100_000])
@pytest.mark.parametrize("kind", ["int", "float"])
def test_csbr_segments_and_split_panels(spx, unit, kind):
    # more than 2^19 ranked columns (several rank segments per panel), panels split into many
    # units with partial slices (small tile_items), a ranked-row count that is not a multiple of
    # the panel height, long rows, empty rows and a very frequent column
    rng = np.random.default_rng(61)
    m, n, E = 20_011, (1 << 21) + 3, 2_000_000
    row = rng.integers(0, m, E)
    col = rng.integers(0, n, E)
    row[:30_000] = 16383          # a long row at a panel edge
    col[30_000:90_000] = 12345    # one very frequent column
    row[90_000:95_000] = m - 1
    row[row % 97 == 5] = 0        # rows without triplets
    perm = rng.permutation(E)
    row, col = row[perm].astype(np.int32), col[perm].astype(np.int32)
    val = synth.values(E, seed=62, kind=kind)
    x = synth.xvec(n, seed=63, kind=kind)
    ref = spmv.reference(m, n, row, col, val, x)
    say("csbr unit", unit, kind)
    A, y = _run(spx, "csbr", m, n, row, col, val, x, tile_items=unit)
    nranked = len(np.unique(col))
    pb, rb = formats.CSBR_PB, formats.CSBR_RB
    rbits = max(rb, (nranked - 1).bit_length())
    assert rbits >= rb + 2                      # at least 4 rank segments per panel
    npan = (len(np.unique(row)) + (1 << pb) - 1) >> pb
    assert A.export("blk_ptr").numel() == npan * (1 << (rbits - rb)) + 1
    if kind == "int":
        _check_int(y, ref, "csbr int unit %d" % unit)
    else:
        _check_float(y, ref, "csbr float unit %d" % unit)
    if unit in (0, 700):
        _check_structure(A, m, n, row, col, val)


def test_csbh_default_block_size_rule(spx, rmat14):
    import torch
    m, n, row, col, d = rmat14
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32),
                    _dev(d["float"][0], torch.float64), (m, n), "csbh")
    assert A.log2_beta == measure.csb_log2_beta(m, n) == 10


@pytest.mark.parametrize("fmt", FMTS)
def test_keep_repeats_option(spx, fmt):
    # sum_duplicates=False keeps each triplet as a stored entry; y is unchanged
    m, n = 300, 200
    row, col = _ragged_matrix(31, m, n, 20_000)
    val = synth.values(len(row), seed=32, kind="int")
    x = synth.xvec(n, seed=33, kind="int")
    ref = spmv.reference(m, n, row, col, val, x)
    if fmt in BCOH:  # built with repeats summed only
        with pytest.raises(spx.SpxError) as e:
            _run(spx, fmt, m, n, row, col, val, x, sum_duplicates=False)
        assert e.value.status == -7
        return
    A, y = _run(spx, fmt, m, n, row, col, val, x, sum_duplicates=False)
    assert A.nnz == len(row)
    _check_int(y, ref, "keep repeats " + fmt)


@pytest.mark.parametrize("fmt", ["rowsplit", "merge"])
@pytest.mark.parametrize("hot", [1, 100, 5000, 10 ** 6])
def test_hot_column_compaction(spx, rmat14, fmt, hot):
    # forced hot-column compaction on the scale-14 matrix: bit-exact on integers, and the exported
    # col_ind (hot entries mapped back) still equals the canonical columns
    m, n, row, col, d = rmat14
    for kind in ("int", "float"):
        val, x, ref = d[kind]
        say("hot", fmt, hot, kind)
        A, y = _run(spx, fmt, m, n, row, col, val, x, hot_columns=hot)
        if kind == "int":
            _check_int(y, ref, "hot %s %d" % (fmt, hot))
        else:
            _check_float(y, ref, "hot %s %d" % (fmt, hot))
        _check_structure(A, m, n, row, col, val)


@pytest.mark.parametrize("fmt", ["rowsplit", "merge"])
@pytest.mark.parametrize("hot", [1, 2, 3])
def test_hot_threshold_beyond_histogram(spx, fmt, hot):
    # three columns with more entries (9000, 7000, 5000) than the count histogram's last bin: the
    # threshold for at most 1 or 2 hot columns is found by bisection on device-side counts, for
    # 3 from the histogram
    rng = np.random.default_rng(71)
    m, n = 20_000, 400
    col = np.concatenate([np.full(9000, 0), np.full(7000, 1), np.full(5000, 2),
                          rng.integers(3, n, 30_000)]).astype(np.int32)
    row = rng.integers(0, m, len(col)).astype(np.int32)
    perm = rng.permutation(len(col))
    row, col = row[perm], col[perm]
    for kind in ("int", "float"):
        val = synth.values(len(row), seed=72, kind=kind)
        x = synth.xvec(n, seed=73, kind=kind)
        ref = spmv.reference(m, n, row, col, val, x)
        say("hot beyond histogram", fmt, hot, kind)
        A, y = _run(spx, fmt, m, n, row, col, val, x, hot_columns=hot)
        if kind == "int":
            _check_int(y, ref, "hot bisection %s %d" % (fmt, hot))
        else:
            _check_float(y, ref, "hot bisection %s %d" % (fmt, hot))
        _check_structure(A, m, n, row, col, val)


# ---------------------------------------------------------------- invariants


@pytest.mark.parametrize("fmt", FMTS)
def test_permutation_and_order_invariance_int(spx, fmt):
    m = n = 1 << 12
    row, col = synth.rmat(12, 16, seed=41)
    val = synth.values(len(row), seed=41, kind="int")
    x = synth.xvec(n, seed=41, kind="int")
    _, y = _run(spx, fmt, m, n, row, col, val, x)
    # (P A Q^T)(Q x) = P (A x)
    P = synth.permutation(m, seed=42)
    Q = synth.permutation(n, seed=43)
    Pinv = np.empty_like(P)
    Pinv[P] = np.arange(m)
    Qinv = np.empty_like(Q)
    Qinv[Q] = np.arange(n)
    _, y2 = _run(spx, fmt, m, n, Pinv[row].astype(np.int32), Qinv[col].astype(np.int32), val,
                 x[Q])
    assert measure.equal_ignoring_zero_sign(y2, y[P])
    # shuffled triplet order: same stored matrix, same y
    S = synth.permutation(len(row), seed=44)
    _, y3 = _run(spx, fmt, m, n, row[S], col[S], val[S], x)
    assert measure.equal_ignoring_zero_sign(y3, y)
    # A 1 = row sums
    ones = np.ones(n)
    _, y4 = _run(spx, fmt, m, n, row, col, val, ones)
    sums = np.zeros(m)
    np.add.at(sums, row, val)
    assert measure.equal_ignoring_zero_sign(y4, sums)


@pytest.mark.parametrize("fmt", ["rowsplit", "merge"])
def test_repeat_runs_bitwise_identical(spx, rmat14, fmt):
    # the CRS products sum every row in a fixed order (the block formats use LDS float atomics
    # and are only held to the product tolerance)
    import torch
    m, n, row, col, d = rmat14
    val, x, _ = d["float"]
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), fmt)
    xd = _dev(x, torch.float64)
    y1 = A.spmv(xd).cpu().numpy()
    y2 = A.spmv(xd).cpu().numpy()
    assert np.array_equal(y1.view(np.int64), y2.view(np.int64))


EXPORTS = {"rowsplit": ("row_ptr", "col_ind", "values", "parts"),
           "merge": ("row_ptr", "col_ind", "values", "parts"),
           "csbh": ("blk_ptr", "packed", "values", "parts"),
           "csb": ("blk_ptr", "packed", "values", "parts"),
           "bcohc": ("blk_ptr", "packed", "values", "parts", "blk_coord"),
           "bcohch": ("blk_ptr", "packed", "values", "parts", "blk_coord"),
           "csbr": ("blk_ptr", "packed", "values", "parts", "col_order", "row_order")}


@pytest.mark.parametrize("fmt", FMTS)
def test_conversion_deterministic(spx, rmat14, fmt):
    # the same triplets convert to bit-identical arrays every time, although some steps run in
    # an order that varies (LDS atomics place entries in the bucketed counts' scatter; the
    # counts and extents they feed do not depend on it)
    import torch
    m, n, row, col, d = rmat14
    val, _, _ = d["float"]
    got = []
    for _ in range(2):
        A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32),
                        _dev(val, torch.float64), (m, n), fmt)
        got.append({a: A.export(a).cpu().numpy().tobytes() for a in EXPORTS[fmt]})
        A.close()
    for a in EXPORTS[fmt]:
        assert got[0][a] == got[1][a], "%s: %s differs between conversions" % (fmt, a)


def test_linearity_float(spx, rmat14):
    import torch
    m, n, row, col, d = rmat14
    val, x1, ref1 = d["float"]
    x2 = synth.values(n, seed=99)
    for fmt in FMTS:
        A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                        (m, n), fmt)
        y1 = A.spmv(_dev(x1, torch.float64)).cpu().numpy()
        y2 = A.spmv(_dev(x2, torch.float64)).cpu().numpy()
        y12 = A.spmv(_dev(2 * x1 - 3 * x2, torch.float64)).cpu().numpy()
        s = ref1["scale"]
        _, _, s2 = spmv.alg1_accurate(ref1["row_ptr"], ref1["col"], ref1["val"], x2)
        assert np.all(np.abs(y12 - (2 * y1 - 3 * y2)) <= 1e-12 * (2 * s + 3 * s2) + 1e-300)


# ---------------------------------------------------------------- errors through the ABI


def test_error_paths(spx):
    import torch
    row = _dev(np.array([0, 5], np.int32), torch.int32)
    col = _dev(np.array([0, 1], np.int32), torch.int32)
    val = _dev(np.array([1.0, 2.0]), torch.float64)
    with pytest.raises(spx.SpxError) as e:
        spx.convert(row, col, val, (5, 5), "merge")
    assert e.value.name == "SPX_ERR_INDEX"
    with pytest.raises(spx.SpxError) as e:
        spx.convert(_dev(np.array([0, -1], np.int32), torch.int32), col, val, (5, 5), "csbh")
    assert e.value.name == "SPX_ERR_INDEX"
    # the same checks with more triplets than one workgroup sorts alone (CRS and CSB keys are
    # then built inside the sort)
    big = 9000
    r = np.arange(big, dtype=np.int32) % 5
    c = np.arange(big, dtype=np.int32) % 7
    v = _dev(np.ones(big), torch.float64)
    for fmt in ("rowsplit", "merge", "csbh", "csb", "csbr"):
        bad_r = r.copy()
        bad_r[4321] = 5
        with pytest.raises(spx.SpxError) as e:
            spx.convert(_dev(bad_r, torch.int32), _dev(c, torch.int32), v, (5, 7), fmt)
        assert e.value.name == "SPX_ERR_INDEX"
        bad_c = c.copy()
        bad_c[8999] = -1
        with pytest.raises(spx.SpxError) as e:
            spx.convert(_dev(r, torch.int32), _dev(bad_c, torch.int32), v, (5, 7), fmt)
        assert e.value.name == "SPX_ERR_INDEX"
    # BCOH keys of a matrix with more than 2^26 rows need more than 64 bits
    for fmt in ("bcohc", "bcohch"):
        with pytest.raises(spx.SpxError) as e:
            spx.convert(row, col, val, ((1 << 26) + 1, 8), fmt)
        assert e.value.name == "SPX_ERR_RANGE"
    # CSBR: more than 2^26 columns; a block size other than its fixed panel height
    with pytest.raises(spx.SpxError) as e:
        spx.convert(row, col, val, (8, (1 << 26) + 1), "csbr")
    assert e.value.name == "SPX_ERR_RANGE"
    with pytest.raises(spx.SpxError) as e:
        spx.convert(_dev(np.array([0, 4], np.int32), torch.int32), col, val, (5, 5), "csbr",
                    log2_beta=5)
    assert e.value.name == "SPX_ERR_UNSUPPORTED"
    A = spx.convert(_dev(np.array([0, 4], np.int32), torch.int32), col, val, (5, 5), "rowsplit")
    buf = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(spx.SpxError) as e:
        A.spmv(buf[0:5], out=buf[3:8])
    assert e.value.name == "SPX_ERR_ALIAS"
    with pytest.raises(TypeError):
        A.spmv(torch.zeros(5, dtype=torch.float32, device="cuda"))
    with pytest.raises(spx.SpxError):
        A.export("blk_ptr")
    A.close()
    with pytest.raises(RuntimeError):
        A.spmv(buf[0:5])


def test_report_and_info(spx, rmat14):
    import torch
    m, n, row, col, d = rmat14
    val = d["float"][0]
    for fmt in FMTS:
        A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                        (m, n), fmt)
        assert A.convert_ms > 0
        assert A.nnz == len(d["float"][2]["col"])
        assert A.bytes >= A.nnz * 12
        assert A.parts > 0


@pytest.mark.parametrize("fmt", BCOH)
@pytest.mark.parametrize("log2_beta", [0, 3, 7])
def test_bcoh_partitions_blocks_and_windows(spx, fmt, log2_beta):
    # enough entries for several balance partitions, more rows than one window, a row longer than
    # the balance target, empty rows, and block sizes from tiny to the default rule
    rng = np.random.default_rng(12)
    m, n = 20000, 9000
    row = np.concatenate([rng.zipf(1.6, 200_000) % m, np.full(70_000, 12345), [m - 1]])
    col = rng.integers(0, n, len(row))
    row, col = row.astype(np.int32), col.astype(np.int32)
    for kind in ("int", "float"):
        val = synth.values(len(row), seed=13, kind=kind)
        x = synth.xvec(n, seed=14, kind=kind)
        ref = spmv.reference(m, n, row, col, val, x)
        A, y = _run(spx, fmt, m, n, row, col, val, x, log2_beta=log2_beta)
        say("  %s log2_beta %d: %d partitions" % (fmt, A.log2_beta, A.parts))
        assert A.parts >= 4
        if kind == "int":
            _check_int(y, ref, fmt)
        else:
            _check_float(y, ref, fmt)
        _check_structure(A, m, n, row, col, val)
