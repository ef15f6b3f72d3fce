"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import curves, formats, measure, mergepath, spmv


def _cells(tokens):
    return [tuple(int(v) for v in t.split(",")) for t in tokens]


# ---------------------------------------------------------------- Algorithm 1 and triplets


def _dense(m, n, row, col, val):
    A = np.zeros((m, n))
    for r, c, v in zip(row, col, val):
        A[r, c] += v
    return A


@pytest.mark.parametrize("seed", range(6))
def test_alg1_matches_dense_matvec_tiny(seed):
    rng = np.random.default_rng(seed)
    m, n = rng.integers(1, 40, size=2)
    E = int(rng.integers(0, 200))
    row = rng.integers(0, m, E).astype(np.int32)
    col = rng.integers(0, n, E).astype(np.int32)
    val = rng.uniform(-1, 1, E)
    x = rng.uniform(-1, 1, n)
    ref = spmv.reference(m, n, row, col, val, x)
    dense = _dense(m, n, row, col, val) @ x
    assert np.allclose(ref["y_ref"], dense, rtol=0, atol=1e-13 * (1 + np.abs(dense).max()))
    assert np.allclose(ref["y_plain"], dense, rtol=0, atol=1e-12 * (1 + np.abs(dense).max()))


@pytest.mark.parametrize("seed", range(4))
def test_alg1_exact_on_integers(seed):
    rng = np.random.default_rng(100 + seed)
    m, n, E = 50, 37, 900
    row = rng.integers(0, m, E).astype(np.int32)
    col = rng.integers(0, n, E).astype(np.int32)
    val = rng.integers(-3, 4, E).astype(np.float64)
    x = rng.integers(-3, 4, n).astype(np.float64)
    ref = spmv.reference(m, n, row, col, val, x)
    exact = np.zeros(m, dtype=object)
    for r, c, v in zip(row, col, val):
        exact[r] += int(v) * int(x[c])
    assert [int(v) for v in ref["y_plain"]] == list(exact)
    assert measure.equal_ignoring_zero_sign(ref["y_plain"], ref["y_ref"])


def test_alg1_special_cases():
    # identity gives x exactly
    n = 33
    x = synth.xvec(n, seed=5)
    idx = np.arange(n, dtype=np.int32)
    r = spmv.reference(n, n, idx, idx, np.ones(n), x)
    assert np.array_equal(r["y_plain"], x) and np.array_equal(r["y_ref"], x)
    # diagonal
    d = synth.values(n, seed=6)
    r = spmv.reference(n, n, idx, idx, d, x)
    assert np.array_equal(r["y_plain"], d * x)
    # nnz = 0 and all rows empty: y is +0
    r = spmv.reference(7, 5, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), np.ones(5))
    assert np.array_equal(r["y_plain"].view(np.int64), np.zeros(7, np.int64))
    assert np.array_equal(r["row_ptr"], np.zeros(8, np.int64))
    # 1 x 1
    r = spmv.reference(1, 1, np.array([0], np.int32), np.array([0], np.int32), np.array([2.5]),
                       np.array([-4.0]))
    assert r["y_plain"][0] == -10.0
    # m != n, one fully dense row among empty ones
    m, n = 5, 300
    row = np.full(n, 3, np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    x = np.arange(n, dtype=np.float64)
    r = spmv.reference(m, n, row, col, val, x)
    assert list(r["y_plain"]) == [0, 0, 0, n * (n - 1) / 2, 0]


def test_negative_zero_products_give_positive_zero():
    # 0 * (-1) = -0; Algorithm 1 starts each row at +0 so the row's result is +0
    r = spmv.reference(2, 2, np.array([0, 1], np.int32), np.array([1, 1], np.int32),
                       np.array([0.0, 1.0]), np.array([1.0, -1.0]))
    assert r["y_plain"][0] == 0.0 and not np.signbit(r["y_plain"][0])
    assert not np.signbit(r["y_ref"][0])


def test_duplicates_summed_in_original_order():
    # three repeats of (0, 0); their sum must be ((v0 + v1) + v2) in input order
    v = np.array([1e16, 1.0, -1e16])
    r, c, s, _ = spmv.canonical_coo(1, 1, np.zeros(3, np.int32), np.zeros(3, np.int32), v)
    assert len(s) == 1 and s[0] == (1e16 + 1.0) + -1e16 == 0.0
    v2 = np.array([1.0, 1e16, -1e16])
    _, _, s2, _ = spmv.canonical_coo(1, 1, np.zeros(3, np.int32), np.zeros(3, np.int32), v2)
    assert s2[0] == (1.0 + 1e16) + -1e16


def test_canonical_matches_dictionary_accumulation():
    rng = np.random.default_rng(7)
    m, n, E = 20, 9, 600
    row = rng.integers(0, m, E).astype(np.int32)
    col = rng.integers(0, n, E).astype(np.int32)
    val = rng.uniform(-1, 1, E)
    acc = {}
    for r, c, v in zip(row, col, val):  # input order
        key = (int(r), int(c))
        acc[key] = acc[key] + v if key in acc else v
    keys = sorted(acc)
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    assert list(zip(cr.tolist(), cc.tolist())) == keys
    assert np.array_equal(cv, np.array([acc[k] for k in keys]))


def test_shuffled_input_gives_identical_crs_on_integers():
    row, col = synth.rmat(10, 8, seed=3)
    val = synth.values(len(row), seed=3, kind="int")
    p = synth.permutation(len(row), seed=9)
    a = spmv.crs(1024, 1024, row, col, val)
    b = spmv.crs(1024, 1024, row[p], col[p], val[p])
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_row_sums_match_triplet_path():
    # A * 1 equals the row sums computed straight from the raw triplets (exact on integers)
    row, col = synth.rmat(11, 16, seed=4)
    val = synth.values(len(row), seed=4, kind="int")
    m = n = 2048
    ones = np.ones(n)
    y = spmv.alg1(*spmv.crs(m, n, row, col, val), ones)
    sums = np.zeros(m)
    np.add.at(sums, row, val)
    assert np.array_equal(y, sums)
    yt = spmv.triplet_spmv(m, row, col, val, ones)
    assert np.array_equal(y, yt)


def test_permutation_invariance_on_integers():
    # (P A Q^T)(Q x) = P (A x)
    m = n = 1024
    row, col = synth.rmat(10, 16, seed=8)
    val = synth.values(len(row), seed=8, kind="int")
    x = synth.xvec(n, seed=8, kind="int")
    P = synth.permutation(m, seed=11)
    Q = synth.permutation(n, seed=12)
    y = spmv.alg1(*spmv.crs(m, n, row, col, val), x)
    Pinv = np.empty_like(P); Pinv[P] = np.arange(m)
    Qinv = np.empty_like(Q); Qinv[Q] = np.arange(n)
    # row i of the new matrix is old row P[i]; column j is old column Q[j]
    y2 = spmv.alg1(*spmv.crs(m, n, Pinv[row].astype(np.int32), Qinv[col].astype(np.int32), val),
                   x[Q])
    assert np.array_equal(y2, y[P])


def test_linearity_within_tolerance():
    m = n = 512
    row, col = synth.rmat(9, 16, seed=2)
    val = synth.values(len(row), seed=2)
    x1 = synth.values(n, seed=21)
    x2 = synth.values(n, seed=22)
    rp, c, v = spmv.crs(m, n, row, col, val)
    _, y1, s1 = spmv.alg1_accurate(rp, c, v, x1)
    _, y2, s2 = spmv.alg1_accurate(rp, c, v, x2)
    _, y12, s12 = spmv.alg1_accurate(rp, c, v, 2.0 * x1 - 3.0 * x2)
    err = np.abs(y12 - (2 * y1 - 3 * y2))
    assert np.all(err <= 1e-14 * (2 * s1 + 3 * s2 + s12) + 1e-300)


def test_accurate_sum_against_exact_rational():
    rng = np.random.default_rng(5)
    # one long ill-conditioned row: large cancelling terms plus small ones
    k = 4000
    a = np.concatenate([rng.uniform(-1, 1, k) * 1e8, rng.uniform(-1, 1, k)])
    xs = np.concatenate([np.ones(k), rng.uniform(-1, 1, k)])
    a = np.concatenate([a, -a[:k]])
    xs = np.concatenate([xs, np.ones(k)])
    n = len(a)
    rp = np.array([0, n], np.int64)
    col = np.arange(n, dtype=np.int32)
    yp, yr, s = spmv.alg1_accurate(rp, col, a, xs)
    exact = sum(Fraction(float(u)) * Fraction(float(v)) for u, v in zip(a, xs))
    exact_f = float(exact)
    assert abs(yr[0] - exact_f) <= 2 * 2.0 ** -53 * abs(exact_f) + 1e-300
    assert s[0] == pytest.approx(float(sum(abs(Fraction(float(u)) * Fraction(float(v)))
                                           for u, v in zip(a, xs))), rel=1e-12)
    # the plain sum is far worse here, which is why the reference is the accurate one
    assert abs(yp[0] - exact_f) > abs(yr[0] - exact_f)


def test_accurate_sum_matches_fsum_random():
    rng = np.random.default_rng(6)
    for _ in range(20):
        k = int(rng.integers(1, 3000))
        a = rng.uniform(-1, 1, k)
        xs = rng.uniform(-1, 1, k)
        _, yr, _ = spmv.alg1_accurate(np.array([0, k], np.int64), np.arange(k, dtype=np.int32), a, xs)
        exact = float(sum(Fraction(float(u)) * Fraction(float(v)) for u, v in zip(a, xs)))
        assert abs(yr[0] - exact) <= 2.0 ** -52 * abs(exact) + 1e-300


def test_rows_reference_matches_full():
    m = n = 2048
    row, col = synth.rmat(11, 16, seed=1)
    val = synth.values(len(row), seed=1)
    x = synth.xvec(n, seed=1)
    full = spmv.reference(m, n, row, col, val, x)
    rows = np.array([0, 1, 5, 100, 2047, 1024])
    rr, yp, yr, s = spmv.rows_reference(m, n, row, col, val, x, rows)
    assert np.array_equal(yp, full["y_plain"][rr])
    assert np.array_equal(yr, full["y_ref"][rr])


# ---------------------------------------------------------------- curves


def test_hilbert_matches_figure(golden):
    for size, *cells in golden("hilbert_figure.txt"):
        k = int(size).bit_length() - 1
        assert curves.hilbert_order(k) == _cells(cells)


def test_zmorton_matches_figure(golden):
    for size, *cells in golden("zmorton_figure.txt"):
        k = int(size).bit_length() - 1
        assert curves.zmorton_order(k) == _cells(cells)


@pytest.mark.parametrize("k", range(0, 8))
def test_hilbert_bijective_unit_steps(k):
    side = 1 << k
    order = curves.hilbert_order(k)
    assert len(set(order)) == side * side
    for (r0, c0), (r1, c1) in zip(order, order[1:]):
        assert abs(r0 - r1) + abs(c0 - c1) == 1  # one index changes, by one (Section 4.1)


@pytest.mark.parametrize("k", [9, 10, 13])
def test_hilbert_array_bijective_large(k):
    side = 1 << k
    rng = np.random.default_rng(k)
    if k <= 10:
        r, c = np.divmod(np.arange(side * side, dtype=np.int64), side)
        d = curves.hilbert_index_array(k, r, c)
        assert np.array_equal(np.sort(d), np.arange(side * side))
    else:
        r = rng.integers(0, side, 2000)
        c = rng.integers(0, side, 2000)
        d = curves.hilbert_index_array(k, r, c)
        assert np.all((d >= 0) & (d < side * side))
    r = rng.integers(0, side, 500)
    c = rng.integers(0, side, 500)
    d = curves.hilbert_index_array(k, r, c)
    assert [curves.hilbert_index(k, a, b) for a, b in zip(r, c)] == d.tolist()


def test_hilbert_unit_steps_k10_vectorised():
    # every consecutive pair of the 1024 x 1024 curve differs by one in exactly one index
    k = 10
    side = 1 << k
    r, c = np.divmod(np.arange(side * side, dtype=np.int64), side)
    d = curves.hilbert_index_array(k, r, c)
    order = np.argsort(d)
    rr, cc = r[order], c[order]
    steps = np.abs(np.diff(rr)) + np.abs(np.diff(cc))
    assert np.all(steps == 1)
    assert rr[0] == 0 and cc[0] == 0


# ---------------------------------------------------------------- merge path


def test_merge_path_matches_figure(golden):
    g = {row[0]: row[1:] for row in golden("merge_path_figure.txt")}
    A = [int(v) for v in g["A"]]
    B = [int(v) for v in g["B"]]
    p = int(g["threads"][0])
    path, merged = mergepath.walk(A, B)
    assert path == _cells(g["path"])
    assert ["%s%d" % (s, v) for s, v in merged] == g["merged"]
    items = (len(A) + len(B)) // p
    assert mergepath.splits(A, B, items) == _cells(g["splits"])
    for i, j in path:
        assert mergepath.is_path_point(A, B, i, j)


@pytest.mark.parametrize("seed", range(10))
def test_merge_walk_equals_stable_merge(seed):
    rng = np.random.default_rng(seed)
    A = sorted(rng.integers(0, 20, int(rng.integers(0, 30))).tolist())
    B = sorted(rng.integers(0, 20, int(rng.integers(0, 30))).tolist())
    _, merged = mergepath.walk(A, B)
    # reference: sort tagged items by (value, list) with A before B on ties, stable within lists
    tagged = sorted([(v, 0, i) for i, v in enumerate(A)] + [(v, 1, i) for i, v in enumerate(B)])
    assert [("A" if t == 0 else "B", v) for v, t, _ in tagged] == merged
    path, _ = mergepath.walk(A, B)
    on = {(i, j) for i, j in path}
    for i in range(len(A) + 1):
        for j in range(len(B) + 1):
            assert mergepath.is_path_point(A, B, i, j) == ((i, j) in on)


def test_merge_spmv_bands_equals_alg1_on_integers():
    m = n = 256
    row, col = synth.rmat(8, 16, seed=6)
    val = synth.values(len(row), seed=6, kind="int")
    x = synth.xvec(n, seed=6, kind="int")
    rp, c, v = spmv.crs(m, n, row, col, val)
    y = spmv.alg1(rp, c, v, x)
    for items in (1, 3, 7, 64, 1000, 10 ** 6):
        yb, carries = mergepath.spmv_bands(rp, c, v, x, items)
        assert np.array_equal(yb, y)


def test_merge_spmv_long_row_spans_bands():
    # one row of 50 entries split over bands of 8 items must carry across 6+ bands
    n = 50
    rp = np.array([0, 0, n, n], np.int64)
    col = np.arange(n, dtype=np.int32)
    v = np.ones(n)
    x = np.arange(n, dtype=np.float64)
    yb, carries = mergepath.spmv_bands(rp, col, v, x, 8)
    assert list(yb) == [0.0, n * (n - 1) / 2, 0.0]
    assert sum(1 for r, _ in carries if r == 1) >= 6


# ---------------------------------------------------------------- block size, break-even


def test_csb_block_size_range():
    assert measure.csb_log2_beta_range(1 << 14) == (7, 10)
    assert measure.csb_log2_beta_range(1 << 24) == (12, 15)
    assert measure.csb_log2_beta_range(10 ** 7) == (12, 15)
    assert measure.csb_log2_beta_range(1) == (0, 3)
    # 4^t >= n boundary
    assert measure.ceil_log2_sqrt(17) == 3 and measure.ceil_log2_sqrt(16) == 2


def test_csb_block_size_rule():
    assert measure.csb_log2_beta(1 << 14, 1 << 14) == 10
    assert measure.csb_log2_beta(1 << 24, 1 << 24) == 13  # budget of 64 KiB of doubles
    assert measure.csb_log2_beta(10 ** 7, 10 ** 7) == 13
    # without an on-chip budget the paper's 16-bit cap applies: n = 2^30 -> range (15, 18) -> 16
    assert measure.csb_log2_beta(1 << 30, 1 << 30, lds_bytes=1 << 40) == 16
    assert measure.csb_log2_beta(1 << 24, 1 << 24, lds_bytes=1 << 40) == 15


def test_break_even_reproduces_paper(golden):
    for fmt, mach, dens, s_crs, s_fmt, c_crs, c_fmt, pub in golden("break_even_tables.txt"):
        nstar = measure.break_even_from_ratios(float(c_fmt), float(c_crs), float(s_crs),
                                               float(s_fmt))
        # tables are rounded to one decimal, so the count is recovered to within ~1%
        assert abs(nstar - float(pub)) <= 0.01 * float(pub) + 0.5, (fmt, nstar, pub)
    assert round(measure.break_even_from_ratios(10.9, 7.8, 2.9, 3.3)) == 26
    assert round(measure.break_even_from_ratios(69.6, 7.8, 2.9, 3.4)) == 420
    # brute force on the definition: the first whole N at which the format's total time is
    # no larger than the reference's
    for cf, cr, sr, sf in [(10, 4, 3, 1), (4, 10, 3, 1), (5, 5, 2, 1), (7, 3, 1, 2)]:
        first = next((N for N in range(0, 100) if cf + N * sf <= cr + N * sr), math.inf)
        nb = measure.break_even(cf, cr, sr, sf)
        assert (math.isinf(nb) and math.isinf(first)) or math.ceil(nb) == first
    assert measure.break_even(5.0, 1.0, 1.0, 1.0) == math.inf
    assert measure.break_even(3.0, 1.0, 2.0, 1.0) == 2.0


def test_scaled_error_metric():
    e = measure.scaled_error([1.0, 0.0, -0.0, 1e-3], [1.0 + 1e-15, 0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0])
    assert e[0] == pytest.approx(1e-15, rel=1e-3) and e[1] == 0 and e[2] == 0 and e[3] == np.inf
    assert measure.equal_ignoring_zero_sign([0.0, -0.0, 1.0], [-0.0, 0.0, 1.0])
    assert not measure.equal_ignoring_zero_sign([1.0], [np.nextafter(1.0, 2.0)])


# ---------------------------------------------------------------- format decoders


def test_check_crs_hand_made():
    # 3x4: row 0 = {(0,1)=2}, row 1 empty, row 2 = {(2,0)=-1, (2,3)=5}
    rp = [0, 1, 1, 3]
    formats.check_crs(3, 4, rp, [1, 0, 3], [2.0, -1.0, 5.0], [0, 2, 2], [1, 0, 3], [2.0, -1.0, 5.0])
    with pytest.raises(AssertionError):
        formats.check_crs(3, 4, rp, [1, 3, 0], [2.0, 5.0, -1.0], [0, 2, 2], [1, 0, 3],
                          [2.0, -1.0, 5.0])
    with pytest.raises(AssertionError):
        formats.check_crs(3, 4, [0, 2, 2, 3], [1, 0, 3], [2.0, -1.0, 5.0], [0, 2, 2], [1, 0, 3],
                          [2.0, -1.0, 5.0])


def test_check_csbh_hand_made():
    # 4x4 matrix, beta = 2 (k=1): blocks (0,0),(0,1),(1,0),(1,1)
    # entries: (0,0)=1, (1,0)=2, (0,1)=3 in block 0; (3,3)=4 in block 3
    # Hilbert order of 2x2 local cells: (0,0),(1,0),(1,1),(0,1)
    blk_ptr = [0, 3, 3, 3, 4]
    packed = [(0 << 16) | 0, (1 << 16) | 0, (0 << 16) | 1, (1 << 16) | 1]
    val = [1.0, 2.0, 3.0, 4.0]
    formats.check_csbh(4, 4, 1, blk_ptr, packed, val, [0, 0, 1, 3], [0, 1, 0, 3],
                       [1.0, 3.0, 2.0, 4.0])
    with pytest.raises(AssertionError):  # row-major instead of Hilbert inside block 0
        formats.check_csbh(4, 4, 1, blk_ptr, [0, 1, 1 << 16, (1 << 16) | 1], [1.0, 3.0, 2.0, 4.0],
                           [0, 0, 1, 3], [0, 1, 0, 3], [1.0, 3.0, 2.0, 4.0])


# ---------------------------------------------------------------- generators (parity unpinned)


def test_rmat_s14_statistics():
    row, col = synth.rmat(14, 16, seed=0)
    assert len(row) == 262144
    key = row.astype(np.int64) * 16384 + col
    u = np.unique(key)
    assert 0.85 < len(u) / len(row) < 0.89
    counts = np.bincount(u // 16384, minlength=16384)
    assert 0.30 < np.mean(counts == 0) < 0.36
    # first-level quadrant frequencies within 5 sigma of (a, b, c, d)
    top_r = row >> 13
    top_c = col >> 13
    E = len(row)
    for (qr, qc), p in {(0, 0): .57, (0, 1): .19, (1, 0): .19, (1, 1): .05}.items():
        f = np.sum((top_r == qr) & (top_c == qc))
        assert abs(f - p * E) < 5 * math.sqrt(E * p * (1 - p))


def test_chunglu_small_statistics():
    n, E = 100_000, 2_000_000
    row, col = synth.chunglu(n, E, 2.1, seed=0)
    assert row.min() >= 0 and row.max() < n and col.min() >= 0 and col.max() < n
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1 / 1.1)
    p0 = w[0] / w.sum()
    f0 = np.mean(row == 0)
    assert abs(f0 - p0) < 5 * math.sqrt(p0 * (1 - p0) / E)


def test_generators_deterministic():
    a = synth.rmat(10, 4, seed=3)
    b = synth.rmat(10, 4, seed=3)
    assert all(np.array_equal(u, v) for u, v in zip(a, b))
    assert not np.array_equal(synth.rmat(10, 4, seed=4)[0], a[0])
    v = synth.values(1000, seed=1, kind="int")
    assert set(np.unique(v).tolist()) <= set(range(-3, 4))
    f = synth.values(100000, seed=1)
    assert f.min() >= -1 and f.max() < 1 and abs(f.mean()) < 0.02


# ---------------------------------------------------------------- reduced-precision forms

from oracle import precision  # noqa: E402


def _bf16_candidates(x):
    # brute force: all bfloat16 values (as float32 bit patterns with 16 zero low bits) around x
    f = np.float32(x)
    hi = int(np.array([f], np.float32).view(np.uint32)[0]) >> 16
    cands = []
    for h in range(hi - 2, hi + 3):
        c = np.array([(h & 0xFFFF) << 16], np.uint32).view(np.float32)[0]
        if np.isfinite(c):
            cands.append((float(c), h & 0xFFFF))
    return cands


def test_bf16_rounding_brute_force():
    rng = np.random.default_rng(17)
    sub = np.ldexp(rng.uniform(0.5, 1, 300), rng.integers(-140, -124, 300))  # near 2^-126
    vals = np.concatenate([rng.uniform(-1, 1, 3000), rng.uniform(-300, 300, 1000),
                           sub, -sub, np.ldexp(rng.uniform(0.5, 1, 200), 127),
                           [1.0, -1.0, 3.0, 255.0, 256.0, 257.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9,
                            1e-3, 2.0 ** -126, 2.0 ** -133, 1.5 * 2.0 ** -133, 2.5 * 2.0 ** -133,
                            2.0 ** -134, 3 * 2.0 ** -135]])
    got = precision.round_bf16(vals)
    for v, g in zip(vals, got):
        cands = _bf16_candidates(v)
        best = min(abs(c - v) for c, _ in cands)
        near = [(c, h) for c, h in cands if abs(c - v) == best]
        if len(near) == 2:  # a tie goes to the even significand
            near = [(c, h) for c, h in near if h % 2 == 0]
        assert g == near[0][0], (v, g, near)
    # integers up to 256 are exact; 257 ties to 256 (even)
    assert list(precision.round_bf16([3.0, -3.0, 256.0, 257.0])) == [3.0, -3.0, 256.0, 256.0]
    # subnormals: spacing 2^-133; 2^-134 ties to 0 (even), 3 2^-135 rounds up to 2^-133
    assert list(precision.round_bf16([2.0 ** -134, 3 * 2.0 ** -135, 1.5 * 2.0 ** -133])) == \
        [0.0, 2.0 ** -133, 2.0 ** -132]
    # overflow: the largest finite value is (2 - 2^-7) 2^127; halfway to 2^128 ties to the even
    # significand, which is the infinity
    big = (2 - 2.0 ** -7) * 2.0 ** 127
    assert precision.round_bf16([big, -big])[0] == big
    assert np.isinf(precision.round_bf16([(2 - 2.0 ** -8) * 2.0 ** 127])[0])
    assert np.array_equal(np.signbit(precision.round_bf16([-0.0, 0.0])), [True, False])
    assert precision.round_bf16([1 + 2 ** -8])[0] == 1.0          # tie -> even
    assert precision.round_bf16([1 + 3 * 2 ** -9])[0] == 1 + 2 ** -7


def test_f32_rounding_and_bound():
    v = np.array([1 + 2 ** -24, 1 + 3 * 2 ** -25, 0.1])
    r = precision.round_f32(v)
    assert r[0] == 1.0 and r[1] == 1 + 2 ** -23
    assert abs(r[2] - 0.1) <= 0.1 * precision.U32
    # the bound covers a brute-force FP32 evaluation of random dot products
    rng = np.random.default_rng(3)
    for k in (1, 10, 1000):
        a = rng.uniform(-1, 1, k)
        x = rng.uniform(-1, 1, k)
        af = a.astype(np.float32)
        xf = x.astype(np.float32)
        acc = np.float32(0)
        for p in af * xf:
            acc = np.float32(acc + p)
        exact = float(sum(Fraction(float(u)) * Fraction(float(w)) for u, w in zip(a, x)))
        s = float(np.sum(np.abs(a * x)))
        assert abs(float(acc) - exact) <= precision.dot_error_bound(k, precision.U32) * s


def test_spmm_equals_dense_product():
    # Y = A X for several right-hand sides against a dense matrix product; integer values keep
    # every sum exact, so equality is bitwise
    rng = np.random.default_rng(11)
    for m, n, E, k in [(7, 5, 20, 3), (1, 9, 6, 4), (12, 1, 15, 2), (6, 6, 0, 5)]:
        row = rng.integers(0, m, E)
        col = rng.integers(0, n, E)
        val = rng.integers(-3, 4, E).astype(np.float64)
        X = rng.integers(-3, 4, (n, k)).astype(np.float64)
        dense = np.zeros((m, n))
        np.add.at(dense, (row, col), val)
        rp, c, v = spmv.crs(m, n, row, col, val)
        Y, R, S = spmv.spmm(rp, c, v, X)
        assert np.array_equal(Y, dense @ X) and np.array_equal(R, dense @ X)
        assert np.array_equal(S, dense_abs(m, n, row, col, val) @ np.abs(X))


def dense_abs(m, n, row, col, val):
    """|A| of the summed entries (repeats summed first, then the absolute value)."""
    d = np.zeros((m, n))
    np.add.at(d, (row, col), val)
    return np.abs(d)


def test_hilbert_prefix_is_block_order():
    # the Hilbert index of level K2 + k of (row, col), shifted right by 2k, is the Hilbert index of
    # level K2 of the block (row >> k, col >> k): the curve visits every aligned sub-square whole
    rng = np.random.default_rng(21)
    for K2, k in [(1, 1), (2, 3), (3, 2), (5, 4)]:
        side = 1 << (K2 + k)
        r = rng.integers(0, side, 4000)
        c = rng.integers(0, side, 4000)
        full = curves.hilbert_index_array(K2 + k, r, c)
        assert np.array_equal(full >> (2 * k), curves.hilbert_index_array(K2, r >> k, c >> k))


def test_bcoh_partitions_and_order():
    from oracle import bcoh
    rng = np.random.default_rng(4)
    # partitions: cover the rows, never span more than WINDOW rows, split where the cumulative
    # raw count crosses a multiple of the target
    m, E = 30000, 500_000
    rows = np.minimum(rng.zipf(1.3, E) - 1, m - 1)
    st = bcoh.partition_starts(m, rows, E)
    assert st[0] == 0 and st[-1] == m and np.all(np.diff(st) > 0)
    assert np.all(np.diff(st) <= bcoh.WINDOW)
    cum = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))])
    t = bcoh.target(E)
    for a, b in zip(st[:-1], st[1:]):  # inside a partition no row crosses a bucket boundary
        inner = np.arange(a + 1, b)
        assert np.all(cum[inner] // t == cum[inner - 1] // t)
        assert (a % bcoh.WINDOW == 0) or a == 0 or cum[a] // t != cum[a - 1] // t
    # order on a small example, checked by brute force against the definitions
    m, n, k = 40, 36, 2
    r = rng.integers(0, m, 300)
    c = rng.integers(0, n, 300)
    st = np.array([0, 13, 29, m])
    for hil in (False, True):
        perm, part, br, bc = bcoh.order(m, n, k, r, c, st, hil)
        K2 = bcoh.ceil_log2(max(-(-m // 4), -(-n // 4)))
        def bkey(i):
            p = int(np.searchsorted(st, r[i], side="right") - 1)
            if hil:
                return (p, curves.hilbert_index(K2 + k, r[i], c[i]))
            return (p, curves.hilbert_index(K2, r[i] >> k, c[i] >> k), r[i], c[i])
        want = sorted(range(len(r)), key=lambda i: (bkey(i), i))
        assert [bkey(i) for i in perm] == [bkey(i) for i in want]


def _bcoh_hand_made():
    """A 4 x 4 matrix with beta = 2 (k = 1), written out by hand.

    Raw triplets: row 0 holds 70000 raw entries (repeats of (0,0) and (0,3)), then (2,1), (3,0),
    (3,1): E = 70003, target = 2^16, so the 65536th raw triplet lies in row 0 and row 1 starts the
    second partition: partitions are rows [0,1) and [1,4).
    Canonical entries: (0,0)=1, (0,3)=2, (2,1)=3, (3,0)=4, (3,1)=5.
    Block Hilbert order (level 1, the figure's 2x2 order over (block row, block column)):
    (0,0), (1,0), (1,1), (0,1).  Hilbert index of level 2 of the entries (figure's 4x4 order):
    (0,0)->0, (0,3)->15, (2,1)->7, (3,0)->5, (3,1)->6.
    """
    raw_rows = np.array([0] * 70000 + [2, 3, 3])
    crow, ccol, cval = [0, 0, 2, 3, 3], [0, 3, 1, 0, 1], [1.0, 2.0, 3.0, 4.0, 5.0]
    part_row, part_blk = [0, 1, 4], [0, 2, 3]
    blk_ptr = [0, 1, 2, 5]
    blk_coord = [(0 << 16) | 0, (0 << 16) | 1, (1 << 16) | 0]
    # BCOHC: partition 0 = blocks (0,0) then (0,1); partition 1 = block (1,0) row by row
    c_packed = [0, 1, (0 << 16) | 1, (1 << 16) | 0, (1 << 16) | 1]
    c_vals = [1.0, 2.0, 3.0, 4.0, 5.0]
    # BCOHCH: partition 1 in Hilbert order of (row, col): (3,0), (3,1), (2,1)
    h_packed = [0, 1, (1 << 16) | 0, (1 << 16) | 1, (0 << 16) | 1]
    h_vals = [1.0, 2.0, 4.0, 5.0, 3.0]
    return (raw_rows, crow, ccol, cval, part_row, part_blk, blk_ptr, blk_coord,
            (c_packed, c_vals), (h_packed, h_vals))


def test_bcoh_decode_and_check_hand_made():
    from oracle import bcoh
    (raw_rows, crow, ccol, cval, part_row, part_blk, blk_ptr, blk_coord, C, H) = _bcoh_hand_made()
    E = len(raw_rows)
    # decode gives the triplets in storage order
    r, c, v = bcoh.decode(1, blk_ptr, blk_coord, *C)
    assert r.tolist() == [0, 0, 2, 3, 3] and c.tolist() == [0, 3, 1, 0, 1]
    assert v.tolist() == [1.0, 2.0, 3.0, 4.0, 5.0]
    r, c, v = bcoh.decode(1, blk_ptr, blk_coord, *H)
    assert r.tolist() == [0, 0, 3, 3, 2] and c.tolist() == [0, 3, 0, 1, 1]
    for hil, (pk, vals) in ((False, C), (True, H)):
        args = dict(m=4, n=4, k=1, raw_rows=raw_rows, E=E, part_row=part_row, part_blk=part_blk,
                    blk_ptr=blk_ptr, blk_coord=blk_coord, packed=pk, values=vals, crow=crow,
                    ccol=ccol, cval=cval, hilbert_entries=hil)
        bcoh.check_bcoh(**args)
        other = H if not hil else C      # the other format's storage order
        bad = [dict(packed=other[0], values=other[1]),                 # wrong order inside a block
               dict(part_row=[0, 4]),                                  # one partition only
               dict(part_blk=[0, 1, 3]),                               # wrong first block
               dict(blk_ptr=[0, 2, 2, 5]),                             # empty block
               dict(blk_coord=[0, 1, (1 << 16) | 1]),                  # block (1,1) instead of (1,0)
               dict(values=list(vals[:4]) + [np.nextafter(vals[4], 9.0)])]   # one value off by 1 ulp
        for b in bad:
            with pytest.raises(AssertionError):
                bcoh.check_bcoh(**dict(args, **b))


def _partition_starts_by_positions(m, raw_rows):
    """Partition starts from the reading, computed through sorted triplet positions: the row after
    the one holding the (j * target)-th raw triplet (1-based, triplets sorted by row) starts a
    partition, for j = 1, 2, ...; so do row 0 and every multiple of the row window."""
    from oracle import bcoh
    srt = sorted(int(r) for r in raw_rows)
    t = bcoh.target(len(srt))
    starts = {0}
    starts.update(range(0, m, bcoh.WINDOW))
    j = 1
    while j * t <= len(srt):
        q = srt[j * t - 1]
        if q + 1 < m:
            starts.add(q + 1)
        j += 1
    return sorted(starts) + [m]


def test_bcoh_partition_starts_brute_force():
    from oracle import bcoh
    rng = np.random.default_rng(11)
    cases = [(30000, np.minimum(rng.zipf(1.3, 500_000) - 1, 29999)),     # heavy head rows
             (20000, rng.integers(0, 20000, 300_000)),                   # uniform
             (9000, np.repeat([3, 8191, 8192, 8999], [200_000, 10, 70_000, 5]))]  # long rows, window edge
    for m, rows in cases:
        got = bcoh.partition_starts(m, rows, len(rows)).tolist()
        assert got == _partition_starts_by_positions(m, rows)


def test_zmorton_array_matches_scalar_and_figure(golden):
    # the vectorised descent agrees with the scalar one on every cell up to 64 x 64, and both with
    # the figure's 8 x 8 order
    for k in range(7):
        side = 1 << k
        r, c = np.divmod(np.arange(side * side), side)
        want = [curves.zmorton_index(k, a, b) for a, b in zip(r, c)]
        assert curves.zmorton_index_array(k, r, c).tolist() == want
    for size, *cells in golden("zmorton_figure.txt"):
        k = int(size).bit_length() - 1
        rc = np.array(_cells(cells))
        assert curves.zmorton_index_array(k, rc[:, 0], rc[:, 1]).tolist() == list(range(len(cells)))


def test_check_csb_zmorton_hand_made():
    # 4x4, beta = 2: block 0 holds (0,0)=1, (0,1)=3, (1,0)=2; block 3 holds (3,3)=4.
    # Z-Morton order inside a 2x2 block (the paper's figure): TL, TR, BL, BR.
    blk_ptr = [0, 3, 3, 3, 4]
    z_packed = [(0 << 16) | 0, (0 << 16) | 1, (1 << 16) | 0, (1 << 16) | 1]
    z_val = [1.0, 3.0, 2.0, 4.0]
    canon = ([0, 0, 1, 3], [0, 1, 0, 3], [1.0, 3.0, 2.0, 4.0])
    formats.check_csb(4, 4, 1, blk_ptr, z_packed, z_val, *canon, "zmorton")
    # the Hilbert order of the same block is not Z-Morton order (and vice versa)
    h_packed = [(0 << 16) | 0, (1 << 16) | 0, (0 << 16) | 1, (1 << 16) | 1]
    h_val = [1.0, 2.0, 3.0, 4.0]
    formats.check_csb(4, 4, 1, blk_ptr, h_packed, h_val, *canon, "hilbert")
    with pytest.raises(AssertionError):
        formats.check_csb(4, 4, 1, blk_ptr, h_packed, h_val, *canon, "zmorton")
    with pytest.raises(AssertionError):
        formats.check_csb(4, 4, 1, blk_ptr, z_packed, z_val, *canon, "hilbert")
    with pytest.raises(AssertionError):   # entry moved to the wrong block
        formats.check_csb(4, 4, 1, [0, 2, 3, 3, 4], z_packed, z_val, *canon, "zmorton")


def test_csbr_check_hand_made():
    # panels of 2 rows (pb = 1) and blocks of 2 ranks (rb = 1), written out by hand.
    # raw triplets (row, col, value): (0,2,1) (0,2,2) (1,0,4) (2,2,5) (2,3,6) (1,2,7) (0,3,8)
    # raw row counts 3, 2, 2: row ranking 0, 1, 2 (the tie by increasing row)
    # raw column counts: col 0 -> 1, col 1 -> 0, col 2 -> 4, col 3 -> 2, so the ranking is
    # col 2, col 3, col 0 (col 1 has no triplet); 3 ranks -> rank field of 2 bits -> 2 segments.
    raw_rows = [0, 0, 1, 2, 2, 1, 0]
    raw_cols = [2, 2, 0, 2, 3, 2, 3]
    canon = ([0, 0, 1, 1, 2, 2], [2, 3, 0, 2, 2, 3], [3.0, 8.0, 4.0, 7.0, 5.0, 6.0])
    order = [2, 3, 0]
    rows = [0, 1, 2]
    # panel 0 (rows 0-1), segment 0 (ranks 0-1): (0,2) (1,2) (0,3); segment 1: (1,0)
    # panel 1 (row 2), segment 0: (2,2) (2,3); segment 1: empty
    blk_ptr = [0, 3, 4, 6, 6]
    packed = [0, 1, 2, 1, 0, 2]    # (rank mod 2) << 1 | (row rank mod 2)
    vals = [3.0, 7.0, 8.0, 4.0, 5.0, 6.0]
    assert formats.csbr_row_order(3, raw_rows).tolist() == rows
    assert formats.csbr_col_order(3, 4, raw_rows, raw_cols, pb=1).tolist() == order
    r, c, panel, crank, rrank = formats.decode_csbr(rows, blk_ptr, packed, order, pb=1, rb=1)
    assert r.tolist() == [0, 1, 0, 1, 2, 2] and c.tolist() == [2, 2, 3, 0, 2, 3]
    assert crank.tolist() == [0, 0, 1, 2, 0, 1]
    ok = dict(m=3, n=4, raw_rows=raw_rows, raw_cols=raw_cols, blk_ptr=blk_ptr, packed=packed,
              val=vals, col_order=order, row_order=rows, canon_row=canon[0], canon_col=canon[1],
              canon_val=canon[2], pb=1, rb=1)
    formats.check_csbr(**ok)
    bad = [dict(packed=[1, 0, 2, 1, 0, 2], val=[7.0, 3.0, 8.0, 4.0, 5.0, 6.0]),  # rows swapped
           dict(col_order=[3, 2, 0]),                                         # ranking
           dict(col_order=[2, 3, 0, 1]),                                      # untouched column
           dict(row_order=[1, 0, 2]),                                         # row ranking
           dict(blk_ptr=[0, 4, 4, 6, 6]),                                     # segment boundary
           dict(blk_ptr=[0, 3, 4, 6]),                                        # segment count
           dict(val=[3.0, 7.0, 8.0, 4.0, 5.0, np.nextafter(6.0, 9.0)])]       # one value 1 ulp off
    for b in bad:
        with pytest.raises(AssertionError):
            formats.check_csbr(**dict(ok, **b))


def test_csbr_ranked_rows_hand_made():
    # rows reordered by the ranking (pb = 1, rb = 1), written out by hand.
    # raw triplets (row, col, value): (3,0,1) (3,1,2) (3,2,3) (1,1,4) (0,2,5) (0,0,6)
    # row counts: row 3 -> 3, row 0 -> 2, row 1 -> 1, row 2 -> 0: row ranking 3, 0, 1 (row 2 has
    # no rank); panel 0 = row ranks 0-1 (rows 3, 0), panel 1 = row rank 2 (row 1).
    # column counts all 2; first/last panel: col 0 (0,0), col 1 (0,1), col 2 (0,0) -> column
    # ranking 0, 2, 1.  (panel, column rank, row rank) of each triplet, in storage order:
    # (0,0,0)=1 (0,0,1)=6 (0,1,0)=3 (0,1,1)=5 | (0,2,0)=2 | panel 1 segment 0 empty | (1,2,2)=4
    raw_rows = [3, 3, 3, 1, 0, 0]
    raw_cols = [0, 1, 2, 1, 2, 0]
    rows, order = [3, 0, 1], [0, 2, 1]
    assert formats.csbr_row_order(4, raw_rows).tolist() == rows
    assert formats.csbr_col_order(4, 3, raw_rows, raw_cols, pb=1).tolist() == order
    blk_ptr = [0, 4, 5, 5, 6]
    packed = [0, 1, 2, 3, 0, 0]
    vals = [1.0, 6.0, 3.0, 5.0, 2.0, 4.0]
    canon = ([0, 0, 1, 3, 3, 3], [0, 2, 1, 0, 1, 2], [6.0, 5.0, 4.0, 1.0, 2.0, 3.0])
    ok = dict(m=4, n=3, raw_rows=raw_rows, raw_cols=raw_cols, blk_ptr=blk_ptr, packed=packed,
              val=vals, col_order=order, row_order=rows, canon_row=canon[0], canon_col=canon[1],
              canon_val=canon[2], pb=1, rb=1)
    formats.check_csbr(**ok)
    r, c, _, _, _ = formats.decode_csbr(rows, blk_ptr, packed, order, pb=1, rb=1)
    y = np.zeros(4)
    np.add.at(y, r, np.asarray(vals) * np.array([1.0, 10.0, 100.0])[c])
    assert y.tolist() == [506.0, 40.0, 0.0, 321.0]
    for b in (dict(row_order=[3, 1, 0]), dict(col_order=[0, 1, 2]),
              dict(blk_ptr=[0, 4, 4, 5, 6])):
        with pytest.raises(AssertionError):
            formats.check_csbr(**dict(ok, **b))


def test_csbr_ranking_ties_and_empty():
    # panels of 2 rows (pb = 1).  Rows 0-6 hold 2, 2, 1, 1, 1, 1, 1 triplets, so the row ranking
    # is 0, 1, 2, 3, 4, 5, 6 (the identity) and a row's panel is row >> 1.
    # Columns 0, 1, 3, 5 have two triplets each, column 4 one, column 2 none:
    #   col 5: rows 4, 0 -> panels 2, 0 (first 0, last 2)
    #   col 1: rows 1, 5 -> panels 0, 2 (first 0, last 2; ties col 5, lower column first)
    #   col 3: rows 2, 3 -> panels 1, 1
    #   col 0: rows 0, 1 -> panels 0, 0
    # ranking: count 2 by (first, last, column): 0 (0,0), 1 (0,2), 5 (0,2), 3 (1,1); then 4.
    rows = [4, 0, 1, 5, 2, 3, 0, 1, 6]
    cols = [5, 5, 1, 1, 3, 3, 0, 0, 4]
    assert formats.csbr_row_order(7, rows).tolist() == [0, 1, 2, 3, 4, 5, 6]
    assert formats.csbr_col_order(7, 6, rows, cols, pb=1).tolist() == [0, 1, 5, 3, 4]
    # one panel for all rows: equal counts fall back to increasing column order
    assert formats.csbr_col_order(7, 6, rows, cols, pb=3).tolist() == [0, 1, 3, 5, 4]
    assert formats.csbr_col_order(3, 3, [], []).tolist() == []
    assert formats.csbr_row_order(3, []).tolist() == []


def test_csbr_ranking_brute_force():
    # tiny random cases against both rules applied row by row and column by column in plain
    # Python
    rng = np.random.default_rng(11)
    for _ in range(200):
        m, n = int(rng.integers(1, 16)), int(rng.integers(1, 12))
        E, pb = int(rng.integers(0, 40)), int(rng.integers(0, 3))
        rows = rng.integers(0, m, E).tolist()
        cols = rng.integers(0, n, E).tolist()
        rk = sorted((-rows.count(r), r) for r in range(m) if rows.count(r) > 0)
        want_rows = [r for _, r in rk]
        assert formats.csbr_row_order(m, rows).tolist() == want_rows
        rank_of = {r: i for i, r in enumerate(want_rows)}
        keyed = []
        for c in range(n):
            mine = [rank_of[r] >> pb for r, cc in zip(rows, cols) if cc == c]
            if mine:
                keyed.append(((-len(mine), min(mine), max(mine), c), c))
        want = [c for _, c in sorted(keyed)]
        assert formats.csbr_col_order(m, n, rows, cols, pb=pb).tolist() == want


def test_parcrs_equals_algorithm1_bitwise():
    # the row-parallel loop sums every row in the same order as Algorithm 1
    rng = np.random.default_rng(6)
    m, n, E = 5000, 4000, 60_000
    row = rng.integers(0, m, E)
    col = rng.integers(0, n, E)
    val = rng.uniform(-1, 1, E)
    x = rng.uniform(-1, 1, n)
    rp, c, v = spmv.crs(m, n, row, col, val)
    y1 = spmv.alg1(rp, c, v, x)
    for chunk in (1, 7, 512):
        y2, used = spmv.parcrs(rp, c, v, x, chunk)
        assert used >= 1
        assert np.array_equal(y1.view(np.int64), y2.view(np.int64))
