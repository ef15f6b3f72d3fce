"""Full-size parity on the benchmark workloads (R-MAT scale 24, the same matrix under a random
relabelling of rows and columns, and the Chung-Lu matrix with rows of up to ~1.8M entries), in
the launch configuration the benchmark times.

The oracle cannot canonicalise 2.7e8 triplets in seconds, so it is checked on sampled outputs:
  * sampled rows (random rows, the longest rows, first and last) against the oracle's Algorithm 1
    restricted to those rows (row-scaled error <= 1e-12), and their CRS slices bit-exactly;
  * sampled CSBH and CSB block rows decoded and compared bit-exactly with the oracle's canonical
    triplets of those rows, with the Hilbert (CSBH) or Z-Morton (CSB) order checked inside every
    block;
  * properties at every size: every merge tile start lies on the merge path; A 1 equals the row
    sums of the raw triplets within the row-scaled tolerance, for all rows.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import curves, measure, spmv

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
FMTS = ["rowsplit", "merge", "csbh", "csb", "bcohc", "bcohch", "csbr"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["rmat24", "rmat24p", "chunglu"])
def big(request):
    import torch

    from ._lib import ensure_built
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    import paper_2502_19284_amd as spx
    spx.use_torch_allocator(True)
    say("generating", request.param)
    w = synth.workload(request.param, seed=0)
    d = lambda a, t: torch.from_numpy(a).to("cuda", dtype=t)
    dev = dict(row=d(w["row"], torch.int32), col=d(w["col"], torch.int32),
               val=d(w["val"], torch.float64), x=d(w["x"], torch.float64))
    counts = np.bincount(w["row"], minlength=w["m"])
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([
        rng.integers(0, w["m"], 1500), np.argsort(counts)[-12:], [0, 1, w["m"] - 1]]))
    say("oracle on %d sampled rows" % len(sample))
    rr, yp, yr, sc = spmv.rows_reference(w["m"], w["n"], w["row"], w["col"], w["val"], w["x"],
                                          sample)
    yield spx, w, dev, (rr, yp, yr, sc)
    del dev
    torch.cuda.empty_cache()


def _convert(spx, w, dev, fmt):
    return spx.convert(dev["row"], dev["col"], dev["val"], (w["m"], w["n"]), fmt)


@pytest.mark.parametrize("fmt", FMTS)
def test_sampled_rows(big, fmt):
    import torch
    spx, w, dev, (rows, yp, yr, sc) = big
    say("full-size", fmt, "rows", len(rows))
    A = _convert(spx, w, dev, fmt)
    y = A.spmv(dev["x"])
    torch.cuda.synchronize()
    got = y[torch.from_numpy(rows).cuda()].cpu().numpy()
    err = measure.scaled_error(got, yr, sc)
    say("  max scaled error %.3g" % err.max())
    assert err.max() <= 1e-12
    A.close()


def test_crs_row_slices_exact(big):
    spx, w, dev, (rows, yp, yr, sc) = big
    A = _convert(spx, w, dev, "merge")
    rp = A.export("row_ptr").cpu().numpy()
    assert rp[0] == 0 and rp[-1] == A.nnz and np.all(np.diff(rp) >= 0)
    # canonical triplets of the sampled rows
    want = np.zeros(w["m"], dtype=bool)
    want[rows] = True
    sel = np.flatnonzero(want[w["row"]])
    cr, cc, cv, _ = spmv.canonical_coo(w["m"], w["n"], w["row"][sel], w["col"][sel],
                                       w["val"][sel])
    col = A.export("col_ind")
    val = A.export("values")
    for r in rows[:200]:
        lo, hi = int(rp[r]), int(rp[r + 1])
        mask = cr == r
        assert hi - lo == int(mask.sum()), r
        if hi > lo:
            assert np.array_equal(col[lo:hi].cpu().numpy(), cc[mask])
            assert np.array_equal(val[lo:hi].cpu().numpy().view(np.int64), cv[mask].view(np.int64))
    # merge tile starts lie on the merge path of (row ends, entry indices)
    co = A.export("parts").cpu().numpy().reshape(-1, 2).astype(np.int64)
    i, j = co[:, 0], co[:, 1]
    nnz = A.nnz
    ok1 = (i == 0) | (j >= nnz) | (rp[np.maximum(i, 1)] <= j)      # A[i-1] <= B[j]
    ok2 = (j == 0) | (i >= w["m"]) | (j - 1 < rp[np.minimum(i + 1, w["m"])])  # B[j-1] < A[i]
    assert np.all(ok1 & ok2)
    assert np.all(np.diff(i + j) >= 0) and (i[-1], j[-1]) == (w["m"], nnz)
    A.close()


@pytest.mark.parametrize("fmt", ["csbh", "csb"])
def test_csb_block_rows_exact(big, fmt):
    spx, w, dev, _ = big
    A = _convert(spx, w, dev, fmt)
    k = A.log2_beta
    beta = 1 << k
    assert k == measure.csb_log2_beta(w["m"], w["n"])
    nbc = (w["n"] + beta - 1) // beta
    nbr = (w["m"] + beta - 1) // beta
    bp = A.export("blk_ptr").cpu().numpy().astype(np.int64)
    assert bp[0] == 0 and bp[-1] == A.nnz and np.all(np.diff(bp) >= 0)
    packed = A.export("packed")
    val = A.export("values")
    for br in sorted({0, nbr // 2, nbr - 1}):
        lo, hi = int(bp[br * nbc]), int(bp[(br + 1) * nbc])
        p = packed[lo:hi].cpu().numpy().view(np.uint32).astype(np.int64)
        v = val[lo:hi].cpu().numpy()
        blk = np.repeat(np.arange(nbc), np.diff(bp[br * nbc:(br + 1) * nbc + 1]))
        lr, lc = p >> 16, p & 0xFFFF
        row = br * beta + lr
        colx = blk * beta + lc
        if fmt == "csbh":
            h = curves.hilbert_index_array(k, lr, lc)
        else:
            h = curves.zmorton_index_array(k, lr, lc)
        same = blk[1:] == blk[:-1]
        assert np.all(h[1:][same] > h[:-1][same])
        sel = np.flatnonzero((w["row"] >= br * beta) & (w["row"] < (br + 1) * beta))
        cr, cc, cv, _ = spmv.canonical_coo(w["m"], w["n"], w["row"][sel], w["col"][sel],
                                           w["val"][sel])
        o = np.lexsort((colx, row))
        assert np.array_equal(row[o], cr) and np.array_equal(colx[o], cc)
        assert np.array_equal(v[o].view(np.int64), cv.view(np.int64))
    A.close()


@pytest.mark.parametrize("fmt", FMTS)
def test_ones_gives_row_sums(big, fmt):
    import torch
    spx, w, dev, _ = big
    A = _convert(spx, w, dev, fmt)
    y = A.spmv(torch.ones(w["n"], dtype=torch.float64, device="cuda")).cpu().numpy()
    sums = np.bincount(w["row"], weights=w["val"], minlength=w["m"])
    scale = np.bincount(w["row"], weights=np.abs(w["val"]), minlength=w["m"])
    # both sides are rounded sums of the same terms: |y - sums| <= 2 k u scale is the bound of two
    # orders of summation of k terms; check the much tighter 1e-12 used for products
    err = measure.scaled_error(y, sums, scale)
    assert err.max() <= 1e-12, err.max()
    A.close()


def _sampled_crs(w, rows):
    """Canonical CRS of the sampled rows (renumbered 0..len-1), as rows_reference builds it."""
    mask = np.zeros(w["m"], dtype=bool)
    mask[rows] = True
    sel = np.flatnonzero(mask[w["row"]])
    local = np.searchsorted(rows, w["row"][sel]).astype(np.int32)
    return spmv.crs(len(rows), w["n"], local, w["col"][sel], w["val"][sel])


@pytest.mark.parametrize("fmt", ["rowsplit", "merge", "csbr", "csbh", "bcohc"])
@pytest.mark.parametrize("vt", ["f32", "bf16"])
def test_sampled_rows_reduced_precision(big, fmt, vt):
    # FP32 / bfloat16 stored values at full size: sampled rows within the FP32 dot-product bound
    # of the oracle on the rounded inputs; the error against the unrounded FP64 oracle is printed
    import torch

    from oracle import precision
    spx, w, dev, (rows, yp, yr, sc) = big
    A = spx.convert(dev["row"], dev["col"], dev["val"], (w["m"], w["n"]), fmt, value_type=vt)
    y = A.spmv(dev["x"].float())
    torch.cuda.synchronize()
    got = y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    rp, cc, cv = _sampled_crs(w, rows)
    rv = precision.round_f32(cv) if vt == "f32" else precision.round_bf16(cv)
    _, yr_r, s_r = spmv.alg1_accurate(rp, cc, rv, precision.round_f32(w["x"]))
    lens = np.diff(rp) + 2
    err = measure.scaled_error(got, yr_r, s_r)
    assert np.all(err <= precision.dot_error_bound(lens, 0.0) + 1e-300)
    e64 = measure.scaled_error(got, yr, sc)
    u = precision.U32 if vt == "f32" else precision.UBF16
    assert np.all(e64 <= precision.dot_error_bound(lens, u))
    say("  %s %s vs FP64 oracle on %d rows: max %.3g median %.3g" % (fmt, vt, len(rows), e64.max(),
                                                                       np.median(e64)))
    A.close()


def test_spmm_sampled_rows(big):
    # Y = A X with 4 column-major right-hand sides (FP32 values) on sampled rows of every column
    import torch

    from oracle import precision
    spx, w, dev, (rows, yp, yr, sc) = big
    k = 4
    X = np.stack([synth.xvec(w["n"], seed=40 + c) for c in range(k)], axis=1)
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda", dtype=torch.float32).t()
    A = spx.convert(dev["row"], dev["col"], dev["val"], (w["m"], w["n"]), "merge",
                    value_type="f32")
    Y = A.spmm(Xd)
    torch.cuda.synchronize()
    got = Y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    rp, cc, cv = _sampled_crs(w, rows)
    _, R, S = spmv.spmm(rp, cc, precision.round_f32(cv), precision.round_f32(X))
    bound = precision.dot_error_bound(np.diff(rp) + 2, 0.0)[:, None]
    err = np.abs(got - R)
    assert np.all(err <= bound * S + 1e-300)
    A.close()
