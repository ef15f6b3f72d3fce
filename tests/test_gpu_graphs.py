"""Products captured in HIP graphs (through torch.cuda.graph) and replayed: every replay equals the
eager product bit for bit, with unrelated eager work between replays; and the serving loop under
several submitting threads.

Bar: bitwise equality with the eager launch for graphs of the CRS formats (their sums have a fixed
order); the block formats (CSB, CSBH, BCOHC, BCOHCH, CSBR) add products into an LDS slice with
float atomics, whose order varies from run to run, so their replays are held to the product
tolerance (row-scaled 1e-12; for their FP32 / bfloat16 forms, which round y to FP32 once, one
FP32 rounding step, 2^-23 of the row scale) instead; for the threaded server, integer-valued
results bit-exact against the oracle.
"""
import sys
import threading

import numpy as np
import pytest

import synth
from oracle import measure, spmv

BLOCK_FORMATS = ("csbh", "csb", "bcohc", "bcohch", "csbr")

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def rmat14():
    row, col = synth.rmat(14, 16, seed=0)
    val = synth.values(len(row), seed=0)
    return (1 << 14), (1 << 14), row, col, val


def _capture(fn):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up on the capture stream (first-call scratch set up outside the graph)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


@pytest.mark.parametrize("fmt,vt", [("merge", "f64"), ("rowsplit", "f64"), ("csbh", "f64"),
                                    ("csb", "f64"), ("bcohc", "f64"), ("bcohch", "f64"),
                                    ("csbr", "f64"), ("merge", "f32"), ("rowsplit", "bf16"),
                                    ("csbr", "f32"), ("csbh", "bf16"), ("bcohch", "f32")])
def test_spmv_graph_replays(spx, rmat14, fmt, vt):
    import torch
    m, n, row, col, val = rmat14
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), fmt, value_type=vt)
    dt = torch.float64 if vt == "f64" else torch.float32
    x = _dev(synth.xvec(n, seed=3), dt)
    y = torch.empty(m, dtype=dt, device="cuda")
    A.spmv(x, out=y)
    torch.cuda.synchronize()
    eager = y.clone()
    scale = None
    if fmt in BLOCK_FORMATS:  # |A| |x| for the tolerance
        ref = spmv.reference(m, n, row, col, val, synth.xvec(n, seed=3))
        scale = ref["scale"]
    g = _capture(lambda: A.spmv(x, out=y))
    for rep in range(3):
        y.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        if scale is None:
            assert torch.equal(y, eager), "%s %s replay %d" % (fmt, vt, rep)
        else:
            # FP64 sums in a varying order; reduced forms then round y to FP32, where two such
            # sums can land one FP32 rounding step apart
            tol = 1e-12 if vt == "f64" else 2.0 ** -23
            err = measure.scaled_error(y.double().cpu().numpy(), eager.double().cpu().numpy(),
                                       scale)
            assert err.max() <= tol, "%s %s replay %d: %.3g" % (fmt, vt, rep, err.max())
    del g
    A.close()


@pytest.mark.parametrize("k", [1, 4, 33])
def test_spmm_graph_replays(spx, rmat14, k):
    import torch
    m, n, row, col, val = rmat14
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), "merge", value_type="f32")
    X = torch.rand((k, n), device="cuda").t()
    Y = torch.empty((k, m), device="cuda").t()
    A.spmm(X, out=Y)
    torch.cuda.synchronize()
    eager = Y.clone()
    g = _capture(lambda: A.spmm(X, out=Y))
    for rep in range(3):
        Y.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(Y, eager), "k=%d replay %d" % (k, rep)
    del g
    A.close()


def test_server_many_submitting_threads(spx):
    # four Python threads submit and wait concurrently (the C calls release the GIL)
    import torch
    mats = []
    for i, (scale, ef) in enumerate([(11, 8), (12, 16), (10, 32)]):
        row, col = synth.rmat(scale, ef, seed=40 + i)
        mats.append((1 << scale, 1 << scale, row, col, synth.values(len(row), seed=i, kind="int")))
    S = spx.Server(slots=3, max_batch=8)
    ids = [S.add_matrix(_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64),
                        (m, n), "merge", value_type="f32")[0] for m, n, r, c, v in mats]
    refs = []
    for m, n, r, c, v in mats:
        x = synth.xvec(n, seed=5, kind="int")
        refs.append((x, spmv.reference(m, n, r, c, v, x)["y_plain"]))
    errors = []

    def worker(t):
        try:
            outs = []
            for q in range(40):
                i = (t + q) % len(mats)
                y = torch.empty(mats[i][0], device="cuda")
                xt = _dev(refs[i][0], torch.float32)
                outs.append((i, y, xt, S.submit(ids[i], xt, y)))
            for i, y, xt, tk in outs:
                S.wait(tk)
                if not measure.equal_ignoring_zero_sign(y.cpu().numpy().astype(np.float64),
                                                        refs[i][1]):
                    errors.append((t, i))
        except Exception as e:  # reported below
            errors.append(repr(e))

    th = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    st = S.stats()
    say("threaded server: %d requests in %d batches" % (st["requests"], st["batches"]))
    assert not errors, errors[:5]
    assert st["requests"] == 160
    S.close()
