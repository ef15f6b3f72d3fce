"""GPU tests of the serving loop (include/spx_serve.h): results of coalesced batches against the
same requests served alone and against the CPU oracle, admission by memory footprint, the plain
one-request-per-launch path, open-loop replay, and argument errors.

Bar: integer-valued SpMV requests are bit-exact against the oracle and alone == in the mix
bitwise for every integer-valued request; float requests y = alpha A x + beta are within
alpha * (FP32 dot-product bound) * |A||x| + u32 * |y| of the oracle's exact value (alpha, beta as
the device forms them in FP32).
"""
import sys

import numpy as np
import pytest

import synth
from oracle import measure, precision, spmv

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


def _matrices(kind):
    """Four small matrices: three R-MAT, one Erdos-Renyi-like with normalised columns."""
    out = []
    for i, (scale, ef) in enumerate([(12, 8), (13, 16), (11, 32)]):
        row, col = synth.rmat(scale, ef, seed=10 + i)
        val = synth.values(len(row), seed=20 + i, kind=kind)
        out.append((1 << scale, 1 << scale, row, col, val))
    n = 3000
    row, col = synth.uniform(n, n, 8 * n, seed=30)
    if kind == "int":
        val = synth.values(len(row), seed=31, kind="int")
    else:  # column-stochastic: each entry 1 / (column count)
        cnt = np.bincount(col, minlength=n).astype(np.float64)
        val = 1.0 / cnt[col]
    out.append((n, n, row, col, val))
    return out


def _oracle(mat, vt, x, kind, d):
    m, n, row, col, val = mat
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    rp, _, _ = spmv.crs_from_canonical(m, cr, cc, cv)
    rv = precision.round_f32(cv) if vt == "f32" else precision.round_bf16(cv)
    y_plain, y_ref, s = spmv.alg1_accurate(rp, cc, rv, precision.round_f32(x))
    if kind == "spmv":
        return y_plain, y_ref, s, 1.0, 0.0, np.diff(rp)
    a = float(np.float32(d))
    b = float((np.float32(1.0) - np.float32(d)) / np.float32(n))  # the device's FP32 arithmetic
    return None, a * y_ref + b, s, a, b, np.diff(rp)


def _check(y, want, what):
    y_plain, y_ref, s, a, b, lens = want
    if y_plain is not None and a == 1.0 and b == 0.0 and np.all(np.round(y_ref) == y_ref):
        assert measure.equal_ignoring_zero_sign(y, y_plain), what
        return
    tol = a * precision.dot_error_bound(lens + 2, 0.0) * s + precision.U32 * np.abs(y_ref)
    err = np.abs(y - y_ref)
    assert np.all(err <= tol + 1e-300), "%s: worst excess %.3g" % (what, float((err - tol).max()))


@pytest.mark.parametrize("vt", ["f32", "bf16"])
@pytest.mark.parametrize("vkind", ["int", "float"])
@pytest.mark.parametrize("fmt", ["merge", "rowsplit"])
def test_serve_alone_and_in_mix(spx, vt, vkind, fmt):
    import torch
    mats = _matrices(vkind)
    S = spx.Server(slots=3, max_batch=16)
    ids = []
    for (m, n, row, col, val) in mats:
        mid, _ = S.add_matrix(_dev(row, torch.int32), _dev(col, torch.int32),
                              _dev(val, torch.float64), (m, n), fmt, value_type=vt)
        ids.append(mid)
    rng = np.random.default_rng(4)
    reqs = []
    for q in range(96):
        i = int(rng.integers(0, len(mats)))
        kind = "spmv" if q % 3 else "pagerank"
        d = 0.85 if vkind == "float" else 0.5
        x = synth.xvec(mats[i][1], seed=100 + q, kind=vkind)
        reqs.append((i, kind, d, x))
    # alone: one request at a time
    alone = []
    for i, kind, d, x in reqs:
        xd = _dev(x, torch.float32)
        yd = torch.empty(mats[i][0], dtype=torch.float32, device="cuda")
        S.wait(S.submit(ids[i], xd, yd, kind, d))
        alone.append(yd.cpu().numpy().astype(np.float64))
    b0 = S.stats()["batches"]
    # in the mix: everything submitted at once (native submission loop), coalesced by the
    # scheduler while earlier batches run
    xs = [_dev(x, torch.float32) for _, _, _, x in reqs]
    ys = [torch.empty(mats[i][0], dtype=torch.float32, device="cuda") for i, _, _, _ in reqs]
    S.replay([S.request(ids[i], xs[q], ys[q], kind, d) for q, (i, kind, d, _) in enumerate(reqs)],
             np.zeros(len(reqs)))
    st = S.stats()
    say("batches for %d mixed requests: %d, widest %d" % (len(reqs), st["batches"] - b0,
                                                          st["max_batch_seen"]))
    assert st["max_batch_seen"] > 1 and st["batches"] - b0 < len(reqs)
    for q, (i, kind, d, x) in enumerate(reqs):
        y = ys[q].cpu().numpy().astype(np.float64)
        want = _oracle(mats[i], vt, x, kind, d)
        _check(alone[q], want, "alone %d" % q)
        _check(y, want, "mix %d" % q)
        if vkind == "int":
            assert measure.equal_ignoring_zero_sign(y, alone[q]), "alone != mix %d" % q
    S.close()


def test_serve_plain_path(spx):
    import torch
    mats = _matrices("int")
    S = spx.Server(coalesce=False)
    ids = [S.add_matrix(_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64),
                        (m, n), "merge", value_type="f32")[0] for m, n, r, c, v in mats]
    xs, ys, tk = [], [], []
    for q in range(40):
        i = q % len(mats)
        x = synth.xvec(mats[i][1], seed=q, kind="int")
        xs.append(x)
        ys.append(torch.empty(mats[i][0], dtype=torch.float32, device="cuda"))
        tk.append(S.submit(ids[i], _dev(x, torch.float32), ys[-1]))
    for t in tk:
        assert S.wait(t) >= 0
    st = S.stats()
    assert st["batches"] == 40 and st["max_batch_seen"] == 1
    for q in range(40):
        i = q % len(mats)
        _check(ys[q].cpu().numpy().astype(np.float64), _oracle(mats[i], "f32", xs[q], "spmv", 0),
               "plain %d" % q)
    S.close()


def test_serve_admission_by_footprint(spx):
    import torch
    mats = _matrices("int")
    m, n, row, col, val = mats[1]
    args = (_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64), (m, n))
    probe = spx.Server()
    _, need = probe.add_matrix(*args, "merge", value_type="f32")
    staging = probe.stats()["bytes_staging"]   # the slots' staging bound for this matrix
    probe.close()
    assert staging > 0
    # room for two matrices and the slots' staging, not for three
    S = spx.Server(memory_budget=int(2.5 * need) + staging)
    a, _ = S.add_matrix(*args, "merge", value_type="f32")
    b, _ = S.add_matrix(*args, "merge", value_type="f32")
    with pytest.raises(spx.SpxError) as e:
        S.add_matrix(*args, "merge", value_type="f32")
    assert e.value.status == -5
    st = S.stats()
    assert st["matrices"] == 2 and st["bytes_resident"] == 2 * need
    assert st["bytes_staging"] == staging
    assert st["bytes_resident"] + st["bytes_staging"] <= st["memory_budget"]
    # without room for the staging, even the first matrix is refused
    T = spx.Server(memory_budget=int(1.5 * need))
    if 1.5 * need < need + staging:
        with pytest.raises(spx.SpxError) as e:
            T.add_matrix(*args, "merge", value_type="f32")
        assert e.value.status == -5
    T.close()
    # a removal returns the bytes; a request in flight is finished first
    x = _dev(synth.xvec(n, seed=1, kind="int"), torch.float32)
    y = torch.empty(m, dtype=torch.float32, device="cuda")
    t = S.submit(a, x, y)
    S.remove_matrix(a)
    S.wait(t)
    _check(y.cpu().numpy().astype(np.float64),
           _oracle(mats[1], "f32", synth.xvec(n, seed=1, kind="int"), "spmv", 0), "removed")
    c, _ = S.add_matrix(*args, "merge", value_type="f32")
    assert S.stats()["matrices"] == 2
    S.close()


def test_serve_replay_poisson(spx):
    import torch
    mats = _matrices("int")
    S = spx.Server(slots=4, max_batch=32)
    ids = [S.add_matrix(_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64),
                        (m, n), "rowsplit", value_type="f32")[0] for m, n, r, c, v in mats]
    rng = np.random.default_rng(7)
    count, rate = 600, 5000.0
    arrival = np.cumsum(rng.exponential(1e6 / rate, count))
    which = rng.integers(0, len(mats), count)
    xs = [_dev(synth.xvec(mats[i][1], seed=i, kind="int"), torch.float32) for i in range(4)]
    ys = [torch.empty(mats[i][0], dtype=torch.float32, device="cuda") for i in which]
    reqs = [S.request(ids[i], xs[i], ys[q]) for q, i in enumerate(which)]
    lat, wall = S.replay(reqs, arrival)
    say("replay: p50 %.1f us  p99 %.1f us  wall %.0f us" % (np.percentile(lat, 50),
                                                           np.percentile(lat, 99), wall))
    assert np.all(lat > 0) and wall > 0
    assert S.stats()["requests"] >= count
    for q, i in enumerate(which):
        _check(ys[q].cpu().numpy().astype(np.float64),
               _oracle(mats[i], "f32", synth.xvec(mats[i][1], seed=i, kind="int"), "spmv", 0),
               "replay %d" % q)
    S.close()


def test_serve_errors(spx):
    import ctypes

    import torch
    mats = _matrices("int")
    m, n, row, col, val = mats[0]
    args = (_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64), (m, n))
    S = spx.Server()
    for fmt, vt in (("csbh", "f32"), ("merge", "f64")):
        with pytest.raises(spx.SpxError) as e:
            S.add_matrix(*args, fmt, value_type=vt)
        assert e.value.status == -7
    mid, _ = S.add_matrix(*args, "merge", value_type="f32")
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    y = torch.zeros(m, dtype=torch.float32, device="cuda")
    L = spx.load()
    t = ctypes.c_uint64()
    for r, code in ((spx.spx.Request(mid + 99, 0, 0.0, x.data_ptr(), y.data_ptr()), -1),
                    (spx.spx.Request(mid, 5, 0.0, x.data_ptr(), y.data_ptr()), -1),
                    (spx.spx.Request(mid, 1, 1.5, x.data_ptr(), y.data_ptr()), -1),
                    (spx.spx.Request(mid, 0, 0.0, None, y.data_ptr()), -1),
                    (spx.spx.Request(mid, 0, 0.0, x.data_ptr(), x.data_ptr()), -4)):
        assert L.spx_server_submit(S._h, ctypes.byref(r), ctypes.byref(t)) == code
    assert L.spx_server_wait(S._h, 12345, None) == -1
    with pytest.raises(spx.SpxError):
        S.remove_matrix(mid + 99)
    assert torch.count_nonzero(y).item() == 0
    S.close()


def test_serve_waits_for_the_stream_producing_x(spx):
    # x is written on a side stream behind a long-running kernel; the request names that stream,
    # so its product must see the final x (not the zeros it held at submission)
    import torch
    mats = _matrices("int")
    m, n, row, col, val = mats[0]
    S = spx.Server(slots=2, max_batch=8)
    mid, _ = S.add_matrix(_dev(row, torch.int32), _dev(col, torch.int32),
                          _dev(val, torch.float64), (m, n), "merge", value_type="f32")
    xh = synth.xvec(n, seed=77, kind="int")
    x_true = _dev(xh, torch.float32)
    side = torch.cuda.Stream()
    for kind in ("spmv", "pagerank"):
        x = torch.zeros(n, dtype=torch.float32, device="cuda")
        y = torch.full((m,), -1.0, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            torch.cuda._sleep(20_000_000)   # a bounded spin, then the copy that produces x
            x.copy_(x_true)
        t = S.submit(mid, x, y, kind=kind, damping=0.85, stream=side)
        S.wait(t)
        torch.cuda.synchronize()
        _check(y.cpu().numpy().astype(np.float64), _oracle(mats[0], "f32", xh, kind, 0.85),
               "stream-ordered " + kind)
    S.close()
