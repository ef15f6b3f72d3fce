"""GPU tests of batched products (include/spx_batch.h): many uneven matrices in one persistent
launch, every plan and the autotuner, HIP graph capture and replay, determinism, errors.

Bar: integer-valued inputs are bit-exact against the oracle; float inputs within the FP32
dot-product bound of oracle.precision.dot_error_bound; two launches and every graph replay equal
the eager launch bit for bit.
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


def _uneven(count, seed, kind):
    """Erdos-Renyi and Chung-Lu matrices with log-uniform rows and average degree."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(300), np.log(40000))))
        deg = float(np.exp(rng.uniform(np.log(4), np.log(64))))
        E = max(1, int(n * deg))
        if i % 2:
            row, col = synth.uniform(n, n, E, seed=seed * 100 + i)
        else:
            row, col = synth.chunglu(n, E, 2.1, seed=seed * 100 + i)
        val = synth.values(E, seed=seed * 100 + i, kind=kind)
        out.append((n, n, row, col, val))
    return out


def _check(mat, vt, x, y, kind, what):
    m, n, row, col, val = mat
    cr, cc, cv, _ = spmv.canonical_coo(m, n, row, col, val)
    rp, _, _ = spmv.crs_from_canonical(m, cr, cc, cv)
    rv = precision.round_f32(cv) if vt == "f32" else precision.round_bf16(cv)
    yp, yr, s = spmv.alg1_accurate(rp, cc, rv, precision.round_f32(x))
    if kind == "int":
        assert measure.equal_ignoring_zero_sign(y, yp), what
    else:
        err = measure.scaled_error(y, yr, s)
        assert np.all(err <= precision.dot_error_bound(np.diff(rp) + 2, 0.0) + 1e-300), what


def _build(spx, mats, vt, fmt="merge", plans=None):
    import torch
    hs = [spx.convert(_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64),
                      (m, n), fmt, value_type=vt) for m, n, r, c, v in mats]
    return hs, spx.Batch(hs, plans)


def _vectors(mats, kind, seed):
    import torch
    xs_h = [synth.xvec(n, seed=seed + i, kind=kind) for i, (m, n, _, _, _) in enumerate(mats)]
    xs = [_dev(x, torch.float32) for x in xs_h]
    ys = [torch.full((m,), float("nan"), dtype=torch.float32, device="cuda")
          for (m, n, _, _, _) in mats]
    return xs_h, xs, ys


@pytest.mark.parametrize("vt", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["int", "float"])
@pytest.mark.parametrize("fmt", ["merge", "rowsplit"])
def test_batch_autotuned(spx, vt, kind, fmt):
    import torch
    mats = _uneven(24, 1, kind)
    hs, B = _build(spx, mats, vt, fmt)
    say("plans", B.plans, B.info())
    assert all(p != "auto" for p in B.plans)
    xs_h, xs, ys = _vectors(mats, kind, 50)
    B.bind(xs, ys)
    B.spmv()
    torch.cuda.synchronize()
    for i, mat in enumerate(mats):
        _check(mat, vt, xs_h[i], ys[i].double().cpu().numpy(), kind, "matrix %d (%s)" % (i, B.plans[i]))
    B.close()


@pytest.mark.parametrize("plan", ["merge4", "merge8", "merge16", "rows512", "rows2048"])
def test_batch_fixed_plans(spx, plan):
    import torch
    mats = _uneven(10, 2, "int")
    if plan.startswith("rows"):  # row tiles need rows of at most 1024 entries: Erdos-Renyi only
        mats = [mt for i, mt in enumerate(mats) if i % 2]
    hs, B = _build(spx, mats, "f32", plans=[plan] * len(mats))
    assert B.plans == [plan] * len(mats)
    xs_h, xs, ys = _vectors(mats, "int", 70)
    B.bind(xs, ys)
    B.spmv()
    torch.cuda.synchronize()
    for i, mat in enumerate(mats):
        _check(mat, "f32", xs_h[i], ys[i].double().cpu().numpy(), "int", "%s %d" % (plan, i))


def test_batch_long_rows_and_hot_columns(spx):
    # rows spanning many merge tiles (carries added by the last tile) and forced hot columns
    import torch
    rng = np.random.default_rng(3)
    mats = []
    for i in range(4):
        m, n = 3000 + i, 5000
        row = np.concatenate([rng.integers(0, m, 30_000), np.full(20_000 * (i + 1), 11)])
        col = rng.integers(0, n, len(row))
        mats.append((m, n, row.astype(np.int32), col.astype(np.int32),
                     synth.values(len(row), seed=i, kind="float")))
    hs = [spx.convert(_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64),
                      (m, n), "merge", value_type="f32", hot_columns=300) for m, n, r, c, v in mats]
    for plans in (None, ["merge4"] * 4, ["merge16"] * 4):
        B = spx.Batch(hs, plans)
        assert all(p.startswith("merge") for p in B.plans)  # rows longer than 1024
        xs_h, xs, ys = _vectors(mats, "float", 90)
        B.bind(xs, ys)
        for rep in range(3):  # counters reset themselves between launches
            B.spmv()
            torch.cuda.synchronize()
            for i, mat in enumerate(mats):
                _check(mat, "f32", xs_h[i], ys[i].double().cpu().numpy(), "float",
                       "long rows %d rep %d" % (i, rep))
        B.close()


def test_batch_graph_replay_and_determinism(spx):
    import torch
    mats = _uneven(16, 4, "float")
    hs, B = _build(spx, mats, "f32")
    xs_h, xs, ys = _vectors(mats, "float", 10)
    B.bind(xs, ys)
    B.spmv()
    torch.cuda.synchronize()
    eager = [y.clone() for y in ys]
    B.spmv()
    torch.cuda.synchronize()
    for a, b in zip(eager, ys):
        assert torch.equal(a, b)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.spmv()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.spmv()
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, (a, b) in enumerate(zip(eager, ys)):
            assert torch.equal(a, b), "replay %d matrix %d" % (rep, i)
    for i, mat in enumerate(mats):
        _check(mat, "f32", xs_h[i], ys[i].double().cpu().numpy(), "float", "graph %d" % i)
    del g
    B.close()


def test_batch_errors(spx):
    import torch
    mats = _uneven(3, 5, "int")
    hs, B = _build(spx, mats, "f32")
    with pytest.raises(spx.SpxError) as e:
        spx.Batch([hs[0], hs[0]])
    assert e.value.status == -1
    m, n, r, c, v = mats[0]
    d = (_dev(r, torch.int32), _dev(c, torch.int32), _dev(v, torch.float64), (m, n))
    for fmt, vt, code in (("csbh", "f64", -7), ("merge", "f64", -7)):
        A = spx.convert(*d, fmt, value_type=vt)
        with pytest.raises(spx.SpxError) as e:
            spx.Batch([A])
        assert e.value.status == code
    C = spx.Batch([hs[0]])
    with pytest.raises(spx.SpxError) as e:  # no vectors bound yet
        C.spmv()
    assert e.value.status == -1
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(spx.SpxError) as e:  # y overlapping x
        C.bind([x], [x[:m]])
    assert e.value.status == -4
    # a matrix with a row longer than 1024 entries cannot take row tiles
    row = np.zeros(3000, np.int32)
    col = np.arange(3000, dtype=np.int32)
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32),
                    _dev(np.ones(3000), torch.float64), (4, 3000), "merge", value_type="f32")
    with pytest.raises(spx.SpxError) as e:
        spx.Batch([A], ["rows512"])
    assert e.value.status == -1
    C.close()
    B.close()
