"""GPU: spx_spmm_noalloc (Y = A X with the scratch in a static device array) against spx_spmm,
through the C ABI.  Two products in a row on the same GPU, the second on a smaller matrix with
fewer right-hand sides, in both layouts and for merge-path and row-split CRS (whose merge tile
starts the entry point builds in the static scratch); integer-valued inputs must agree bit for bit,
float inputs to the bit as well (the same kernels and summation order).  Sizes beyond the static
scratch are refused before any device work."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch

    from ._lib import ensure_built
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ensure_built()
    import paper_2502_19284_amd as spx
    spx.use_torch_allocator(True)
    return spx, spx.load()


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _operands(n, m, k, layout, dt, seed, kind):
    import torch
    X = np.stack([synth.xvec(n, seed=seed + c, kind=kind) for c in range(k)], axis=1)
    if layout == "col":
        Xd = _dev(X.T, dt).t()                       # column-major n x k, ld = n
        Y1 = torch.full((k, m), 7.0, dtype=dt, device="cuda").t()
        Y2 = torch.full((k, m), -3.0, dtype=dt, device="cuda").t()
        return Xd, Y1, Y2, Xd.stride(1), Y1.stride(1), 0
    Xd = _dev(X, dt)                                 # row-major n x k, ld = k
    Y1 = torch.full((m, k), 7.0, dtype=dt, device="cuda")
    Y2 = torch.full((m, k), -3.0, dtype=dt, device="cuda")
    return Xd, Y1, Y2, Xd.stride(0), Y1.stride(0), 1


def _both(spx, L, A, Xd, Y1, Y2, ldx, ldy, code, k):
    """Y1 = A X by spx_spmm, Y2 by spx_spmm_noalloc; returns both on the host."""
    import torch
    P = ctypes.c_void_p
    st = torch.cuda.current_stream().cuda_stream
    assert L.spx_spmm(A.handle, k, P(Xd.data_ptr()), ldx, P(Y1.data_ptr()), ldy, code, P(st)) == 0
    s2 = L.spx_spmm_noalloc(A.handle, k, P(Xd.data_ptr()), ldx, P(Y2.data_ptr()), ldy, code, P(st))
    assert s2 == 0, L.spx_last_error_message()
    torch.cuda.synchronize()
    return Y1.cpu().numpy(), Y2.cpu().numpy()


@pytest.mark.parametrize("fmt", ["merge", "rowsplit"])
@pytest.mark.parametrize("layout", ["col", "row"])
@pytest.mark.parametrize("kind", ["int", "float"])
def test_noalloc_matches_spmm_twice(lib, fmt, layout, kind):
    import torch
    spx, L = lib
    cases = [(12, 16, 6), (10, 9, 3)]   # (R-MAT scale, edge factor, k); the second is smaller
    for i, (scale, ef, k) in enumerate(cases):
        m = n = 1 << scale
        row, col = synth.rmat(scale, ef, seed=70 + i)
        val = synth.values(len(row), seed=70 + i, kind=kind)
        say("noalloc", fmt, layout, kind, "call", i + 1, "m", m, "k", k)
        A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                        (m, n), fmt)
        Xd, Y1, Y2, ldx, ldy, code = _operands(n, m, k, layout, torch.float64, 80 + 10 * i, kind)
        a, b = _both(spx, L, A, Xd, Y1, Y2, ldx, ldy, code, k)
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), (fmt, layout, kind, i)
        A.close()


def test_noalloc_fp32_matrix_and_hot_rows(lib):
    # FP32 stored values with forced hot-column compaction (the hot rows of X are staged too)
    import torch
    spx, L = lib
    for i, (scale, k) in enumerate([(13, 8), (11, 2)]):
        m = n = 1 << scale
        row, col = synth.rmat(scale, 16, seed=90 + i)
        val = synth.values(len(row), seed=90 + i, kind="int")
        A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                        (m, n), "merge", value_type="f32", hot_columns=500)
        Xd, Y1, Y2, ldx, ldy, code = _operands(n, m, k, "col", torch.float32, 95 + i, "int")
        a, b = _both(spx, L, A, Xd, Y1, Y2, ldx, ldy, code, k)
        assert np.array_equal(a.view(np.int32), b.view(np.int32))
        A.close()


def test_noalloc_refuses_beyond_static_scratch(lib):
    # 2^22 rows and columns with k = 2 column-major: the X and Y staging alone need 128 MiB
    import torch
    spx, L = lib
    m = n = 1 << 22
    row = _dev(np.array([0, m - 1], np.int32), torch.int32)
    col = _dev(np.array([5, n - 1], np.int32), torch.int32)
    A = spx.convert(row, col, _dev(np.array([1.0, 2.0]), torch.float64), (m, n), "merge")
    X = torch.ones((2, n), dtype=torch.float64, device="cuda").t()
    Y = torch.zeros((2, m), dtype=torch.float64, device="cuda").t()
    P = ctypes.c_void_p
    st = L.spx_spmm_noalloc(A.handle, 2, P(X.data_ptr()), n, P(Y.data_ptr()), m, 0, None)
    assert st == -3 and b"scratch" in L.spx_last_error_message()
    torch.cuda.synchronize()
    assert float(Y.abs().sum()) == 0.0     # nothing was launched
    A.close()
