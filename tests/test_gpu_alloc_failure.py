"""GPU: device allocation failures through the allocator hook (spx_set_allocator).

For every format's conversion and for the first product with several right-hand sides (which
grows the handle's scratch), an allocator that fails its k-th call, for every k up to the number
of allocations the call makes, must give SPX_ERR_NOMEM, leave *out NULL (conversion), free every
temporary (torch's allocated bytes back at their baseline), and leave the library usable."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
FMTS = ["rowsplit", "merge", "csbh", "csb", "bcohc", "bcohch", "csbr"]


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
    yield spx
    spx.use_torch_allocator(True)


_INSTALLED = []   # the installed hook's callbacks must outlive its installation


class Hook:
    """Allocator routed to torch's caching allocator that counts calls and fails the fail_at-th
    (0: never)."""

    def __init__(self, spx, fail_at=0):
        import torch
        from paper_2502_19284_amd import spx as B
        self.calls = 0
        self.fail_at = fail_at

        def alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.calls == self.fail_at:
                return None
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0))

        def free(ptr, stream, ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)
        self.refs = (B.ALLOC_FN(alloc), B.FREE_FN(free))
        assert spx.load().spx_set_allocator(self.refs[0], self.refs[1], None) == 0
        _INSTALLED[:] = [self]


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _convert_raw(spx, L, desc, fmt):
    """spx_convert through the C ABI with *out preset to a non-NULL value."""
    from paper_2502_19284_amd import spx as B
    opts = B.ConvertOpts(1, 0, 1, 0, -1, 0)
    h = ctypes.c_void_p(0x1234)
    st = L.spx_convert(ctypes.byref(desc), B.FORMATS[fmt], ctypes.byref(opts), None,
                       ctypes.byref(h), None)
    return st, h


@pytest.mark.parametrize("fmt", FMTS)
def test_conversion_fails_cleanly_at_every_allocation(spx, fmt):
    import torch
    from paper_2502_19284_amd import spx as B
    L = spx.load()
    m = n = 1 << 12
    row, col = synth.rmat(12, 16, seed=5)
    val = synth.values(len(row), seed=5)
    r, c, v = _dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64)
    desc = B.CooDesc(m, n, len(row), ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                     ctypes.c_void_p(v.data_ptr()), 0)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    counter = Hook(spx)
    st, h = _convert_raw(spx, L, desc, fmt)
    assert st == 0 and h.value
    total = counter.calls
    assert L.spx_matrix_destroy(h) == 0
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    say(fmt, "allocations per conversion:", total)
    for k in range(1, total + 1):
        Hook(spx, fail_at=k)
        st, h = _convert_raw(spx, L, desc, fmt)
        assert st == -5, (fmt, k, st, L.spx_last_error_message())
        assert h.value is None, (fmt, k)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base, (fmt, k)
    # the library still converts once allocations succeed again
    Hook(spx)
    st, h = _convert_raw(spx, L, desc, fmt)
    assert st == 0 and h.value
    assert L.spx_matrix_destroy(h) == 0


@pytest.mark.parametrize("fmt", ["rowsplit", "merge"])
def test_spmm_scratch_failure_leaves_handle_usable(spx, fmt):
    import torch
    from oracle import measure, spmv
    L = spx.load()
    m = n = 1 << 11
    row, col = synth.rmat(11, 16, seed=6)
    val = synth.values(len(row), seed=6, kind="int")
    k = 5
    X = np.stack([synth.xvec(n, seed=60 + j, kind="int") for j in range(k)], axis=1)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    Hook(spx)
    A = spx.convert(_dev(row, torch.int32), _dev(col, torch.int32), _dev(val, torch.float64),
                    (m, n), fmt)
    Xd = _dev(X.T, torch.float64).t()
    Y = torch.empty((k, m), dtype=torch.float64, device="cuda").t()
    P = ctypes.c_void_p
    for j in range(1, 8):          # the first product grows up to six scratch buffers
        Hook(spx, fail_at=j)
        st = L.spx_spmm(A.handle, k, P(Xd.data_ptr()), n, P(Y.data_ptr()), m, 0, None)
        if st == 0:
            break
        assert st == -5, (fmt, j, L.spx_last_error_message())
    Hook(spx)
    A.spmm(Xd, out=Y)
    torch.cuda.synchronize()
    rp, cc, cv = spmv.crs(m, n, row, col, val)
    Yp, _, _ = spmv.spmm(rp, cc, cv, X)
    assert measure.equal_ignoring_zero_sign(Y.cpu().numpy(), Yp)
    A.close()
    del Xd, Y
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
