"""The C ABI without a GPU: the library loads, exports every declared entry point, and rejects
invalid arguments before touching a device."""
import ctypes
import math
import re
import subprocess

import numpy as np
import pytest

import paper_2502_19284_amd as spx
from paper_2502_19284_amd import spx as B
from oracle import measure

from ._lib import ensure_built


@pytest.fixture(scope="module")
def L():
    return ensure_built()


def test_exports_every_declared_symbol(L):
    names = spx.header_functions()
    assert len(names) >= 11
    out = subprocess.run(["nm", "-D", "--defined-only", spx.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (spx_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def test_status_strings(L):
    for code, name in B.STATUS.items():
        assert L.spx_status_string(code).decode() == name
    assert L.spx_status_string(-99).decode() == "SPX_ERR_UNKNOWN"
    assert spx.version().count(".") == 2


def test_opts_default(L):
    o = B.ConvertOpts(7, 7, 7, 7, 7, 7)
    assert L.spx_convert_opts_default(ctypes.byref(o)) == 0
    assert (o.sum_duplicates, o.log2_beta, o.validate, o.tile_items, o.hot_columns,
            o.value_type) == (1, 0, 1, 0, -1, 0)
    assert L.spx_convert_opts_default(None) == -1


def _convert(L, desc, fmt=1, opts=None):
    h = ctypes.c_void_p(12345)
    st = L.spx_convert(ctypes.byref(desc) if desc is not None else None, fmt,
                       ctypes.byref(opts) if opts is not None else None, None, ctypes.byref(h),
                       None)
    return st, h


def test_convert_argument_errors(L):
    fake = ctypes.c_void_p(0x1000)
    good = dict(m=4, n=4, nnz=3, row=fake, col=fake, val=fake, val_type=0)
    st, h = _convert(L, None)
    assert st == -1
    assert L.spx_convert(None, 1, None, None, None, None) == -1
    cases = [
        (dict(good, m=-1), -1),
        (dict(good, nnz=-5), -1),
        (dict(good, nnz=2 ** 31), -3),
        (dict(good, val_type=3), -7),
        (dict(good, row=None), -1),
        (dict(good, val=None), -1),
        (dict(good, m=0), -2),
    ]
    for kw, code in cases:
        d = B.CooDesc(kw["m"], kw["n"], kw["nnz"], kw["row"], kw["col"], kw["val"],
                      kw["val_type"])
        st, h = _convert(L, d)
        assert st == code, (kw, st, L.spx_last_error_message())
        assert h.value is None  # *out cleared on every error
        assert L.spx_last_error_message().decode() != ""
    d = B.CooDesc(**good)
    st, _ = _convert(L, d, fmt=9)
    assert st == -1
    assert "format" in L.spx_last_error_message().decode()
    st, _ = _convert(L, d, opts=B.ConvertOpts(2, 0, 1, 0, -1))
    assert st == -1
    st, _ = _convert(L, d, opts=B.ConvertOpts(1, 17, 1, 0, -1))
    assert st == -1
    st, _ = _convert(L, d, opts=B.ConvertOpts(1, 0, 1, -3, -1))
    assert st == -1
    st, _ = _convert(L, d, opts=B.ConvertOpts(1, 0, 1, 0, -2))
    assert st == -1
    st, _ = _convert(L, d, fmt=1, opts=B.ConvertOpts(1, 0, 1, 100, -1))
    assert st == -7
    st, _ = _convert(L, d, fmt=1, opts=B.ConvertOpts(1, 0, 1, 0, -1, 5))
    assert st == -1
    for fmt in (4, 5):  # BCOHC / BCOHCH: summed repeats only
        st, _ = _convert(L, d, fmt=fmt, opts=B.ConvertOpts(0, 0, 1, 0, -1, 0))
        assert st == -7
    # CSBR (6): panels of fixed height
    st, _ = _convert(L, d, fmt=6, opts=B.ConvertOpts(1, 5, 1, 0, -1, 0))
    assert st == -7
    st, _ = _convert(L, d, fmt=7)
    assert st == -1


def test_handle_argument_errors(L):
    P = ctypes.c_void_p
    assert L.spx_spmv(None, P(0x1000), P(0x2000), None) == -1
    assert L.spx_spmv_f32(None, P(0x1000), P(0x2000), None) == -1
    info = B.MatrixInfo()
    assert L.spx_matrix_get_info(None, ctypes.byref(info)) == -1
    assert L.spx_matrix_export(None, 0, None, 0, None, None) == -1
    assert L.spx_matrix_destroy(None) == 0


def test_allocator_hook_pairing(L):
    assert L.spx_set_allocator(B.ALLOC_FN(lambda a, b, c: None), B.FREE_FN(), None) == -1
    assert L.spx_set_allocator(B.ALLOC_FN(), B.FREE_FN(), None) == 0


def test_break_even_matches_oracle(L):
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b, c, d = rng.uniform(0, 10, 4)
        assert spx.break_even(a, b, c, d) == pytest.approx(measure.break_even(a, b, c, d))
    assert math.isinf(spx.break_even(5, 1, 1, 1))
    assert math.isinf(spx.break_even(5, 1, 1, 2))
    # faster product and no slower conversion: ahead from the first product
    assert spx.break_even(1, 2, 3, 2) == 0.0 == measure.break_even(1, 2, 3, 2)
    # the paper's counts through the product's formula (times in ParCRS units)
    t_par = 1 / 2.9
    assert round(spx.break_even(10.9 * t_par, 7.8 * t_par, t_par, 1 / 3.3)) == 26


def test_server_argument_errors(L):
    o = B.ServerOpts()
    assert L.spx_server_opts_default(ctypes.byref(o)) == 0
    assert (o.memory_budget, o.slots, o.max_batch, o.coalesce, o.poll_us) == (64 << 30, 4, 32, 1, 0)
    h = ctypes.c_void_p()
    for field, bad in (("slots", 0), ("slots", 17), ("max_batch", 0), ("max_batch", 65),
                       ("memory_budget", 0), ("poll_us", -1), ("poll_us", 1001)):
        b = B.ServerOpts()
        L.spx_server_opts_default(ctypes.byref(b))
        setattr(b, field, bad)
        assert L.spx_server_create(ctypes.byref(b), ctypes.byref(h)) == -1, field
        assert h.value is None
    assert L.spx_server_create(ctypes.byref(o), None) == -1
    t = ctypes.c_uint64()
    r = B.Request(1, 0, 0.85, None, None)
    assert L.spx_server_submit(None, ctypes.byref(r), ctypes.byref(t)) == -1
    assert L.spx_server_wait(None, 1, None) == -1
    assert L.spx_server_remove_matrix(None, 1) == -1
    assert L.spx_server_get_stats(None, None) == -1
    assert L.spx_server_replay(None, None, None, 0, None, None) == -1
    assert L.spx_server_add_matrix(None, None, 1, None, None, None, None) == -1
    assert L.spx_server_destroy(None) == 0
