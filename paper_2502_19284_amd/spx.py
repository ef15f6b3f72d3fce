"""ctypes binding of libspx (include/spx.h): argument marshalling only.

Every step of conversion and product runs in the library's HIP kernels; this module only checks
tensor dtypes/devices, passes raw device pointers and the current torch stream, and turns status
codes into exceptions.  torch supplies device memory and streams.  If libspx.so is missing the
import of the binding's entry points fails loudly (there is no CPU fallback).
"""
import atexit
import ctypes
import os
import weakref

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPX_LIBRARY") or os.path.join(_PKG, "libspx.so")

SPX_OK = 0
STATUS = {0: "SPX_OK", -1: "SPX_ERR_INVALID_ARG", -2: "SPX_ERR_INDEX", -3: "SPX_ERR_RANGE",
          -4: "SPX_ERR_ALIAS", -5: "SPX_ERR_NOMEM", -6: "SPX_ERR_HIP", -7: "SPX_ERR_UNSUPPORTED",
          -8: "SPX_ERR_DEVICE"}
FORMATS = {"rowsplit": 0, "merge": 1, "csbh": 2, "csb": 3, "bcohc": 4, "bcohch": 5, "csbr": 6}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}
LAYOUTS = {"col": 0, "row": 1}
VALUE_TYPES = {"f64": 0, "f32": 1, "bf16": 2}
VALUE_TORCH = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}
ARRAYS = {"row_ptr": (0, torch.int32), "col_ind": (1, torch.int32), "values": (2, torch.float64),
          "blk_ptr": (3, torch.int32), "packed": (4, torch.int32), "parts": (5, torch.int32),
          "blk_coord": (6, torch.int32), "col_order": (7, torch.int32),
          "row_order": (8, torch.int32)}


class SpxError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = STATUS.get(status, "SPX_ERR_UNKNOWN")
        super().__init__("%s: %s" % (self.name, message))


class CooDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("val_type", ctypes.c_int32)]


class ConvertOpts(ctypes.Structure):
    _fields_ = [("sum_duplicates", ctypes.c_int32), ("log2_beta", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("tile_items", ctypes.c_int32),
                ("hot_columns", ctypes.c_int32), ("value_type", ctypes.c_int32)]


class ConvertReport(ctypes.Structure):
    _fields_ = [("convert_ms", ctypes.c_float), ("nnz_out", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("log2_beta", ctypes.c_int32),
                ("parts", ctypes.c_int32), ("sort_split_keys", ctypes.c_int64),
                ("sort_levels", ctypes.c_int32), ("sort_first_fused", ctypes.c_int32)]


class MatrixInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("format", ctypes.c_int32), ("log2_beta", ctypes.c_int32),
                ("bytes", ctypes.c_int64), ("parts", ctypes.c_int64),
                ("value_type", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("min_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("coalesce", ctypes.c_int32),
                ("poll_us", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_int32), ("kind", ctypes.c_int32), ("damping", ctypes.c_float),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("stream", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("max_batch_seen", ctypes.c_int64), ("bytes_resident", ctypes.c_int64),
                ("memory_budget", ctypes.c_int64), ("matrices", ctypes.c_int32),
                ("in_flight", ctypes.c_int32), ("bytes_staging", ctypes.c_int64)]


REQUEST_KINDS = {"spmv": 0, "pagerank": 1}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_alloc_refs = None
_atexit_set = False
_live = weakref.WeakSet()  # open Matrix handles
_live_containers = weakref.WeakSet()


def load(path=LIB_PATH):
    """Load libspx.so and declare its signatures.  Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libspx.so not found at %s: build it with "
                           "paper_2502_19284_amd.build.build()" % path)
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.spx_convert_opts_default.argtypes = [ctypes.POINTER(ConvertOpts)]
    L.spx_convert.argtypes = [ctypes.POINTER(CooDesc), ctypes.c_int32, ctypes.POINTER(ConvertOpts),
                              P, ctypes.POINTER(P), ctypes.POINTER(ConvertReport)]
    L.spx_spmv.argtypes = [P, P, P, P]
    L.spx_spmv_f32.argtypes = [P, P, P, P]
    L.spx_spmv_f32.restype = ctypes.c_int32
    L.spx_spmm.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int64,
                           ctypes.c_int32, P]
    L.spx_spmm.restype = ctypes.c_int32
    L.spx_matrix_get_info.argtypes = [P, ctypes.POINTER(MatrixInfo)]
    L.spx_matrix_export.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_int64), P]
    L.spx_matrix_destroy.argtypes = [P]
    L.spx_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    for f in (L.spx_convert_opts_default, L.spx_convert, L.spx_spmv, L.spx_matrix_get_info,
              L.spx_matrix_export, L.spx_matrix_destroy, L.spx_set_allocator):
        f.restype = ctypes.c_int32
    L.spx_server_opts_default.argtypes = [ctypes.POINTER(ServerOpts)]
    L.spx_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]
    L.spx_server_destroy.argtypes = [P]
    L.spx_server_add_matrix.argtypes = [P, ctypes.POINTER(CooDesc), ctypes.c_int32,
                                        ctypes.POINTER(ConvertOpts), P,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64)]
    L.spx_server_remove_matrix.argtypes = [P, ctypes.c_int32]
    L.spx_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.spx_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
    L.spx_server_replay.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    L.spx_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    for f in (L.spx_server_opts_default, L.spx_server_create, L.spx_server_destroy,
              L.spx_server_add_matrix, L.spx_server_remove_matrix, L.spx_server_submit,
              L.spx_server_wait, L.spx_server_replay, L.spx_server_get_stats):
        f.restype = ctypes.c_int32
    L.spx_batch_create.argtypes = [ctypes.POINTER(P), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), P, ctypes.POINTER(P),
                                   ctypes.POINTER(ctypes.c_int32)]
    L.spx_batch_bind.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), P]
    L.spx_batch_spmv.argtypes = [P, P]
    L.spx_batch_get_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32)]
    L.spx_batch_destroy.argtypes = [P]
    for f in (L.spx_batch_create, L.spx_batch_bind, L.spx_batch_spmv, L.spx_batch_get_info,
              L.spx_batch_destroy):
        f.restype = ctypes.c_int32
    L.spx_profile_enable.argtypes = [ctypes.c_int32]
    L.spx_profile_enable.restype = ctypes.c_int32
    L.spx_profile_collect.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]
    L.spx_profile_collect.restype = ctypes.c_int32
    L.spx_break_even.argtypes = [ctypes.c_double] * 4
    L.spx_break_even.restype = ctypes.c_double
    L.spx_spmm_noalloc.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64, P, ctypes.c_int64,
                                   ctypes.c_int32, P]
    L.spx_spmm_noalloc.restype = ctypes.c_int32
    L.spx_probe_gather.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P, P]
    L.spx_probe_gather.restype = ctypes.c_int32
    L.spx_probe_out_len.argtypes = []
    L.spx_probe_out_len.restype = ctypes.c_int64
    L.spx_status_string.argtypes = [ctypes.c_int32]
    L.spx_status_string.restype = ctypes.c_char_p
    L.spx_last_error_message.argtypes = []
    L.spx_last_error_message.restype = ctypes.c_char_p
    L.spx_version.argtypes = []
    L.spx_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status):
    if status != SPX_OK:
        msg = load().spx_last_error_message().decode()
        raise SpxError(status, msg)


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def use_torch_allocator(enable=True):
    """Route the library's device allocations through torch's caching allocator."""
    global _alloc_refs
    L = load()
    if not enable:
        _check(L.spx_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _alloc_refs = None
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0))
        except Exception:  # out of memory or invalid request -> NULL -> SPX_ERR_NOMEM
            return None

    def _free(ptr, stream, ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    refs = (ALLOC_FN(_alloc), FREE_FN(_free))
    _check(L.spx_set_allocator(refs[0], refs[1], None))
    _alloc_refs = refs
    _register_shutdown()


def _register_shutdown():
    global _atexit_set
    if not _atexit_set:
        atexit.register(_shutdown)
        _atexit_set = True


def _shutdown():
    """At exit, while torch is still alive: free live handles, then drop the allocator hook."""
    global _alloc_refs
    for srv in list(_live_containers):  # servers and batches first: they use matrices
        try:
            srv.close()
        except Exception:
            pass
    for mat in list(_live):
        try:
            mat.close()
        except Exception:
            pass
    if _lib is not None and _alloc_refs is not None:
        _lib.spx_set_allocator(ALLOC_FN(), FREE_FN(), None)
        _alloc_refs = None


def profile_enable(enable=True):
    """Start (clearing earlier records) or stop per-kernel HIP-event timing in the library."""
    _check(load().spx_profile_enable(1 if enable else 0))


def profile_collect():
    """Per-kernel launch statistics since profile_enable: {name: dict(launches, total_ms,
    min_ms, max_ms, avg_ms)}.  Waits for the recorded events."""
    L = load()
    cnt = ctypes.c_int32(0)
    _check(L.spx_profile_collect(None, 0, ctypes.byref(cnt)))
    buf = (KernelStat * max(cnt.value, 1))()
    _check(L.spx_profile_collect(buf, cnt.value, ctypes.byref(cnt)))
    out = {}
    for i in range(cnt.value):
        s = buf[i]
        out[s.name.decode()] = dict(launches=int(s.launches), total_ms=s.total_ms,
                                    min_ms=s.min_ms, max_ms=s.max_ms,
                                    avg_ms=s.total_ms / max(s.launches, 1))
    return out


def probe_gather(x, window, n, out=None, stream=None):
    """n random 8-byte loads from the first `window` doubles of the float64 device tensor x
    (library kernel); returns the per-thread sums tensor (timing is the caller's)."""
    _dev_tensor(x, torch.float64, "x")
    if window > x.numel():
        raise ValueError("window beyond x")
    L = load()
    if out is None:
        out = torch.empty(int(L.spx_probe_out_len()), dtype=torch.float64, device=x.device)
    _check(L.spx_probe_gather(ctypes.c_void_p(x.data_ptr()), int(window), int(n),
                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def break_even(conv_fmt, conv_ref, spmv_ref, spmv_fmt):
    """Products after which a format pays for its longer conversion (inf if it is not faster)."""
    return float(load().spx_break_even(conv_fmt, conv_ref, spmv_ref, spmv_fmt))


def _dev_tensor(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


class Matrix:
    """A converted matrix held by libspx.  Use .spmv(x) for y = A x."""

    def __init__(self, handle, fmt, report):
        self._h = handle
        self.format = fmt
        self.convert_ms = float(report.convert_ms)
        self.sort_split_keys = int(report.sort_split_keys)
        self.sort_levels = int(report.sort_levels)
        self.sort_first_fused = int(report.sort_first_fused)
        info = MatrixInfo()
        _check(load().spx_matrix_get_info(self._h, ctypes.byref(info)))
        self.shape = (info.m, info.n)
        self.nnz = int(info.nnz)
        self.bytes = int(info.bytes)
        self.log2_beta = int(info.log2_beta)
        self.parts = int(info.parts)
        self.value_type = int(info.value_type)
        self.vec_dtype = torch.float64 if self.value_type == 0 else torch.float32
        _live.add(self)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("matrix was destroyed")
        return self._h

    def spmv(self, x, out=None, stream=None):
        """y = A x on the current (or given) stream; returns y of length m.  FP64 matrices take
        and return float64 vectors, FP32/bfloat16 matrices float32 vectors."""
        m, n = self.shape
        dt = self.vec_dtype
        _dev_tensor(x, dt, "x")
        if x.numel() != n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), n))
        if out is None:
            out = torch.empty(m, dtype=dt, device=x.device)
        _dev_tensor(out, dt, "out")
        if out.numel() != m:
            raise ValueError("out has %d entries, expected %d" % (out.numel(), m))
        fn = load().spx_spmv if self.value_type == 0 else load().spx_spmv_f32
        _check(fn(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  _stream_ptr(stream)))
        return out

    def spmm(self, X, out=None, stream=None):
        """Y = A X for an n x k device tensor X (float64 for FP64 matrices, float32 otherwise).
        The layout follows X's strides: column-major (stride (1, ld), e.g. the transpose of a
        contiguous k x n tensor) or row-major (stride (ld, 1)).  Y is created in the same layout
        unless `out` (m x k, either layout) is given.  Returns Y."""
        m, n = self.shape
        dt = self.vec_dtype
        if not isinstance(X, torch.Tensor) or X.dim() != 2:
            raise TypeError("X must be a 2-D tensor")
        if X.dtype != dt or not X.is_cuda:
            raise TypeError("X must be a %s CUDA tensor" % dt)
        if X.shape[0] != n:
            raise ValueError("X has %d rows, expected %d" % (X.shape[0], n))
        k = X.shape[1]
        lx, ldx = _layout_of(X)
        if out is None:
            out = (torch.empty((k, m), dtype=dt, device=X.device).t() if lx == 0
                   else torch.empty((m, k), dtype=dt, device=X.device))
        if not isinstance(out, torch.Tensor) or out.dim() != 2 or out.dtype != dt or \
                not out.is_cuda or tuple(out.shape) != (m, k):
            raise TypeError("out must be an m x k %s CUDA tensor" % dt)
        ly, ldy = _layout_of(out)
        if ly != lx:
            raise ValueError("X and out must have the same layout")
        _check(load().spx_spmm(self.handle, k, ctypes.c_void_p(X.data_ptr()), ldx,
                               ctypes.c_void_p(out.data_ptr()), ldy, lx, _stream_ptr(stream)))
        return out

    def export(self, name, stream=None):
        """Copy one of the handle's arrays into a new device tensor."""
        which, dtype = ARRAYS[name]
        if name == "values":
            dtype = VALUE_TORCH[self.value_type]
        L = load()
        need = ctypes.c_int64(-1)
        st = L.spx_matrix_export(self.handle, which, None, 0, ctypes.byref(need), None)
        if need.value < 0:  # the array does not exist for this format
            _check(st)
        nelem = need.value // torch.empty(0, dtype=dtype).element_size()
        t = torch.empty(nelem, dtype=dtype, device=torch.cuda.current_device())
        _check(L.spx_matrix_export(self.handle, which, ctypes.c_void_p(t.data_ptr()),
                                   need.value, None, _stream_ptr(stream)))
        return t

    def close(self):
        if self._h is not None:
            load().spx_matrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __repr__(self):
        return "Matrix(%s, shape=%s, nnz=%d)" % (self.format, self.shape, self.nnz)


PLANS = {"auto": 0, "merge4": 1, "merge8": 2, "merge16": 3, "rows512": 4, "rows2048": 5}
PLAN_NAMES = {v: k for k, v in PLANS.items()}


class Batch:
    """Products of many CRS matrices (FP32 / bfloat16 values) in one persistent launch
    (include/spx_batch.h).  plans: None (autotune every matrix) or one PLANS name per matrix.
    The matrices must stay open while the batch exists."""

    def __init__(self, matrices, plans=None, stream=None):
        L = load()
        cnt = len(matrices)
        hs = (ctypes.c_void_p * cnt)(*[A.handle for A in matrices])
        pl = None if plans is None else (ctypes.c_int32 * cnt)(*[PLANS[p] for p in plans])
        chosen = (ctypes.c_int32 * cnt)()
        h = ctypes.c_void_p()
        _check(L.spx_batch_create(hs, cnt, pl, _stream_ptr(stream), ctypes.byref(h), chosen))
        self._h = h
        self.matrices = list(matrices)
        self.plans = [PLAN_NAMES[c] for c in chosen]
        self._bound = None
        _live_containers.add(self)
        _register_shutdown()

    def bind(self, xs, ys, stream=None):
        """Use float32 device vectors xs[i] (n_i) and ys[i] (m_i) for the following products."""
        if len(xs) != len(self.matrices) or len(ys) != len(self.matrices):
            raise ValueError("one x and one y per matrix")
        for A, x, y in zip(self.matrices, xs, ys):
            _dev_tensor(x, torch.float32, "x")
            _dev_tensor(y, torch.float32, "y")
            if x.numel() != A.shape[1] or y.numel() != A.shape[0]:
                raise ValueError("vector length does not match its matrix")
        cnt = len(xs)
        px = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
        py = (ctypes.c_void_p * cnt)(*[y.data_ptr() for y in ys])
        _check(load().spx_batch_bind(self._h, px, py, _stream_ptr(stream)))
        self._bound = (list(xs), list(ys))

    def spmv(self, stream=None):
        """y_i = A_i x_i for every matrix: one launch on the current (or given) stream."""
        _check(load().spx_batch_spmv(self._h, _stream_ptr(stream)))

    def info(self):
        it = ctypes.c_int64()
        wg = ctypes.c_int32()
        _check(load().spx_batch_get_info(self._h, ctypes.byref(it), ctypes.byref(wg)))
        return {"items": it.value, "workgroups": wg.value}

    def close(self):
        if self._h is not None:
            load().spx_batch_destroy(self._h)
            self._h = None
            self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over resident matrices (include/spx_serve.h).  Matrices are admitted by their
    footprint bound against memory_budget; requests against one matrix that wait together are
    coalesced into one product with several right-hand sides (coalesce=True), or served one per
    launch in arrival order (coalesce=False, the plain path)."""

    def __init__(self, memory_budget=None, slots=None, max_batch=None, coalesce=True,
                 poll_us=None):
        L = load()
        o = ServerOpts()
        _check(L.spx_server_opts_default(ctypes.byref(o)))
        if memory_budget is not None:
            o.memory_budget = int(memory_budget)
        if slots is not None:
            o.slots = int(slots)
        if max_batch is not None:
            o.max_batch = int(max_batch)
        if poll_us is not None:
            o.poll_us = int(poll_us)
        o.coalesce = 1 if coalesce else 0
        h = ctypes.c_void_p()
        _check(L.spx_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.max_batch = o.max_batch if coalesce else 1
        self._shapes = {}
        self._held = {}  # ticket -> (x, y) kept alive until waited for
        _live_containers.add(self)
        _register_shutdown()

    def add_matrix(self, row, col, val, shape, fmt="merge", value_type="f32", hot_columns=-1,
                   stream=None):
        """Convert device triplets and keep them resident; returns (matrix id, footprint bound)."""
        m, n = shape
        _dev_tensor(row, torch.int32, "row")
        _dev_tensor(col, torch.int32, "col")
        _dev_tensor(val, torch.float64, "val")
        if not (row.numel() == col.numel() == val.numel()):
            raise ValueError("row, col and val must have the same length")
        L = load()
        coo = CooDesc(m, n, row.numel(), row.data_ptr(), col.data_ptr(), val.data_ptr(), 0)
        opts = ConvertOpts()
        _check(L.spx_convert_opts_default(ctypes.byref(opts)))
        opts.hot_columns = int(hot_columns)
        opts.value_type = VALUE_TYPES[value_type]
        mid = ctypes.c_int32()
        nb = ctypes.c_int64()
        _check(L.spx_server_add_matrix(self._h, ctypes.byref(coo), FORMATS[fmt], ctypes.byref(opts),
                                       _stream_ptr(stream), ctypes.byref(mid), ctypes.byref(nb)))
        self._shapes[mid.value] = (m, n)
        return mid.value, nb.value

    def remove_matrix(self, mid):
        _check(load().spx_server_remove_matrix(self._h, int(mid)))
        self._shapes.pop(mid, None)

    def request(self, mid, x, y, kind="spmv", damping=0.85, stream=None):
        """A Request struct for submit / replay (x, y: float32 device vectors).  The product waits
        for the work enqueued on `stream` (default: the current stream) before the submission."""
        _dev_tensor(x, torch.float32, "x")
        _dev_tensor(y, torch.float32, "y")
        return Request(int(mid), REQUEST_KINDS[kind], float(damping), x.data_ptr(), y.data_ptr(),
                       _stream_ptr(stream))

    def submit(self, mid, x, y, kind="spmv", damping=0.85, stream=None):
        """Queue y = A x (kind 'spmv') or y = d A x + (1 - d) / n ('pagerank'); returns a ticket.
        The product waits for the work enqueued on `stream` (default: current) before the call."""
        r = self.request(mid, x, y, kind, damping, stream)
        t = ctypes.c_uint64()
        _check(load().spx_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._held[t.value] = (x, y)
        return t.value

    def wait(self, ticket):
        """Block until the request is done; returns its latency in microseconds."""
        lat = ctypes.c_double()
        try:
            _check(load().spx_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(lat)))
        finally:
            self._held.pop(ticket, None)
        return lat.value

    def replay(self, requests, arrival_us):
        """Submit requests[i] (Request structs from request()) at arrival_us[i] microseconds after
        the call starts, wait for all; returns (latencies in us as a list, wall time in us).  The
        caller keeps the request vectors alive for the duration of the call."""
        import numpy as np
        cnt = len(requests)
        arr = (Request * cnt)(*requests)
        at = np.ascontiguousarray(arrival_us, dtype=np.float64)
        if len(at) != cnt:
            raise ValueError("one arrival time per request")
        lat = np.empty(cnt, dtype=np.float64)
        wall = ctypes.c_double()
        _check(load().spx_server_replay(
            self._h, arr, at.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cnt,
            lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(wall)))
        return lat, wall.value

    def stats(self):
        st = ServerStats()
        _check(load().spx_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None:
            load().spx_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _layout_of(t):
    """(layout code, leading dimension) of a 2-D tensor: column-major when the row stride is 1."""
    rows, k = t.shape
    s0, s1 = t.stride()
    if k == 1 and (s0 == 1 or rows <= 1):
        return LAYOUTS["col"], max(rows, 1)
    if s0 == 1 or rows <= 1:
        return LAYOUTS["col"], max(s1, rows, 1)
    if s1 == 1:
        return LAYOUTS["row"], s0
    raise ValueError("operand must be column-major (stride (1, ld)) or row-major (stride (ld, 1))")


def convert(row, col, val, shape, fmt="merge", sum_duplicates=True, log2_beta=0,
            tile_items=0, hot_columns=-1, value_type="f64", stream=None):
    """Convert device triplets (int32 row, int32 col, float64 val) to a Matrix of format `fmt`
    ('rowsplit', 'merge', 'csbh', 'csb', 'bcohc', 'bcohch' or 'csbr').  hot_columns: -1
    automatic, 0 off, k > 0 at most k columns
    in the compact x copy (CRS formats).  value_type: 'f64', or 'f32' / 'bf16' stored values
    (CRS formats; products then take float32 x and y)."""
    if fmt not in FORMATS:
        raise ValueError("unknown format %r (expected one of %s)" % (fmt, sorted(FORMATS)))
    m, n = int(shape[0]), int(shape[1])
    _dev_tensor(row, torch.int32, "row")
    _dev_tensor(col, torch.int32, "col")
    _dev_tensor(val, torch.float64, "val")
    E = row.numel()
    if col.numel() != E or val.numel() != E:
        raise ValueError("row, col and val must have the same length")
    desc = CooDesc(m, n, E, ctypes.c_void_p(row.data_ptr() if E else 0),
                   ctypes.c_void_p(col.data_ptr() if E else 0),
                   ctypes.c_void_p(val.data_ptr() if E else 0), 0)
    if value_type not in VALUE_TYPES:
        raise ValueError("unknown value_type %r" % (value_type,))
    opts = ConvertOpts(1 if sum_duplicates else 0, int(log2_beta), 1, int(tile_items),
                       int(hot_columns), VALUE_TYPES[value_type])
    rep = ConvertReport()
    h = ctypes.c_void_p()
    L = load()
    _check(L.spx_convert(ctypes.byref(desc), FORMATS[fmt], ctypes.byref(opts),
                         _stream_ptr(stream), ctypes.byref(h), ctypes.byref(rep)))
    return Matrix(h, fmt, rep)


def version():
    return load().spx_version().decode()


def header_functions():
    """Names of the entry points declared in include/*.h."""
    import glob
    import re
    names = set()
    for hdr in sorted(glob.glob(os.path.join(_PKG, "..", "include", "*.h"))):
        with open(hdr) as f:
            text = f.read()
        names.update(re.findall(r"^\s*(?:const\s+)?[a-z_][a-z_0-9]*\*?\s+\**(spx_[a-z_0-9]+)\(", text, re.M))
    return sorted(names)

