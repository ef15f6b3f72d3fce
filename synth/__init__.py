"""Seeded synthetic inputs: R-MAT, Chung-Lu and uniform (Erdos-Renyi) triplet matrices, values
and dense vectors.

This package generates inputs only; it holds none of the SpMV method's arithmetic, so both the
oracle's tests and the GPU path take their inputs from here.  Every draw is a pure function of
(seed, stream, counter) (SplitMix64 used as a counter-based generator), so results do not depend
on the number of host threads.

Workload recipes (matrix shapes follow the power-law workloads the method targets):
  * ``rmat(scale, edge_factor)``: m = n = 2**scale, E = edge_factor * 2**scale raw entries,
    quadrant probabilities (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) by default.
  * ``chunglu(n, E, gamma)``: rows and columns drawn independently with weight (i+1)^(-1/(gamma-1)).
  * ``uniform(m, n, E)``: rows and columns uniform.
Raw entries may repeat; repeats are summed by the conversion.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

STREAM_STRUCT = 0
STREAM_VAL = 1
STREAM_X = 2
STREAM_PERM = 3


def build():
    """Compile libsynth.so with gcc (host code, OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src,
                           "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
    lib.synth_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.synth_rmat.restype = None
    lib.synth_chunglu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_uint64, i32p, i32p]
    lib.synth_chunglu.restype = ctypes.c_int
    lib.synth_uniform.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint64, i32p, i32p]
    lib.synth_uniform.restype = None
    lib.synth_values.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                 f64p]
    lib.synth_values.restype = None
    lib.synth_u64.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, u64p]
    lib.synth_u64.restype = None
    lib.synth_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_draw.restype = ctypes.c_uint64
    _lib = lib
    return lib


def draw(seed, stream, ctr):
    """One raw 64-bit draw of (seed, stream, counter)."""
    return int(_load().synth_draw(seed, stream, ctr))


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=0):
    """R-MAT raw coordinates: returns (row, col) int32 arrays of length edge_factor * 2**scale."""
    E = int(edge_factor) << int(scale)
    row = np.empty(E, np.int32)
    col = np.empty(E, np.int32)
    _load().synth_rmat(int(scale), E, a, b, c, seed, row, col)
    return row, col


def chunglu(n, E, gamma=2.1, seed=0):
    """Chung-Lu power-law raw coordinates: (row, col) int32 arrays of length E."""
    row = np.empty(int(E), np.int32)
    col = np.empty(int(E), np.int32)
    if _load().synth_chunglu(int(n), int(E), gamma, seed, row, col) != 0:
        raise MemoryError("synth_chunglu: allocation failed")
    return row, col


def uniform(m, n, E, seed=0):
    """Uniformly random raw coordinates: (row, col) int32 arrays of length E."""
    row = np.empty(int(E), np.int32)
    col = np.empty(int(E), np.int32)
    _load().synth_uniform(int(m), int(n), int(E), seed, row, col)
    return row, col


def values(length, seed=0, stream=STREAM_VAL, kind="float"):
    """Float64 values: kind 'float' = uniform(-1, 1); kind 'int' = integers in {-3..3}."""
    out = np.empty(int(length), np.float64)
    _load().synth_values(int(length), seed, stream, 0 if kind == "float" else 1, out)
    return out


def xvec(n, seed=0, kind="float"):
    """Dense input vector x of length n (stream 2)."""
    return values(n, seed, STREAM_X, kind)


def permutation(n, seed=1):
    """Random permutation of range(n) (argsort of counter-based 64-bit keys, stream 3)."""
    keys = np.empty(int(n), np.uint64)
    _load().synth_u64(int(n), seed, STREAM_PERM, keys)
    return np.argsort(keys, kind="stable").astype(np.int64)


def workload(name, seed=0, kind="float"):
    """Named workloads: returns dict(m, n, row, col, val, x).

    rmat14  : R-MAT scale 14, edge factor 16
    rmat24  : R-MAT scale 24, edge factor 16
    chunglu : Chung-Lu gamma 2.1, n = 10**7, E = 2*10**8
    rmatS   : R-MAT of scale S (e.g. 'rmat18')
    rmatSp  : R-MAT of scale S under a random relabelling of rows and of columns (row r becomes
              permutation(m, seed + 1)[r], column c becomes permutation(n, seed + 2)[c]); same
              entries, values and x, with the generator's index locality removed
    """
    relabel = name.startswith("rmat") and name.endswith("p")
    if relabel:
        name = name[:-1]
    if name == "chunglu":
        n = 10_000_000
        row, col = chunglu(n, 200_000_000, 2.1, seed)
        m = n
    elif name.startswith("rmat"):
        s = int(name[4:])
        row, col = rmat(s, 16, seed=seed)
        m = n = 1 << s
    else:
        raise ValueError("unknown workload " + name)
    if relabel:
        row = permutation(m, seed + 1).astype(np.int32)[row]
        col = permutation(n, seed + 2).astype(np.int32)[col]
    val = values(len(row), seed, STREAM_VAL, kind)
    x = xvec(n, seed, kind)
    return dict(m=m, n=n, row=row, col=col, val=val, x=x)
