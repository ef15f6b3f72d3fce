"""Build and load the oracle's C loops (ref.c) with gcc.  Test infrastructure only."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile liboracle.so (plain C, no contraction of multiply-add, no vector flags)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-fopenmp", "-shared", "-std=c11", os.path.join(_HERE, "ref.c"), "-o",
                           tmp, "-lm"])
    os.replace(tmp, LIB_PATH)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = ctypes.CDLL(LIB_PATH)
    i64 = ctypes.c_int64
    p_i64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    p_i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    p_f64 = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    L.ref_sum_runs.argtypes = [i64, p_i64, p_i64, p_f64, p_f64]
    L.ref_alg1.argtypes = [i64, p_i64, p_i32, p_f64, p_f64, p_f64]
    L.ref_alg1_accurate.argtypes = [i64, p_i64, p_i32, p_f64, p_f64, p_f64, p_f64, p_f64]
    L.ref_triplet_spmv.argtypes = [i64, p_i32, p_i32, p_f64, p_f64, i64, p_f64]
    L.ref_parcrs.argtypes = [i64, p_i64, p_i32, p_f64, p_f64, p_f64, i64]
    L.ref_parcrs.restype = ctypes.c_int
    for f in (L.ref_sum_runs, L.ref_alg1, L.ref_alg1_accurate, L.ref_triplet_spmv):
        f.restype = None
    _lib = L
    return L
