"""CPU oracle for SpKAdd -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never calls it.

``spkadd(batch, cols=None)`` computes the requested output columns of
B = A_1 + ... + A_k (Section II-A) with the plain definition written in
``oracle.c``: concatenate the (column, row, value) triples, sort them by
(column, row), and reduce each run in 80-bit long double.  It returns canonical CSC
plus, for each entry, the sum of magnitudes s and the run length t that the
tolerance bound needs.

``spkadd_ordered(batch, cols=None)`` gives the same pattern with every value the
sequential sum of its terms in input order, in the inputs' own precision (the order
in which Algorithm 5 visits the inputs of a column, Section II-C).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_lib(force: bool = False, src: str | None = None, out: str | None = None) -> str:
    """Compile oracle.c (or `src`) into a shared library."""
    src = src or os.path.join(_HERE, "oracle.c")
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _bind(path: str):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_spkadd.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P, P, ctypes.c_int32,
                                  P, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64]
    lib.oracle_spkadd.restype = ctypes.c_int64
    if hasattr(lib, "oracle_spkadd_ordered"):
        lib.oracle_spkadd_ordered.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P, P,
                                              ctypes.c_int32, P, ctypes.c_int64, P, P, P, P, ctypes.c_int64]
        lib.oracle_spkadd_ordered.restype = ctypes.c_int64
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        _lib = _bind(_LIB_PATH)
    return _lib


@dataclass
class OracleResult:
    colptr: np.ndarray   # int64 (ncols+1,)
    rowidx: np.ndarray   # int32 (nnz,)
    val: np.ndarray      # longdouble (nnz,): sum of the stored input entries
    abs: np.ndarray      # longdouble (nnz,): sum of their magnitudes
    mult: np.ndarray     # int32 (nnz,): number of stored input entries at the position

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


def spkadd(batch, cols=None, lib=None) -> OracleResult:
    """Columns `cols` (all when None) of the sum of the k inputs of `batch`."""
    lib = lib or _load()
    k, n = batch.k, batch.n
    colptr_rows = [np.ascontiguousarray(batch.colptr[i]) for i in range(k)]
    cp = (ctypes.c_void_p * k)(*[a.ctypes.data for a in colptr_rows])
    ri = (ctypes.c_void_p * k)(*[a.ctypes.data for a in batch.rowidx])
    if batch.vals:
        dtype = 0 if batch.vals[0].dtype == np.float32 else 1
        vp = (ctypes.c_void_p * k)(*[a.ctypes.data for a in batch.vals])
    else:
        dtype, vp = -1, None
    if cols is None:
        cols_arr, ncols = None, n
        cap = sum(int(batch.colptr[i, n]) for i in range(k))
    else:
        cols_arr = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
        ncols = int(cols_arr.shape[0])
        cap = int(sum((batch.colptr[i, cols_arr + 1] - batch.colptr[i, cols_arr]).sum() for i in range(k)))
    out_cp = np.zeros(ncols + 1, dtype=np.int64)
    out_r = np.empty(max(cap, 1), dtype=np.int32)
    out_v = np.empty(max(cap, 1), dtype=np.longdouble)
    out_a = np.empty(max(cap, 1), dtype=np.longdouble)
    out_t = np.empty(max(cap, 1), dtype=np.int32)
    nnz = lib.oracle_spkadd(batch.m, n, k, cp, ri, vp, dtype,
                            None if cols_arr is None else cols_arr.ctypes.data, ncols,
                            out_cp.ctypes.data, out_r.ctypes.data, out_v.ctypes.data, out_a.ctypes.data,
                            out_t.ctypes.data, max(cap, 1))
    if nnz < 0:
        raise ValueError(f"oracle_spkadd failed ({nnz})")
    return OracleResult(out_cp, out_r[:nnz].copy(), out_v[:nnz].copy(), out_a[:nnz].copy(), out_t[:nnz].copy())


@dataclass
class OrderedResult:
    colptr: np.ndarray   # int64 (ncols+1,)
    rowidx: np.ndarray   # int32 (nnz,)
    val: np.ndarray      # the inputs' dtype (nnz,): sequential sum in input order
    mult: np.ndarray     # int32 (nnz,)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


def spkadd_ordered(batch, cols=None, lib=None) -> OrderedResult:
    """Columns `cols` (all when None) of the sum with every value added in input order
    in the inputs' precision."""
    lib = lib or _load()
    k, n = batch.k, batch.n
    if not batch.vals:
        raise ValueError("the ordered sum needs values")
    dt = batch.vals[0].dtype
    dtype = 0 if dt == np.float32 else 1
    colptr_rows = [np.ascontiguousarray(batch.colptr[i]) for i in range(k)]
    cp = (ctypes.c_void_p * k)(*[a.ctypes.data for a in colptr_rows])
    ri = (ctypes.c_void_p * k)(*[a.ctypes.data for a in batch.rowidx])
    vp = (ctypes.c_void_p * k)(*[a.ctypes.data for a in batch.vals])
    if cols is None:
        cols_arr, ncols = None, n
        cap = sum(int(batch.colptr[i, n]) for i in range(k))
    else:
        cols_arr = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
        ncols = int(cols_arr.shape[0])
        cap = int(sum((batch.colptr[i, cols_arr + 1] - batch.colptr[i, cols_arr]).sum() for i in range(k)))
    out_cp = np.zeros(ncols + 1, dtype=np.int64)
    out_r = np.empty(max(cap, 1), dtype=np.int32)
    out_v = np.empty(max(cap, 1), dtype=np.float64)
    out_t = np.empty(max(cap, 1), dtype=np.int32)
    nnz = lib.oracle_spkadd_ordered(batch.m, n, k, cp, ri, vp, dtype,
                                    None if cols_arr is None else cols_arr.ctypes.data, ncols,
                                    out_cp.ctypes.data, out_r.ctypes.data, out_v.ctypes.data, out_t.ctypes.data,
                                    max(cap, 1))
    if nnz < 0:
        raise ValueError(f"oracle_spkadd_ordered failed ({nnz})")
    return OrderedResult(out_cp, out_r[:nnz].copy(), out_v[:nnz].astype(dt), out_t[:nnz].copy())
