"""The paper's comparison algorithms on the GPU, for measuring the hash method against
(include/spkadd_baselines.h).  Argument marshalling only; every step runs in the
library's kernels.

* heap_add: the k-way heap merge of Algorithm 3 (HeapAdd, Section II-C) through
  spkadd_heap_add (one thread per column, its heap in LDS).
* tree_add: the 2-way tree of Section II-B -- lg k rounds, each summing pairs of the
  previous round's matrices with the k = 2 SpKAdd of spkadd.h (an odd matrix out is
  carried to the next round).
"""
from __future__ import annotations

import ctypes

from . import binding

HEAP_MAX_K = 128


def _heap_fn():
    f = binding.lib().spkadd_heap_add
    if f.argtypes is None:
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        f.argtypes = [I32, I32, I32, P, P, P, ctypes.c_int, P, P, P, I64, ctypes.POINTER(I64), P]
        f.restype = ctypes.c_int
    return f


def heap_add(m, colptrs, rowidxs, values, stream=None):
    """B = A_1 + ... + A_k by the k-way heap merge (sorted input columns).  Inputs are
    k-lists of device tensors; returns (colptr, rowidx, values) of B as device tensors."""
    import torch
    k = len(colptrs)
    n = colptrs[0].shape[0] - 1
    dtype = binding.SPKADD_F64 if values[0].dtype == torch.float64 else binding.SPKADD_F32
    dev = colptrs[0].device
    cap = sum(int(r.shape[0]) for r in rowidxs)
    colptr_c = torch.empty(n + 1, dtype=torch.int32, device=dev)
    rowidx_c = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    values_c = torch.empty(max(cap, 1), dtype=values[0].dtype, device=dev)
    pc = binding.PtrArray(colptrs)
    pr = binding.PtrArray(rowidxs, non_null=True, fallback=rowidx_c.data_ptr())
    pv = binding.PtrArray(values, non_null=True, fallback=values_c.data_ptr())
    nnz = ctypes.c_int64(0)
    binding._check(_heap_fn()(m, n, k, pc.arr, pr.arr, pv.arr, dtype, ctypes.c_void_p(colptr_c.data_ptr()),
                              ctypes.c_void_p(rowidx_c.data_ptr()), ctypes.c_void_p(values_c.data_ptr()), cap,
                              ctypes.byref(nnz), binding._stream_ptr(stream)))
    z = int(nnz.value)
    return colptr_c, rowidx_c[:z], values_c[:z]


def tree_add(m, colptrs, rowidxs, values, opts=None, stream=None):
    """B = A_1 + ... + A_k by a balanced tree of 2-way sums (lg k rounds)."""
    level = list(zip(colptrs, rowidxs, values))
    while len(level) > 1:
        nxt = []
        for a in range(0, len(level) - 1, 2):
            (c1, r1, v1), (c2, r2, v2) = level[a], level[a + 1]
            nxt.append(binding.spkadd(m, [c1, c2], [r1, r2], [v1, v2], opts, stream))
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]
