"""Streaming SpKAdd: a running sum over inputs that arrive in batches (the paper's
conclusions, Section V, leave streaming SpKAdd as future work).  Each
arriving batch A_1..A_b is added together with the running sum S in one k-way sum,
S <- S + A_1 + ... + A_b (k = b + 1), so every entry of S is read once per batch
instead of once per input as in an incremental 2-way scheme.  Host orchestration
only: every sum runs in the library's kernels (spkadd.h).
"""
from __future__ import annotations

from . import binding


class StreamingSum:
    """Running sum of m x n CSC matrices on the device.

    add(colptrs, rowidxs, values) takes one batch (k-lists of device tensors, as
    binding.spkadd); result() returns (colptr, rowidx, values) of the sum so far, or
    None before the first batch.

    The sums run on `stream` (torch's current stream when None); each new sum's
    outputs are allocated on that stream (binding.spkadd), so dropping the previous
    running sum cannot release its memory to other streams while the new sum still
    reads it."""

    def __init__(self, m: int, n: int, opts=None, stream=None):
        self.m, self.n = m, n
        self.opts, self.stream = opts, stream
        self.sum = None
        self.batches = 0

    def add(self, colptrs, rowidxs, values):
        if not colptrs:
            return
        for c in colptrs:
            if c.shape[0] != self.n + 1:
                raise ValueError(f"colptr of length {c.shape[0]}, expected n + 1 = {self.n + 1}")
        cps, ris, vas = list(colptrs), list(rowidxs), list(values)
        if self.sum is not None:
            c, r, v = self.sum
            cps, ris, vas = [c] + cps, [r] + ris, [v] + vas
        self.sum = binding.spkadd(self.m, cps, ris, vas, self.opts, self.stream)
        self.batches += 1

    def result(self):
        return self.sum
