"""Helpers of the GPU parity tests: upload a batch, run SpKAdd through the C ABI,
compare with the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import workloads

F32_UNIT = 2.0 ** -24
F64_UNIT = 2.0 ** -53


def note(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a failing run says which one."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_device(batch: workloads.CSCBatch, dev="cuda:0"):
    import torch
    cps = [torch.from_numpy(np.ascontiguousarray(batch.colptr[i])).to(dev) for i in range(batch.k)]
    ris = [torch.from_numpy(r).to(dev) for r in batch.rowidx]
    vas = [torch.from_numpy(v).to(dev) for v in batch.vals]
    return cps, ris, vas


def run_gpu(batch: workloads.CSCBatch, opts=None, stats=False, device_out=False):
    """(colptr int64, rowidx, values[, stats]) of B computed by the GPU library."""
    import torch
    from paper_2112_10223_amd import binding
    cps, ris, vas = to_device(batch)
    n = batch.n
    dtype = binding.SPKADD_F64 if batch.vals[0].dtype == np.float64 else binding.SPKADD_F32
    plan = binding.spkadd_plan(batch.m, n, cps, ris, dtype, opts)
    try:
        colptr_c = torch.empty(n + 1, dtype=torch.int32, device="cuda:0")
        nnz = binding.spkadd_symbolic(plan, colptr_c)
        rowidx_c = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda:0")[:nnz]
        vals_c = torch.empty(max(nnz, 1), dtype=vas[0].dtype if vas else torch.float32, device="cuda:0")[:nnz]
        binding.spkadd_numeric(plan, vas, rowidx_c, vals_c)
        torch.cuda.synchronize()
        st = binding.spkadd_get_stats(plan)
    finally:
        plan.free()
    if device_out:
        out = (colptr_c, rowidx_c, vals_c)
    else:
        out = (colptr_c.cpu().numpy().astype(np.int64), rowidx_c.cpu().numpy(), vals_c.cpu().numpy())
    return (*out, st) if stats else out


def value_bound(batch, ref):
    """Per-entry tolerance max(k, t) * u * sum|a| (u = 2^-24 for fp32, 2^-53 for fp64).

    t is the number of stored input entries summed into the output entry.  With
    sorted inputs t <= k and the bound is k * u * sum|a|; an input column that repeats
    a row (unsorted-input mode) can make t exceed k, and a sum of t terms in any order
    is within (t - 1) * u / (1 - (t - 1) * u) * sum|a| of the exact sum."""
    unit = F64_UNIT if batch.vals[0].dtype == np.float64 else F32_UNIT
    terms = np.maximum(np.int64(batch.k), ref.mult.astype(np.int64)).astype(np.longdouble)
    return terms * np.longdouble(unit) * ref.abs


def assert_matches(batch, got, ref, cols=None, exact_values=False):
    """colptr and rowidx bit-exact; values bit-exact or within the tolerance."""
    colptr, rowidx, vals = got[:3]
    if cols is None:
        assert np.array_equal(colptr, ref.colptr), "colptr differs"
        assert np.array_equal(rowidx, ref.rowidx), "rowidx differs"
        gv = vals
    else:
        cols = np.asarray(cols)
        counts = colptr[cols + 1] - colptr[cols]
        assert np.array_equal(counts, np.diff(ref.colptr)), "column counts differ"
        sel = np.concatenate([np.arange(colptr[j], colptr[j + 1]) for j in cols]) if len(cols) else \
            np.zeros(0, np.int64)
        assert np.array_equal(rowidx[sel], ref.rowidx), "rows differ"
        gv = vals[sel]
    if exact_values:
        assert np.array_equal(gv.astype(np.float64), ref.val.astype(np.float64)), "values differ"
    else:
        idx = None
        if batch.vals[0].dtype == np.float32:
            # fast pass in float64: the margins (2^-40 of the bound, 2^-50 * sum|a|) exceed
            # every rounding of these float64 steps, so an entry passing here is within
            # the bound; the others are checked exactly below
            s64 = ref.abs.astype(np.float64)
            bound64 = np.maximum(np.float64(batch.k), ref.mult.astype(np.float64)) * F32_UNIT * s64
            diff64 = np.abs(gv.astype(np.float64) - ref.val.astype(np.float64))
            idx = np.nonzero(~(diff64 <= bound64 * (1.0 - 2.0 ** -40) - 2.0 ** -50 * s64))[0]
            if idx.shape[0] == 0:
                return
        sub = ref if idx is None else _Sub(ref, idx)
        sv = gv if idx is None else gv[idx]
        diff = np.abs(sv.astype(np.longdouble) - sub.val)
        bound = value_bound(batch, sub)
        bad = diff > bound
        assert not bad.any(), f"{int(bad.sum())} values outside k*u*sum|a| (max excess {float((diff - bound).max())})"


class _Sub:
    """The entries idx of an oracle result (val, abs, mult)."""

    def __init__(self, ref, idx):
        self.val, self.abs, self.mult = ref.val[idx], ref.abs[idx], ref.mult[idx]


def check_properties(batch, colptr, rowidx):
    """Invariants that hold at any size: colptr monotone from 0, rows in range and
    strictly ascending per column, nnz(B) <= sum nnz(A_i), nnz(B(:,j)) >= max_i nnz(A_i(:,j))."""
    n, m = batch.n, batch.m
    assert colptr.shape == (n + 1,) and colptr[0] == 0
    counts = np.diff(colptr)
    assert (counts >= 0).all()
    assert colptr[-1] == rowidx.shape[0] <= batch.nnz_in
    for i in range(batch.k):
        assert (counts >= np.diff(batch.colptr[i])).all()
    if rowidx.shape[0]:
        assert rowidx.min() >= 0 and rowidx.max() < m
        d = np.diff(rowidx.astype(np.int64))
        inner = np.ones(d.shape[0], bool)
        b = colptr[1:-1] - 1
        b = b[(b >= 0) & (b < d.shape[0])]
        inner[b] = False
        assert (d[inner] > 0).all(), "rows not strictly ascending within a column"


def check_properties_device(batch, colptr_d, rowidx_d):
    """check_properties with the row checks done on the device (large outputs)."""
    import torch
    n, m = batch.n, batch.m
    colptr = colptr_d.cpu().numpy().astype(np.int64)
    assert colptr.shape == (n + 1,) and colptr[0] == 0
    counts = np.diff(colptr)
    assert (counts >= 0).all()
    assert colptr[-1] == rowidx_d.shape[0] <= batch.nnz_in
    for i in range(batch.k):
        assert (counts >= np.diff(batch.colptr[i])).all()
    nnz = rowidx_d.shape[0]
    if nnz:
        assert int(rowidx_d.min()) >= 0 and int(rowidx_d.max()) < m
        d = rowidx_d[1:] - rowidx_d[:-1]
        inner = torch.ones(nnz - 1, dtype=torch.bool, device=rowidx_d.device)
        b = colptr[1:-1] - 1
        b = b[(b >= 0) & (b < nnz - 1)]
        inner[torch.from_numpy(b).to(rowidx_d.device)] = False
        assert bool((d[inner] > 0).all()), "rows not strictly ascending within a column"
    return colptr


def gather_columns(colptr, rowidx_d, vals_d, cols):
    """Compact host copies (colptr of the selection, rows, values) of the listed output columns."""
    import torch
    cols = np.asarray(cols, dtype=np.int64)
    counts = colptr[cols + 1] - colptr[cols]
    sel = np.concatenate([np.arange(colptr[j], colptr[j + 1]) for j in cols]) if len(cols) else np.zeros(0, np.int64)
    idx = torch.from_numpy(sel).to(rowidx_d.device)
    sub_colptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return sub_colptr, rowidx_d[idx].cpu().numpy(), vals_d[idx].cpu().numpy()


def host_threads() -> int:
    """Worker threads for host-side checks: the cores in this process's affinity mask,
    at most 16 (the host share of one GPU)."""
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def column_chunks(batch, target_entries=1 << 22):
    """Contiguous column ranges of about target_entries input entries each (a column
    heavier than that is a chunk of its own)."""
    u = np.zeros(batch.n, dtype=np.int64)
    for i in range(batch.k):
        u += np.diff(batch.colptr[i]).astype(np.int64)
    csum = np.concatenate([[0], np.cumsum(u)])
    bounds = [0]
    while bounds[-1] < batch.n:
        s = bounds[-1]
        e = int(np.searchsorted(csum, csum[s] + target_entries, side="right")) - 1
        bounds.append(min(batch.n, max(e, s + 1)))
    return [(bounds[t], bounds[t + 1]) for t in range(len(bounds) - 1)]


def oracle_check_all(batch, colptr, rowidx, vals, exact=False, target_entries=1 << 22):
    """Every output column of a GPU result against the oracle.

    colptr, rowidx, vals: host arrays of the GPU's B (colptr int64).  The oracle runs
    on column chunks in host threads (its C routine runs without the interpreter lock);
    each chunk is compared as it completes: counts and rows bit-exact, values bit-exact
    or within max(k, t) * u * sum|a|.  Returns the number of entries checked."""
    import concurrent.futures as cf
    assert colptr.shape == (batch.n + 1,) and colptr[0] == 0
    assert int(colptr[-1]) == rowidx.shape[0] == vals.shape[0]
    chunks = column_chunks(batch, target_entries)

    def one(ch):
        s, e = ch
        cols = np.arange(s, e, dtype=np.int64)
        ref = oracle.spkadd(batch, cols=cols)
        o0, o1 = int(colptr[s]), int(colptr[e])
        sub_cp = colptr[s:e + 1] - o0
        got = (sub_cp, rowidx[o0:o1], vals[o0:o1])
        assert_matches(batch, got, ref, exact_values=exact)
        return o1 - o0

    checked = 0
    with cf.ThreadPoolExecutor(host_threads()) as ex:
        for c in ex.map(one, chunks):
            checked += c
    assert checked == rowidx.shape[0]
    return checked
