"""GPU parity of the ordered mode (SPKADD_FLAG_ORDERED) against the oracle's ordered sum.

In this mode every value of B is the sequential sum of its terms in input order, in
the values' own precision, so the GPU must reproduce the oracle's ordered sum bit for
bit (colptr and rows as always).  Values spread over many binades make the order of
the additions visible in the last bits; the cases reach wave columns (bitmap and hash
accumulators), both workgroup bins and row windows.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import note, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_10223_amd import binding
    binding.lib()


def _opts(**kw):
    from paper_2112_10223_amd import binding
    flags = kw.pop("flags", 0) | binding.SPKADD_FLAG_ORDERED
    return binding.make_opts(flags=flags, **kw)


def _spread(batch, seed):
    """The same pattern with each value scaled by a seeded power of two in [2^-20, 2^12]:
    sums of such terms round differently in different orders."""
    rng = np.random.default_rng(seed)
    vals = [(v * np.exp2(rng.integers(-20, 13, size=v.shape[0]))).astype(v.dtype) for v in batch.vals]
    return workloads.CSCBatch(batch.m, batch.n, batch.colptr, batch.rowidx, vals)


def _check(batch, opts, stats=False):
    ref = oracle.spkadd_ordered(batch)
    got = run_gpu(batch, opts, stats=stats)
    assert np.array_equal(got[0], ref.colptr), "colptr differs"
    assert np.array_equal(got[1], ref.rowidx), "rowidx differs"
    bad = got[2].view(np.uint8).reshape(-1, got[2].itemsize) != ref.val.view(np.uint8).reshape(-1, ref.val.itemsize)
    nbad = int(bad.any(axis=1).sum())
    assert nbad == 0, f"{nbad} of {ref.nnz} values differ from the input-order sum"
    return got


def test_order_matters_here():
    """The test values do distinguish orders: the ordered sum differs from the sum in
    reversed input order on many entries."""
    b = _spread(workloads.er(1000, 300, 32, 100.0, seed=3, values="f32"), 1)
    fwd = oracle.spkadd_ordered(b)
    rev = oracle.spkadd_ordered(b.select(list(range(b.k))[::-1]))
    assert np.array_equal(fwd.rowidx, rev.rowidx)
    assert int((fwd.val != rev.val).sum()) > 10000


@pytest.mark.parametrize("values", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(1000, 1000, 4, 8.0), (1000, 300, 32, 100.0), (65536, 2000, 32, 16.0),
                                   (1 << 20, 500, 12, 40.0), (3000, 200, 64, 14.0), (500, 300, 130, 2.0),
                                   (200, 100, 1, 5.0)])
def test_wave_columns(values, shape):
    m, n, k, d = shape
    note(f"ordered wave columns m={m} n={n} k={k} d={d} values={values}")
    b = _spread(workloads.er(m, n, k, d, seed=m % 997 + k, values=values), k)
    _check(b, _opts())


@pytest.mark.parametrize("values", ["f32", "f64"])
@pytest.mark.parametrize("force_bin,window_cap", [(-1, 0), (1, 0), (2, 0), (2, 64), (-1, 128), (1, 700)])
def test_every_bin(values, force_bin, window_cap):
    """Columns from empty through both workgroup bins to row windows (forced or not)."""
    from tests.test_gpu_parity import _ragged_batch
    note(f"ordered every bin force_bin={force_bin} window_cap={window_cap} values={values}")
    base = _ragged_batch(seed=21, k=6, m=20000, values="f32")
    if values == "f64":
        base = base.astype(np.float64)
    b = _spread(base, 2)
    got = _check(b, _opts(force_bin=force_bin, window_cap=window_cap), stats=True)
    if force_bin == 2:
        assert got[3]["n_windows"] > 0


@pytest.mark.parametrize("accum_mode", [1, 2])
def test_accumulators_and_rmat_windows(accum_mode):
    """Hash-only and bitmap-only accumulators; R-MAT columns long enough for windows."""
    note(f"ordered accum_mode={accum_mode} + R-MAT windows")
    b = _spread(workloads.er(50000, 400, 24, 20.0, seed=5, values="f32"), 3)
    _check(b, _opts(accum_mode=accum_mode))
    r = _spread(workloads.rmat(14, 16, 12, seed=6, values="normal"), 4)
    got = _check(r, _opts(accum_mode=accum_mode, window_cap=512), stats=True)
    assert got[3]["n_window_cols"] > 0


def test_integer_values_equal_plain():
    """Integer-valued inputs: every order is exact, so the ordered result equals the
    default path's bit for bit."""
    note("ordered integer values")
    b = workloads.er(20000, 500, 16, 40.0, seed=9, values="int32f")
    plain = run_gpu(b)
    got = _check(b, _opts())
    for x, y in zip(plain, got):
        assert np.array_equal(x, y)


def test_flags_and_rerun():
    """UNSORTED_OUT is ignored (the output stays sorted); UNSORTED_IN is refused; a
    second numeric pass with new values on the same plan is ordered too."""
    import torch
    from paper_2112_10223_amd import binding
    from tests.gpu_util import to_device
    note("ordered flags and rerun")
    b = _spread(workloads.er(8000, 300, 10, 60.0, seed=11, values="f32"), 5)
    _check(b, _opts(flags=binding.SPKADD_FLAG_UNSORTED_OUT))
    cps, ris, vas = to_device(b)
    with pytest.raises(binding.SpkaddError) as ei:
        binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, _opts(flags=binding.SPKADD_FLAG_UNSORTED_IN))
    assert ei.value.status == binding.SPKADD_ERR_UNSUPPORTED
    with pytest.raises(binding.SpkaddError) as ei:
        binding.Batch(binding.SPKADD_F32, 4, 100, 16, _opts())
    assert ei.value.status == binding.SPKADD_ERR_UNSUPPORTED
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, _opts(force_bin=2, window_cap=200))
    try:
        cp = torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0")
        nnz = binding.spkadd_symbolic(plan, cp)
        r = torch.empty(nnz, dtype=torch.int32, device="cuda:0")
        v = torch.empty(nnz, dtype=torch.float32, device="cuda:0")
        for seed in (6, 7):
            b2 = _spread(b, seed)
            _, _, vas2 = to_device(b2)
            binding.spkadd_numeric(plan, vas2, r, v)
            torch.cuda.synchronize()
            ref = oracle.spkadd_ordered(b2)
            assert np.array_equal(r.cpu().numpy(), ref.rowidx)
            assert np.array_equal(v.cpu().numpy().view(np.uint32), ref.val.view(np.uint32))
    finally:
        plan.free()
