"""The no-allocation entry point (spkadd_sum_noalloc) through the C ABI, against the
existing spkadd_plan / spkadd_symbolic / spkadd_numeric entry points and the oracle.

Two calls in a row share the library's scratch array, the second with a smaller input
than the first (so stale contents of the first are under the second's workspace).
colptr and rows bit-exact; values bit-exact for integer-valued inputs and within
max(k, t) * u * sum|a| of the oracle otherwise.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, note, run_gpu, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_10223_amd import binding
    binding.lib()


def _noalloc(batch, cap=None, opts=None):
    import torch
    from paper_2112_10223_amd import binding
    cps, ris, vas = to_device(batch)
    cap = batch.nnz_in if cap is None else cap
    dev = "cuda:0"
    colptr_c = torch.full((batch.n + 1,), -7, dtype=torch.int32, device=dev)
    rowidx_c = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)[:cap]
    values_c = torch.zeros(max(cap, 1), dtype=vas[0].dtype, device=dev)[:cap]
    nnz = binding.spkadd_sum_noalloc(batch.m, cps, ris, vas, colptr_c, rowidx_c, values_c, opts)
    torch.cuda.synchronize()
    return nnz, (colptr_c.cpu().numpy().astype(np.int64), rowidx_c[:nnz].cpu().numpy(),
                 values_c[:nnz].cpu().numpy())


def _same_as_plan_path(batch, exact, opts=None):
    nnz, got = _noalloc(batch, opts=opts)
    want = run_gpu(batch, opts)
    assert nnz == int(want[0][-1])
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    ref = oracle.spkadd(batch)
    assert_matches(batch, got, ref, exact_values=exact)
    if exact:
        assert np.array_equal(got[2], want[2])


@pytest.mark.parametrize("values", ["int32f", "f32", "f64"])
def test_two_calls_second_smaller(values):
    """Every bin (wave, workgroup, row windows) in the first call; a smaller input in
    the second."""
    from tests.test_gpu_parity import _ragged_batch
    note(f"noalloc two calls values={values}")
    big = _ragged_batch(seed=31, k=8, m=20000, values="int32f" if values == "int32f" else "f32")
    if values == "f64":
        big = big.astype(np.float64)
    small = workloads.er(3000, 200, 5, 20.0, seed=32, values=values)
    for b in (big, small):
        _same_as_plan_path(b, exact=values == "int32f")


def test_headline_shape_then_tiny():
    """k = 32 ER over 65 536 rows (20 000 columns), then a 1000 x 1000 k = 4 input."""
    note("noalloc headline shape then tiny")
    _same_as_plan_path(workloads.er(65536, 20000, 32, 16.0, seed=33, values="int32f"), exact=True)
    _same_as_plan_path(workloads.config1(values="int32f"), exact=True)


def test_options_and_errors():
    """Forced windows and the ordered mode run in the scratch array too; too small an
    output capacity is refused with colptr(B) and nnz(B) written; an input whose
    workspace exceeds the array is refused before any device work."""
    import torch
    from paper_2112_10223_amd import binding
    note("noalloc options and errors")
    b = workloads.er(20000, 300, 6, 300.0, seed=34, values="f32")
    _same_as_plan_path(b, exact=False, opts=binding.make_opts(force_bin=2, window_cap=256))
    nnz, got = _noalloc(b, opts=binding.make_opts(flags=binding.SPKADD_FLAG_ORDERED))
    ref = oracle.spkadd_ordered(b)
    assert np.array_equal(got[1], ref.rowidx) and np.array_equal(got[2].view(np.uint32), ref.val.view(np.uint32))
    need = int(ref.colptr[-1])
    with pytest.raises(binding.SpkaddError) as ei:
        _noalloc(b, cap=need - 1)
    assert ei.value.status == binding.SPKADD_ERR_INVALID
    # too many columns for the scratch array: n = 4 194 304 needs about 72 MB
    n = 1 << 22
    cp = [torch.zeros(n + 1, dtype=torch.int32, device="cuda:0")]
    ri = [torch.zeros(1, dtype=torch.int32, device="cuda:0")]
    va = [torch.zeros(1, dtype=torch.float32, device="cuda:0")]
    out_cp = torch.empty(n + 1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(binding.SpkaddError) as ei:
        binding.spkadd_sum_noalloc(10, cp, ri, va, out_cp, torch.empty(1, dtype=torch.int32, device="cuda:0"),
                                   torch.empty(1, device="cuda:0"))
    assert ei.value.status == binding.SPKADD_ERR_UNSUPPORTED
    # and the entry point still works afterwards
    _same_as_plan_path(workloads.config1(values="int32f"), exact=True)
