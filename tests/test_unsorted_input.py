"""GPU parity of the unsorted-input mode (SPKADD_FLAG_UNSORTED_IN) against the CPU
oracle, which sorts the (column, row, value) triples itself and so needs no input
order.

Every input column is shuffled (rows and values together), and some columns repeat a
row; the result must equal the oracle's sum of the same entries: colptr and rowidx
bit-exact, values bit-exact for integer-valued inputs and within k * u * sum|a|
otherwise.  The cases reach every accumulator family and each fallback of the window
histogram and partition (more inputs than the on-chip segment table, more windows in
a column than on-chip cursors).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, note, run_gpu

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
    flags = kw.pop("flags", 0) | binding.SPKADD_FLAG_UNSORTED_IN
    return binding.make_opts(flags=flags, **kw)


def _shuffled(batch, seed, dup_every=0, repeats=1):
    """The same entries, each input column in a random order; with dup_every > 0 every
    dup_every-th non-empty column of each input also repeats its first row (`repeats`
    more times, each copy with the value of the first)."""
    rng = np.random.default_rng(seed)
    cps, rows, vals = [], [], []
    for i in range(batch.k):
        cp = batch.colptr[i].astype(np.int64)
        r_out, v_out, cp_out = [], [], [0]
        for j in range(batch.n):
            s, e = cp[j], cp[j + 1]
            r, v = batch.rowidx[i][s:e], batch.vals[i][s:e]
            if dup_every and e > s and j % dup_every == 0:
                r = np.concatenate([r, np.repeat(r[:1], repeats)])
                v = np.concatenate([v, np.repeat(v[:1], repeats)])
            perm = rng.permutation(len(r))
            r_out.append(r[perm])
            v_out.append(v[perm])
            cp_out.append(cp_out[-1] + len(r))
        cps.append(np.array(cp_out, np.int32))
        rows.append(np.concatenate(r_out).astype(np.int32) if r_out else np.zeros(0, np.int32))
        vals.append(np.concatenate(v_out).astype(batch.vals[i].dtype) if v_out else np.zeros(0, batch.vals[i].dtype))
    return workloads.CSCBatch(batch.m, batch.n, np.stack(cps), rows, vals)


def _check(b, opts, exact=True, windows=None):
    ref = oracle.spkadd(b)
    got = run_gpu(b, opts, stats=True)
    assert_matches(b, got[:3], ref, exact_values=exact)
    if windows is not None:
        assert got[3]["n_windows"] >= windows
    return got[3]


@pytest.mark.parametrize("values", ["int32f", "f32", "f64"])
def test_every_bin(values):
    """Columns from empty through the wave and workgroup bins to row windows."""
    from tests.test_gpu_parity import _ragged_batch
    note(f"unsorted every_bin values={values}")
    base = _ragged_batch(seed=31, k=6, m=20000, values="int32f" if values == "int32f" else "f32")
    if values == "f64":
        base = workloads.CSCBatch(base.m, base.n, base.colptr, base.rowidx, [v.astype(np.float64) for v in base.vals])
    b = _shuffled(base, seed=1, dup_every=5)
    st = _check(b, _opts(), exact=values == "int32f")
    assert st["n_window_cols"] > 0 and st["n_wave_cols"] > 0 and st["n_wg_cols"] > 0


@pytest.mark.parametrize("accum_mode", [1, 2])
def test_accumulators(accum_mode):
    note(f"unsorted accum_mode={accum_mode}")
    b = _shuffled(workloads.er(3000, 400, 9, 30.0, seed=8, values="int32f"), seed=2, dup_every=3)
    _check(b, _opts(accum_mode=accum_mode))


@pytest.mark.parametrize("window_cap", [64, 700])
def test_windows_refined(window_cap):
    """Every column through row windows, small windows: several refinement levels over
    skewed R-MAT rows."""
    note(f"unsorted windows window_cap={window_cap}")
    b = _shuffled(workloads.rmat(12, 8, 5, seed=12, values="int32f"), seed=3, dup_every=7)
    st = _check(b, _opts(force_bin=2, window_cap=window_cap), windows=1)
    assert st["window_levels"] >= 1


def test_more_inputs_than_the_segment_table():
    """k = 1100 (> 1024): the window passes walk the inputs one by one."""
    note("unsorted k=1100")
    b = _shuffled(workloads.er(5000, 6, 1100, 3.0, seed=21, values="int32f"), seed=4, dup_every=2)
    _check(b, _opts(force_bin=2, window_cap=512), windows=6)


def test_more_windows_than_on_chip_cursors():
    """A column split into more than 4096 windows: global counters and cursors."""
    note("unsorted many windows")
    b = _shuffled(workloads.er(100000, 2, 9, 1000.0, seed=22, fixed=True, values="int32f"), seed=5)
    _check(b, _opts(force_bin=2, window_cap=2), windows=8192)


def test_numeric_rerun_and_validation():
    """A second numeric pass with new values gathers them again; VALIDATE accepts
    unsorted rows and still rejects rows out of range."""
    import torch
    from paper_2112_10223_amd import binding
    from tests.gpu_util import to_device
    note("unsorted rerun + validate")
    b = _shuffled(workloads.er(4000, 50, 7, 200.0, seed=23, values="int32f"), seed=6, dup_every=4)
    cps, ris, vas = to_device(b)
    opts = _opts(flags=binding.SPKADD_FLAG_VALIDATE, force_bin=2, window_cap=256)
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, opts)
    try:
        colptr_c = torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0")
        nnz = binding.spkadd_symbolic(plan, colptr_c)
        rowidx_c = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda:0")
        vals_c = torch.empty(max(nnz, 1), dtype=torch.float32, device="cuda:0")
        for scale in (1.0, -2.0):
            vs = [v * scale for v in vas]
            binding.spkadd_numeric(plan, vs, rowidx_c, vals_c)
            torch.cuda.synchronize()
            b2 = workloads.CSCBatch(b.m, b.n, b.colptr, b.rowidx, [v * np.float32(scale) for v in b.vals])
            ref = oracle.spkadd(b2)
            got = (colptr_c.cpu().numpy().astype(np.int64), rowidx_c[:nnz].cpu().numpy(), vals_c[:nnz].cpu().numpy())
            assert_matches(b2, got, ref, exact_values=True)
    finally:
        plan.free()
    bad = [r.clone() for r in ris]
    bad[2][5] = b.m  # a row out of range
    with pytest.raises(binding.SpkaddError):
        binding.spkadd_plan(b.m, b.n, cps, bad, binding.SPKADD_F32, opts).free()


def test_sorted_input_same_result():
    """Sorted input under the flag gives the result of the default path."""
    note("unsorted flag on sorted input")
    from paper_2112_10223_amd import binding
    b = workloads.rmat(11, 8, 4, seed=24, values="int32f")
    ref = run_gpu(b, binding.make_opts(force_bin=2, window_cap=256))
    got = run_gpu(b, _opts(force_bin=2, window_cap=256))
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("force", [False, True])
def test_real_values_many_repeats(force):
    """Real values (N(0,1) on R-MAT rows) with rows repeated within input columns so
    that an output entry sums more terms than there are inputs (t > k): the values
    must lie within t * u * sum|a| of the oracle's, through every accumulator and
    through refined row windows."""
    note(f"unsorted real values, repeats, windows forced={force}")
    b = _shuffled(workloads.rmat(12, 8, 3, seed=25, values="normal"), seed=7, dup_every=2, repeats=20)
    ref = oracle.spkadd(b)
    assert int(ref.mult.max()) > b.k
    opts = _opts(force_bin=2, window_cap=256) if force else _opts()
    got = run_gpu(b, opts, stats=True)
    assert_matches(b, got[:3], ref)
    if force:
        assert got[3]["n_windows"] > 0
