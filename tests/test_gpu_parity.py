"""GPU parity: the HIP path through the C ABI against the CPU oracle.

colptr and rowidx must match bit-exactly.  Integer-valued inputs must give
bit-exact values.  Real values must lie within |c - c_ref| <= k * u * sum|a|
(u = 2^-24 fp32, 2^-53 fp64).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, check_properties, note, run_gpu

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
    return binding.make_opts(**kw)


@pytest.mark.parametrize("values", ["int32f", "f32", "int64f", "f64"])
def test_config1(values):
    note(f"config1 values={values}")
    batch = workloads.config1(values=values)
    got = run_gpu(batch)
    ref = oracle.spkadd(batch)
    assert_matches(batch, got, ref, exact_values=values.startswith("int"))


@pytest.mark.parametrize("seed", range(24))
def test_small_random(seed):
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.integers(1, 300))
    n = int(rng.integers(1, 120))
    k = int(rng.integers(1, 9))
    d = float(rng.choice([0.0, 0.5, 3.0, 20.0, 200.0]))
    values = ["int32f", "f32", "f64", "int64f"][seed % 4]
    note(f"small_random seed={seed} m={m} n={n} k={k} d={d} values={values}")
    batch = workloads.er(m, n, k, d, seed=seed, values=values)
    got = run_gpu(batch)
    ref = oracle.spkadd(batch)
    assert_matches(batch, got, ref, exact_values=values.startswith("int"))


def _ragged_batch(seed=5, k=6, m=20000, values="int32f", sizes=None):
    """Columns whose sizes span every bin: empty, wave sub-bins, both workgroup
    bins and the window bin."""
    if sizes is None:
        sizes = [0, 1, 3, 10, 40, 64, 65, 100, 170, 200, 250, 300, 500, 700, 900, 1100, 1500, 2500, 3000, 3500,
                 6000, 9000]
    n = len(sizes) * 3
    per = np.array([sizes[j % len(sizes)] for j in range(n)], dtype=np.float64) / k
    masks_cp = np.zeros((k, n + 1), np.int32)
    rows, vals = [[] for _ in range(k)], [[] for _ in range(k)]
    rng = np.random.default_rng(seed)
    for j in range(n):
        for i in range(k):
            c = int(min(m, rng.poisson(per[j]) if per[j] > 0 else 0))
            r = np.sort(rng.choice(m, size=c, replace=False)).astype(np.int32)
            rows[i].append(r)
            if values == "int32f":
                vals[i].append(rng.integers(-3, 4, size=c).astype(np.float32))
            else:
                vals[i].append(((rng.integers(0, 1 << 24, size=c) - (1 << 23)) * 2.0 ** -23).astype(np.float32))
            masks_cp[i, j + 1] = masks_cp[i, j] + c
    return workloads.CSCBatch(m, n, masks_cp, [np.concatenate(r) for r in rows], [np.concatenate(v) for v in vals])


@pytest.mark.parametrize("force_bin,window_cap", [(-1, 0), (0, 0), (1, 0), (2, 0), (2, 64), (-1, 128), (1, 700),
                                                  (2, 1000)])
def test_forced_bins(force_bin, window_cap):
    note(f"forced_bins force_bin={force_bin} window_cap={window_cap}")
    batch = _ragged_batch()
    got = run_gpu(batch, _opts(force_bin=force_bin, window_cap=window_cap), stats=True)
    ref = oracle.spkadd(batch)
    assert_matches(batch, got, ref, exact_values=True)
    st = got[3]
    if force_bin == 2:
        assert st["n_window_cols"] == batch.n - st["n_empty_cols"]


@pytest.mark.parametrize("m", [100000, 1 << 20])
def test_workgroup_bitmap_and_hash_agree(m):
    """Workgroup units (both workgroup bins, row windows) through the workgroup bitmap
    (windows and columns at most 2^17 rows wide) and through hash tables only give the
    same bits and match the oracle.  With m = 2^20 the sparse window columns have
    windows wider than 2^17 rows, so one launch mixes bitmap and hash windows, and the
    workgroup-bin columns stay on hash tables; with m = 100000 every workgroup unit
    takes the bitmap.  The largest columns hold more entries per window than the
    workgroup's registers (dense windows: every entry adds)."""
    note(f"workgroup bitmap vs hash m={m}")
    sizes = [1200, 2000, 2900, 4000, 5000, 9000, 60000, 200000]
    batch = _ragged_batch(seed=9, k=6, m=m, sizes=sizes)
    ref = oracle.spkadd(batch)
    bm = run_gpu(batch, stats=True)
    hs = run_gpu(batch, _opts(accum_mode=1), stats=True)
    assert bm[3]["n_window_cols"] > 0 and bm[3]["n_wg_cols"] > 0
    assert_matches(batch, bm, ref, exact_values=True)
    for x, y in zip(bm[:3], hs[:3]):
        assert np.array_equal(x, y)
    # forced windows with a small capacity: many narrow windows, dense ones too
    fw = run_gpu(batch, _opts(force_bin=2, window_cap=256), stats=True)
    assert_matches(batch, fw, ref, exact_values=True)
    # fp32 values: within the tolerance
    bf = _ragged_batch(seed=10, k=6, m=m, sizes=sizes, values="f32")
    assert_matches(bf, run_gpu(bf), oracle.spkadd(bf))


def test_workgroup_bitmap_dense_windows():
    """Windows of at most 256 rows holding more entries than the workgroup's registers
    (k = 24 inputs, ~80% of rows present in each): every entry adds into the zeroed
    staging area."""
    note("workgroup bitmap dense windows")
    batch = _ragged_batch(seed=11, k=24, m=5000, sizes=[100000, 60000, 3000])
    u = sum(np.diff(batch.colptr[i]).astype(np.int64) for i in range(batch.k))
    assert u.max() > 5000 * 24 * 0.6
    ref = oracle.spkadd(batch)
    for opts in (_opts(force_bin=2, window_cap=256), _opts(force_bin=2, window_cap=256, accum_mode=1)):
        got = run_gpu(batch, opts, stats=True)
        assert got[3]["n_windows"] > batch.n
        assert_matches(batch, got, ref, exact_values=True)


def test_unsorted_input_in_windows_validated():
    """An input whose rows are not ascending in window columns: SPKADD_FLAG_VALIDATE
    rejects it in spkadd_plan, before any window is built."""
    from paper_2112_10223_amd import binding
    note("unsorted input in windows")
    b = workloads.er(20000, 4, 3, 3000.0, seed=5, values="int32f")  # u ~ 9000 > cap: window columns
    rng = np.random.default_rng(3)
    for j in range(b.n):
        s, e = int(b.colptr[0, j]), int(b.colptr[0, j + 1])
        b.rowidx[0][s:e] = rng.permutation(b.rowidx[0][s:e])
    with pytest.raises(binding.SpkaddError) as err:
        run_gpu(b, _opts(flags=binding.SPKADD_FLAG_VALIDATE))
    assert err.value.status == binding.SPKADD_ERR_INVALID


@pytest.mark.parametrize("seed", range(16))
def test_random_options(seed):
    """Seeded random shapes and option combinations (bins forced or automatic, window
    capacity, wave limit, accumulator choice, bin merging, unsorted output, fp32 and
    fp64), each against the oracle: colptr and rows exact, values exact for integer
    inputs (per column as sets when the output order is free)."""
    from paper_2112_10223_amd import binding
    rng = np.random.default_rng(1000 + seed)
    m = int(rng.choice([1, 7, 300, 5000, 65536, 131072, 300000, 1 << 20]))
    n = int(rng.integers(1, 400))
    k = int(rng.choice([1, 2, 3, 8, 32, 65, 130]))
    d = float(min(m * 0.8, rng.choice([0.5, 4.0, 20.0, 200.0, 2000.0]) / max(1, k // 8)))
    values = str(rng.choice(["int32f", "int64f", "f32", "f64"]))
    kw = {}
    if rng.random() < 0.4:
        kw["force_bin"] = int(rng.choice([0, 1, 2]))
    if rng.random() < 0.4:
        kw["window_cap"] = int(rng.choice([64, 256, 1000, 4096]))
    if rng.random() < 0.3:
        kw["wave_max"] = int(rng.choice([256, 512, 768]))
    kw["accum_mode"] = int(rng.choice([0, 0, 1, 2]))
    kw["wave_merge"] = int(rng.integers(0, 2))
    unsorted = rng.random() < 0.3
    if unsorted:
        kw["flags"] = binding.SPKADD_FLAG_UNSORTED_OUT
    note(f"random options seed={seed} m={m} n={n} k={k} d={d:.2f} values={values} {kw}")
    batch = workloads.er(m, n, k, d, seed=77 + seed, values=values)
    ref = oracle.spkadd(batch)
    got = run_gpu(batch, _opts(**kw))
    if unsorted:
        got = _sorted_columns(got)
    assert_matches(batch, got, ref, exact_values=values.startswith("int"))


def _sorted_columns(got):
    """(colptr, rows, values) with each column's entries ordered by row."""
    colptr, rows, vals = got[:3]
    rows = rows.copy()
    vals = vals.copy()
    for j in range(len(colptr) - 1):
        s, e = int(colptr[j]), int(colptr[j + 1])
        o = np.argsort(rows[s:e], kind="stable")
        rows[s:e] = rows[s:e][o]
        vals[s:e] = vals[s:e][o]
    return colptr, rows, vals


@pytest.mark.parametrize("accum_mode", [0, 1])
def test_unsorted_output(accum_mode):
    """SPKADD_FLAG_UNSORTED_OUT: every column holds the same (row, value) pairs as the
    sorted output, in any order (the hash accumulators skip their sort; the bitmap
    ones stay sorted).  Wave bins, both workgroup bins and row windows, hash tables
    only (accum_mode 1) and the default choice."""
    from paper_2112_10223_amd import binding
    note(f"unsorted output accum_mode={accum_mode}")
    batches = [_ragged_batch(seed=12, k=6, m=1 << 20), workloads.er(300000, 400, 8, 30.0, seed=13, values="int32f")]
    for batch in batches:
        ref = oracle.spkadd(batch)
        for extra in ({}, {"force_bin": 2, "window_cap": 256}):
            got = run_gpu(batch, _opts(flags=binding.SPKADD_FLAG_UNSORTED_OUT, accum_mode=accum_mode, **extra))
            assert_matches(batch, _sorted_columns(got), ref, exact_values=True)
    # the flag changes nothing where the result is sorted anyway
    b = workloads.er(65536, 300, 32, 16.0, seed=14, values="int32f")
    plain = run_gpu(b)
    assert all(np.array_equal(x, y) for x, y in zip(plain, run_gpu(b, _opts(flags=binding.SPKADD_FLAG_UNSORTED_OUT))))


def test_sliding_windows_match_plain():
    """Forcing the sliding hash must reproduce the plain result bit for bit on
    colptr / rowidx (Algorithms 7-8 change only where the table lives)."""
    note("sliding_windows_match_plain")
    batch = workloads.er(50000, 300, 16, 40.0, seed=21, values="int32f")
    plain = run_gpu(batch)
    slid = run_gpu(batch, _opts(force_bin=2, window_cap=96), stats=True)
    assert slid[3]["n_windows"] > batch.n
    assert np.array_equal(plain[0], slid[0]) and np.array_equal(plain[1], slid[1])
    assert np.array_equal(plain[2], slid[2])


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("shape", [(65536, 1500, 32, 16.0), (10000, 800, 8, 40.0), (1, 300, 5, 0.5),
                                   (131072, 300, 16, 30.0), (777, 500, 64, 6.0)])
def test_accum_modes(mode, shape):
    """Hash tables and the bitmap accumulator give the same result (wave bins)."""
    m, n, k, d = shape
    note(f"accum_mode={mode} m={m} n={n} k={k} d={d}")
    for values in ("int32f", "int64f"):
        batch = workloads.er(m, n, k, d, seed=m + k, values=values)
        got = run_gpu(batch, _opts(accum_mode=mode))
        assert_matches(batch, got, oracle.spkadd(batch), exact_values=True)
    batch = workloads.er(m, n, k, d, seed=m + k + 1, values="f32")
    assert_matches(batch, run_gpu(batch, _opts(accum_mode=mode, bitmap_ratio=4.0)), oracle.spkadd(batch))


@pytest.mark.parametrize("merge", [0, 1])
def test_wave_bin_merging(merge):
    """Merged and separate wave bins give the same result.  Column lengths
    Poisson(40 * 8) straddle the E=5 / E=6 edge, so the auto rule merges them."""
    note(f"wave_merge={merge}")
    for values, exact in (("int32f", True), ("f32", False)):
        batch = workloads.er(20000, 600, 8, 40.0, seed=77 + merge, values=values)
        got = run_gpu(batch, _opts(wave_merge=merge))
        assert_matches(batch, got, oracle.spkadd(batch), exact_values=exact)
        for mode in (1, 2):
            got = run_gpu(batch, _opts(wave_merge=merge, accum_mode=mode))
            assert_matches(batch, got, oracle.spkadd(batch), exact_values=exact)


def test_degenerate_hash():
    note("degenerate_hash")
    batch = workloads.er(3000, 200, 5, 30.0, seed=8, values="int32f")
    got = run_gpu(batch, _opts(hash_mode=1))
    ref = oracle.spkadd(batch)
    assert_matches(batch, got, ref, exact_values=True)
    got = run_gpu(batch, _opts(hash_mode=1, force_bin=2, window_cap=64))
    assert_matches(batch, got, ref, exact_values=True)


def test_load_factors_and_wave_limit():
    note("load_factors_and_wave_limit")
    batch = _ragged_batch(seed=9, values="f32")
    ref = oracle.spkadd(batch)
    for kw in [dict(load_factor_sym=0.9, load_factor_num=0.5), dict(load_factor_sym=0.2, load_factor_num=0.25),
               dict(wave_max=64), dict(wave_max=256, window_fill=0.3)]:
        got = run_gpu(batch, _opts(**kw))
        assert_matches(batch, got, ref)


def test_edge_shapes():
    import torch
    note("edge_shapes")
    # k = 1: B is A_1 itself
    b1 = workloads.er(500, 300, 1, 6.0, seed=2, values="f32")
    got = run_gpu(b1)
    assert np.array_equal(got[0], b1.colptr[0].astype(np.int64))
    assert np.array_equal(got[1], b1.rowidx[0]) and np.array_equal(got[2], b1.vals[0])
    # m = 1 (every column has at most one row), n = 1 (one column)
    for m, n, d in [(1, 400, 0.7), (700, 1, 300.0), (2, 3, 1.0)]:
        b = workloads.er(m, n, 7, d, seed=3, values="int32f")
        assert_matches(b, run_gpu(b), oracle.spkadd(b), exact_values=True)
    # all-empty inputs
    b = workloads.er(100, 50, 3, 0.0, seed=4, values="f32")
    got = run_gpu(b)
    assert got[0].sum() == 0 and got[1].shape == (0,)
    # fully dense columns: every input holds every row
    mask = np.ones((64, 5), bool)
    vals = [np.full((64, 5), float(i + 1), np.float32) for i in range(4)]
    b = workloads.from_dense([mask] * 4, vals)
    assert_matches(b, run_gpu(b), oracle.spkadd(b), exact_values=True)
    # n = 0 and m = 0
    from paper_2112_10223_amd import binding
    e = [torch.zeros(1, dtype=torch.int32, device="cuda:0")]
    plan = binding.spkadd_plan(10, 0, e, [None], binding.SPKADD_F32)
    cp = torch.empty(1, dtype=torch.int32, device="cuda:0")
    assert binding.spkadd_symbolic(plan, cp) == 0 and int(cp.item()) == 0
    plan.free()
    e = [torch.zeros(4, dtype=torch.int32, device="cuda:0")] * 2
    plan = binding.spkadd_plan(0, 3, e, [None, None], binding.SPKADD_F32)
    cp = torch.empty(4, dtype=torch.int32, device="cuda:0")
    assert binding.spkadd_symbolic(plan, cp) == 0 and cp.cpu().tolist() == [0, 0, 0, 0]
    binding.spkadd_numeric(plan, [None, None], None, None)
    plan.free()


@pytest.mark.parametrize("n", [16383, 16384, 65536, 100003, 131072, 131073, 200000])
def test_scan_lengths(n):
    """colptr(B) over column counts of every length around the scan's tile and path
    limits (one workgroup up to 2^17 columns, tile sums beyond)."""
    note(f"scan_lengths n={n}")
    b = workloads.er(40, n, 2, 0.6, seed=n % 9973, values="int32f")
    assert_matches(b, run_gpu(b), oracle.spkadd(b), exact_values=True)


def test_same_row_everywhere_and_large_k():
    note("same_row_everywhere_and_large_k")
    k, m, n = 200, 1000, 40
    cp = np.tile(np.arange(n + 1, dtype=np.int32), (k, 1))
    rows = [np.full(n, 7, np.int32) for _ in range(k)]
    vals = [np.full(n, 1.0, np.float32) for _ in range(k)]
    b = workloads.CSCBatch(m, n, cp, rows, vals)
    got = run_gpu(b)
    assert np.array_equal(got[0], np.arange(n + 1)) and (got[1] == 7).all() and (got[2] == k).all()
    for fb in (1, 2):
        got = run_gpu(b, _opts(force_bin=fb, window_cap=64))
        assert np.array_equal(got[0], np.arange(n + 1)) and (got[1] == 7).all() and (got[2] == k).all()


def _csc_from_columns(m, cols_per_input, dtype=np.float32, seed=0):
    """A CSCBatch from per-input lists of per-column row arrays (sorted, unique), with
    small integer values (exact in any summation order)."""
    rng = np.random.default_rng(seed)
    k, n = len(cols_per_input), len(cols_per_input[0])
    colptr = np.zeros((k, n + 1), np.int32)
    rows, vals = [], []
    for i, cols in enumerate(cols_per_input):
        colptr[i, 1:] = np.cumsum([len(c) for c in cols])
        r = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
        rows.append(r)
        vals.append(rng.integers(-3, 4, size=r.size).astype(dtype))
    return workloads.CSCBatch(m, n, colptr, rows, vals)


def test_windows_long_runs_and_skewed_runs():
    """Window columns whose inputs hold long runs of rows: uniform ones keep equal row
    ranges and the ordered pass per input, skewed ones (rows crowding the low indices)
    take quantile windows and the chunked pass, and columns of shorter runs the chunked
    pass too; all in one launch, against the oracle."""
    note("windows_long_runs_and_skewed_runs")
    rng = np.random.default_rng(31)
    m, k = 1 << 20, 4
    cols = [[] for _ in range(k)]
    for j in range(24):
        for i in range(k):
            if j < 8:  # uniform, 2048 rows per input
                r = rng.choice(m, size=2048, replace=False)
            elif j < 16:  # skewed, 2048 rows per input
                r = np.unique(np.minimum((rng.pareto(1.2, size=4000) * 200).astype(np.int64), m - 1))[:2048]
            else:  # shorter runs (1 000 rows per input)
                r = rng.choice(m, size=1000, replace=False)
            cols[i].append(np.sort(r))
    b = _csc_from_columns(m, cols, seed=32)
    got = run_gpu(b, stats=True)
    assert got[3]["n_window_cols"] == 24 and got[3]["n_windows"] > 24
    assert_matches(b, got, oracle.spkadd(b), exact_values=True)


def test_windows_more_inputs_than_the_segment_table():
    """Window columns of sorted inputs with more inputs than the boundary pass's segment
    table (one wavefront per input walks its rows), against the oracle."""
    note("windows_more_inputs_than_the_segment_table")
    rng = np.random.default_rng(33)
    m, k, n = 40000, 1100, 5
    cols = [[np.sort(rng.choice(m, size=int(rng.integers(0, 7)), replace=False)) for _ in range(n)]
            for _ in range(k)]
    b = _csc_from_columns(m, cols, seed=34)
    got = run_gpu(b, _opts(force_bin=2, window_cap=512), stats=True)
    assert got[3]["n_windows"] > n
    assert_matches(b, got, oracle.spkadd(b), exact_values=True)


def test_permutation_invariance():
    note("permutation_invariance")
    batch = workloads.er(5000, 500, 12, 25.0, seed=17, values="int32f")
    base = run_gpu(batch)
    perm = np.random.default_rng(3).permutation(batch.k)
    other = run_gpu(batch.select(perm))
    for x, y in zip(base, other):
        assert np.array_equal(x, y)


def test_numeric_rerun_new_values():
    """spkadd_numeric may run again with new values on the same pattern."""
    import torch
    from paper_2112_10223_amd import binding
    from tests.gpu_util import to_device
    note("numeric_rerun_new_values")
    b1 = workloads.er(4000, 300, 6, 30.0, seed=31, values="int32f")
    b2 = workloads.CSCBatch(b1.m, b1.n, b1.colptr, b1.rowidx, [(v * 2 + 1).astype(np.float32) for v in b1.vals])
    cps, ris, vas1 = to_device(b1)
    _, _, vas2 = to_device(b2)
    plan = binding.spkadd_plan(b1.m, b1.n, cps, ris, binding.SPKADD_F32)
    cp = torch.empty(b1.n + 1, dtype=torch.int32, device="cuda:0")
    nnz = binding.spkadd_symbolic(plan, cp)
    r = torch.empty(nnz, dtype=torch.int32, device="cuda:0")
    v = torch.empty(nnz, dtype=torch.float32, device="cuda:0")
    for b, vas in ((b1, vas1), (b2, vas2), (b1, vas1)):
        binding.spkadd_numeric(plan, vas, r, v)
        torch.cuda.synchronize()
        ref = oracle.spkadd(b)
        assert_matches(b, (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), ref,
                       exact_values=True)
    plan.free()


def test_state_and_validation_errors():
    import torch
    from paper_2112_10223_amd import binding
    from tests.gpu_util import to_device
    note("state_and_validation_errors")
    b = workloads.er(100, 20, 2, 5.0, seed=1)
    cps, ris, vas = to_device(b)
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32)
    with pytest.raises(binding.SpkaddError) as ei:
        binding.spkadd_numeric(plan, vas, torch.empty(1, dtype=torch.int32, device="cuda:0"),
                               torch.empty(1, device="cuda:0"))
    assert ei.value.status == binding.SPKADD_ERR_STATE
    plan.free()
    # an unsorted column is rejected when validation is on
    bad = [r.clone() for r in ris]
    j = int(np.argmax(np.diff(b.colptr[0])))
    s = int(b.colptr[0, j])
    bad[0][s], bad[0][s + 1] = ris[0][s + 1].item(), ris[0][s].item()
    with pytest.raises(binding.SpkaddError) as ei:
        binding.spkadd_plan(b.m, b.n, cps, bad, binding.SPKADD_F32, _opts(flags=binding.SPKADD_FLAG_VALIDATE))
    assert ei.value.status == binding.SPKADD_ERR_INVALID
    # row out of range
    bad = [r.clone() for r in ris]
    bad[1][0] = b.m
    with pytest.raises(binding.SpkaddError):
        binding.spkadd_plan(b.m, b.n, cps, bad, binding.SPKADD_F32, _opts(flags=binding.SPKADD_FLAG_VALIDATE))
    # valid input passes validation
    binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, _opts(flags=binding.SPKADD_FLAG_VALIDATE)).free()


def _hstack(batches):
    """The columns of several batches (same m and k) side by side."""
    k, m, n = batches[0].k, batches[0].m, sum(x.n for x in batches)
    colptr = np.zeros((k, n + 1), dtype=np.int32)
    rows, vals = [], []
    for i in range(k):
        off = pos = 0
        for x in batches:
            colptr[i, pos:pos + x.n] = x.colptr[i][:-1] + off
            pos += x.n
            off += int(x.colptr[i][-1])
        colptr[i, n] = off
        rows.append(np.concatenate([x.rowidx[i] for x in batches]))
        vals.append(np.concatenate([x.vals[i] for x in batches]))
    return workloads.CSCBatch(m, n, colptr, rows, vals)


def test_plan_without_waiting():
    """spkadd_plan returns before the device has binned the columns; the symbolic pass
    takes the wave bins in one launch and then waits for the plan.  A plan freed or
    queried before its symbolic pass, and a symbolic pass on another stream than the
    plan, still give the oracle's result."""
    import torch
    from paper_2112_10223_amd import binding
    from tests.gpu_util import to_device
    note("plan_without_waiting")
    # every wave bin, workgroup columns and windowed columns in one input
    b = _hstack([workloads.er(6000, 40, 24, d, seed=s, values="int32f") for s, d in
                 enumerate([0.5, 2.0, 3.5, 6.0, 9.0, 12.0, 17.0, 22.0, 30.0, 40.0, 80.0, 200.0])])
    ref = oracle.spkadd(b)
    cps, ris, vas = to_device(b)
    opts = _opts(window_cap=2048)  # workgroup columns up to 2048 entries, windows above
    # freed before its symbolic pass
    binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, opts).free()
    # queried before its symbolic pass
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, opts)
    st = binding.spkadd_get_stats(plan)
    assert st["nnz_out"] == -1 and st["n_wave_cols"] > 0 and st["n_wg_cols"] > 0 and st["n_window_cols"] > 0
    cp = torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0")
    nnz = binding.spkadd_symbolic(plan, cp)
    r = torch.empty(nnz, dtype=torch.int32, device="cuda:0")
    v = torch.empty(nnz, dtype=torch.float32, device="cuda:0")
    binding.spkadd_numeric(plan, vas, r, v)
    torch.cuda.synchronize()
    assert_matches(b, (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), ref, exact_values=True)
    plan.free()
    # plan on one stream, the passes on another
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, opts, stream=s1)
    cp2 = torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0")
    with torch.cuda.stream(s2):
        nnz2 = binding.spkadd_symbolic(plan, cp2, stream=s2)
        r2 = torch.empty(nnz2, dtype=torch.int32, device="cuda:0")
        v2 = torch.empty(nnz2, dtype=torch.float32, device="cuda:0")
        binding.spkadd_numeric(plan, vas, r2, v2, stream=s2)
    s2.synchronize()
    assert_matches(b, (cp2.cpu().numpy().astype(np.int64), r2.cpu().numpy(), v2.cpu().numpy()), ref,
                   exact_values=True)
    plan.free()


def test_trace_records_kernels():
    from paper_2112_10223_amd import binding
    import torch
    from tests.gpu_util import to_device
    note("trace_records_kernels")
    b = workloads.config1()
    cps, ris, vas = to_device(b)
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32, _opts(flags=binding.SPKADD_FLAG_TRACE))
    cp = torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0")
    nnz = binding.spkadd_symbolic(plan, cp)
    r = torch.empty(nnz, dtype=torch.int32, device="cuda:0")
    v = torch.empty(nnz, dtype=torch.float32, device="cuda:0")
    binding.spkadd_numeric(plan, vas, r, v)
    tr = binding.spkadd_trace(plan)
    names = [t[0] for t in tr]
    assert "bounds" in names and any(x.startswith("sym_") for x in names) and any(x.startswith("num_") for x in names)
    assert all(ms >= 0 for _, ms in tr)
    plan.free()
    # numeric-only tracing records nothing before spkadd_numeric, then its launches
    plan = binding.spkadd_plan(b.m, b.n, cps, ris, binding.SPKADD_F32,
                               _opts(flags=binding.SPKADD_FLAG_TRACE_NUMERIC))
    binding.spkadd_symbolic(plan, cp)
    assert binding.spkadd_trace(plan) == []
    binding.spkadd_numeric(plan, vas, r, v)
    names = [t[0] for t in binding.spkadd_trace(plan)]
    assert any(x.startswith("num_") for x in names)
    assert all(x.startswith(("num_", "put_ptrs_num")) for x in names)
    # a NULL value pointer of a non-empty input is rejected on the host
    import ctypes
    nulls = (ctypes.c_void_p * b.k)(*([None] * b.k))
    st = binding.lib().spkadd_numeric(plan.handle, ctypes.cast(nulls, ctypes.c_void_p), r.data_ptr(), v.data_ptr(),
                                      binding._stream_ptr(None))
    assert st == binding.SPKADD_ERR_INVALID
    plan.free()


# ---- full-size workloads: every output column against the column-chunked oracle ----
def _full_check(batch, got, exact=False):
    """got = (colptr, rowidx, values) on the device: the invariants on the device, then
    every column against the oracle on the host's cores."""
    from tests.gpu_util import check_properties_device, oracle_check_all
    colptr = check_properties_device(batch, got[0], got[1])
    rows = got[1].cpu().numpy()
    vals = got[2].cpu().numpy()
    n_checked = oracle_check_all(batch, colptr, rows, vals, exact=exact)
    print(f"checked all {batch.n} columns, {n_checked} entries", flush=True)


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("values", ["f32", "f64", "int32f"])
def test_config2_full(values):
    note(f"config2 full values={values}")
    batch = workloads.config2(values=values)
    got = run_gpu(batch, stats=True, device_out=True)
    assert got[3]["n_wave_cols"] > 0
    _full_check(batch, got, exact=values.startswith("int"))


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_config3_full():
    note("config3 full (R-MAT scale 20, k=64)")
    batch = workloads.config3()
    got = run_gpu(batch, stats=True, device_out=True)
    st = got[3]
    print("config3 stats", st, flush=True)
    assert st["n_window_cols"] > 0
    _full_check(batch, got)


@pytest.mark.slow
@pytest.mark.timeout(900)
@pytest.mark.parametrize("window", [0, 524288])
def test_config4_full(window):
    note(f"config4 full window={window}")
    batch = workloads.config4(window=window)
    got = run_gpu(batch, stats=True, device_out=True)
    assert got[3]["n_window_cols"] == batch.n
    _full_check(batch, got)
