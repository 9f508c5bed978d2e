"""GPU tests of the autotuner (include/spkadd_tune.h): it measures settings on the
caller's inputs, every setting keeps colptr(B), the chosen one is cached under the
inputs' shape class and gives results that match the CPU oracle."""
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
    binding.tune_clear()
    yield
    binding.tune_clear()


def _tune(batch, **kw):
    from paper_2112_10223_amd import binding
    cps, ris, vas = to_device(batch)
    dtype = binding.SPKADD_F64 if batch.vals[0].dtype == np.float64 else binding.SPKADD_F32
    return binding.tune(batch.m, cps, ris, vas, dtype, **kw)


@pytest.mark.parametrize("case", ["er", "rmat", "windows"])
def test_tune_matches_oracle(case):
    import torch
    from paper_2112_10223_amd import binding
    note(f"tune {case}")
    if case == "er":
        b = workloads.er(8192, 4096, 16, 24.0, seed=41, values="int32f")
    elif case == "rmat":
        b = workloads.rmat(12, 8, 8, seed=42, values="int32f")
    else:  # columns longer than a workgroup table: the row-window parameters are searched
        b = workloads.er(400000, 12, 6, 1500.0, seed=43, values="int32f")
    best, rep, trials = _tune(b, reps=2)
    assert rep["trials"] == len(trials) >= 10 and rep["failed"] == 0
    assert all(t["status"] == 0 and t["same_colptr"] and t["ms"] > 0 for t in trials)
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    assert min(t["ms"] for t in trials) <= rep["best_ms"] + 1e-9
    # the window parameters are searched when some column is too long for a wavefront
    _, _, _, st = run_gpu(b, stats=True)
    long_cols = st["n_wg_cols"] + st["n_window_cols"] > 0
    assert long_cols == (case != "er")
    if case == "windows":
        assert st["n_window_cols"] > 0
    caps = {t["opts"]["window_cap"] for t in trials}
    assert (len(caps) > 1) == long_cols
    # cached under the inputs' shape class, with the same rule as the host-side key
    key = binding.tune_key(b.m, b.n, b.k, b.nnz_in, binding.SPKADD_F32)
    props = torch.cuda.get_device_properties(0)
    host = binding.tune_key(b.m, b.n, b.k, b.nnz_in, binding.SPKADD_F32, arch=key.arch.decode(),
                            cus=props.multi_processor_count)
    assert [getattr(key, f) for f, _ in binding.TuneKey._fields_] == \
        [getattr(host, f) for f, _ in binding.TuneKey._fields_]
    assert rep["key"]["u_log2"] == key.u_log2
    cached = binding.tune_lookup(key)
    assert cached is not None
    for f in binding.TUNED_FIELDS:
        assert getattr(cached, f) == getattr(best, f)
    got = run_gpu(b, opts=cached)
    assert_matches(b, got, oracle.spkadd(b), exact_values=True)


def test_tune_errors():
    from paper_2112_10223_amd import binding
    note("tune errors")
    b = workloads.er(100, 10, 2, 3.0, seed=1, values="int32f")
    with pytest.raises(binding.SpkaddError):
        _tune(b, reps=0)
    bad = binding.make_opts(wave_max=5000)
    with pytest.raises(binding.SpkaddError) as e:
        _tune(b, base=bad, reps=1)
    assert e.value.status == binding.SPKADD_ERR_INVALID


def _request_dicts(batches, values_dtype):
    import torch
    reqs = []
    for b in batches:
        cps, ris, vas = to_device(b)
        cap = max(b.nnz_in, 1)
        reqs.append(dict(m=b.m, colptrs=cps, rowidxs=ris, values=vas,
                         colptr_c=torch.empty(b.n + 1, dtype=torch.int32, device="cuda:0"),
                         rowidx_c=torch.empty(cap, dtype=torch.int32, device="cuda:0"),
                         values_c=torch.empty(cap, dtype=values_dtype, device="cuda:0"), cap_c=cap))
    return reqs


def test_batch_tuner_matches_oracle():
    """The batched-path tuner on a sample of the request distribution (k up to 64, with
    requests too long for a batched run): every trial keeps each request's nnz(B), the
    best setting is cached under the sample's key (kind 1), and batched runs with it
    (the too-large requests through the one-request path) match the oracle."""
    import torch
    from paper_2112_10223_amd import binding
    note("batch tuner")
    batches = workloads.request_stream(36, seed=93, max_nnz=1 << 18, values="int32f")
    batches += [workloads.er(3000, 40, 64, 10.0, seed=94, values="int32f"),     # k = 64
                workloads.er(20000, 10, 40, 100.0, seed=95, values="int32f")]   # u ~ 4000: workgroup or too large
    reqs = _request_dicts(batches, torch.float32)
    best, rep, trials = binding.tune_batch(reqs, binding.SPKADD_F32, reps=1)
    assert rep["trials"] == len(trials) >= 8 and rep["failed"] == 0, rep
    assert all(t["status"] == 0 and t["same_nnz"] and t["ms"] > 0 for t in trials)
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    assert {t["opts"]["batch_run_size"] for t in trials} >= {8, 16, 32}
    assert {t["opts"]["batch_wave_max"] for t in trials} >= {512, 768}
    key = binding.tune_key_batch(len(batches), sum(b.m for b in batches), sum(b.n for b in batches),
                                 sum(b.k for b in batches), sum(b.nnz_in for b in batches))
    assert key.kind == 1 and rep["key"]["kind"] == 1 and rep["key"]["u_log2"] == key.u_log2
    cached = binding.tune_lookup(key)
    assert cached is not None
    for f in binding.BATCH_TUNED_FIELDS:
        assert getattr(cached, f) == getattr(best, f)
    # every request with the tuned setting, against the oracle
    R = best.batch_run_size
    bt = binding.Batch(binding.SPKADD_F32, R, sum(b.n for b in batches), sum(b.k for b in batches), cached)
    for g in range(0, len(reqs), R):
        grp = reqs[g:g + R]
        for q in grp:
            q["colptr_c"].fill_(-7)
        bt.run(grp, use_graph=True)
        nnz, st = bt.results()
        for b, q, z, s in zip(batches[g:g + R], grp, nnz, st):
            ref = oracle.spkadd(b)
            if s == binding.SPKADD_REQ_TOO_LARGE:
                cp, r, v = binding.spkadd(b.m, q["colptrs"], q["rowidxs"], q["values"], cached)
                got = (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy())
            else:
                assert s == binding.SPKADD_REQ_OK and z == ref.nnz
                got = (q["colptr_c"].cpu().numpy().astype(np.int64), q["rowidx_c"][:z].cpu().numpy(),
                       q["values_c"][:z].cpu().numpy())
            assert_matches(b, got, ref, exact_values=True)
    bt.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("kw", [dict(batch_wave_max=512, batch_wg_max=2048, batch_wg_threads=512),
                                dict(batch_wave_max=256, batch_wg_max=256), dict(batch_wg_threads=512)])
def test_batch_cutoffs_and_workgroup_size(kw):
    """Lower wavefront and workgroup cutoffs and 512-thread workgroups: columns move
    between the slots (and to the one-request path), results stay exact."""
    import torch
    from paper_2112_10223_amd import binding
    note(f"batch cutoffs {kw}")
    batches = workloads.request_stream(20, seed=96, max_nnz=1 << 18, values="int32f")
    batches.append(workloads.er(6000, 30, 8, 300.0, seed=97, values="int32f"))  # u ~ 2400
    reqs = _request_dicts(batches, torch.float32)
    opts = binding.make_opts(**kw)
    bt = binding.Batch(binding.SPKADD_F32, len(reqs), sum(b.n for b in batches), sum(b.k for b in batches), opts)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    wg_max = kw.get("batch_wg_max", 4096)
    for b, q, z, s in zip(batches, reqs, nnz, st):
        u = sum(np.diff(b.colptr[i]).astype(np.int64) for i in range(b.k))
        too_large = bool((u > wg_max).any() or (b.m > (1 << 17) and (u > kw.get("batch_wave_max", 1024)).any()))
        assert (s == binding.SPKADD_REQ_TOO_LARGE) == too_large
        if too_large:
            continue
        ref = oracle.spkadd(b)
        got = (q["colptr_c"].cpu().numpy().astype(np.int64), q["rowidx_c"][:z].cpu().numpy(),
               q["values_c"][:z].cpu().numpy())
        assert_matches(b, got, ref, exact_values=True)
    bt.close()
    with pytest.raises(binding.SpkaddError):
        binding.Batch(binding.SPKADD_F32, 4, 100, 16, binding.make_opts(batch_wave_max=2048))
    with pytest.raises(binding.SpkaddError):
        binding.Batch(binding.SPKADD_F32, 4, 100, 16, binding.make_opts(batch_wave_max=1024, batch_wg_max=512))
    with pytest.raises(binding.SpkaddError):
        binding.Batch(binding.SPKADD_F32, 4, 100, 16, binding.make_opts(batch_wg_threads=384))
    torch.cuda.synchronize()
