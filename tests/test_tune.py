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
