"""CPU tests of the C ABI: the library loads, exports every declared entry point,
and rejects bad arguments on the host before any device work."""
import ctypes

import pytest

from paper_2112_10223_amd import binding


@pytest.fixture(scope="module")
def L():
    return binding.lib()


def test_exports_every_declared_symbol(L):
    names = binding.declared_functions()
    assert "spkadd_plan" in names and "spkadd_symbolic" in names and "spkadd_numeric" in names
    assert "spkadd_free" in names
    for name in names:
        assert hasattr(L, name), name


def test_opts_default(L):
    o = binding.Opts()
    o.force_bin = 5
    L.spkadd_opts_default(ctypes.byref(o))
    assert o.force_bin == -1 and o.flags == 0 and o.window_cap == 0


def _plan(L, m=4, n=3, k=1, colptr=True, rowidx=True, dtype=0, opts=None, out=True):
    h = ctypes.c_void_p()
    fake = (ctypes.c_void_p * max(k, 1))(*([0x1000] * max(k, 1)))
    return L.spkadd_plan(ctypes.byref(h) if out else None, m, n, k, fake if colptr else None,
                         fake if rowidx else None, dtype, ctypes.byref(opts) if opts else None, None)


@pytest.mark.parametrize("kw", [dict(out=False), dict(k=0), dict(k=-3), dict(m=-1), dict(n=-1),
                                dict(m=2 ** 31 - 1), dict(colptr=False), dict(rowidx=False), dict(dtype=7)])
def test_plan_rejects_bad_arguments(L, kw):
    assert _plan(L, **kw) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_last_error()


@pytest.mark.parametrize("field,value", [("force_bin", 3), ("force_bin", -2), ("hash_mode", 2), ("wave_max", 2048),
                                         ("window_cap", -1), ("window_cap", 1 << 20), ("load_factor_sym", 0.99),
                                         ("load_factor_num", 0.75), ("window_fill", 1.5)])
def test_plan_rejects_bad_options(L, field, value):
    o = binding.make_opts()
    setattr(o, field, value)
    assert _plan(L, opts=o) == binding.SPKADD_ERR_INVALID


def test_plan_null_colptr_entry(L):
    h = ctypes.c_void_p()
    cps = (ctypes.c_void_p * 2)(0x1000, 0)
    assert L.spkadd_plan(ctypes.byref(h), 4, 3, 2, cps, cps, 0, None, None) == binding.SPKADD_ERR_INVALID


def test_calls_on_null_plan(L):
    n = ctypes.c_int64()
    assert L.spkadd_symbolic(None, None, ctypes.byref(n), None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_numeric(None, None, None, None, None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_free(None) == binding.SPKADD_OK
    assert L.spkadd_trace_count(None) == 0
    st = binding.Stats()
    assert L.spkadd_get_stats(None, ctypes.byref(st)) == binding.SPKADD_ERR_INVALID


def test_batch_argument_checks_without_gpu():
    """Argument checks of the batch API that return before any device call."""
    import ctypes
    from paper_2112_10223_amd import binding
    L = binding.lib()
    h = ctypes.c_void_p()
    assert L.spkadd_batch_create(ctypes.byref(h), binding.SPKADD_F32, 0, 10, 10, None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_batch_create(ctypes.byref(h), 7, 4, 10, 10, None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_batch_create(None, binding.SPKADD_F32, 4, 10, 10, None) == binding.SPKADD_ERR_INVALID
    o = binding.make_opts(accum_mode=5)
    assert L.spkadd_batch_create(ctypes.byref(h), binding.SPKADD_F32, 4, 10, 10, ctypes.byref(o)) == \
        binding.SPKADD_ERR_INVALID
    assert L.spkadd_batch_run(None, None, 1, 0, None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_batch_results(None, None, None) == binding.SPKADD_ERR_INVALID
    assert L.spkadd_batch_destroy(None) == binding.SPKADD_OK
    assert b"NULL" in L.spkadd_last_error() or len(L.spkadd_last_error()) > 0


def test_heap_baseline_argument_errors(L):
    """spkadd_heap_add rejects bad arguments on the host, before any device work."""
    import ctypes
    from paper_2112_10223_amd import baselines, binding
    f = baselines._heap_fn()
    nnz = ctypes.c_int64(0)
    arr = (ctypes.c_void_p * 1)(ctypes.c_void_p(0x1000))
    out = ctypes.c_void_p(0x2000)
    assert f(10, 10, 0, arr, arr, arr, 0, out, out, out, 0, ctypes.byref(nnz), None) == binding.SPKADD_ERR_INVALID
    assert f(10, 10, baselines.HEAP_MAX_K + 1, arr, arr, arr, 0, out, out, out, 0, ctypes.byref(nnz),
             None) == binding.SPKADD_ERR_INVALID
    assert f(-1, 10, 1, arr, arr, arr, 0, out, out, out, 0, ctypes.byref(nnz), None) == binding.SPKADD_ERR_INVALID
    assert f(10, 10, 1, arr, arr, arr, 5, out, out, out, 0, ctypes.byref(nnz), None) == binding.SPKADD_ERR_INVALID
    assert f(10, 10, 1, arr, arr, arr, 0, out, None, None, 4, ctypes.byref(nnz), None) == binding.SPKADD_ERR_INVALID
