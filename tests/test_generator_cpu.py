"""Host checks of the seeded generators' portable Poisson sampler (the one the device
generator shares): its counts follow Poisson(d) and, up to d = 500 where both invert
the CDF, agree with the libm-based sampler column by column except where a uniform
falls within rounding of a CDF step."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("d", [0.5, 16.0, 300.0, 655.36])
def test_portable_counts_match_libm_sampler(d):
    m, n = 65536, 4000
    a = workloads.er(m, n, 1, d, seed=77, values="int32f", portable=True)
    b = workloads.er(m, n, 1, d, seed=77, values="int32f")
    ca, cb = np.diff(a.colptr[0]), np.diff(b.colptr[0])
    if d <= 500:  # (above 500 the libm-based sampler switches to a normal approximation)
        assert (ca == cb).mean() >= 0.999
    # Poisson(d): mean d, variance d (n columns: the sample mean within 6 standard errors)
    assert abs(ca.mean() - d) < 6 * np.sqrt(d / n)
    assert 0.85 * d < ca.var() < 1.15 * d
    # the same columns drawn the same way: where the counts agree, the rows agree too
    same = np.nonzero(ca == cb)[0][:50]
    for j in same:
        assert np.array_equal(a.column(0, j)[0], b.column(0, j)[0])


def test_request_specs_are_the_stream():
    """request_stream is request_from_spec over request_specs; the filter keeps only
    requests whose expected input entries are within the bound."""
    specs = workloads.request_specs(6, max_nnz=1 << 18)
    reqs = workloads.request_stream(6, max_nnz=1 << 18, values="int32f")
    for s, r in zip(specs, reqs):
        assert s.expected_nnz <= 1 << 18
        assert (r.k, r.m, r.n) == (s.k, s.m, s.n)
        again = workloads.request_from_spec(s, "int32f")
        assert np.array_equal(again.colptr, r.colptr)
        assert all(np.array_equal(x, y) for x, y in zip(again.rowidx, r.rowidx))
    ks = [s.k for s in workloads.request_specs(400)]
    assert min(ks) >= 2 and max(ks) <= 64
