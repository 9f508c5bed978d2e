"""Host checks of the comparison the GPU parity tests use (tests/gpu_util.py): values
just inside max(k, t) * u * sum|a| of the oracle pass, values just outside fail, for
fp32 (float64 fast pass plus exact recheck) and fp64 (exact check)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, value_bound


@pytest.mark.parametrize("values", ["f32", "f64"])
def test_bound_edges(values):
    b = workloads.er(300, 200, 9, 20.0, seed=3, values=values)
    ref = oracle.spkadd(b)
    dt = b.vals[0].dtype.type
    bound = value_bound(b, ref)
    exact = ref.val.astype(dt)
    got = (ref.colptr, ref.rowidx, exact)
    assert_matches(b, got, ref)
    # move every 37th value as far as the bound allows (inside), then one entry just past it
    inside = exact.copy()
    for i in range(0, len(inside), 37):
        target = ref.val[i] + bound[i] * np.longdouble(0.999)
        v = dt(target)
        while np.abs(np.longdouble(v) - ref.val[i]) > bound[i]:
            v = np.nextafter(v, dt(ref.val[i]))
        inside[i] = v
    assert_matches(b, (ref.colptr, ref.rowidx, inside), ref)
    i = int(np.argmax(ref.abs))
    outside = exact.copy()
    v = dt(ref.val[i] + bound[i] * np.longdouble(1.001))
    while np.abs(np.longdouble(v) - ref.val[i]) <= bound[i]:
        v = np.nextafter(v, dt(np.inf))
    outside[i] = v
    with pytest.raises(AssertionError):
        assert_matches(b, (ref.colptr, ref.rowidx, outside), ref)
