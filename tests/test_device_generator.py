"""The device copy of the ER generator (workloads/gen_device.hip) draws the same
matrices as the host generator, entry for entry: column pointers, rows and values."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("values", ["f32", "int32f", "f64", "int64f"])
def test_device_equals_host(values):
    import torch
    specs = workloads.request_specs(12, seed=31337, max_nnz=1 << 21)
    # plus the densest shapes of the distribution: density 1e-2 over 65536 rows
    # (Poisson mean 655), a short matrix where columns can fill, and k = 64
    specs.append(workloads.RequestSpec(1, 3, 65536, 300, np.array([1e-2, 5e-3, 1e-4]), 99))
    specs.append(workloads.RequestSpec(2, 4, 256, 2000, np.array([1e-2, 1e-2, 2e-3, 1e-4]), 99))
    specs.append(workloads.RequestSpec(3, 64, 3000, 500, np.full(64, 3e-3), 99))
    for s in specs:
        note(f"device generator k={s.k} m={s.m} n={s.n} values={values}")
        host = workloads.request_from_spec(s, values)
        cps, ris, vas = workloads.device_request(s, values)
        torch.cuda.synchronize()
        for i in range(s.k):
            assert np.array_equal(cps[i].cpu().numpy(), host.colptr[i]), (s, i)
            assert np.array_equal(ris[i].cpu().numpy(), host.rowidx[i]), (s, i)
            assert np.array_equal(vas[i].cpu().numpy().view(np.uint8), host.vals[i].view(np.uint8)), (s, i)
