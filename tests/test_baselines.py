"""GPU parity of the comparison baselines (include/spkadd_baselines.h,
paper_2112_10223_amd/baselines.py) against the CPU oracle: the k-way heap merge of
Algorithm 3 and the 2-way tree of Section II-B must give B exactly as the oracle does
(colptr and rowidx bit-exact; values bit-exact for integer-valued inputs, else within
k * u * sum|a|)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, note, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_10223_amd import binding
    binding.lib()


CASES = [  # m, n, k, d, values
    (300, 120, 5, 6.0, "int32f"),
    (65536, 700, 32, 16.0, "f32"),
    (2000, 400, 3, 0.0, "f32"),        # every column empty
    (5000, 64, 128, 2.0, "int32f"),    # the heap's largest k
    (40, 90, 1, 5.0, "f64"),           # k = 1
    (20000, 50, 9, 900.0, "f64"),      # long columns
]


@pytest.mark.parametrize("algo", ["heap", "tree"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_baseline_matches_oracle(algo, case):
    import torch
    from paper_2112_10223_amd import baselines
    m, n, k, d, values = CASES[case]
    note(f"baseline {algo} m={m} n={n} k={k} d={d} values={values}")
    b = workloads.er(m, n, k, d, seed=400 + case, values=values)
    cps, ris, vas = to_device(b)
    fn = baselines.heap_add if algo == "heap" else baselines.tree_add
    c, r, v = fn(m, cps, ris, vas)
    torch.cuda.synchronize()
    got = (c.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy())
    assert_matches(b, got, oracle.spkadd(b), exact_values=values.startswith("int"))


def test_rmat_skewed_columns():
    import torch
    from paper_2112_10223_amd import baselines
    note("baseline heap+tree rmat")
    b = workloads.rmat(12, 8, 16, seed=77, values="int32f")
    cps, ris, vas = to_device(b)
    ref = oracle.spkadd(b)
    for fn in (baselines.heap_add, baselines.tree_add):
        c, r, v = fn(b.m, cps, ris, vas)
        torch.cuda.synchronize()
        assert_matches(b, (c.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), ref,
                       exact_values=True)
