"""Host-side checks of the measurement harness (no device): the committed rocprofv3
traffic summary belongs to the current kernel sources and counts the same algorithmic
bytes as bench.py's formula, the column-to-kernel mapping used for the roofline
matches the library's binning on the headline workload, and --gpus above 1 is refused."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_num_wave_e10_config2.md")


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_traffic_summary_is_current(bench):
    from paper_2112_10223_amd import profiling
    rec = profiling.read_traffic_summary(TRAFFIC)
    for key in ("kernel", "fetch_kib_per_dispatch", "write_kib_per_dispatch", "traffic_bytes_per_launch",
                "alg_bytes_per_launch", "source_sha"):
        assert key in rec, key
    # taken on the sources the library is built from (a kernel change needs new counters)
    assert rec["source_sha"] == bench.source_sha()
    assert 1.0 <= float(rec["traffic_over_alg"]) < 1.5
    assert bench.measured_traffic("num_wave_e10", "config2") == int(rec["traffic_bytes_per_launch"])


def test_algorithmic_bytes_of_the_dominant_kernel(bench):
    """(4 + v)(u_j + c_j) + 4k + 4 summed over the columns of num_wave_e10 on the k=32
    ER workload, with c_j from the oracle, equals the committed figure."""
    import oracle
    import workloads
    from paper_2112_10223_amd import profiling
    batch = workloads.config2("f32")
    u = sum(np.diff(batch.colptr[i]).astype(np.int64) for i in range(batch.k))
    names = bench.kernel_of_column(u, cap=3072)
    assert set(names) == {"num_wave_e10"}  # Poisson(512) columns: the merged E=8/10 bin
    ref = oracle.spkadd(batch)
    c = np.diff(ref.colptr)
    alg = int(((4 + 4) * (u + c) + 4 * batch.k + 4).sum())
    assert alg == int(profiling.read_traffic_summary(TRAFFIC)["alg_bytes_per_launch"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_reversed_columns(bench):
    """--unsorted-in input: every column's entries in reverse order, nothing else moved."""
    import workloads
    b = workloads.er(50, 7, 3, 4.0, seed=3, values="int32f")
    r = bench.reversed_columns(b)
    assert np.array_equal(r.colptr, b.colptr)
    for i in range(b.k):
        for j in range(b.n):
            s, e = b.colptr[i][j], b.colptr[i][j + 1]
            assert np.array_equal(r.rowidx[i][s:e], b.rowidx[i][s:e][::-1])
            assert np.array_equal(r.vals[i][s:e], b.vals[i][s:e][::-1])
