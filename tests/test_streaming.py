"""GPU parity of the streaming sum (paper_2112_10223_amd/streaming.py): batches added
one after another into a running sum equal the oracle's sum of every input."""
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


@pytest.mark.parametrize("sizes", [[1], [3, 1, 4], [8, 8, 8, 8], [2, 0, 5]])
def test_streaming_matches_oracle(sizes):
    import torch
    from paper_2112_10223_amd.streaming import StreamingSum
    note(f"streaming batches={sizes}")
    k = sum(sizes)
    b = workloads.er(4000, 300, k, 25.0, seed=500 + len(sizes), values="int32f")
    cps, ris, vas = to_device(b)
    s = StreamingSum(b.m, b.n)
    at = 0
    for sz in sizes:
        s.add(cps[at:at + sz], ris[at:at + sz], vas[at:at + sz])
        at += sz
    c, r, v = s.result()
    torch.cuda.synchronize()
    assert s.batches == sum(1 for sz in sizes if sz)
    assert_matches(b, (c.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), oracle.spkadd(b),
                   exact_values=True)


def test_streaming_windows():
    """Batches whose columns need row windows (a long running sum)."""
    import torch
    from paper_2112_10223_amd import binding
    from paper_2112_10223_amd.streaming import StreamingSum
    note("streaming windows")
    b = workloads.rmat(12, 8, 12, seed=501, values="int32f")
    cps, ris, vas = to_device(b)
    s = StreamingSum(b.m, b.n, opts=binding.make_opts(force_bin=2, window_cap=256))
    for at in range(0, 12, 4):
        s.add(cps[at:at + 4], ris[at:at + 4], vas[at:at + 4])
    c, r, v = s.result()
    torch.cuda.synchronize()
    assert_matches(b, (c.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), oracle.spkadd(b),
                   exact_values=True)


def test_streaming_on_a_side_stream():
    """Sums on a stream other than torch's current one, with other work allocating on
    the current stream between batches: every running sum dropped while the next sum
    still reads it keeps its memory until that stream has passed it."""
    import torch
    from paper_2112_10223_amd.streaming import StreamingSum
    note("streaming side stream")
    b = workloads.er(20000, 2000, 12, 40.0, seed=502, values="int32f")
    cps, ris, vas = to_device(b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    s = StreamingSum(b.m, b.n, stream=side)
    junk = []
    for at in range(0, 12, 3):
        s.add(cps[at:at + 3], ris[at:at + 3], vas[at:at + 3])
        junk.append(torch.full((1 << 20,), 7, dtype=torch.int32, device="cuda:0"))  # current-stream allocations
    c, r, v = s.result()
    side.synchronize()
    torch.cuda.synchronize()
    assert_matches(b, (c.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy()), oracle.spkadd(b),
                   exact_values=True)
