"""Host-side checks of the streaming sum (no device): shapes are checked before any
library call, and an empty batch leaves the sum untouched."""
import pytest


def test_streaming_rejects_wrong_shape_and_ignores_empty_batches():
    torch = pytest.importorskip("torch")
    from paper_2112_10223_amd.streaming import StreamingSum
    s = StreamingSum(10, 4)
    s.add([], [], [])
    assert s.result() is None and s.batches == 0
    bad = torch.zeros(3, dtype=torch.int32)  # n + 1 = 5 expected
    with pytest.raises(ValueError):
        s.add([bad], [torch.zeros(0, dtype=torch.int32)], [torch.zeros(0)])
    assert s.result() is None and s.batches == 0
