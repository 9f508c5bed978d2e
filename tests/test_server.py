"""GPU tests of the serving loop (include/spkadd_server.h): every request's result is
the same when it is served alone and when it is served in a mix with other requests
arriving concurrently, and matches the CPU oracle."""
import threading

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


def _mixed(seed, count, values="int32f"):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        k = int(rng.integers(1, 10))
        m = int(rng.integers(1, 70000)) if t % 3 else int(rng.integers(1, 2000))
        n = int(rng.integers(0, 150))
        d = min(float(rng.uniform(0, 30)), 0.9 * m)
        if 2 * k * d > 900:
            d = 900.0 / (2 * k)
        out.append(workloads.er(m, n, k, d, seed=seed * 997 + t, values=values))
    return out


_side = []


def _side_stream():
    import torch
    if not _side:
        _side.append(torch.cuda.Stream())
    return _side[0]


def _submit(srv, b):
    import torch
    with torch.cuda.stream(_side_stream()):  # (the null stream refuses work while lanes capture)
        cps, ris, vas = to_device(b)
        torch.cuda.current_stream().synchronize()
    cap = max(int(sum(int(b.colptr[i, b.n]) for i in range(b.k))), 1)
    return srv.submit(b.m, cps, ris, vas, cap), (cps, ris, vas)


def _collect(srv, tk):
    import torch
    from paper_2112_10223_amd import binding
    res = srv.wait(tk, timeout=60.0)
    assert res["status"] == binding.SPKADD_REQ_OK, res
    with torch.cuda.stream(_side_stream()):  # (the null stream refuses work while lanes capture)
        cp, r, v = srv.outputs(res)
        out = (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy())
    srv.release(tk)
    return res, out


@pytest.mark.parametrize("n_streams,depth", [(1, 1), (2, 2)])
def test_server_alone_vs_mix(n_streams, depth):
    from paper_2112_10223_amd import binding
    note(f"server alone vs mix streams={n_streams} depth={depth}")
    targets = _mixed(7, 16)
    targets.append(workloads.er(20000, 12, 3, 2000.0, seed=5, values="int32f"))  # too large for a batch (u > 4096)
    others = _mixed(8, 40)
    srv = binding.Server(n_streams=n_streams, max_batch=16, max_columns=4096, max_inputs=256, depth=depth)
    alone = []
    for b in targets:
        tk, keep = _submit(srv, b)
        alone.append(_collect(srv, tk))
    # the same requests again, interleaved with others from a second thread
    tickets = {}
    keeps = []

    def submit_others():
        for b in others:
            tk, keep = _submit(srv, b)
            keeps.append(keep)
            tickets[("o", len(tickets))] = (tk, b)

    th = threading.Thread(target=submit_others)
    th.start()
    mine = []
    for b in targets:
        tk, keep = _submit(srv, b)
        keeps.append(keep)
        mine.append(tk)
    th.join()
    for i, (tk, b) in enumerate(zip(mine, targets)):
        res, got = _collect(srv, tk)
        ra, ga = alone[i]
        assert res["nnz"] == ra["nnz"]
        for x, y in zip(got, ga):
            assert np.array_equal(x, y)
        assert_matches(b, got, oracle.spkadd(b), exact_values=True)
        if i == len(targets) - 1:
            assert res["path"] == 1 and ra["path"] == 1
    for (tk, b) in tickets.values():
        res, got = _collect(srv, tk)
        assert_matches(b, got, oracle.spkadd(b), exact_values=True)
    info = srv.info()
    n_req = 2 * len(targets) + len(others)
    assert info["batched"] == n_req and info["large"] == 2 and info["runs"] >= 1
    # released output blocks were reused by later requests of the same size class
    assert info["allocations"] < n_req and info["held_bytes"] == 0 and info["pooled_bytes"] > 0
    srv.close()


def test_server_tight_budget_and_real_values():
    """A budget that holds only a few requests' outputs at a time: admission waits
    for releases, every result is still right."""
    from paper_2112_10223_amd import binding
    note("server tight budget")
    reqs = _mixed(11, 24, "f32")
    srv = binding.Server(n_streams=3, max_batch=4, max_columns=4096, max_inputs=256, hbm_budget=2 << 20)
    pend = []
    for b in reqs:
        tk, keep = _submit(srv, b)
        pend.append((tk, b, keep))
    for tk, b, _ in pend:
        res, got = _collect(srv, tk)
        assert_matches(b, got, oracle.spkadd(b))
    info = srv.info()
    assert info["held_bytes"] == 0 and info["pooled_bytes"] <= 2 << 20
    srv.close()


def test_server_errors():
    import torch
    from paper_2112_10223_amd import binding
    note("server errors")
    srv = binding.Server(max_columns=64, max_inputs=16, hbm_budget=1 << 20)
    b = workloads.er(100, 100, 2, 1.0, seed=3, values="int32f")  # more columns than one run holds
    with pytest.raises(binding.SpkaddError):
        _submit(srv, b)
    with pytest.raises(binding.SpkaddError):
        srv.wait(12345, timeout=0.1)
    b = workloads.er(100, 10, 2, 1.0, seed=3, values="int32f")
    tk, keep = _submit(srv, b)
    res, got = _collect(srv, tk)
    with pytest.raises(binding.SpkaddError):
        srv.release(tk)  # already released
    torch.cuda.synchronize()
    srv.close()


def _stream_mix(seed, count, values):
    """Requests of the served workload's distribution (k ~ U{2..64}), a bounded sample
    (expected input entries <= 2^19), plus requests with columns too long for a batched
    run (they take the one-request lane, row windows included)."""
    out = workloads.request_stream(count, seed=seed, max_nnz=1 << 19, values=values)
    out += [workloads.er(65536, 60, 64, 400.0, seed=seed + 1, values=values),   # u ~ 25600: windows
            workloads.er(20000, 12, 64, 100.0, seed=seed + 2, values=values)]   # u ~ 6400
    return out


@pytest.mark.parametrize("values", ["int32f", "f32"])
def test_server_request_stream_alone_vs_mix(values):
    """Every request of a sample of the served workload (k up to 64, large requests
    in the one-request lane) gives the same result alone and in a concurrent mix:
    colptr and rows bit-exact, values bit-exact for integer-valued inputs and, for real
    values, both within the oracle's tolerance (so within twice it of each other)."""
    import numpy as np
    from paper_2112_10223_amd import binding
    note(f"server request stream alone vs mix values={values}")
    targets = _stream_mix(91, 20, values)
    others = _stream_mix(92, 30, values)
    srv = binding.Server(n_streams=2, max_batch=8, max_columns=1 << 17, max_inputs=8 * 64, depth=1)
    alone = []
    for b in targets:
        tk, keep = _submit(srv, b)
        alone.append(_collect(srv, tk))
    tickets, keeps = [], []

    def submit_others():
        for b in others:
            tk, keep = _submit(srv, b)
            keeps.append(keep)
            tickets.append((tk, b))

    th = threading.Thread(target=submit_others)
    th.start()
    mine = []
    for b in targets:
        tk, keep = _submit(srv, b)
        keeps.append(keep)
        mine.append(tk)
    th.join()
    exact = values.startswith("int")
    lanes = []
    for i, (tk, b) in enumerate(zip(mine, targets)):
        res, got = _collect(srv, tk)
        ra, ga = alone[i]
        assert res["nnz"] == ra["nnz"]
        assert np.array_equal(got[0], ga[0]) and np.array_equal(got[1], ga[1])
        ref = oracle.spkadd(b)
        assert_matches(b, got, ref, exact_values=exact)
        assert_matches(b, ga, ref, exact_values=exact)
        if exact:
            assert np.array_equal(got[2], ga[2])
        lanes.append(res["path"])
    assert lanes[-1] == 1 and lanes[-2] == 1 and sum(lanes) < len(lanes)
    for tk, b in tickets:
        res, got = _collect(srv, tk)
        assert_matches(b, got, oracle.spkadd(b), exact_values=exact)
    info = srv.info()
    assert info["held_bytes"] == 0
    srv.close()
