"""GPU parity of the batched launch (include/spkadd_batch.h) against the CPU oracle.

Each request of a batch is checked on its own: colptr and rowidx bit-exact, values
bit-exact for integer-valued inputs and within k * u * sum|a| otherwise.  Runs through
the captured hipGraph are replayed with new requests and host work in between, and
every replay is checked.
"""
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


def _random_batches(seed, count, values="int32f"):
    """Small requests of mixed shapes: short and long columns, tall matrices (hash
    accumulator) and short ones (bitmap), empty columns, an empty matrix."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        kind = t % 5
        k = int(rng.integers(1, 13))
        if kind == 0:
            m, n, d = int(rng.integers(1, 600)), int(rng.integers(1, 200)), float(rng.uniform(0.5, 8))
        elif kind == 1:
            m, n, d = int(rng.integers(9000, 140000)), int(rng.integers(1, 120)), float(rng.uniform(2, 40))
        elif kind == 2:
            m, n, d = int(rng.integers(2000, 20000)), int(rng.integers(1, 300)), float(rng.uniform(0, 3))
        elif kind == 3:
            m, n, d = int(rng.integers(100, 3000)), int(rng.integers(1, 60)), float(rng.uniform(20, 80))
        else:
            m, n, d = int(rng.integers(1, 50)), int(rng.integers(0, 30)), float(rng.uniform(0, 5))
        d = min(d, m * 0.9)
        if 2 * k * d > 900:  # keep columns within a wavefront (u <= 1024)
            d = 900.0 / (2 * k)
        out.append(workloads.er(m, n, k, d, seed=seed * 1000 + t, values=values))
    return out


def _requests(batches, cap_scale=1.0):
    import torch
    reqs, keep = [], []
    for b in batches:
        cps, ris, vas = to_device(b)
        nnz_in = int(sum(int(b.colptr[i, b.n]) for i in range(b.k)))
        cap = int(nnz_in * cap_scale)
        colptr_c = torch.full((b.n + 1,), -7, dtype=torch.int32, device="cuda:0")
        rowidx_c = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda:0")
        values_c = torch.zeros(max(cap, 1), dtype=vas[0].dtype if vas else torch.float32, device="cuda:0")
        reqs.append(dict(m=b.m, colptrs=cps, rowidxs=ris, values=vas, colptr_c=colptr_c, rowidx_c=rowidx_c,
                         values_c=values_c, cap_c=cap))
        keep.append((cps, ris, vas))
    return reqs


def _check_all(batches, reqs, nnz, status, exact):
    from paper_2112_10223_amd import binding
    for b, q, z, st in zip(batches, reqs, nnz, status):
        assert st == binding.SPKADD_REQ_OK
        ref = oracle.spkadd(b)
        assert z == int(ref.colptr[-1])
        got = (q["colptr_c"].cpu().numpy().astype(np.int64), q["rowidx_c"][:z].cpu().numpy(),
               q["values_c"][:z].cpu().numpy())
        assert_matches(b, got, ref, exact_values=exact)


def _batch(dtype, nreq, cols, inputs, **kw):
    from paper_2112_10223_amd import binding
    return binding.Batch(dtype, nreq, cols, inputs, binding.make_opts(**kw) if kw else None)


# fused_cols: 0 = default (these runs are small enough for the fused launches, one
# kernel per pass), -1 = one launch per (wave bin, accumulator)
@pytest.mark.parametrize("values,use_graph,fused_cols", [
    ("int32f", False, 0), ("int32f", True, 0), ("int32f", False, -1), ("int32f", True, -1), ("f32", True, 0),
    ("f32", True, -1), ("int64f", True, 0), ("int64f", True, -1), ("f64", False, 0), ("f64", False, -1)])
def test_batch_matches_oracle(values, use_graph, fused_cols):
    import torch
    from paper_2112_10223_amd import binding
    note(f"batch values={values} graph={use_graph} fused_cols={fused_cols}")
    batches = _random_batches(3, 25, values)
    reqs = _requests(batches)
    dtype = binding.SPKADD_F64 if values in ("f64", "int64f") else binding.SPKADD_F32
    bt = _batch(dtype, 64, 20000, 2000, batch_fused_cols=fused_cols)
    bt.run(reqs, use_graph=use_graph)
    nnz, st = bt.results()
    torch.cuda.synchronize()
    _check_all(batches, reqs, nnz, st, exact=values.startswith("int"))
    info = bt.info()
    assert info["fused_runs"] == (1 if fused_cols == 0 else 0)
    assert info["kernels_per_run"] == 9 if fused_cols == 0 else info["kernels_per_run"] > 9
    if use_graph:
        assert info["graphs_captured"] == 1 and info["graph_replays"] == 1
    bt.close()


def test_batch_fused_threshold():
    """Runs with more columns than batch_fused_cols launch per slot, smaller ones fused;
    both right, the same batch object."""
    from paper_2112_10223_amd import binding
    note("batch fused threshold")
    bt = _batch(binding.SPKADD_F32, 64, 20000, 2000, batch_fused_cols=400)
    big = _random_batches(13, 20, "int32f")
    small = [b for b in _random_batches(14, 20, "int32f") if 0 < b.n <= 100][:3]
    assert sum(b.n for b in big) > 400 and 0 < sum(b.n for b in small) <= 400
    for batches in (big, small, big):
        reqs = _requests(batches)
        bt.run(reqs, use_graph=True)
        nnz, st = bt.results()
        _check_all(batches, reqs, nnz, st, exact=True)
    info = bt.info()
    assert info["fused_runs"] == 1 and info["graphs_captured"] == 2 and info["graph_replays"] == 3
    bt.close()


@pytest.mark.parametrize("mode,fused_cols", [(1, 0), (2, 0), (1, -1), (2, -1)])
def test_batch_accumulators(mode, fused_cols):
    from paper_2112_10223_amd import binding
    note(f"batch accum_mode={mode} fused_cols={fused_cols}")
    batches = _random_batches(5, 15, "int32f")
    reqs = _requests(batches)
    bt = _batch(binding.SPKADD_F32, 32, 10000, 1000, accum_mode=mode, batch_fused_cols=fused_cols)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    _check_all(batches, reqs, nnz, st, exact=True)
    bt.close()


def test_batch_graph_replays():
    """Three runs through one captured graph (same launch shape, new requests each
    time), with host work between them; every run is checked."""
    from paper_2112_10223_amd import binding
    note("batch graph replays")
    bt = _batch(binding.SPKADD_F32, 64, 20000, 2000)
    for rep in range(3):
        batches = _random_batches(11, 25, "int32f") if rep == 0 else _random_batches(11 + rep, 25, "int32f")
        reqs = _requests(batches)
        bt.run(reqs, use_graph=True)
        nnz, st = bt.results()
        _check_all(batches, reqs, nnz, st, exact=True)  # host work between replays
    info = bt.info()
    assert info["graph_replays"] == 3
    bt.close()


def test_batch_covering_graph_reused():
    """A run whose launch shape is covered by an earlier run's captured graph replays
    that graph (its extra launches find no columns) instead of capturing a new one,
    and its results are still right."""
    from paper_2112_10223_amd import binding
    note("batch covering graph")
    bt = _batch(binding.SPKADD_F32, 64, 20000, 2000)
    batches = _random_batches(41, 30, "int32f")
    reqs = _requests(batches)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    _check_all(batches, reqs, nnz, st, exact=True)
    sub = batches[3:9]
    reqs = _requests(sub)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    _check_all(sub, reqs, nnz, st, exact=True)
    info = bt.info()
    assert info["graphs_captured"] == 1 and info["graph_reuses"] == 1 and info["graph_replays"] == 2
    bt.close()


def test_batch_too_large_and_capacity():
    import torch
    from paper_2112_10223_amd import binding
    note("batch too large / capacity")
    small = _random_batches(21, 6, "int32f")
    big = workloads.er(5000, 10, 4, 1500.0, seed=99, values="int32f")  # u about 6000 > 4096
    batches = small[:3] + [big] + small[3:]
    reqs = _requests(batches)
    # request 1 gets too little room for its output
    ref1 = oracle.spkadd(batches[1])
    need = int(ref1.colptr[-1])
    assert need > 2
    reqs[1]["cap_c"] = need - 1
    bt = _batch(binding.SPKADD_F32, 16, 5000, 500)
    bt.run(reqs, use_graph=False)
    nnz, st = bt.results()
    torch.cuda.synchronize()
    assert st[3] == binding.SPKADD_REQ_TOO_LARGE
    assert st[1] == binding.SPKADD_REQ_CAPACITY and nnz[1] == need
    assert np.array_equal(reqs[1]["colptr_c"].cpu().numpy().astype(np.int64), ref1.colptr)
    assert (reqs[1]["rowidx_c"].cpu().numpy() == -7).all()  # nothing written
    ok = [i for i in range(len(batches)) if i not in (1, 3)]
    _check_all([batches[i] for i in ok], [reqs[i] for i in ok], [nnz[i] for i in ok], [st[i] for i in ok], True)
    bt.close()


@pytest.mark.parametrize("values", ["int32f", "f32", "f64"])
def test_batch_workgroup_columns(values):
    """Columns with 1024 < u <= 4096 entries (requests of at most 2^17 rows) are
    computed inside the batched run by the workgroup bitmap; wider requests or longer
    columns are reported too large.  Mixed with wave-sized requests."""
    import torch
    from paper_2112_10223_amd import binding
    note(f"batch workgroup columns values={values}")
    batches = _random_batches(51, 8, values)
    batches.insert(2, workloads.er(6000, 40, 5, 500.0, seed=52, values=values))     # u ~ 2500
    batches.insert(5, workloads.er(131072, 30, 12, 300.0, seed=53, values=values))  # u ~ 3600, m = 2^17
    batches.append(workloads.er(40000, 25, 3, 500.0, seed=54, values=values))       # u ~ 1500
    too_long = workloads.er(3000, 10, 3, 2000.0, seed=55, values=values)             # u ~ 6000
    too_wide = workloads.er(140000, 10, 4, 400.0, seed=56, values=values)            # m > 2^17
    batches += [too_long, too_wide]
    reqs = _requests(batches)
    dtype = binding.SPKADD_F64 if values == "f64" else binding.SPKADD_F32
    bt = _batch(dtype, 32, 20000, 2000)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    torch.cuda.synchronize()
    assert st[-2] == binding.SPKADD_REQ_TOO_LARGE and st[-1] == binding.SPKADD_REQ_TOO_LARGE
    _check_all(batches[:-2], reqs[:-2], nnz[:-2], st[:-2], exact=values.startswith("int"))
    bt.close()


def test_batch_long_requests_and_many_bounds_blocks():
    """Requests of up to 70 001 columns (their colptr scans run several tiles and a
    ragged tail); a 300 000-column batch spreads the bounds pass over hundreds of
    blocks."""
    from paper_2112_10223_amd import binding
    note("batch long requests")
    batches = [workloads.er(200, 70001, 3, 0.7, seed=61, values="int32f"),
               workloads.er(5000, 16385, 4, 2.0, seed=62, values="int32f"),
               workloads.er(50, 1, 2, 3.0, seed=63, values="int32f"),
               workloads.er(3000, 40000, 2, 1.5, seed=64, values="int32f")]
    bt = _batch(binding.SPKADD_F32, 8, 300000, 64)
    for use_graph in (False, True):
        reqs = _requests(batches)
        bt.run(reqs, use_graph=use_graph)
        nnz, st = bt.results()
        _check_all(batches, reqs, nnz, st, exact=True)
    bt.close()


def test_batch_many_requests():
    """More requests than the kernels keep in on-chip memory (1024): the column to
    request search then reads the request table in device memory."""
    from paper_2112_10223_amd import binding
    note("batch many requests")
    rng = np.random.default_rng(71)
    batches = [workloads.er(int(rng.integers(1, 300)), int(rng.integers(0, 5)), int(rng.integers(1, 4)),
                            float(rng.uniform(0, 4)), seed=7100 + t, values="int32f") for t in range(1100)]
    bt = _batch(binding.SPKADD_F32, 1100, 5000, 3300)
    reqs = _requests(batches)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    _check_all(batches, reqs, nnz, st, exact=True)
    bt.close()


def test_batch_equals_plain_path():
    """The batched and the one-request launches give identical bits on the same
    requests (integer-valued inputs: every order of summation is exact)."""
    from paper_2112_10223_amd import binding
    note("batch vs plain")
    batches = _random_batches(31, 12, "int32f")
    reqs = _requests(batches)
    bt = _batch(binding.SPKADD_F32, 16, 10000, 500)
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    for b, q, z in zip(batches, reqs, nnz):
        cps, ris, vas = to_device(b)
        cp, r, v = binding.spkadd(b.m, cps, ris, vas)
        assert np.array_equal(cp.cpu().numpy(), q["colptr_c"].cpu().numpy())
        assert np.array_equal(r.cpu().numpy(), q["rowidx_c"][:z].cpu().numpy())
        assert np.array_equal(v.cpu().numpy(), q["values_c"][:z].cpu().numpy())
    bt.close()


def test_batch_argument_errors():
    import torch
    from paper_2112_10223_amd import binding
    note("batch argument errors")
    bt = _batch(binding.SPKADD_F32, 2, 100, 4)
    b = workloads.er(50, 10, 3, 2.0, seed=1, values="int32f")
    reqs = _requests([b, b, b])
    with pytest.raises(binding.SpkaddError):
        bt.run(reqs)  # three requests, room for two
    reqs = _requests([workloads.er(50, 80, 3, 2.0, seed=1, values="int32f")] * 2)
    with pytest.raises(binding.SpkaddError):
        bt.run(reqs)  # 160 columns, room for 100
    with pytest.raises(binding.SpkaddError):
        bt.results()  # no run yet
    torch.cuda.synchronize()
    bt.close()


def _stream_batches(seed, count, values, max_nnz=1 << 19):
    """Requests of the batched workload's distribution (k ~ U{2..64}, m and n
    log-uniform in [256, 65536], per-matrix density log-uniform in [1e-4, 1e-2]),
    requests above max_nnz expected input entries redrawn, plus fixed requests at the
    edge of the one-input-per-lane layout (k = 63 and 64) in wave, workgroup and
    too-large columns."""
    out = workloads.request_stream(count, seed=seed, max_nnz=max_nnz, values=values)
    out += [workloads.er(3000, 50, 64, 5.0, seed=seed + 1, values=values),      # k = 64, u ~ 320
            workloads.er(60000, 40, 63, 10.0, seed=seed + 2, values=values),    # k = 63, hash wave columns
            workloads.er(800, 30, 64, 14.0, seed=seed + 3, values=values),      # k = 64, u ~ 900
            workloads.er(5000, 20, 64, 40.0, seed=seed + 4, values=values),     # k = 64, u ~ 2560: workgroup
            workloads.er(20000, 12, 64, 100.0, seed=seed + 5, values=values)]   # k = 64, u ~ 6400: too large
    return out


@pytest.mark.parametrize("values", ["int32f", "f32", "f64"])
def test_batch_request_stream(values):
    """Requests drawn from the batched workload's own distribution, k up to 64 (and
    exactly 63 and 64), each against the oracle; the requests the run reports too large
    go through the one-request path and are checked as well."""
    import torch
    from paper_2112_10223_amd import binding
    note(f"batch request stream values={values}")
    batches = _stream_batches(81, 40, values)
    assert max(b.k for b in batches) == 64
    reqs = _requests(batches)
    dtype = binding.SPKADD_F64 if values == "f64" else binding.SPKADD_F32
    bt = _batch(dtype, len(batches), sum(b.n for b in batches), sum(b.k for b in batches))
    bt.run(reqs, use_graph=True)
    nnz, st = bt.results()
    torch.cuda.synchronize()
    exact = values.startswith("int")
    big = [i for i, s in enumerate(st) if s == binding.SPKADD_REQ_TOO_LARGE]
    assert len(batches) - 1 in big
    ok = [i for i in range(len(batches)) if i not in big]
    _check_all([batches[i] for i in ok], [reqs[i] for i in ok], [nnz[i] for i in ok], [st[i] for i in ok], exact)
    for i in big:
        b = batches[i]
        cps, ris, vas = to_device(b)
        cp, r, v = binding.spkadd(b.m, cps, ris, vas)
        torch.cuda.synchronize()
        got = (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy())
        assert_matches(b, got, oracle.spkadd(b), exact_values=exact)
    bt.close()
