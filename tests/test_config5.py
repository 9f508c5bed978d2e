"""The batched / served workload at its stated shape, against the oracle.

The first 1000 requests of the unfiltered request distribution (k ~ U{2..64}, m and n
log-uniform in [256, 65536], per-matrix density log-uniform in [1e-4, 1e-2], fp32
values) are drawn on the device and served together by the serving loop (a 64 GB
output budget; requests with columns too long for a batched run take the one-request
lane).  Every request of at most 2^24 input entries, and a seeded sample of 50 larger
ones, is checked against the oracle on the host: colptr and rows bit-exact, values
within max(k, t) * 2^-24 * sum|a|.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import assert_matches, host_threads, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_10223_amd import binding
    binding.lib()


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_served_pool_against_oracle():
    import torch
    from paper_2112_10223_amd import binding
    pool_size = 1000
    specs = workloads.request_specs(pool_size)
    note(f"config5 pool of {pool_size}: drawing on the device")
    inputs = []
    for s in specs:
        cps, ris, vas = workloads.device_request(s, "f32")
        fb = cps[0].data_ptr()
        nnz = int(sum(int(r.shape[0]) for r in ris))
        inputs.append((binding.PtrArray(cps, True, fb), binding.PtrArray(ris, True, fb),
                       binding.PtrArray(vas, True, fb), nnz))
    torch.cuda.synchronize()
    nnz_in = np.array([x[3] for x in inputs])
    small = np.nonzero(nnz_in <= (1 << 24))[0]
    large = np.nonzero(nnz_in > (1 << 24))[0]
    chosen = set(small.tolist()) | set(np.random.default_rng(5).choice(large, size=min(50, len(large)),
                                                                        replace=False).tolist())
    note(f"config5: {len(small)} requests <= 2^24 entries, {len(large)} larger; serving all together")
    srv = binding.Server(binding.SPKADD_F32, n_streams=1, max_batch=8, max_columns=8 * 65536, max_inputs=8 * 64,
                         hbm_budget=64 << 30)
    side = torch.cuda.Stream()
    tickets = [srv.submit(s.m, cp, ri, va, max(z, 1)) for s, (cp, ri, va, z) in zip(specs, inputs)]
    outputs, lanes = {}, 0
    for i, tk in enumerate(tickets):
        res = srv.wait(tk, timeout=600.0)
        assert res["status"] == binding.SPKADD_REQ_OK, (i, res)
        lanes += res["path"]
        if i in chosen:
            with torch.cuda.stream(side):  # (the null stream refuses work while the lanes capture)
                cp, r, v = srv.outputs(res)
                outputs[i] = (cp.cpu().numpy().astype(np.int64), r.cpu().numpy(), v.cpu().numpy())
        srv.release(tk)
    srv.close()
    assert 0 < lanes < pool_size  # both the batched runs and the one-request lane served
    note(f"config5: checking {len(chosen)} requests against the oracle ({lanes} took the one-request lane)")

    def host_inputs(i):
        """The request's inputs as drawn on the device, on the host.  The device
        generator draws the host generator's matrices bit for bit (the device
        generator's own test), so these are the seeded inputs of request i."""
        cp, ri, va, _ = inputs[i]
        k = len(cp)
        colptr = np.stack([cp.tensors[t].cpu().numpy() for t in range(k)])
        rows = [ri.tensors[t].cpu().numpy() for t in range(k)]
        vals = [va.tensors[t].cpu().numpy() for t in range(k)]
        return workloads.CSCBatch(specs[i].m, specs[i].n, colptr, rows, vals)

    def check(i, batch):
        got = outputs.pop(i)
        assert_matches(batch, got, oracle.spkadd(batch))
        return batch.nnz_in

    checked, done = 0, 0
    with cf.ThreadPoolExecutor(host_threads()) as ex:
        pending = []
        for i in sorted(chosen):
            pending.append(ex.submit(check, i, host_inputs(i)))
            while len(pending) >= 2 * host_threads() or (pending and pending[0].done()):
                checked += pending.pop(0).result()
                done += 1
                if done % 100 == 0:
                    print(f"config5: {done} of {len(chosen)} checked", flush=True)
        for f in pending:
            checked += f.result()
    del inputs
    torch.cuda.empty_cache()
    print(f"config5: {len(chosen)} requests, {checked} input entries checked against the oracle", flush=True)
