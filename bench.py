#!/usr/bin/env python3
"""SpKAdd benchmark on one MI355X.

One step is the whole hot path of the method on one batch of synthetic inputs:
spkadd_plan (upper bounds, bins, windows), spkadd_symbolic (per-column output
counts and colptr(B)), and spkadd_numeric (hash accumulation, in-LDS sort,
write-out).  Inputs are resident in HBM and outputs are preallocated before the
timed region.  The default workload is k=32 Erdos-Renyi CSC matrices,
65,536 x 65,536, Poisson(16) rows per column, fp32.

Prints one JSON line: input nnz/s over the timed steps, the roofline entry of the
dominant kernel (algorithmic bytes per launch / mean launch time, from HIP events
recorded by the library on the launch stream), and the CPU oracle timed on the
host on the same inputs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBPS = 8000.0
METRIC = "SpKAdd input nnz/s + % HBM peak; served p50/p99 latency vs plain launches"

WORKLOADS = {
    "config2": ("k=32 Erdos-Renyi CSC 65536x65536, Poisson(16) rows/column, fp32 U(-1,1)",
                lambda: workloads.config2("f32")),
    "config2_f64": ("k=32 Erdos-Renyi CSC 65536x65536, Poisson(16) rows/column, fp64 U(-1,1)",
                    lambda: workloads.config2("f64")),
    "config1": ("k=4 Erdos-Renyi CSC 1000x1000, Poisson(8) rows/column, fp32 U(-1,1)",
                lambda: workloads.config1("f32")),
    "config3": ("k=64 R-MAT (a=.57,b=c=.19) 2^20x2^20, edge factor 16, fp32 N(0,1)",
                lambda: workloads.config3("normal")),
    "config4": ("k=128 tall-skinny 2^24x1024, 4096 uniform rows/column, fp32 U(-1,1)",
                lambda: workloads.config4("f32")),
}

WAVE_E = [1, 2, 3, 4, 5, 6, 8, 10, 12, 16]


def kernel_of_column(u: np.ndarray, cap: int, wave_max: int = 1024, merge: bool = True) -> np.ndarray:
    """Name of the numeric kernel each column goes to under the default options
    (mirrors the library's binning by u_j, and its merging of two adjacent
    populous wave bins)."""
    names = np.empty(u.shape[0], dtype=object)
    names[:] = "empty"
    e = (u + 63) // 64
    for E in reversed(WAVE_E):
        names[(u > 0) & (u <= wave_max) & (e <= E)] = f"num_wave_e{E}"
    if merge:
        counts = {E: int(np.sum(names == f"num_wave_e{E}")) for E in WAVE_E}
        total = sum(counts.values())
        prev = None
        for E in WAVE_E:
            if counts[E] == 0:
                continue
            if prev is not None and 16 * counts[prev] >= total and 16 * counts[E] >= total and 2 * E <= 3 * prev:
                names[names == f"num_wave_e{prev}"] = f"num_wave_e{E}"
                prev = None
            else:
                prev = E
    names[(u > wave_max) & (u <= min(cap, 2048))] = "num_wg256"
    names[(u > max(wave_max, min(cap, 2048))) & (u <= cap)] = "num_wg512"
    names[u > cap] = "num_window"
    return names


# kernel sources whose change makes a committed traffic summary stale, by trace-name prefix
_KERNEL_SOURCES = {
    "num_wave": ("hash_kernels.hip", "wave_kernels.hip", "wave_device.h", "hash_common.h", "device.h", "internal.h"),
    "num_window": ("bitmap_wg.hip", "bitmap_wg_device.h", "hash_kernels.hip", "hash_common.h", "device.h",
                   "internal.h"),
}


def source_sha(kernel: str = "num_wave") -> str:
    """Hash of the sources the kernel (by trace name) is compiled from."""
    files = next((v for key, v in _KERNEL_SOURCES.items() if kernel.startswith(key)), None)
    if files is None:
        files = tuple(sorted(f for f in os.listdir(os.path.join(ROOT, "paper_2112_10223_amd", "csrc"))
                             if f.endswith((".hip", ".h"))))
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(ROOT, "paper_2112_10223_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/traffic_<kernel>_<workload>.md), or None when there is none or the
    kernel sources changed since the counters were taken."""
    from paper_2112_10223_amd import profiling
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = profiling.read_traffic_summary(path)
    if rec.get("source_sha") != source_sha(kernel):
        return None
    return int(rec["traffic_bytes_per_launch"])


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)  # one elementwise kernel: reads nbytes, writes nbytes
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps, "source_sha": source_sha()}))


# serving loop defaults: one batched stream, one run in flight, at most 8 requests per
# run, two one-request lanes for the requests too large for a batched run
SERVER_CONFIG = {"n_streams": 1, "depth": 1, "max_batch": 8, "large_streams": 2}
# the policies the served workload is swept over before it is measured
SERVER_CANDIDATES = [
    {"n_streams": 1, "depth": 1, "max_batch": 8, "large_streams": 2},
    {"n_streams": 2, "depth": 1, "max_batch": 8, "large_streams": 2},
    {"n_streams": 2, "depth": 1, "max_batch": 4, "large_streams": 2},
    {"n_streams": 4, "depth": 1, "max_batch": 4, "large_streams": 2},
    {"n_streams": 2, "depth": 1, "max_batch": 8, "large_streams": 4},
    {"n_streams": 4, "depth": 1, "max_batch": 4, "large_streams": 4},
    {"n_streams": 4, "depth": 1, "max_batch": 8, "large_streams": 2},
    {"n_streams": 6, "depth": 1, "max_batch": 4, "large_streams": 2},
]
SERVE_BUDGET = 64 << 30  # bytes of output memory the admitted requests may hold
BYTES_PER_INPUT_NNZ = 20  # algorithmic bytes of a batched request per input entry (fp32, cf ~ 1)


class RequestPool:
    """Requests of the served workload drawn on the device: the first `size` shapes of
    the unfiltered request distribution (workloads.request_specs: k ~ U{2..64}, m, n
    log-uniform in [256, 65536], density log-uniform in [1e-4, 1e-2] per matrix), their
    inputs resident in HBM."""

    def __init__(self, size: int, values: str = "f32", seed: int = workloads.SEED + 5):
        import torch
        from paper_2112_10223_amd import binding
        self.specs = workloads.request_specs(size, seed=seed)
        self.reqs = []
        for sp in self.specs:
            cps, ris, vas = workloads.device_request(sp, values)
            fb = cps[0].data_ptr()
            nnz = int(sum(int(r.shape[0]) for r in ris))
            self.reqs.append(dict(m=sp.m, n=sp.n, k=sp.k, nnz_in=nnz, cap_c=max(nnz, 1),
                                  colptrs=binding.PtrArray(cps, True, fb), rowidxs=binding.PtrArray(ris, True, fb),
                                  values=binding.PtrArray(vas, True, fb)))
        torch.cuda.synchronize()
        self.nnz_in = sum(q["nnz_in"] for q in self.reqs)
        self.max_cap = max(q["cap_c"] for q in self.reqs)
        self.max_n = max(q["n"] for q in self.reqs)


class PlainRunner:
    """The one-request path (plan, symbolic, numeric) with outputs in one of `slots`
    preallocated buffers (a buffer per concurrent stream)."""

    def __init__(self, pool: RequestPool, slots: int = 4):
        import torch
        dev = "cuda:0"
        self.out = [(torch.empty(pool.max_n + 1, dtype=torch.int32, device=dev),
                     torch.empty(pool.max_cap, dtype=torch.int32, device=dev),
                     torch.empty(pool.max_cap, dtype=torch.float32, device=dev)) for _ in range(slots)]

    def run(self, q, stream, slot: int = 0, opts=None):
        from paper_2112_10223_amd import binding
        cp, r, v = self.out[slot]
        p = binding.spkadd_plan(q["m"], q["n"], q["colptrs"], q["rowidxs"], binding.SPKADD_F32, opts, stream)
        binding.spkadd_symbolic(p, cp[:q["n"] + 1], stream)
        binding.spkadd_numeric(p, q["values"], r, v, stream)
        p.free()


def _pct(v, p):
    return round(float(np.percentile(np.asarray(v) * 1e3, p)), 3)


def _plain_latencies(plain, reqs, arrivals, stream, opts, wait_until):
    """(a) one-request launches at their arrival times, in order, on one stream; (a') the
    same from four host threads, each with its own stream, taking the requests in
    arrival order.  Latencies and spans of both."""
    import threading
    import torch
    from paper_2112_10223_amd import binding
    lat_plain = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, a in zip(reqs, arrivals):
        wait_until(t0, a)
        plain.run(q, stream, 0, opts)
        torch.cuda.synchronize()
        lat_plain.append(time.perf_counter() - t0 - a)
    span_plain = time.perf_counter() - t0
    # (a') plain on 4 streams: 4 host threads take the requests in arrival order
    lat_p4 = [0.0] * len(reqs)
    nxt = [0]
    lock = threading.Lock()
    streams = [torch.cuda.Stream() for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def worker(w, st):
        sp = binding._stream_ptr(st)
        while True:
            with lock:
                i = nxt[0]
                nxt[0] += 1
            if i >= len(reqs):
                return
            wait_until(t0, arrivals[i])
            plain.run(reqs[i], sp, w, opts)
            st.synchronize()
            lat_p4[i] = time.perf_counter() - t0 - arrivals[i]

    ths = [threading.Thread(target=worker, args=(w, st)) for w, st in enumerate(streams)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    span_p4 = time.perf_counter() - t0
    return lat_plain, span_plain, lat_p4, span_p4


def measure_served(pool: RequestPool, plain: PlainRunner, picks, plain_service_s: float, load: float, seed: int,
                   opts=None, server_config: dict | None = None, baselines: bool = True) -> dict:
    """Poisson arrivals at `load` times the rate one-request launches sustain on one
    stream (1 / mean plain service time); arrival t brings pool request picks[t].
    (a) plain: each request at its arrival time, in order, one at a time; (a') the
    same from four host threads, each with its own stream; (b) served: a submitter
    thread hands each request to the serving loop at its arrival time.  Latency =
    completion - arrival; p50 / p99 over all arrivals."""
    import threading
    import torch
    from paper_2112_10223_amd import binding
    rng = np.random.default_rng(seed)
    rate = load / plain_service_s
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(picks)))
    reqs = [pool.reqs[i] for i in picks]
    nnz_in = sum(q["nnz_in"] for q in reqs)

    def wait_until(t0, t):
        while True:
            left = t - (time.perf_counter() - t0)
            if left <= 0:
                return
            if left > 2e-4:
                time.sleep(left - 1e-4)

    stream = binding._stream_ptr(None)
    lat_plain, lat_p4, span_plain, span_p4 = [0.0], [0.0], 1.0, 1.0
    if baselines:
        lat_plain, span_plain, lat_p4, span_p4 = _plain_latencies(plain, reqs, arrivals, stream, opts, wait_until)
    # (b) the serving loop
    sc = dict(SERVER_CONFIG, **(server_config or {}))
    srv = binding.Server(binding.SPKADD_F32, n_streams=sc["n_streams"], max_batch=sc["max_batch"],
                         max_columns=max(sc["max_batch"] * pool.max_n, 1 << 17), max_inputs=sc["max_batch"] * 64,
                         hbm_budget=SERVE_BUDGET, depth=sc["depth"], opts=opts, large_streams=sc["large_streams"])
    tickets = [None] * len(reqs)

    def submitter(t0s):
        for i, (q, a) in enumerate(zip(reqs, arrivals)):
            wait_until(t0s, a)
            tickets[i] = srv.submit(q["m"], q["colptrs"], q["rowidxs"], q["values"], q["cap_c"])

    # warm-up: the pool once through the server, all at once (captures the launch
    # shapes of full runs, which cover most smaller ones later)
    warm = [srv.submit(q["m"], q["colptrs"], q["rowidxs"], q["values"], q["cap_c"]) for q in pool.reqs]
    for tk in warm:
        srv.wait(tk)
        srv.release(tk)
    info0 = srv.info()
    t0 = time.perf_counter()
    th = threading.Thread(target=submitter, args=(t0,))
    th.start()
    lat_srv, paths, qwait, run = [], [], [], []
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0)
        res = srv.wait(tickets[i])
        lat_srv.append(res["t_done"] - res["t_submit"])
        qwait.append(res["t_start"] - res["t_submit"])
        run.append(res["t_done"] - res["t_start"])
        paths.append(res["path"])
        srv.release(tickets[i])
    th.join()
    span_srv = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    timed = {key: info[key] - info0[key] for key in ("runs", "batched", "large", "allocations", "graphs_captured",
                                                     "graph_reuses")}
    lane = [x for x, p in zip(lat_srv, paths) if p == 1]
    served = {"p50_ms": _pct(lat_srv, 50), "p99_ms": _pct(lat_srv, 99), "nnz_per_s": nnz_in / span_srv,
              "one_request_lane": {"share": round(len(lane) / len(reqs), 4),
                                   "p50_ms": _pct(lane, 50) if lane else None,
                                   "p99_ms": _pct(lane, 99) if lane else None},
              "p50_admission_wait_ms": _pct(qwait, 50), "p50_run_ms": _pct(run, 50), "timed_region": timed}
    if not baselines:
        return {"arrival_rate_per_s": round(rate, 1), "load_vs_plain": load, "arrivals": len(reqs), "server": sc,
                "served": served}
    return {"arrival_rate_per_s": round(rate, 1), "load_vs_plain": load, "arrivals": len(reqs), "server": sc,
            "plain": {"p50_ms": _pct(lat_plain, 50), "p99_ms": _pct(lat_plain, 99), "nnz_per_s": nnz_in / span_plain},
            "plain_4_streams": {"p50_ms": _pct(lat_p4, 50), "p99_ms": _pct(lat_p4, 99),
                                "nnz_per_s": nnz_in / span_p4},
            "served": served,
            "p99_speedup_vs_plain": round(_pct(lat_plain, 99) / max(_pct(lat_srv, 99), 1e-9), 3),
            "p99_speedup_vs_plain_4_streams": round(_pct(lat_p4, 99) / max(_pct(lat_srv, 99), 1e-9), 3)}


def batched_throughput(pool: RequestPool, plain: PlainRunner, opts, run_size: int, reps: int = 3) -> dict:
    """Every pool request through batched runs of run_size requests (two batch objects
    alternate, each with an output arena of its largest group; graphs captured in a
    warm-up pass); the requests a run reports too large go through the one-request
    path.  Best of reps; also the device time of one run against its host call."""
    import torch
    from paper_2112_10223_amd import binding
    stream = binding._stream_ptr(None)
    groups = [pool.reqs[i:i + run_size] for i in range(0, len(pool.reqs), run_size)]
    cols = max(sum(q["n"] for q in g) for g in groups)
    inputs = max(sum(q["k"] for q in g) for g in groups)
    arena_entries = max(sum(q["cap_c"] for q in g) for g in groups)
    arena_cols = max(sum(q["n"] + 1 for q in g) for g in groups)
    bts = [binding.Batch(binding.SPKADD_F32, run_size, cols, inputs, opts) for _ in range(2)]
    arenas = [(torch.empty(arena_cols, dtype=torch.int32, device="cuda:0"),
               torch.empty(arena_entries, dtype=torch.int32, device="cuda:0"),
               torch.empty(arena_entries, dtype=torch.float32, device="cuda:0")) for _ in range(2)]
    runs = []
    for gi, g in enumerate(groups):
        cp, r, v = arenas[gi & 1]
        oc = oe = 0
        rq = []
        for q in g:
            rq.append(dict(m=q["m"], colptrs=q["colptrs"], rowidxs=q["rowidxs"], values=q["values"],
                           colptr_c=cp[oc:oc + q["n"] + 1], rowidx_c=r[oe:oe + q["cap_c"]],
                           values_c=v[oe:oe + q["cap_c"]], cap_c=q["cap_c"], src=q))
            oc += q["n"] + 1
            oe += q["cap_c"]
        runs.append(rq)
    large = []

    def one_pass():
        large.clear()
        pending = [None, None]
        for gi, rq in enumerate(runs):
            bt = bts[gi & 1]
            if pending[gi & 1] is not None:
                _, st = bt.results()
                large.extend(x["src"] for x, s in zip(pending[gi & 1], st) if s == binding.SPKADD_REQ_TOO_LARGE)
            bt.run(rq, use_graph=True, stream=stream)
            pending[gi & 1] = rq
        for slot in (0, 1):
            if pending[slot] is not None:
                _, st = bts[slot].results()
                large.extend(x["src"] for x, s in zip(pending[slot], st) if s == binding.SPKADD_REQ_TOO_LARGE)
        for q in large:
            plain.run(q, stream, 0, opts)

    one_pass()  # warm-up (captures the graphs)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        t0 = time.perf_counter()
        one_pass()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    # one run of the largest group by device time (events on the stream) against its
    # host call: the gap is host preparation and launch
    gi = max(range(len(runs)), key=lambda x: sum(q["cap_c"] for q in runs[x]))
    torch.cuda.synchronize()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ea.record()
    bts[0].run(runs[gi], use_graph=True, stream=stream)
    eb.record()
    t_host = time.perf_counter() - t0
    eb.synchronize()
    t_wall = time.perf_counter() - t0
    info = bts[0].info()
    for bt in bts:
        bt.close()
    nnz_batched = pool.nnz_in - sum(q["nnz_in"] for q in large)
    return {"run_size": run_size, "ms": round(best * 1e3, 3), "nnz_per_s": pool.nnz_in / best,
            "gbps_alg": round(BYTES_PER_INPUT_NNZ * pool.nnz_in / best / 1e9, 1),
            "hbm_frac_alg": round(BYTES_PER_INPUT_NNZ * pool.nnz_in / best / 1e9 / HBM_PEAK_GBPS, 4),
            "too_large_routed_plain": len(large), "input_nnz_in_batched_runs": int(nnz_batched),
            "kernels_per_run": info["kernels_per_run"],
            "one_run": {"requests": len(runs[gi]), "input_nnz": int(sum(q["src"]["nnz_in"] for q in runs[gi])),
                        "device_ms": round(ea.elapsed_time(eb), 4), "host_call_ms": round(t_host * 1e3, 4),
                        "wall_ms": round(t_wall * 1e3, 4)}}


def alone_vs_mix(pool_size: int, picks, rate: float, seed: int, opts=None, server_config: dict | None = None) -> dict:
    """The bit-exact check of the served results on the integer-valued twin of the pool
    (same patterns, values in {-3..3}): every pool request served alone, then every
    arrival served in the mix at the given rate; each result's digest (colptr, rows and
    values weighted by position, exact in int64 / fp64) must equal its alone digest."""
    import threading
    import torch
    from paper_2112_10223_amd import binding
    pool = RequestPool(pool_size, values="int32f")
    sc = dict(SERVER_CONFIG, **(server_config or {}))
    srv = binding.Server(binding.SPKADD_F32, n_streams=sc["n_streams"], max_batch=sc["max_batch"],
                         max_columns=max(sc["max_batch"] * pool.max_n, 1 << 17), max_inputs=sc["max_batch"] * 64,
                         hbm_budget=SERVE_BUDGET, depth=sc["depth"], opts=opts, large_streams=sc["large_streams"])

    side = torch.cuda.Stream()  # (the null stream refuses work while the server's lanes capture)

    def digest(res):
        with torch.cuda.stream(side):
            cp, r, v = srv.outputs(res)
            w = torch.arange(r.numel(), device=r.device, dtype=torch.int64) % 1021 + 1
            wc = torch.arange(cp.numel(), device=cp.device, dtype=torch.int64) % 1019 + 1
            return (int(res["nnz"]), int((cp.to(torch.int64) * wc).sum()), int((r.to(torch.int64) * w).sum()),
                    float((v.to(torch.float64) * w.to(torch.float64)).sum()))

    alone = []
    for q in pool.reqs:
        tk = srv.submit(q["m"], q["colptrs"], q["rowidxs"], q["values"], q["cap_c"])
        res = srv.wait(tk)
        alone.append(digest(res))
        srv.release(tk)
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(picks)))
    tickets = [None] * len(picks)

    def submitter(t0):
        for t, (i, a) in enumerate(zip(picks, arrivals)):
            while time.perf_counter() - t0 < a:
                time.sleep(0)
            q = pool.reqs[i]
            tickets[t] = srv.submit(q["m"], q["colptrs"], q["rowidxs"], q["values"], q["cap_c"])

    th = threading.Thread(target=submitter, args=(time.perf_counter(),))
    th.start()
    same = lanes = 0
    for t, i in enumerate(picks):
        while tickets[t] is None:
            time.sleep(0)
        res = srv.wait(tickets[t])
        lanes += res["path"]
        same += int(digest(res) == alone[i])
        srv.release(tickets[t])
    th.join()
    srv.close()
    del pool
    torch.cuda.empty_cache()
    return {"values": "integer-valued twin of the pool (exact in any summation order)", "arrivals": len(picks),
            "server": sc, "identical_to_alone": same, "differing": len(picks) - same, "one_request_lane": lanes}


def measure_config5(pool_size: int = 1000, arrivals: int = 10000, side_arrivals: int = 2000,
                    tune_sample: int = 250, policy_arrivals: int = 1500) -> dict:
    """The batched / served workload at its stated size: a pool of pool_size requests of
    the unfiltered request distribution (inputs drawn on the device), Poisson arrival
    streams of `arrivals` requests drawn from the pool at load 0.8 (and side_arrivals at
    loads 0.5 and 1.5) with a 64 GB output budget; batched throughput with the default
    and the tuned batch setting (spkadd_tune_batch on a sample of the pool) against one
    plain launch sequence per request; and the bit-exact alone-vs-mix check of every
    arrival at load 0.8 on the pool's integer-valued twin."""
    import torch
    from paper_2112_10223_amd import binding
    t_gen = time.perf_counter()
    pool = RequestPool(pool_size)
    t_gen = time.perf_counter() - t_gen
    plain = PlainRunner(pool)
    stream = binding._stream_ptr(None)
    # one-request service time of every pool request (after one warm pass)
    for q in pool.reqs:
        plain.run(q, stream)
    torch.cuda.synchronize()
    svc = []
    t_all = time.perf_counter()
    for q in pool.reqs:
        t0 = time.perf_counter()
        plain.run(q, stream)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t0)
    t_all = time.perf_counter() - t_all
    mean_svc = float(np.mean(svc))
    big = [q["nnz_in"] > (1 << 24) for q in pool.reqs]
    out = {"pool": {"requests": pool_size, "input_nnz": int(pool.nnz_in), "requests_over_2^24": int(sum(big)),
                    "largest_input_nnz": int(max(q["nnz_in"] for q in pool.reqs)),
                    "generation_s": round(t_gen, 2),
                    "sample": f"the first {pool_size} requests of the unfiltered distribution (k ~ U{{2..64}}, "
                              "m, n log-U[256, 65536], density log-U[1e-4, 1e-2] per matrix, fp32 U(-1,1)), "
                              "drawn on the device; arrivals pick pool requests uniformly"},
           "budget_bytes": SERVE_BUDGET,
           "plain": {"mean_service_ms": round(mean_svc * 1e3, 4), "p99_service_ms": _pct(svc, 99),
                     "nnz_per_s": pool.nnz_in / t_all,
                     "gbps_alg": round(BYTES_PER_INPUT_NNZ * pool.nnz_in / t_all / 1e9, 1)}}
    # batched throughput: default vs tuned
    default = binding.make_opts()
    out["batched_default"] = batched_throughput(pool, plain, default, 40)
    rng = np.random.default_rng(11)
    sample_idx = sorted(rng.choice(pool_size, size=min(tune_sample, pool_size), replace=False).tolist())
    # the tuner's sample, each request with its own outputs (carved from one arena)
    tot = sum(pool.reqs[i]["cap_c"] for i in sample_idx)
    tc = sum(pool.reqs[i]["n"] + 1 for i in sample_idx)
    a_cp = torch.empty(tc, dtype=torch.int32, device="cuda:0")
    a_r = torch.empty(tot, dtype=torch.int32, device="cuda:0")
    a_v = torch.empty(tot, dtype=torch.float32, device="cuda:0")
    sample = []
    oc = oe = 0
    for i in sample_idx:
        q = pool.reqs[i]
        sample.append(dict(m=q["m"], colptrs=q["colptrs"], rowidxs=q["rowidxs"], values=q["values"],
                           colptr_c=a_cp[oc:oc + q["n"] + 1], rowidx_c=a_r[oe:oe + q["cap_c"]],
                           values_c=a_v[oe:oe + q["cap_c"]], cap_c=q["cap_c"]))
        oc += q["n"] + 1
        oe += q["cap_c"]
    best, rep, trials = binding.tune_batch(sample, binding.SPKADD_F32, reps=2)
    del sample, a_cp, a_r, a_v
    torch.cuda.empty_cache()
    out["batch_tuner"] = {"sample_requests": len(sample_idx), "trials": rep["trials"], "failed": rep["failed"],
                          "default_ms": round(rep["default_ms"], 3), "best_ms": round(rep["best_ms"], 3),
                          "best": {f: getattr(best, f) for f in binding.BATCH_TUNED_FIELDS}}
    out["batched_tuned"] = batched_throughput(pool, plain, best, best.batch_run_size)
    out["batched_speedup_tuned_vs_plain"] = round(out["batched_tuned"]["nnz_per_s"] / out["plain"]["nnz_per_s"], 3)
    out["batched_speedup_tuned_vs_default"] = round(out["batched_tuned"]["nnz_per_s"] /
                                                    out["batched_default"]["nnz_per_s"], 3)
    # serving policy: a short stream at load 0.8 through each candidate (batched streams,
    # requests per run, one-request lanes); the lowest p99, then p50, serves the streams
    # measured below
    picks = np.random.default_rng(105).integers(0, pool_size, size=policy_arrivals).tolist()
    sweep = []
    for cand in SERVER_CANDIDATES:
        r = measure_served(pool, plain, picks, mean_svc, 0.8, 5, opts=best, server_config=cand, baselines=False)
        sweep.append({"server": r["server"], "p50_ms": r["served"]["p50_ms"], "p99_ms": r["served"]["p99_ms"]})
    chosen = min(sweep, key=lambda x: (x["p99_ms"], x["p50_ms"]))["server"]
    out["serve_policy"] = {"arrivals": policy_arrivals, "load_vs_plain": 0.8, "sweep": sweep, "chosen": chosen}
    # served
    served = []
    for load, count, seed in ((0.8, arrivals, 7), (0.5, side_arrivals, 8), (1.5, side_arrivals, 9)):
        picks = np.random.default_rng(100 + seed).integers(0, pool_size, size=count).tolist()
        served.append(measure_served(pool, plain, picks, mean_svc, load, seed, opts=best, server_config=chosen))
    out["served"] = served
    del plain, pool
    torch.cuda.empty_cache()
    picks = np.random.default_rng(107).integers(0, pool_size, size=arrivals).tolist()
    out["alone_vs_mix"] = alone_vs_mix(pool_size, picks, 0.8 / mean_svc, 7, opts=best, server_config=chosen)
    return out


def cpu_baseline(batch, max_cols: int | None = None):
    import oracle
    n = batch.n if max_cols is None else min(batch.n, max_cols)
    cols = None if n == batch.n else np.arange(n, dtype=np.int64)
    nnz_in = int(sum(int(batch.colptr[i, n]) for i in range(batch.k)))
    t0 = time.perf_counter()
    oracle.spkadd(batch, cols=cols)
    dt = time.perf_counter() - t0
    return {"value": nnz_in / dt, "unit": "input nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (concatenate, qsort, reduce in long double; one thread) on columns 0..{n - 1} "
                      f"of the same inputs ({nnz_in} input nnz), {dt:.2f} s"}


def cpu_baseline_all_cores(batch):
    """The same oracle over column chunks on every core of the host's share (threads:
    the oracle's C routine runs without the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    threads = max(1, len(os.sched_getaffinity(0)))
    chunks = np.array_split(np.arange(batch.n, dtype=np.int64), threads * 4)
    oracle.spkadd(batch, cols=chunks[0][:1])  # library loaded before timing
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda c: oracle.spkadd(batch, cols=c), chunks))
    dt = time.perf_counter() - t0
    return {"value": batch.nnz_in / dt, "unit": "input nnz/s", "cores": threads, "kind": "oracle",
            "sample": f"the oracle on all {batch.n} columns in {len(chunks)} chunks over {threads} threads, {dt:.2f} s"}


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth: a device-to-device copy of nbytes (read + write),
    best of reps, GB/s."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    return round(2 * nbytes / (best * 1e-3) / 1e9, 1)


def compare_algorithms(m, cps, ris, vas, nnz_out, hash_ms, reps=3):
    """The paper's algorithm comparison on this workload, on the GPU: the hash k-way
    sum (the timed steps above) against the k-way heap merge (Algorithm 3) and the
    2-way tree (Section II-B), each a whole call with its allocations, mean of `reps`
    after one warm-up; nnz(B) checked against the hash result."""
    import torch
    from paper_2112_10223_amd import baselines
    res = {"hash_ms": round(hash_ms, 4)}
    for name, fn in (("heap", baselines.heap_add), ("tree", baselines.tree_add)):
        c, _, _ = fn(m, cps, ris, vas)
        torch.cuda.synchronize()
        ok = int(c[-1].item()) == nnz_out
        t0 = time.perf_counter()
        for _ in range(reps):
            fn(m, cps, ris, vas)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_nnz_agrees"] = ok
        res[f"{name}_over_hash"] = round(ms / hash_ms, 2)
    return res


def reversed_columns(batch):
    """The same matrices with every column's entries in descending row order."""
    import workloads
    rows, vals = [], []
    for i in range(batch.k):
        cp = batch.colptr[i].astype(np.int64)
        lens = np.diff(cp)
        # entry p of column j moves to cp[j] + cp[j+1] - 1 - p
        ends = np.repeat(cp[:-1] + cp[1:] - 1, lens)
        src = ends - np.arange(cp[-1], dtype=np.int64)
        rows.append(np.ascontiguousarray(batch.rowidx[i][src]))
        vals.append(np.ascontiguousarray(batch.vals[i][src]))
    return workloads.CSCBatch(batch.m, batch.n, batch.colptr, rows, vals)


def host_cpu() -> dict:
    """The host the CPU baseline runs on: cores in this process's affinity mask,
    all online cores, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"affinity_cores": len(os.sched_getaffinity(0)), "nproc": os.cpu_count(), "model": model}


def measure_workload(name: str, batch, steps: int, warmup: int, trace_steps: int, trace: bool = True,
                     flags: int = 0, tune: bool = False) -> dict:
    """Times `steps` steps (plan + symbolic + numeric on resident inputs, outputs
    preallocated) of one workload after `warmup` untimed ones; the numeric launches of
    the timed steps carry HIP events (SPKADD_FLAG_TRACE_NUMERIC) for the roofline of
    the dominant kernel, and `trace_steps` more untimed steps trace every launch for
    the phase breakdown."""
    import torch
    from paper_2112_10223_amd import binding
    k, m, n = batch.k, batch.m, batch.n
    f64 = batch.vals[0].dtype == np.float64
    vbytes = 8 if f64 else 4
    dev = torch.device("cuda:0")
    cps = [torch.from_numpy(np.ascontiguousarray(batch.colptr[i])).to(dev) for i in range(k)]
    ris = [torch.from_numpy(r).to(dev) for r in batch.rowidx]
    vas = [torch.from_numpy(v).to(dev) for v in batch.vals]
    dtype = binding.SPKADD_F64 if f64 else binding.SPKADD_F32
    opts = binding.make_opts(flags=flags | (binding.SPKADD_FLAG_TRACE_NUMERIC if trace else 0))
    opts_all = binding.make_opts(flags=flags | binding.SPKADD_FLAG_TRACE)
    tuned = None
    if tune:  # the autotuner on this workload; the timed steps then use its choice
        best, rep, trials = binding.tune(m, cps, ris, vas, dtype, reps=5)
        for o in (opts, opts_all):
            for f in binding.TUNED_FIELDS:
                setattr(o, f, getattr(best, f))
        tuned = {"default_ms": round(rep["default_ms"], 4), "best_ms": round(rep["best_ms"], 4),
                 "trials": rep["trials"], "failed": rep["failed"],
                 "best": {f: getattr(best, f) for f in binding.TUNED_FIELDS},
                 "sweep": [{"changed": {f: v for f, v in t["opts"].items() if v != trials[0]["opts"][f]},
                            "ms": round(t["ms"], 4)} for t in trials]}

    # output sizes: one untimed call
    plan = binding.spkadd_plan(m, n, cps, ris, dtype, opts)
    colptr_c = torch.empty(n + 1, dtype=torch.int32, device=dev)
    nnz_out = binding.spkadd_symbolic(plan, colptr_c)
    stats = binding.spkadd_get_stats(plan)
    plan.free()
    rowidx_c = torch.empty(max(nnz_out, 1), dtype=torch.int32, device=dev)
    vals_c = torch.empty(max(nnz_out, 1), dtype=vas[0].dtype, device=dev)
    nnz_in = batch.nnz_in

    # pointer arrays and the stream handle are marshalled once; every step still
    # runs the whole path on the device
    pcp, pri, pva = binding.PtrArray(cps), binding.PtrArray(ris), binding.PtrArray(vas, non_null=True)
    stream = binding._stream_ptr(None)
    host_s = {"plan": 0.0, "symbolic": 0.0, "numeric": 0.0}
    step_events = []  # (start, end) of each timed step on the launch stream
    collect_steps = [False]

    def step(o):
        if collect_steps[0]:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            step_events.append(ev)
        t_a = time.perf_counter()
        p = binding.spkadd_plan(m, n, pcp, pri, dtype, o, stream)
        t_b = time.perf_counter()
        binding.spkadd_symbolic(p, colptr_c, stream)
        t_c = time.perf_counter()
        binding.spkadd_numeric(p, pva, rowidx_c, vals_c, stream)
        t_d = time.perf_counter()
        host_s["plan"] += t_b - t_a
        host_s["symbolic"] += t_c - t_b
        host_s["numeric"] += t_d - t_c
        if collect_steps[0]:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            step_events.append(ev)
        return p

    def run(nsteps, o, collect):
        """nsteps steps; a plan is freed (after reading its trace) once the next one is
        queued, so no step waits for the previous one to drain."""
        prev, traces = None, []
        for _ in range(nsteps):
            p = step(o)
            if prev is not None:
                if collect:
                    traces.append(binding.spkadd_trace(prev))
                prev.free()
            prev = p
        return prev, traces

    last, _ = run(warmup, opts, False)
    if last is not None:
        last.free()
    torch.cuda.synchronize()
    for kk in host_s:
        host_s[kk] = 0.0
    collect_steps[0] = True
    t0 = time.perf_counter()
    last, traces = run(steps, opts, trace)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    collect_steps[0] = False
    step_ms = [step_events[2 * i].elapsed_time(step_events[2 * i + 1]) for i in range(len(step_events) // 2)]
    step_ms_q = {f"p{q}": round(float(np.percentile(step_ms, q)), 4) for q in (10, 50, 90)} if step_ms else None
    if trace:
        traces.append(binding.spkadd_trace(last))
    last.free()
    ms_per_step = (t1 - t0) * 1e3 / steps
    host_call_ms = {kk: round(v * 1e3 / steps, 4) for kk, v in host_s.items()}

    def mean_by_kernel(trs):
        per = {}
        for tr in trs:
            for kname, ms in tr:
                per.setdefault(kname, []).append(ms)
        return {kname: float(np.mean(v)) for kname, v in per.items()}

    mean_ms = mean_by_kernel(traces)  # numeric launches of the timed steps
    last, tr_all = run(trace_steps, opts_all, True)
    if last is not None:
        tr_all.append(binding.spkadd_trace(last))
        last.free()
    torch.cuda.synchronize()
    all_ms = mean_by_kernel(tr_all)
    phase_ms = {"plan": 0.0, "symbolic": 0.0, "numeric": 0.0}
    for kname, ms in all_ms.items():
        ph = "numeric" if kname.startswith(("num_", "put_ptrs_num", "uwin_gather")) else \
            "symbolic" if kname.startswith(("sym_", "scan", "win_colsum")) else "plan"
        phase_ms[ph] += ms

    # algorithmic bytes of the numeric kernels, per launch
    u = np.zeros(n, dtype=np.int64)
    for i in range(k):
        u += np.diff(batch.colptr[i]).astype(np.int64)
    cnt = np.diff(colptr_c.cpu().numpy().astype(np.int64))
    cap = stats["window_cap"]
    kern = kernel_of_column(u, cap)
    roofline = None
    num_kernels = [kname for kname in mean_ms if kname.startswith("num_") and kname != "num_ordered"]
    if not num_kernels:  # timed without events: fall back to the traced pass
        mean_ms = all_ms
        num_kernels = [kname for kname in mean_ms if kname.startswith("num_") and kname != "num_ordered"]
    if num_kernels:
        dom = max(num_kernels, key=lambda x: mean_ms[x])
        sel = kern == dom
        alg_bytes = int(((4 + vbytes) * (u[sel] + cnt[sel]) + 4 * k + 4).sum())
        achieved = alg_bytes / (mean_ms[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": measured_traffic(dom, name),
                    "alg_bytes_per_launch": alg_bytes, "mean_launch_ms": round(mean_ms[dom], 5),
                    "units_per_launch": int(sel.sum())}

    b_alg = (8 + vbytes) * nnz_in + (4 + vbytes) * nnz_out + 12 * k * (n + 1) + 12 * (n + 1)
    b_min = (4 + vbytes) * (nnz_in + nnz_out) + 4 * (k + 1) * (n + 1)  # every byte read or written once
    rec = {
        "ms_per_step": round(ms_per_step, 4),
        "steps": steps,
        "warmup": warmup,
        "value": nnz_in / (ms_per_step * 1e-3),
        "unit": "input nnz/s",
        "dtype": "f64" if f64 else "f32",
        "k": k, "m": m, "n": n, "nnz_in": nnz_in, "nnz_out": nnz_out,
        "hbm_gbps_alg_step": round(b_alg / (ms_per_step * 1e-3) / 1e9, 1),
        "hbm_frac_alg_step": round(b_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "hbm_gbps_min_step": round(b_min / (ms_per_step * 1e-3) / 1e9, 1),
        "step_ms": step_ms_q,
        "phase_ms": {kk: round(v, 4) for kk, v in phase_ms.items()},
        "host_call_ms": host_call_ms,
        "kernel_ms": {kk: round(v, 5) for kk, v in sorted(all_ms.items())},
        "bins": {kk: stats[kk] for kk in ("n_wave_cols", "n_wg_cols", "n_window_cols", "n_windows")},
        "roofline": roofline,
    }
    if tuned is not None:
        rec["tune"] = tuned
    rec["_device"] = (cps, ris, vas, nnz_out)  # for the algorithm comparison (removed before printing)
    return rec


# the other single-GPU workloads timed beside the headline one: (name, timed steps, warm-up steps)
SUB_WORKLOADS = [("config2_f64", 20, 3), ("config4", 5, 2), ("config3", 3, 2)]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-trace", action="store_true", help="time without per-kernel events")
    ap.add_argument("--trace-steps", type=int, default=3, help="untimed steps with every launch traced")
    ap.add_argument("--tune", action="store_true", help="autotune the launch parameters on the workload first")
    ap.add_argument("--unsorted-in", action="store_true",
                    help="every input column reversed (descending rows), planned with SPKADD_FLAG_UNSORTED_IN")
    ap.add_argument("--unsorted-out", action="store_true",
                    help="rows of each output column in any order (hash accumulators skip their sort)")
    ap.add_argument("--ordered", action="store_true", help="values summed in input order (SPKADD_FLAG_ORDERED)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison with the heap-merge and 2-way-tree baselines")
    ap.add_argument("--served", type=int, default=10000,
                    help="arrivals of the served stream at load 0.8 (0 = skip the batched / served workload)")
    ap.add_argument("--served-pool", type=int, default=1000,
                    help="distinct requests of the served workload (drawn on the device)")
    ap.add_argument("--no-sub", action="store_true",
                    help="time only --workload (not also the fp64, tall-skinny and R-MAT workloads)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched runs of the served pool (runs of 40), e.g. for a kernel trace of the "
                         "runs without the serving threads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the SpKAdd path here is single-GPU.",
              file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration:
        copy_calibration()
        return 0
    from paper_2112_10223_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    if args.batched_only:
        pool = RequestPool(args.served_pool)
        rec = batched_throughput(pool, PlainRunner(pool), binding.make_opts(), 40, reps=1)
        print(json.dumps({"batched_only": rec, "pool_requests": args.served_pool}))
        return 0

    desc, make = WORKLOADS[args.workload]
    batch = make()
    if args.unsorted_in:
        batch = reversed_columns(batch)
    flags = (binding.SPKADD_FLAG_UNSORTED_OUT if args.unsorted_out else 0) | \
        (binding.SPKADD_FLAG_UNSORTED_IN if args.unsorted_in else 0) | \
        (binding.SPKADD_FLAG_ORDERED if args.ordered else 0)
    head = measure_workload(args.workload, batch, args.steps, args.warmup, args.trace_steps, not args.no_trace,
                            flags, args.tune)
    cps, ris, vas, nnz_out = head.pop("_device")
    k, m, n = batch.k, batch.m, batch.n
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "input nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic (seeded generator; paper's R-MAT family, no public datasets)",
        "config": {"workload": f"{args.workload}: {desc}", "k": k, "m": m, "n": n, "nnz_in": batch.nnz_in,
                   "nnz_out": nnz_out, "parallelism": "single GPU",
                   "output_order": "any" if args.unsorted_out else "sorted",
                   "input_order": "descending (reversed columns)" if args.unsorted_in else "ascending",
                   "summation": "input order" if args.ordered else "any order"},
    }
    for key in ("hbm_gbps_alg_step", "hbm_frac_alg_step", "hbm_gbps_min_step", "step_ms"):
        out[key] = head[key]
    out["copy_gbps"] = copy_bandwidth()
    for key in ("phase_ms", "host_call_ms", "kernel_ms", "bins", "roofline"):
        out[key] = head[key]
    out["cpu_baseline"] = None
    if "tune" in head:
        out["tune"] = head["tune"]
    if not args.no_compare and not args.unsorted_in and k <= 128:
        out["algorithms"] = compare_algorithms(m, cps, ris, vas, nnz_out, head["ms_per_step"])
    if not args.no_cpu_baseline:
        out["cpu_host"] = host_cpu()
        out["cpu_baseline"] = cpu_baseline(batch)
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(batch)
    del cps, ris, vas, batch
    torch.cuda.empty_cache()
    if args.served > 0:
        out["config5"] = measure_config5(pool_size=args.served_pool, arrivals=args.served)
        torch.cuda.empty_cache()
    if not args.no_sub and not (args.unsorted_in or args.unsorted_out or args.ordered or args.tune):
        subs = {}
        for wname, wsteps, wwarm in SUB_WORKLOADS:
            if wname == args.workload:
                continue
            wdesc, wmake = WORKLOADS[wname]
            wb = wmake()
            rec = measure_workload(wname, wb, wsteps, wwarm, 1)
            rec.pop("_device")
            rec["workload"] = f"{wname}: {wdesc}"
            for key in ("host_call_ms", "kernel_ms", "step_ms"):
                rec.pop(key, None)
            subs[wname] = rec
            del wb
            torch.cuda.empty_cache()
        out["workloads"] = subs
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
