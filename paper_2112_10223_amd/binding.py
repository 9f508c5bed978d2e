"""ctypes binding of the SpKAdd C ABI (include/spkadd.h).

This layer only marshals arguments: torch device tensors are turned into raw
pointers and the current torch stream into a hipStream_t.  Every step of the
computation runs in the HIP kernels of libspkadd.so.  If the library has not been
built, importing the binding raises; nothing falls back to a CPU path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspkadd.so")

SPKADD_OK, SPKADD_ERR_INVALID, SPKADD_ERR_OOM, SPKADD_ERR_HIP, SPKADD_ERR_STATE, SPKADD_ERR_OVERFLOW, \
    SPKADD_ERR_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "OOM", 3: "HIP", 4: "STATE", 5: "OVERFLOW", 6: "UNSUPPORTED"}
SPKADD_F32, SPKADD_F64 = 0, 1
SPKADD_FLAG_VALIDATE, SPKADD_FLAG_TRACE, SPKADD_FLAG_TRACE_NUMERIC, SPKADD_FLAG_UNSORTED_OUT = 1, 2, 4, 8
SPKADD_FLAG_UNSORTED_IN = 16
SPKADD_FLAG_ORDERED = 32
SPKADD_BIN_AUTO, SPKADD_BIN_WAVE, SPKADD_BIN_WG, SPKADD_BIN_WINDOW = -1, 0, 1, 2
SPKADD_ACCUM_AUTO, SPKADD_ACCUM_HASH, SPKADD_ACCUM_BITMAP = 0, 1, 2
SPKADD_REQ_OK, SPKADD_REQ_TOO_LARGE, SPKADD_REQ_CAPACITY = 0, 1, 2


class SpkaddError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"SPKADD_ERR_{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("force_bin", ctypes.c_int32), ("window_cap", ctypes.c_int32),
                ("hash_mode", ctypes.c_int32), ("wave_max", ctypes.c_int32), ("load_factor_sym", ctypes.c_float),
                ("load_factor_num", ctypes.c_float), ("window_fill", ctypes.c_float),
                ("accum_mode", ctypes.c_int32), ("bitmap_ratio", ctypes.c_float), ("wave_merge", ctypes.c_int32),
                ("batch_fused_cols", ctypes.c_int32), ("batch_wave_max", ctypes.c_int32),
                ("batch_wg_max", ctypes.c_int32), ("batch_wg_threads", ctypes.c_int32),
                ("batch_run_size", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("nnz_in", ctypes.c_int64), ("nnz_out", ctypes.c_int64), ("n_empty_cols", ctypes.c_int32),
                ("n_wave_cols", ctypes.c_int32), ("n_wg_cols", ctypes.c_int32), ("n_window_cols", ctypes.c_int32),
                ("n_windows", ctypes.c_int32), ("window_levels", ctypes.c_int32), ("window_cap", ctypes.c_int32),
                ("wave_max", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("colptr_c", ctypes.c_void_p), ("rowidx_c", ctypes.c_void_p), ("values_c", ctypes.c_void_p),
                ("cap_c", ctypes.c_int64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("graphs_captured", ctypes.c_int32), ("graph_replays", ctypes.c_int32),
                ("kernels_per_run", ctypes.c_int32), ("graph_reuses", ctypes.c_int32),
                ("fused_runs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def declared_functions():
    """Names of the functions declared in include/*.h (for the export check)."""
    import re
    inc = os.path.join(os.path.dirname(HERE), "include")
    names = []
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(spkadd_[a-z0-9_]+)\s*\(", text,
                                flags=re.M)
    return sorted(set(names))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.spkadd_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.spkadd_opts_default.restype = None
        L.spkadd_plan.argtypes = [ctypes.POINTER(P), I32, I32, I32, P, P, ctypes.c_int, ctypes.POINTER(Opts), P]
        L.spkadd_plan.restype = ctypes.c_int
        L.spkadd_symbolic.argtypes = [P, P, ctypes.POINTER(I64), P]
        L.spkadd_symbolic.restype = ctypes.c_int
        L.spkadd_numeric.argtypes = [P, P, P, P, P]
        L.spkadd_numeric.restype = ctypes.c_int
        L.spkadd_free.argtypes = [P]
        L.spkadd_free.restype = ctypes.c_int
        L.spkadd_last_error.argtypes = []
        L.spkadd_last_error.restype = ctypes.c_char_p
        L.spkadd_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.spkadd_get_stats.restype = ctypes.c_int
        L.spkadd_trace_count.argtypes = [P]
        L.spkadd_trace_count.restype = I32
        L.spkadd_trace_get.argtypes = [P, I32, ctypes.c_char_p, I32, ctypes.POINTER(ctypes.c_float)]
        L.spkadd_trace_get.restype = ctypes.c_int
        L.spkadd_trace_reset.argtypes = [P]
        L.spkadd_trace_reset.restype = ctypes.c_int
        L.spkadd_sum_noalloc.argtypes = [I32, I32, I32, P, P, P, ctypes.c_int, ctypes.POINTER(Opts), P, P, P, I64,
                                         ctypes.POINTER(I64), P]
        L.spkadd_sum_noalloc.restype = ctypes.c_int
        L.spkadd_batch_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, I32, I64, I64, ctypes.POINTER(Opts)]
        L.spkadd_batch_create.restype = ctypes.c_int
        L.spkadd_batch_run.argtypes = [P, ctypes.POINTER(Request), I32, I32, P]
        L.spkadd_batch_run.restype = ctypes.c_int
        L.spkadd_batch_results.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I32)]
        L.spkadd_batch_results.restype = ctypes.c_int
        L.spkadd_batch_get_info.argtypes = [P, ctypes.POINTER(BatchInfo)]
        L.spkadd_batch_get_info.restype = ctypes.c_int
        L.spkadd_batch_destroy.argtypes = [P]
        L.spkadd_batch_destroy.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != SPKADD_OK:
        raise SpkaddError(status, lib().spkadd_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if isinstance(stream, ctypes.c_void_p):
        return stream
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


class PtrArray:
    """A host array of device pointers built once from k tensors, for callers that
    pass the same inputs many times.  Keeps the tensors alive.  With
    non_null=True, pointers of empty tensors (which torch reports as 0) are replaced
    by another input's pointer; they are never read through."""

    def __init__(self, tensors, non_null: bool = False, fallback: int = 0):
        self.tensors = list(tensors)
        ptrs = [t.data_ptr() if t is not None else 0 for t in self.tensors]
        if non_null:
            fill = next((q for q in ptrs if q), fallback)
            ptrs = [q or fill for q in ptrs]
        self.arr = (ctypes.c_void_p * len(ptrs))(*ptrs)

    def __len__(self):
        return len(self.tensors)


def _ptr_array(tensors, non_null: bool = False):
    if isinstance(tensors, PtrArray):
        return tensors.arr
    return PtrArray(tensors, non_null).arr


def make_opts(**kw) -> Opts:
    o = Opts()
    lib().spkadd_opts_default(ctypes.byref(o))
    for key, val in kw.items():
        if val is not None:
            setattr(o, key, val)
    return o


class Plan:
    """Owning handle of an spkadd_plan_t."""

    def __init__(self, handle, m, n, k, dtype):
        self.handle = handle
        self.m, self.n, self.k, self.dtype = m, n, k, dtype
        self.nnz = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self.handle:
            lib().spkadd_free(self.handle)
            self.handle = None


def spkadd_plan(m, n, colptrs, rowidxs, dtype=SPKADD_F32, opts: Opts | None = None, stream=None) -> Plan:
    """colptrs / rowidxs: k int32 device tensors each (torch), or PtrArray objects.
    stream: a torch stream, a raw hipStream_t (int or ctypes.c_void_p), or None for
    torch's current stream."""
    k = len(colptrs)
    h = ctypes.c_void_p()
    cp = _ptr_array(colptrs)
    ri = _ptr_array(rowidxs)
    _check(lib().spkadd_plan(ctypes.byref(h), m, n, k, ctypes.cast(cp, ctypes.c_void_p),
                             ctypes.cast(ri, ctypes.c_void_p), dtype,
                             ctypes.byref(opts) if opts is not None else None, _stream_ptr(stream)))
    return Plan(h, m, n, k, dtype)


def spkadd_symbolic(plan: Plan, colptr_c, stream=None) -> int:
    nnz = ctypes.c_int64()
    _check(lib().spkadd_symbolic(plan.handle, colptr_c.data_ptr(), ctypes.byref(nnz), _stream_ptr(stream)))
    plan.nnz = int(nnz.value)
    return plan.nnz


def spkadd_numeric(plan: Plan, values, rowidx_c, values_c, stream=None) -> None:
    va = _ptr_array(values, non_null=True)
    _check(lib().spkadd_numeric(plan.handle, ctypes.cast(va, ctypes.c_void_p),
                                rowidx_c.data_ptr() if rowidx_c is not None else None,
                                values_c.data_ptr() if values_c is not None else None, _stream_ptr(stream)))


def spkadd_free(plan: Plan) -> None:
    plan.free()


def spkadd_get_stats(plan: Plan) -> dict:
    s = Stats()
    _check(lib().spkadd_get_stats(plan.handle, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in Stats._fields_}


def spkadd_trace(plan: Plan, reset: bool = True) -> list:
    """[(kernel name, ms)] of the launches recorded under SPKADD_FLAG_TRACE."""
    out = []
    buf = ctypes.create_string_buffer(64)
    ms = ctypes.c_float()
    for i in range(lib().spkadd_trace_count(plan.handle)):
        _check(lib().spkadd_trace_get(plan.handle, i, buf, 64, ctypes.byref(ms)))
        out.append((buf.value.decode(), float(ms.value)))
    if reset:
        lib().spkadd_trace_reset(plan.handle)
    return out


def spkadd(m, colptrs, rowidxs, values, opts: Opts | None = None, stream=None):
    """B = A_1 + ... + A_k on the device: plan, symbolic, numeric, free.

    Inputs are k-lists of device tensors (int32 colptr[n+1], int32 rowidx, float32 or
    float64 values).  Returns (colptr, rowidx, values) of B as device tensors."""
    import contextlib
    import torch
    n = colptrs[0].shape[0] - 1
    dtype = SPKADD_F64 if values[0].dtype == torch.float64 else SPKADD_F32
    dev = colptrs[0].device
    # the outputs are allocated on the stream the work runs on, so that torch's caching
    # allocator does not hand their memory (or, once they are dropped, that of a
    # running sum fed back as an input) to other work before this stream reaches it
    ctx = contextlib.nullcontext()
    if stream is not None and not isinstance(stream, torch.cuda.Stream):
        raw = stream.value if isinstance(stream, ctypes.c_void_p) else int(stream)
        stream = torch.cuda.ExternalStream(raw, device=dev) if raw else None
    if stream is not None and stream != torch.cuda.current_stream(dev):
        ctx = torch.cuda.stream(stream)
    plan = spkadd_plan(m, n, colptrs, rowidxs, dtype, opts, stream)
    try:
        with ctx:
            colptr_c = torch.empty(n + 1, dtype=torch.int32, device=dev)
            nnz = spkadd_symbolic(plan, colptr_c, stream)
            rowidx_c = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)[:nnz]
            values_c = torch.empty(max(nnz, 1), dtype=values[0].dtype, device=dev)[:nnz]
        spkadd_numeric(plan, values, rowidx_c, values_c, stream)
    finally:
        plan.free()
    return colptr_c, rowidx_c, values_c


SPKADD_NOALLOC_SCRATCH_BYTES = 64 << 20


def spkadd_sum_noalloc(m, colptrs, rowidxs, values, colptr_c, rowidx_c, values_c, opts: Opts | None = None,
                       stream=None) -> int:
    """The no-allocation entry point: plan, symbolic and numeric in one call, the
    device workspace in the library's static scratch array.  The caller's output
    tensors hold colptr(B) (n + 1) and up to len(rowidx_c) entries.  Returns nnz(B)."""
    import torch
    k = len(colptrs)
    n = int(colptrs[0].shape[0]) - 1
    dtype = SPKADD_F64 if values[0].dtype == torch.float64 else SPKADD_F32
    cp = _ptr_array(colptrs)
    ri = _ptr_array(rowidxs)
    va = _ptr_array(values, non_null=True)
    cap = int(rowidx_c.shape[0])
    if int(values_c.shape[0]) < cap or int(colptr_c.shape[0]) != n + 1:
        raise ValueError("output tensors do not match n and the capacity")
    nnz = ctypes.c_int64(-1)
    _check(lib().spkadd_sum_noalloc(m, n, k, ctypes.cast(cp, ctypes.c_void_p), ctypes.cast(ri, ctypes.c_void_p),
                                    ctypes.cast(va, ctypes.c_void_p), dtype,
                                    ctypes.byref(opts) if opts is not None else None, colptr_c.data_ptr(),
                                    rowidx_c.data_ptr() if cap else None, values_c.data_ptr() if cap else None,
                                    cap, ctypes.byref(nnz), _stream_ptr(stream)))
    return int(nnz.value)


def request_array(requests):
    """(ctypes array of spkadd_request, objects to keep alive) from request dicts: m,
    colptrs, rowidxs, values (k device tensors or PtrArray each), colptr_c, rowidx_c,
    values_c (device tensors) and cap_c."""
    arr = (Request * len(requests))()
    keep = []
    for r, q in enumerate(requests):
        # inputs without entries still need a device pointer (never read through)
        fb = q["colptr_c"].data_ptr()
        cps = q["colptrs"] if isinstance(q["colptrs"], PtrArray) else PtrArray(q["colptrs"], True, fb)
        ris = q["rowidxs"] if isinstance(q["rowidxs"], PtrArray) else PtrArray(q["rowidxs"], True, fb)
        vas = q["values"] if isinstance(q["values"], PtrArray) else PtrArray(q["values"], True, fb)
        keep += [cps, ris, vas, q["colptr_c"], q["rowidx_c"], q["values_c"]]
        n = q["colptr_c"].shape[0] - 1
        arr[r] = Request(q["m"], n, len(cps), ctypes.cast(cps.arr, ctypes.c_void_p).value,
                         ctypes.cast(ris.arr, ctypes.c_void_p).value, ctypes.cast(vas.arr, ctypes.c_void_p).value,
                         q["colptr_c"].data_ptr(), q["rowidx_c"].data_ptr() or None,
                         q["values_c"].data_ptr() or None, int(q["cap_c"]))
    return arr, keep


class Batch:
    """Owning handle of an spkadd_batch_t (include/spkadd_batch.h).

    run() takes a list of requests, each a dict with m, colptrs, rowidxs, values (k
    device tensors or PtrArray each), colptr_c, rowidx_c, values_c (device tensors)
    and cap_c.  The pointer arrays are kept alive until the next run."""

    def __init__(self, dtype, max_requests, max_columns, max_inputs, opts: Opts | None = None):
        h = ctypes.c_void_p()
        _check(lib().spkadd_batch_create(ctypes.byref(h), dtype, max_requests, max_columns, max_inputs,
                                         ctypes.byref(opts) if opts is not None else None))
        self.handle = h
        self._keep = []
        self.nreq = 0

    def run(self, requests, use_graph: bool = True, stream=None) -> None:
        arr, keep = request_array(requests)
        _check(lib().spkadd_batch_run(self.handle, arr, len(requests), 1 if use_graph else 0, _stream_ptr(stream)))
        self._keep = keep
        self.nreq = len(requests)

    def results(self):
        nnz = (ctypes.c_int64 * self.nreq)()
        st = (ctypes.c_int32 * self.nreq)()
        _check(lib().spkadd_batch_results(self.handle, nnz, st))
        return list(nnz), list(st)

    def info(self) -> dict:
        i = BatchInfo()
        _check(lib().spkadd_batch_get_info(self.handle, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in BatchInfo._fields_}

    def close(self):
        if self.handle:
            lib().spkadd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SPKADD_REQ_ERROR = 3


class ServerConfig(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("large_streams", ctypes.c_int32), ("max_columns", ctypes.c_int64),
                ("max_inputs", ctypes.c_int64), ("hbm_budget", ctypes.c_uint64),
                ("opts", ctypes.POINTER(Opts))]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("error", ctypes.c_int32), ("path", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("nnz", ctypes.c_int64), ("colptr_c", ctypes.c_void_p),
                ("rowidx_c", ctypes.c_void_p), ("values_c", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_int64), ("batched", ctypes.c_int64), ("large", ctypes.c_int64),
                ("allocations", ctypes.c_int64), ("held_bytes", ctypes.c_uint64), ("pooled_bytes", ctypes.c_uint64),
                ("graphs_captured", ctypes.c_int32), ("graph_reuses", ctypes.c_int32)]


def _server_fns():
    L = lib()
    if not hasattr(L, "_server_bound"):
        P = ctypes.c_void_p
        L.spkadd_server_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(ServerConfig)]
        L.spkadd_server_create.restype = ctypes.c_int
        L.spkadd_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.spkadd_server_submit.restype = ctypes.c_int
        L.spkadd_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result), ctypes.c_double]
        L.spkadd_server_wait.restype = ctypes.c_int
        L.spkadd_server_release.argtypes = [P, ctypes.c_uint64]
        L.spkadd_server_release.restype = ctypes.c_int
        L.spkadd_server_now.argtypes = [P]
        L.spkadd_server_now.restype = ctypes.c_double
        L.spkadd_server_get_info.argtypes = [P, ctypes.POINTER(ServerInfo)]
        L.spkadd_server_get_info.restype = ctypes.c_int
        L.spkadd_server_destroy.argtypes = [P]
        L.spkadd_server_destroy.restype = ctypes.c_int
        L.spkadd_batch_ready.argtypes = [P]
        L.spkadd_batch_ready.restype = ctypes.c_int32
        L._server_bound = True
    return L


_hip = None


def _hip_runtime():
    """The HIP runtime library (for copies out of server-owned device memory)."""
    global _hip
    if _hip is None:
        import torch  # noqa: F401  (loads the runtime torch was built with)
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
        _hip.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        _hip.hipStreamCreateWithFlags.restype = ctypes.c_int
        _hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipStreamSynchronize.restype = ctypes.c_int
    return _hip


class Server:
    """Owning handle of an spkadd_server_t (include/spkadd_server.h)."""

    def __init__(self, dtype=SPKADD_F32, n_streams=1, max_batch=8, max_columns=1 << 20, max_inputs=1 << 14,
                 hbm_budget=64 << 30, opts: Opts | None = None, depth=1, large_streams=0):
        L = _server_fns()
        self._opts = opts
        cfg = ServerConfig(dtype, n_streams, max_batch, depth, large_streams, max_columns, max_inputs, hbm_budget,
                           ctypes.pointer(opts) if opts is not None else None)
        h = ctypes.c_void_p()
        _check(L.spkadd_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self.handle = h
        self.dtype = dtype
        self._keep = {}

    def now(self) -> float:
        return _server_fns().spkadd_server_now(self.handle)

    def submit(self, m, colptrs, rowidxs, values, cap) -> int:
        """k device tensors (or PtrArray) each; cap = output capacity in entries."""
        import torch
        fb = 0
        for t in (colptrs.tensors if isinstance(colptrs, PtrArray) else list(colptrs)):
            if isinstance(t, torch.Tensor) and t.data_ptr():
                fb = t.data_ptr()
                break
        cps = colptrs if isinstance(colptrs, PtrArray) else PtrArray(colptrs, True, fb)
        ris = rowidxs if isinstance(rowidxs, PtrArray) else PtrArray(rowidxs, True, fb)
        vas = values if isinstance(values, PtrArray) else PtrArray(values, True, fb)
        n = (colptrs.tensors[0] if isinstance(colptrs, PtrArray) else colptrs[0]).shape[0] - 1
        req = Request(m, n, len(cps), ctypes.cast(cps.arr, ctypes.c_void_p).value,
                      ctypes.cast(ris.arr, ctypes.c_void_p).value, ctypes.cast(vas.arr, ctypes.c_void_p).value,
                      None, None, None, int(cap))
        tk = ctypes.c_uint64()
        _check(_server_fns().spkadd_server_submit(self.handle, ctypes.byref(req), ctypes.byref(tk)))
        self._keep[tk.value] = (cps, ris, vas, n)
        return tk.value

    def wait(self, ticket: int, timeout: float = -1.0) -> dict:
        r = Result()
        _check(_server_fns().spkadd_server_wait(self.handle, ticket, ctypes.byref(r), timeout))
        out = {name: getattr(r, name) for name, _ in Result._fields_}
        out["n"] = self._keep[ticket][3]
        return out

    def outputs(self, res: dict):
        """Copies of a completed ticket's colptr(B), rows and values (torch, device),
        made on torch's current stream, which is synchronised before returning (the
        ticket's arrays may be reused once it is released).  While the server's threads
        capture graphs, the legacy (null) stream refuses work: call this under a
        torch.cuda.stream of its own."""
        import torch
        n, z = res["n"], max(res["nnz"], 0)
        vdt = torch.float64 if self.dtype == SPKADD_F64 else torch.float32
        cp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        r = torch.empty(max(z, 1), dtype=torch.int32, device="cuda")[:z]
        v = torch.empty(max(z, 1), dtype=vdt, device="cuda")[:z]
        hip = _hip_runtime()
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        for dst, src, nbytes in ((cp, res["colptr_c"], 4 * (n + 1)), (r, res["rowidx_c"], 4 * z),
                                 (v, res["values_c"], v.element_size() * z)):
            if nbytes:
                err = hip.hipMemcpyAsync(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src), ctypes.c_size_t(nbytes),
                                         3, st)
                if err != 0:
                    raise RuntimeError(f"hipMemcpyAsync failed: {err}")
        err = hip.hipStreamSynchronize(st)
        if err != 0:
            raise RuntimeError(f"hipStreamSynchronize failed: {err}")
        return cp, r, v

    def info(self) -> dict:
        i = ServerInfo()
        _check(_server_fns().spkadd_server_get_info(self.handle, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in ServerInfo._fields_}

    def release(self, ticket: int) -> None:
        _check(_server_fns().spkadd_server_release(self.handle, ticket))
        self._keep.pop(ticket, None)

    def close(self):
        if self.handle:
            _server_fns().spkadd_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- autotuner (include/spkadd_tune.h) ----

class TuneKey(ctypes.Structure):
    _fields_ = [("arch", ctypes.c_char * 64), ("cus", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("m_log2", ctypes.c_int32), ("n_log2", ctypes.c_int32), ("k_log2", ctypes.c_int32),
                ("u_log2", ctypes.c_int32), ("kind", ctypes.c_int32)]


class TuneTrial(ctypes.Structure):
    _fields_ = [("opts", Opts), ("ms", ctypes.c_double), ("status", ctypes.c_int32), ("same_colptr", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int32), ("failed", ctypes.c_int32), ("default_ms", ctypes.c_double),
                ("best_ms", ctypes.c_double), ("key", TuneKey)]


TUNED_FIELDS = ("wave_max", "accum_mode", "bitmap_ratio", "wave_merge", "load_factor_sym", "load_factor_num",
                "window_cap", "window_fill")
BATCH_TUNED_FIELDS = ("accum_mode", "bitmap_ratio", "batch_fused_cols", "batch_wave_max", "batch_wg_max",
                      "batch_wg_threads", "batch_run_size")


def _tune_fns():
    L = lib()
    if not hasattr(L, "_tune_bound"):
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.spkadd_tune_key_for.argtypes = [I32, I32, I32, I64, ctypes.c_int, ctypes.POINTER(TuneKey)]
        L.spkadd_tune_key_for.restype = ctypes.c_int
        L.spkadd_tune.argtypes = [I32, I32, I32, P, P, P, ctypes.c_int, ctypes.POINTER(Opts), I32,
                                  ctypes.POINTER(Opts), ctypes.POINTER(TuneReport), ctypes.POINTER(TuneTrial), I32, P]
        L.spkadd_tune.restype = ctypes.c_int
        L.spkadd_tune_lookup.argtypes = [ctypes.POINTER(TuneKey), ctypes.POINTER(Opts), ctypes.POINTER(I32)]
        L.spkadd_tune_lookup.restype = ctypes.c_int
        L.spkadd_tune_store.argtypes = [ctypes.POINTER(TuneKey), ctypes.POINTER(Opts), ctypes.c_double]
        L.spkadd_tune_store.restype = ctypes.c_int
        L.spkadd_tune_size.argtypes = []
        L.spkadd_tune_size.restype = I32
        L.spkadd_tune_save.argtypes = [ctypes.c_char_p]
        L.spkadd_tune_save.restype = ctypes.c_int
        L.spkadd_tune_load.argtypes = [ctypes.c_char_p]
        L.spkadd_tune_load.restype = ctypes.c_int
        L.spkadd_tune_clear.argtypes = []
        L.spkadd_tune_clear.restype = None
        L.spkadd_tune_key_for_batch.argtypes = [I32, I64, I64, I64, I64, ctypes.c_int, ctypes.POINTER(TuneKey)]
        L.spkadd_tune_key_for_batch.restype = ctypes.c_int
        L.spkadd_tune_batch.argtypes = [ctypes.POINTER(Request), I32, ctypes.c_int, ctypes.POINTER(Opts), I32,
                                        ctypes.POINTER(Opts), ctypes.POINTER(TuneReport), ctypes.POINTER(TuneTrial),
                                        I32, P]
        L.spkadd_tune_batch.restype = ctypes.c_int
        L._tune_bound = True
    return L


def opts_dict(o: Opts) -> dict:
    return {name: getattr(o, name) for name, _ in Opts._fields_}


def tune_key(m, n, k, nnz_in, dtype=SPKADD_F32, arch=None, cus=None) -> TuneKey:
    """The shape class of an SpKAdd; on the current device unless arch and cus are given
    (then computed here with the same rule, without a device)."""
    if arch is None or cus is None:
        key = TuneKey()
        _check(_tune_fns().spkadd_tune_key_for(m, n, k, nnz_in, dtype, ctypes.byref(key)))
        return key

    def clog2(x):
        return 0 if x <= 1 else int(x - 1).bit_length()
    u = (nnz_in + n - 1) // n if n > 0 else 0
    return TuneKey(arch.encode(), cus, dtype, clog2(m), clog2(n), clog2(k), clog2(u) if n > 0 else 0, 0)


def tune_key_batch(nreq, sum_m, sum_n, sum_k, nnz_in, dtype=SPKADD_F32) -> TuneKey:
    """The shape class (kind 1) of a set of batched requests on the current device."""
    key = TuneKey()
    _check(_tune_fns().spkadd_tune_key_for_batch(nreq, sum_m, sum_n, sum_k, nnz_in, dtype, ctypes.byref(key)))
    return key


def tune_batch(requests, dtype=SPKADD_F32, base: Opts | None = None, reps=3, stream=None, max_trials=64):
    """Runs the batched-path tuner on a sample of requests (dicts as Batch.run takes);
    returns (best Opts, report dict, [trial dicts])."""
    arr, keep = request_array(requests)
    best = Opts()
    rep = TuneReport()
    trials = (TuneTrial * max_trials)()
    _check(_tune_fns().spkadd_tune_batch(arr, len(requests), dtype, ctypes.byref(base) if base is not None else None,
                                         reps, ctypes.byref(best), ctypes.byref(rep), trials, max_trials,
                                         _stream_ptr(stream)))
    del keep
    report = {"trials": rep.trials, "failed": rep.failed, "default_ms": rep.default_ms, "best_ms": rep.best_ms,
              "key": {name: (getattr(rep.key, name).decode() if name == "arch" else getattr(rep.key, name))
                      for name, _ in TuneKey._fields_}}
    out = []
    for t in trials[:min(rep.trials, max_trials)]:
        out.append({"opts": {f: getattr(t.opts, f) for f in BATCH_TUNED_FIELDS}, "ms": t.ms, "status": t.status,
                    "same_nnz": bool(t.same_colptr)})
    return best, report, out


def tune(m, colptrs, rowidxs, values, dtype=SPKADD_F32, base: Opts | None = None, reps=5, stream=None,
         max_trials=64):
    """Runs the tuner on these inputs; returns (best Opts, report dict, [trial dicts])."""
    n = colptrs[0].shape[0] - 1
    cp = _ptr_array(colptrs)
    ri = _ptr_array(rowidxs)
    va = _ptr_array(values, non_null=True)
    best = Opts()
    rep = TuneReport()
    trials = (TuneTrial * max_trials)()
    _check(_tune_fns().spkadd_tune(m, n, len(colptrs), ctypes.cast(cp, ctypes.c_void_p),
                                   ctypes.cast(ri, ctypes.c_void_p), ctypes.cast(va, ctypes.c_void_p), dtype,
                                   ctypes.byref(base) if base is not None else None, reps, ctypes.byref(best),
                                   ctypes.byref(rep), trials, max_trials, _stream_ptr(stream)))
    report = {"trials": rep.trials, "failed": rep.failed, "default_ms": rep.default_ms, "best_ms": rep.best_ms,
              "key": {name: (getattr(rep.key, name).decode() if name == "arch" else getattr(rep.key, name))
                      for name, _ in TuneKey._fields_}}
    out = []
    for t in trials[:min(rep.trials, max_trials)]:
        out.append({"opts": {f: getattr(t.opts, f) for f in TUNED_FIELDS}, "ms": t.ms, "status": t.status,
                    "same_colptr": bool(t.same_colptr)})
    return best, report, out


def tune_lookup(key: TuneKey, opts: Opts | None = None):
    """Opts with the cached setting of key applied (a copy of opts, or the defaults),
    or None when the cache has no entry."""
    o = Opts()
    if opts is None:
        lib().spkadd_opts_default(ctypes.byref(o))
    else:
        ctypes.pointer(o)[0] = opts
    found = ctypes.c_int32()
    _check(_tune_fns().spkadd_tune_lookup(ctypes.byref(key), ctypes.byref(o), ctypes.byref(found)))
    return o if found.value else None


def tune_store(key: TuneKey, opts: Opts, ms: float = -1.0) -> None:
    _check(_tune_fns().spkadd_tune_store(ctypes.byref(key), ctypes.byref(opts), ms))


def tune_size() -> int:
    return _tune_fns().spkadd_tune_size()


def tune_save(path: str) -> None:
    _check(_tune_fns().spkadd_tune_save(os.fsencode(path)))


def tune_load(path: str) -> None:
    _check(_tune_fns().spkadd_tune_load(os.fsencode(path)))


def tune_clear() -> None:
    _tune_fns().spkadd_tune_clear()
