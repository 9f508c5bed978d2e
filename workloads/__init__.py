"""Seeded synthetic CSC inputs for SpKAdd (shared by the GPU tests and the CPU oracle).

The C module ``gen.c`` draws the sparsity patterns and values.  This module holds
none of the method's arithmetic.  The recipes follow the paper's generator family
(R-MAT, Section IV-A):

* ``er``   -- each column holds c distinct uniformly drawn rows, with c ~ Poisson(d)
  or a fixed count.  This is the Erdos-Renyi pattern (R-MAT a=b=c=d=1/4) restricted
  to one column.
* ``rmat`` -- k independent R-MAT matrices (a, b, c, d).  Duplicate edges of a
  matrix are removed, and no vertex permutation is applied.

Every batch is k matrices of the same shape m x n in CSC form.  A batch holds
int32 colptr (k, n+1), a list of int32 row arrays (rows strictly ascending in each
column) and a list of value arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgen.so")
_lib = None

SEED = 211210223

VALUE_KINDS = {
    "f32": 0,      # fp32 U(-1,1) on the 2^-23 grid
    "f64": 1,      # fp64 U(-1,1) on the 2^-52 grid
    "int32f": 2,   # fp32 integers in {-3..3}
    "normal": 3,   # fp32 N(0,1)
    "int64f": 4,   # fp64 integers in {-3..3}
    "pos": 5,      # fp32 U(0,1] on the 2^-23 grid
}
VALUE_DTYPES = {0: np.float32, 1: np.float64, 2: np.float32, 3: np.float32, 4: np.float64, 5: np.float32}


def build_lib(force: bool = False) -> str:
    """Compile gen.c into libgen.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "gen.c"), "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gen_er_counts.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_int64, P, P]
        lib.gen_er_counts.restype = ctypes.c_int
        lib.gen_er_fill.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int64, P, P, P, ctypes.c_int32]
        lib.gen_er_fill.restype = ctypes.c_int
        lib.gen_rmat.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int32, P, P, P,
                                 ctypes.c_int32, P]
        lib.gen_rmat.restype = ctypes.c_int
        lib.gen_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P]
        lib.gen_uniform.restype = None
        _lib = lib
    return _lib


@dataclass
class CSCBatch:
    """k same-shape CSC matrices on the host."""

    m: int
    n: int
    colptr: np.ndarray                 # int32 (k, n+1)
    rowidx: list                       # k int32 arrays
    vals: list = field(default_factory=list)  # k value arrays (float32 or float64)

    @property
    def k(self) -> int:
        return len(self.rowidx)

    @property
    def nnz(self) -> list:
        return [int(r.shape[0]) for r in self.rowidx]

    @property
    def nnz_in(self) -> int:
        return int(sum(self.nnz))

    @property
    def dtype(self):
        return self.vals[0].dtype if self.vals else None

    def select(self, idx) -> "CSCBatch":
        """The sub-batch of the inputs listed in idx (same order)."""
        return CSCBatch(self.m, self.n, self.colptr[list(idx)].copy(),
                        [self.rowidx[i] for i in idx], [self.vals[i] for i in idx] if self.vals else [])

    def column(self, i: int, j: int):
        """(rows, vals) of column j of input i."""
        s, e = int(self.colptr[i, j]), int(self.colptr[i, j + 1])
        return self.rowidx[i][s:e], (self.vals[i][s:e] if self.vals else None)

    def astype(self, dtype) -> "CSCBatch":
        return CSCBatch(self.m, self.n, self.colptr, self.rowidx, [v.astype(dtype) for v in self.vals])


def _ptrs(arrays):
    return (ctypes.c_void_p * len(arrays))(*[a.ctypes.data for a in arrays])


def er(m: int, n: int, k: int, d: float, *, seed: int = SEED, fixed: bool = False, window: int = 0,
       values: str = "f32", portable: bool = False) -> CSCBatch:
    """k ER matrices m x n; each column holds c distinct uniform rows.

    c ~ Poisson(d), or c = round(d) when ``fixed``.  A positive ``window`` draws
    each column's rows from `window` consecutive rows at a seeded per-column
    offset (the same offset in all k inputs).  ``portable`` draws the Poisson counts
    with the sampler the device generator (gen_device.hip) shares, so the device can
    produce the same matrices (d <= 700, no window)."""
    lib = _load()
    colptr = np.zeros((k, n + 1), dtype=np.int32)
    nnz = np.zeros(k, dtype=np.int64)
    mode = 1 if fixed else 2 if portable else 0
    rc = lib.gen_er_counts(seed, m, n, k, mode, float(d), window, colptr.ctypes.data, nnz.ctypes.data)
    if rc != 0:
        raise ValueError("ER input too large for int32 column pointers")
    kind = VALUE_KINDS[values]
    rows = [np.empty(int(z), dtype=np.int32) for z in nnz]
    vals = [np.empty(int(z), dtype=VALUE_DTYPES[kind]) for z in nnz]
    rc = lib.gen_er_fill(seed, m, n, k, window, colptr.ctypes.data, _ptrs(rows), _ptrs(vals), kind)
    if rc != 0:
        raise MemoryError("generator allocation failed")
    return CSCBatch(m, n, colptr, rows, vals)


def rmat(scale: int, edge_factor: int, k: int, *, a=0.57, b=0.19, c=0.19, seed: int = SEED,
         values: str = "normal") -> CSCBatch:
    """k independent R-MAT matrices 2^scale x 2^scale with edge_factor * 2^scale edges
    each; duplicates removed per matrix."""
    lib = _load()
    n = 1 << scale
    edges = edge_factor * n
    kind = VALUE_KINDS[values]
    colptr = np.zeros((k, n + 1), dtype=np.int32)
    rows = [np.empty(edges, dtype=np.int32) for _ in range(k)]
    vals = [np.empty(edges, dtype=VALUE_DTYPES[kind]) for _ in range(k)]
    nnz = np.zeros(k, dtype=np.int64)
    rc = lib.gen_rmat(seed, scale, edges, a, b, c, k, colptr.ctypes.data, _ptrs(rows), _ptrs(vals), kind,
                      nnz.ctypes.data)
    if rc != 0:
        raise MemoryError("generator allocation failed")
    rows = [r[: int(z)].copy() for r, z in zip(rows, nnz)]
    vals = [v[: int(z)].copy() for v, z in zip(vals, nnz)]
    return CSCBatch(n, n, colptr, rows, vals)


def uniform(count: int, *, seed: int = SEED, tag: int = 17) -> np.ndarray:
    """`count` U(0,1) draws of stream (seed, tag)."""
    out = np.empty(count, dtype=np.float64)
    _load().gen_uniform(seed, tag, count, out.ctypes.data)
    return out


def from_dense(masks, values=None) -> CSCBatch:
    """A batch from k dense (m, n) stored-entry masks (and optional value arrays);
    used for hand-built cases."""
    masks = [np.asarray(mk, dtype=bool) for mk in masks]
    m, n = masks[0].shape
    colptr = np.zeros((len(masks), n + 1), dtype=np.int32)
    rows, vals = [], []
    for i, mk in enumerate(masks):
        r_list, v_list = [], []
        for j in range(n):
            rr = np.nonzero(mk[:, j])[0]
            r_list.append(rr)
            if values is not None:
                v_list.append(np.asarray(values[i])[rr, j])
            colptr[i, j + 1] = colptr[i, j] + len(rr)
        rows.append(np.concatenate(r_list).astype(np.int32) if r_list else np.zeros(0, np.int32))
        if values is not None:
            dt = np.asarray(values[i]).dtype
            vals.append(np.concatenate(v_list).astype(dt) if v_list else np.zeros(0, dt))
    return CSCBatch(m, n, colptr, rows, vals)


# The five workloads of the benchmark plan, by name.  Each returns a CSCBatch.
def config1(values: str = "f32") -> CSCBatch:
    """k=4 ER 1000 x 1000, Poisson(8) distinct rows per column."""
    return er(1000, 1000, 4, 8.0, seed=SEED + 1, values=values)


def config2(values: str = "f32") -> CSCBatch:
    """k=32 ER 65,536 x 65,536, Poisson(16) distinct rows per column."""
    return er(65536, 65536, 32, 16.0, seed=SEED + 2, values=values)


def config3(values: str = "normal") -> CSCBatch:
    """k=64 R-MAT scale 20 (a=.57, b=c=.19, d=.05), edge factor 16, N(0,1) values."""
    return rmat(20, 16, 64, seed=SEED + 3, values=values)


def config4(values: str = "f32", window: int = 0) -> CSCBatch:
    """k=128 tall-skinny 2^24 x 1024, exactly 4,096 distinct uniform rows per column
    (window > 0: rows drawn from a per-column window of that many rows)."""
    return er(1 << 24, 1024, 128, 4096, seed=SEED + 4, fixed=True, window=window, values=values)


def stack(batches) -> CSCBatch:
    """One batch from several batches of the same shape (their matrices in order)."""
    m, n = batches[0].m, batches[0].n
    colptr = np.concatenate([b.colptr for b in batches], axis=0)
    return CSCBatch(m, n, colptr, [r for b in batches for r in b.rowidx], [v for b in batches for v in b.vals])


@dataclass
class RequestSpec:
    """The shape of one request of the batched / served workload (draw number t of the
    stream): k matrices m x n, matrix i with density dens[i] and seed matrix_seed(i)."""

    t: int
    k: int
    m: int
    n: int
    dens: np.ndarray
    seed: int

    def matrix_seed(self, i: int) -> int:
        return self.seed * 7919 + self.t * 131 + i

    @property
    def expected_nnz(self) -> float:
        return float(self.dens.sum()) * self.m * self.n


def request_specs(count: int, *, seed: int = SEED + 5, max_nnz: int | None = None):
    """Shapes of the batched / served workload: k ~ U{2..64}; m and n independent
    log-uniform in [256, 65536]; each of the k matrices with its own density,
    log-uniform in [1e-4, 1e-2].  With max_nnz, requests whose expected input nnz
    exceeds it are redrawn (a bounded sample of the small-request part of the stream)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0
    while len(out) < count:
        t += 1
        k = int(rng.integers(2, 65))
        m = int(round(np.exp(rng.uniform(np.log(256), np.log(65536)))))
        n = int(round(np.exp(rng.uniform(np.log(256), np.log(65536)))))
        dens = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), size=k))
        if max_nnz is not None and float(dens.sum()) * m * n > max_nnz:
            continue
        out.append(RequestSpec(t, k, m, n, dens, seed))
    return out


def request_from_spec(spec: RequestSpec, values: str = "f32") -> CSCBatch:
    """The request's matrices on the host: matrix i holds Poisson(dens[i] * m) distinct
    uniform rows per column (the portable sampler, so device_request draws the same)."""
    return stack([er(spec.m, spec.n, 1, float(d * spec.m), seed=spec.matrix_seed(i), values=values, portable=True)
                  for i, d in enumerate(spec.dens)])


def request_stream(count: int, *, seed: int = SEED + 5, max_nnz: int | None = None, values: str = "f32"):
    """Requests of the batched / served workload on the host (request_specs, then
    request_from_spec)."""
    return [request_from_spec(s, values) for s in request_specs(count, seed=seed, max_nnz=max_nnz)]


# ---- the same ER matrices drawn on the device (gen_device.hip) ----
_DEV_LIB_PATH = os.path.join(_HERE, "libgendev.so")
_dev_lib = None


def build_device_lib(force: bool = False) -> str:
    """Compile gen_device.hip for gfx950 into libgendev.so next to it."""
    if force or not os.path.exists(_DEV_LIB_PATH):
        tmp = _DEV_LIB_PATH + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-Wno-unused-command-line-argument", "-o", tmp,
                               os.path.join(_HERE, "gen_device.hip")])
        os.replace(tmp, _DEV_LIB_PATH)
    return _DEV_LIB_PATH


def _load_dev():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB_PATH):
            raise ImportError(f"{_DEV_LIB_PATH} is not built (workloads.build_device_lib())")
        lib = ctypes.CDLL(_DEV_LIB_PATH)
        P = ctypes.c_void_p
        lib.gendev_er_counts.argtypes = [ctypes.c_int, ctypes.c_longlong, ctypes.c_longlong, P, P, P, P, P]
        lib.gendev_er_counts.restype = ctypes.c_int
        lib.gendev_er_fill.argtypes = [ctypes.c_int, ctypes.c_longlong, ctypes.c_longlong, P, P, P, P, ctypes.c_int, P]
        lib.gendev_er_fill.restype = ctypes.c_int
        _dev_lib = lib
    return _dev_lib


def device_request(spec: RequestSpec, values: str = "f32", device: str = "cuda:0", stream=None):
    """The request's matrices drawn on the device: (colptrs, rowidxs, values), k torch
    tensors each, equal to request_from_spec(spec, values) entry for entry."""
    import torch
    lib = _load_dev()
    kind = VALUE_KINDS[values]
    if kind == VALUE_KINDS["normal"]:
        raise ValueError("normal values are drawn on the host only")
    k, m, n = spec.k, spec.m, spec.n
    s = torch.cuda.current_stream(device) if stream is None else stream
    sp = ctypes.c_void_p(s.cuda_stream)
    seeds = (ctypes.c_uint64 * k)(*[spec.matrix_seed(i) for i in range(k)])
    means = (ctypes.c_double * k)(*[float(d * m) for d in spec.dens])
    cp = torch.empty((k, n + 1), dtype=torch.int32, device=device)
    cps = [cp[i] for i in range(k)]
    cpp = (ctypes.c_void_p * k)(*[c.data_ptr() for c in cps])
    nnz = torch.empty(k, dtype=torch.int64, device=device)
    if lib.gendev_er_counts(k, m, n, seeds, means, cpp, ctypes.c_void_p(nnz.data_ptr()), sp) != 0:
        raise RuntimeError("device generator: counts failed")
    z = nnz.cpu().tolist()  # (waits for the counts)
    if min(z) < 0:
        raise ValueError("ER input too large for int32 column pointers")
    dt = torch.float32 if VALUE_DTYPES[kind] == np.float32 else torch.float64
    ris = [torch.empty(max(int(v), 1), dtype=torch.int32, device=device)[:int(v)] for v in z]
    vas = [torch.empty(max(int(v), 1), dtype=dt, device=device)[:int(v)] for v in z]
    rp = (ctypes.c_void_p * k)(*[r.data_ptr() for r in ris])
    vp = (ctypes.c_void_p * k)(*[v.data_ptr() for v in vas])
    if lib.gendev_er_fill(k, m, n, seeds, cpp, rp, vp, kind, sp) != 0:
        raise RuntimeError("device generator: fill failed")
    return cps, ris, vas
