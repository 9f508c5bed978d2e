"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every pin takes the oracle's library handle, so the same checks can be run
against deliberately broken copies of the oracle.  Those copies are built in a
temporary directory by the mutation test, and each broken copy must fail at least
one pin.

The sources of truth:
* the hand-worked Fig. 1-style example (tests/golden), summed by hand;
* dense brute force: stored-entry masks OR-ed and values summed in float64
  (Section II-A, the problem statement);
* scipy's sparse "+" for k = 2 (Section II-A: for k = 2 SpKAdd is Python's "+"
  on scipy sparse matrices);
* closed forms for ER inputs: E[nnz(B(:,j))] = m (1 - (1 - d/m)^k) when each
  input column holds a uniform random subset of expected size d;
* invariants: nnz(B) <= sum nnz(A_i) (Section II-A), per-column
  nnz(B(:,j)) >= max_i nnz(A_i(:,j)), rows strictly ascending, and invariance
  under any permutation of the k inputs.
"""
from __future__ import annotations

import os

import numpy as np

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _parse_pairs(text):
    out = []
    for tok in text.split():
        r, v = tok.split(":")
        out.append((int(r), float(v)))
    return out


def load_fig1():
    """(batch, expected {col: [(row, val)]}, expected multiplicities) of the hand example."""
    meta, inputs, outputs, mults = {}, {}, {}, {}
    with open(os.path.join(GOLDEN, "fig1_hand_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, _, rest = line.partition(":")
            parts = head.split()
            if parts[0] in ("m", "n", "k") and not rest:
                meta[parts[0]] = int(parts[1])
            elif parts[0] == "input":
                inputs[(int(parts[1]), int(parts[3]))] = _parse_pairs(rest)
            elif parts[0] == "output":
                outputs[int(parts[2])] = _parse_pairs(rest)
            elif parts[0] == "mult":
                mults[int(parts[2])] = _parse_pairs(rest)
    m, n, k = meta["m"], meta["n"], meta["k"]
    masks = [np.zeros((m, n), bool) for _ in range(k)]
    vals = [np.zeros((m, n), np.float64) for _ in range(k)]
    for (i, j), pairs in inputs.items():
        for r, v in pairs:
            masks[i][r, j] = True
            vals[i][r, j] = v
    return workloads.from_dense(masks, vals), outputs, mults


def pin_fig1(lib):
    batch, outputs, mults = load_fig1()
    res = oracle.spkadd(batch, lib=lib)
    for j in range(batch.n):
        s, e = res.colptr[j], res.colptr[j + 1]
        got = [(int(r), float(v)) for r, v in zip(res.rowidx[s:e], res.val[s:e])]
        assert got == outputs.get(j, []), (j, got)
        if j in mults:
            assert [(int(r), int(t)) for r, t in zip(res.rowidx[s:e], res.mult[s:e])] == \
                [(r, int(t)) for r, t in mults[j]]


def _random_dense_case(rng, m, n, k, density, int_values):
    masks, vals = [], []
    for _ in range(k):
        mk = rng.random((m, n)) < density
        if int_values:
            v = rng.integers(-3, 4, size=(m, n)).astype(np.float64)   # includes stored zeros
        else:
            v = (rng.integers(0, 1 << 24, size=(m, n)) - (1 << 23)).astype(np.float64) * 2.0 ** -23
        masks.append(mk)
        vals.append(v)
    return masks, vals


def pin_dense_brute_force(lib, seeds=range(40)):
    for seed in seeds:
        rng = np.random.default_rng(seed)
        m = int(rng.integers(1, 13))
        n = int(rng.integers(1, 13))
        k = int(rng.integers(1, 7))
        density = float(rng.choice([0.0, 0.1, 0.3, 0.7, 1.0]))
        masks, vals = _random_dense_case(rng, m, n, k, density, int_values=bool(seed % 2))
        batch = workloads.from_dense(masks, [v.astype(np.float32) for v in vals])
        res = oracle.spkadd(batch, lib=lib)
        stored = np.zeros((m, n), bool)
        total = np.zeros((m, n), np.float64)
        mag = np.zeros((m, n), np.float64)
        mult = np.zeros((m, n), np.int64)
        for mk, v in zip(masks, vals):
            v32 = v.astype(np.float32).astype(np.float64)
            stored |= mk
            total += np.where(mk, v32, 0.0)
            mag += np.where(mk, np.abs(v32), 0.0)
            mult += mk
        assert res.colptr[0] == 0 and res.colptr.shape == (n + 1,)
        for j in range(n):
            s, e = res.colptr[j], res.colptr[j + 1]
            rows = np.nonzero(stored[:, j])[0]
            assert np.array_equal(res.rowidx[s:e], rows), (seed, j)
            assert np.array_equal(res.val[s:e].astype(np.float64), total[rows, j]), (seed, j)
            assert np.array_equal(res.abs[s:e].astype(np.float64), mag[rows, j]), (seed, j)
            assert np.array_equal(res.mult[s:e], mult[rows, j]), (seed, j)


def pin_scipy_k2(lib):
    import scipy.sparse as sp
    batch = workloads.er(300, 200, 2, 9.0, seed=99, values="pos").astype(np.float64)
    res = oracle.spkadd(batch, lib=lib)
    mats = [sp.csc_matrix((batch.vals[i], batch.rowidx[i], batch.colptr[i]), shape=(batch.m, batch.n))
            for i in range(2)]
    ref = (mats[0] + mats[1]).tocsc()
    ref.sort_indices()
    assert np.array_equal(res.colptr, ref.indptr.astype(np.int64))
    assert np.array_equal(res.rowidx, ref.indices)
    # two positive doubles: the wide sum rounded once to double is exactly scipy's sum
    assert np.array_equal(res.val.astype(np.float64), ref.data)


def pin_er_closed_form(lib):
    m, n, k, d = 1000, 3000, 4, 8.0
    batch = workloads.er(m, n, k, d, seed=7)
    res = oracle.spkadd(batch, lib=lib)
    per_col = np.diff(res.colptr).astype(np.float64)
    expect = m * (1.0 - (1.0 - d / m) ** k)
    # the per-column count is a sum of m weakly dependent indicators; its variance
    # is close to its mean, so the mean over n columns has sd ~ sqrt(expect / n)
    assert abs(per_col.mean() - expect) < 6.0 * np.sqrt(expect / n), (per_col.mean(), expect)
    # inputs alone: mean column count d
    for i in range(k):
        assert abs(np.diff(batch.colptr[i]).mean() - d) < 6.0 * np.sqrt(d / n)


def pin_invariants(lib, batch=None):
    batch = batch or workloads.er(500, 400, 6, 5.0, seed=11, values="int32f")
    res = oracle.spkadd(batch, lib=lib)
    k, n = batch.k, batch.n
    assert res.nnz <= batch.nnz_in
    counts = np.diff(res.colptr)
    for i in range(k):
        assert np.all(counts >= np.diff(batch.colptr[i]))
    for j in range(n):
        s, e = res.colptr[j], res.colptr[j + 1]
        rows = res.rowidx[s:e]
        assert np.all(np.diff(rows) > 0)
        union = np.unique(np.concatenate([batch.column(i, j)[0] for i in range(k)]))
        assert np.array_equal(rows, union)
    assert int(res.mult.sum()) == batch.nnz_in
    perm = np.random.default_rng(5).permutation(k)
    res_p = oracle.spkadd(batch.select(perm), lib=lib)
    assert np.array_equal(res.colptr, res_p.colptr)
    assert np.array_equal(res.rowidx, res_p.rowidx)
    assert np.array_equal(res.val, res_p.val)


def pin_k1_identity(lib):
    batch = workloads.er(200, 150, 1, 6.0, seed=3)
    res = oracle.spkadd(batch, lib=lib)
    assert np.array_equal(res.colptr, batch.colptr[0].astype(np.int64))
    assert np.array_equal(res.rowidx, batch.rowidx[0])
    assert np.array_equal(res.val.astype(np.float32), batch.vals[0])
    assert np.all(res.mult == 1)


def pin_column_subset(lib):
    batch = workloads.er(400, 300, 5, 7.0, seed=13)
    full = oracle.spkadd(batch, lib=lib)
    cols = np.array([299, 0, 17, 17, 150], dtype=np.int64)
    sub = oracle.spkadd(batch, cols=cols, lib=lib)
    for c, j in enumerate(cols):
        a = slice(full.colptr[j], full.colptr[j + 1])
        b = slice(sub.colptr[c], sub.colptr[c + 1])
        assert np.array_equal(full.rowidx[a], sub.rowidx[b])
        assert np.array_equal(full.val[a], sub.val[b])


# ---- the ordered sum (input order, the inputs' precision) ----
def pin_ordered_hand(lib):
    """Worked by hand in binary32 / binary64 round-to-nearest-even.  With u the unit
    roundoff (2^-24 or 2^-53): 1 + u is a tie between 1 and 1 + 2u and rounds to the
    even 1, so the input order (1, u, u) sums to exactly 1; the order (u, u, 1) first
    gives 2u exactly and then 1 + 2u, which is representable.  The wide sum of either
    is 1 + 2u."""
    for dt, u in ((np.float32, 2.0 ** -24), (np.float64, 2.0 ** -53)):
        # column 0: inputs hold 1, u, u at row 0; column 1: u, u, 1; column 2: only
        # inputs 1 and 2 store row 3 (3 then -3: an explicit zero stays stored)
        cp = np.array([[0, 1, 2, 2], [0, 1, 2, 3], [0, 1, 2, 3]], np.int32)
        rows = [np.array([0, 0], np.int32), np.array([0, 0, 3], np.int32), np.array([0, 0, 3], np.int32)]
        vals = [np.array([1.0, u], dt), np.array([u, u, 3.0], dt), np.array([u, 1.0, -3.0], dt)]
        batch = workloads.CSCBatch(4, 3, cp, rows, vals)
        res = oracle.spkadd_ordered(batch, lib=lib)
        assert res.colptr.tolist() == [0, 1, 2, 3]
        assert res.rowidx.tolist() == [0, 0, 3]
        assert res.val.dtype == dt
        assert res.val[0] == dt(1.0), res.val[0]
        assert res.val[1] == dt(1.0 + 2 * u), res.val[1]
        assert res.val[2] == dt(0.0)
        assert res.mult.tolist() == [3, 3, 2]


def pin_ordered_dense_brute_force(lib, seeds=range(30)):
    """Dense brute force: each position's running sum kept in a dense array of the
    inputs' dtype and updated input by input (numpy adds in that dtype)."""
    for seed in seeds:
        rng = np.random.default_rng(500 + seed)
        m, n, k = int(rng.integers(1, 11)), int(rng.integers(1, 11)), int(rng.integers(1, 9))
        dt = np.float32 if seed % 2 == 0 else np.float64
        density = float(rng.choice([0.2, 0.5, 0.9]))
        masks = [rng.random((m, n)) < density for _ in range(k)]
        # values spread over many binades, so that the order of the additions matters
        vals = [(rng.uniform(-1, 1, size=(m, n)) * np.exp2(rng.integers(-30, 12, size=(m, n)))).astype(dt)
                for _ in range(k)]
        batch = workloads.from_dense(masks, vals)
        res = oracle.spkadd_ordered(batch, lib=lib)
        acc = np.zeros((m, n), dt)
        seen = np.zeros((m, n), bool)
        for mk, v in zip(masks, vals):
            first = mk & ~seen
            later = mk & seen
            acc[first] = v[first]
            acc[later] = acc[later] + v[later]
            seen |= mk
        for j in range(n):
            s, e = res.colptr[j], res.colptr[j + 1]
            rows = np.nonzero(seen[:, j])[0]
            assert np.array_equal(res.rowidx[s:e], rows), (seed, j)
            assert np.array_equal(res.val[s:e].view(np.uint8), acc[rows, j].view(np.uint8)), (seed, j)


def pin_ordered_agrees_with_plain(lib):
    """Same pattern and term counts as the plain oracle; the values equal its wide sum
    for integer-valued inputs and lie within k * u * sum|a| of it otherwise."""
    for values in ("int32f", "f32", "f64"):
        batch = workloads.er(400, 200, 9, 12.0, seed=21, values=values)
        plain = oracle.spkadd(batch, lib=lib)
        res = oracle.spkadd_ordered(batch, lib=lib)
        assert np.array_equal(res.colptr, plain.colptr) and np.array_equal(res.rowidx, plain.rowidx)
        assert np.array_equal(res.mult, plain.mult)
        if values == "int32f":
            assert np.array_equal(res.val.astype(np.float64), plain.val.astype(np.float64))
        else:
            unit = 2.0 ** -53 if values == "f64" else 2.0 ** -24
            diff = np.abs(res.val.astype(np.longdouble) - plain.val)
            assert (diff <= batch.k * np.longdouble(unit) * plain.abs).all()


ALL_PINS = [pin_fig1, pin_dense_brute_force, pin_scipy_k2, pin_er_closed_form, pin_invariants,
            pin_k1_identity, pin_column_subset, pin_ordered_hand, pin_ordered_dense_brute_force,
            pin_ordered_agrees_with_plain]
