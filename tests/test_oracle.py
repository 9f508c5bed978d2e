"""CPU tests: the oracle against its pins, and broken copies of it against the same pins."""
import os
import re
import shutil

import numpy as np
import pytest

import oracle
import workloads
from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_oracle_pin(pin):
    pin(oracle._load())


def test_oracle_empty_shapes():
    # n = 0: only colptr[0] = 0
    b = workloads.CSCBatch(5, 0, np.zeros((2, 1), np.int32), [np.zeros(0, np.int32)] * 2,
                           [np.zeros(0, np.float32)] * 2)
    r = oracle.spkadd(b)
    assert r.nnz == 0 and np.array_equal(r.colptr, [0])
    # m = 0 and all-empty inputs: flat colptr
    b = workloads.CSCBatch(0, 4, np.zeros((3, 5), np.int32), [np.zeros(0, np.int32)] * 3,
                           [np.zeros(0, np.float32)] * 3)
    r = oracle.spkadd(b)
    assert r.nnz == 0 and np.array_equal(r.colptr, np.zeros(5))


def test_oracle_rejects_bad_rows():
    b = workloads.CSCBatch(4, 1, np.array([[0, 1]], np.int32), [np.array([7], np.int32)],
                           [np.array([1.0], np.float32)])
    with pytest.raises(ValueError):
        oracle.spkadd(b)


# Plausible mistakes, each planted in a private copy of oracle.c; the pins must catch every one.
MUTATIONS = {
    "sort_ignores_row": ("if (a->row != b->row) return a->row < b->row ? -1 : 1;", ""),
    "keeps_last_value": ("sum += T[r_end].val;", "sum = T[r_end].val;"),
    "wrong_sign": ("sum += T[r_end].val;", "sum -= T[r_end].val;"),
    "drops_last_input_entry": ("p < colptr[i][j + 1]; p++", "p + 1 < colptr[i][j + 1]; p++"),
    "colptr_off_by_one": ("out_colptr[c + 1] = nnz;", "out_colptr[c] = nnz;"),
    "skips_last_input": ("for (int32_t i = 0; i < k; i++) {\n      for (int64_t p",
                         "for (int32_t i = 0; i + 1 < k; i++) {\n      for (int64_t p"),
    "row_from_wrong_array": ("T[w].row = rowidx[i][p];", "T[w].row = rowidx[0][p % (colptr[0][n] > 0 ? colptr[0][n] : 1)];"),
    "magnitude_signed": ("mag += T[r_end].val < 0 ? -T[r_end].val : T[r_end].val;", "mag += T[r_end].val;"),
    # the ordered sum
    "ordered_reverse_inputs": ("if (x->src != y->src) return x->src < y->src ? -1 : 1;",
                               "if (x->src != y->src) return x->src > y->src ? -1 : 1;"),
    "ordered_wide_accumulator": ("float acc = (float)E[at].v;", "double acc = E[at].v;"),
    "ordered_drops_first_term": ("float acc = (float)E[at].v;", "float acc = 0.0f;"),
    "ordered_f64_in_f32": ("double acc = E[at].v;", "float acc = (float)E[at].v;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
    text = open(src).read()
    old, new = MUTATIONS[name]
    assert old in text, name
    mutated = tmp_path / "oracle_mut.c"
    mutated.write_text(text.replace(old, new, 1))
    lib_path = oracle.build_lib(force=True, src=str(mutated), out=str(tmp_path / "liboracle_mut.so"))
    lib = oracle._bind(lib_path)
    failures = 0
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(lib)
        except Exception:  # an assertion, or an error the broken oracle reports
            failures += 1
    assert failures > 0, f"no pin caught mutation {name}"
