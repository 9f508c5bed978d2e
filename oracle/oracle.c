/*
 * CPU oracle for SpKAdd -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * this code.  The GPU library never links, calls or includes it, and this file
 * shares nothing with the GPU library.
 *
 * What it computes (Section II-A, "The problem"): B = A_1 + ... + A_k for k
 * same-shape CSC matrices.  The result is written as the plain definition, not as
 * any of the paper's accumulators:
 *   - pattern(B) is the union of the stored patterns of the inputs.  Algorithms 5
 *     and 6 never test a value, so explicit zeros and cancellations stay stored.
 *   - B(r,j) is the sum of every stored input entry at (r,j).
 *   - Output is canonical CSC with rows strictly ascending in each column.  This is
 *     the "sorted output" option of Algorithm 5.
 * Method: concatenate every (column, row, value) triple, sort by (column, row)
 * with the C library's qsort, and reduce each run of equal keys.  The reduction
 * uses a wide accumulator (x86 80-bit long double).  For every entry the oracle
 * also reports the sum of magnitudes s = sum |a| and the run length t; the
 * tolerance bound needs both.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  int64_t col; /* position of the column in the requested column list */
  int32_t row;
  int32_t pad;
  long double val;
} triple_t;

static int cmp_triple(const void* pa, const void* pb) {
  const triple_t* a = (const triple_t*)pa;
  const triple_t* b = (const triple_t*)pb;
  if (a->col != b->col) return a->col < b->col ? -1 : 1;
  if (a->row != b->row) return a->row < b->row ? -1 : 1;
  return 0;
}

/*
 * m, n, k     : shape and number of inputs (all inputs are m x n).
 * colptr[i]   : int32[n+1] column pointers of input i (host memory).
 * rowidx[i]   : int32 row indices of input i.
 * vals[i]     : values of input i (float when dtype == 0, double when dtype == 1);
 *               vals may be NULL when dtype == -1 (pattern only; values read as 0).
 * cols, ncols : the output columns to compute, in the order given (cols == NULL
 *               means all n columns in order).
 * out_colptr  : int64[ncols+1], out_colptr[0] = 0.
 * out_rowidx, out_val, out_abs, out_mult : arrays of capacity out_cap receiving,
 *               per output entry, the row, the sum, the sum of magnitudes and the
 *               number of input entries that were added.
 * Returns nnz of the requested output columns, -1 on bad arguments or allocation
 * failure, -2 if out_cap is too small.
 */
int64_t oracle_spkadd(int64_t m, int64_t n, int32_t k, const int32_t* const* colptr,
                      const int32_t* const* rowidx, const void* const* vals, int32_t dtype,
                      const int64_t* cols, int64_t ncols, int64_t* out_colptr, int32_t* out_rowidx,
                      long double* out_val, long double* out_abs, int32_t* out_mult, int64_t out_cap) {
  if (m < 0 || n < 0 || k < 1 || !colptr || !rowidx || !out_colptr) return -1;
  if (dtype != -1 && !vals) return -1;
  if (!cols) ncols = n;

  /* 1. concatenate the triples of the requested columns */
  int64_t total = 0;
  for (int64_t c = 0; c < ncols; c++) {
    int64_t j = cols ? cols[c] : c;
    if (j < 0 || j >= n) return -1;
    for (int32_t i = 0; i < k; i++) total += (int64_t)colptr[i][j + 1] - colptr[i][j];
  }
  triple_t* T = (triple_t*)malloc(sizeof(triple_t) * (size_t)(total > 0 ? total : 1));
  if (!T) return -1;
  int64_t w = 0;
  for (int64_t c = 0; c < ncols; c++) {
    int64_t j = cols ? cols[c] : c;
    for (int32_t i = 0; i < k; i++) {
      for (int64_t p = colptr[i][j]; p < colptr[i][j + 1]; p++) {
        T[w].col = c;
        T[w].row = rowidx[i][p];
        T[w].pad = 0;
        if (dtype == 0)
          T[w].val = (long double)((const float*)vals[i])[p];
        else if (dtype == 1)
          T[w].val = (long double)((const double*)vals[i])[p];
        else
          T[w].val = 0.0L;
        if (T[w].row < 0 || T[w].row >= m) {
          free(T);
          return -1;
        }
        w++;
      }
    }
  }

  /* 2. sort by (column, row) */
  qsort(T, (size_t)total, sizeof(triple_t), cmp_triple);

  /* 3. reduce every run of equal (column, row) */
  int64_t nnz = 0;
  int64_t q = 0;
  out_colptr[0] = 0;
  for (int64_t c = 0; c < ncols; c++) {
    while (q < total && T[q].col == c) {
      int64_t r_end = q;
      long double sum = 0.0L, mag = 0.0L;
      while (r_end < total && T[r_end].col == c && T[r_end].row == T[q].row) {
        sum += T[r_end].val;
        mag += T[r_end].val < 0 ? -T[r_end].val : T[r_end].val;
        r_end++;
      }
      if (nnz >= out_cap) {
        free(T);
        return -2;
      }
      if (out_rowidx) out_rowidx[nnz] = T[q].row;
      if (out_val) out_val[nnz] = sum;
      if (out_abs) out_abs[nnz] = mag;
      if (out_mult) out_mult[nnz] = (int32_t)(r_end - q);
      nnz++;
      q = r_end;
    }
    /* 4. column pointer of the next column */
    out_colptr[c + 1] = nnz;
  }
  free(T);
  return nnz;
}

/*
 * Ordered sums (the SPKADD_FLAG_ORDERED mode) -- TEST INFRASTRUCTURE ONLY.
 *
 * Algorithm 5 (Section II-C) takes the inputs of a column in order i = 1..k and adds
 * every entry into the slot of its row.  Summed that way in the inputs' own
 * precision, each output value is the sequential sum of its terms in input order:
 * c = a_first, then c = c + a_next for each later term, one rounding per addition.
 * Terms of the same input (a repeated row of an unsorted column) come in their stored
 * order.  The pattern is the same union as oracle_spkadd's.
 *
 * Method: list every (column, row, input, position, value) entry, sort by all four
 * keys, and fold each run of equal (column, row) left to right in float (dtype 0) or
 * double (dtype 1).  Arguments as oracle_spkadd (vals required); out_val receives
 * each sum widened to double (exact), out_mult the number of terms.
 */
typedef struct {
  int64_t col;
  int64_t pos;
  int32_t row;
  int32_t src;
  double v;
} oentry_t;

static int cmp_oentry(const void* pa, const void* pb) {
  const oentry_t* x = (const oentry_t*)pa;
  const oentry_t* y = (const oentry_t*)pb;
  if (x->col != y->col) return x->col < y->col ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  if (x->src != y->src) return x->src < y->src ? -1 : 1;
  if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
  return 0;
}

int64_t oracle_spkadd_ordered(int64_t m, int64_t n, int32_t k, const int32_t* const* colptr,
                              const int32_t* const* rowidx, const void* const* vals, int32_t dtype,
                              const int64_t* cols, int64_t ncols, int64_t* out_colptr, int32_t* out_rowidx,
                              double* out_val, int32_t* out_mult, int64_t out_cap) {
  if (m < 0 || n < 0 || k < 1 || !colptr || !rowidx || !out_colptr || !vals) return -1;
  if (dtype != 0 && dtype != 1) return -1;
  if (!cols) ncols = n;
  int64_t count = 0;
  for (int64_t c = 0; c < ncols; c++) {
    const int64_t col = cols ? cols[c] : c;
    if (col < 0 || col >= n) return -1;
    for (int32_t src = 0; src < k; src++) count += (int64_t)colptr[src][col + 1] - colptr[src][col];
  }
  oentry_t* E = (oentry_t*)malloc(sizeof(oentry_t) * (size_t)(count > 0 ? count : 1));
  if (!E) return -1;
  int64_t fill = 0;
  for (int64_t c = 0; c < ncols; c++) {
    const int64_t col = cols ? cols[c] : c;
    for (int32_t src = 0; src < k; src++) {
      for (int64_t at = colptr[src][col]; at < colptr[src][col + 1]; at++) {
        oentry_t* x = &E[fill++];
        x->col = c;
        x->pos = at;
        x->src = src;
        x->row = rowidx[src][at];
        x->v = dtype == 0 ? (double)((const float*)vals[src])[at] : ((const double*)vals[src])[at];
        if (x->row < 0 || x->row >= m) {
          free(E);
          return -1;
        }
      }
    }
  }
  qsort(E, (size_t)count, sizeof(oentry_t), cmp_oentry);
  int64_t out = 0, at = 0;
  out_colptr[0] = 0;
  for (int64_t c = 0; c < ncols; c++) {
    while (at < count && E[at].col == c) {
      int64_t stop = at + 1;
      while (stop < count && E[stop].col == c && E[stop].row == E[at].row) stop++;
      if (out >= out_cap) {
        free(E);
        return -2;
      }
      double result;
      if (dtype == 0) {
        float acc = (float)E[at].v;
        for (int64_t t = at + 1; t < stop; t++) acc = acc + (float)E[t].v;
        result = (double)acc;
      } else {
        double acc = E[at].v;
        for (int64_t t = at + 1; t < stop; t++) acc = acc + E[t].v;
        result = acc;
      }
      out_rowidx[out] = E[at].row;
      out_val[out] = result;
      if (out_mult) out_mult[out] = (int32_t)(stop - at);
      out++;
      at = stop;
    }
    out_colptr[c + 1] = out;
  }
  free(E);
  return out;
}
