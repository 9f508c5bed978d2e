/*
 * Seeded synthetic CSC inputs for SpKAdd workloads.
 *
 * This module only draws random sparsity patterns and values.  It holds none of
 * the arithmetic of the method (no accumulation, hashing or merging); both the
 * GPU library's tests and the CPU oracle are fed from it.
 *
 * Randomness: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used as a counter-based generator.  Every
 * (matrix i, column j) has its own stream key, so any column can be regenerated
 * on its own and results do not depend on the number of threads.
 *
 * Pattern families (the paper's R-MAT generator, Section IV-A):
 *   - ER: each column holds c distinct rows drawn uniformly (c either fixed or
 *     Poisson(d)); this is R-MAT with a=b=c=d=1/4 restricted to one column.
 *   - RMAT: classic recursive-quadrant R-MAT edges (a,b,c,d), duplicates removed
 *     per matrix, no vertex permutation.
 * Output: per matrix CSC with int32 colptr[n+1] (colptr[0]=0) and rows strictly
 * ascending within each column.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ull

static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
/* ctr-th output of the SplitMix64 sequence whose state starts at `key`. */
static inline uint64_t draw(uint64_t key, uint64_t ctr) { return sm64_mix(key + (ctr + 1) * GOLDEN); }

/* Stream key for (seed, tag, i, j). */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j) {
  uint64_t h = sm64_mix(seed + GOLDEN);
  h = sm64_mix(h ^ (tag * 0xD1B54A32D192ED03ull));
  h = sm64_mix(h ^ (i * 0xABC98388FB8FAC03ull + 1));
  h = sm64_mix(h ^ (j * 0x8CB92BA72F3D8DD7ull + 2));
  return h;
}

enum { TAG_COUNT = 1, TAG_ROWS = 2, TAG_VALS = 3, TAG_OFFSET = 4, TAG_RMAT = 5 };

enum {
  VAL_F32_GRID = 0,   /* fp32 U(-1,1) on the 2^-23 grid */
  VAL_F64_GRID = 1,   /* fp64 U(-1,1) on the 2^-52 grid */
  VAL_INT_F32 = 2,    /* fp32 integers uniform in {-3..3} */
  VAL_NORMAL_F32 = 3, /* fp32 N(0,1) (Box-Muller) */
  VAL_INT_F64 = 4,    /* fp64 integers uniform in {-3..3} */
  VAL_POS_F32 = 5,    /* fp32 U(0,1) on the 2^-23 grid, strictly positive */
};

static inline double u01_open(uint64_t u) { return ((double)(u >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

static void write_value(void* vals, int64_t pos, int kind, uint64_t key, uint64_t ctr) {
  uint64_t u = draw(key, 2 * ctr);
  switch (kind) {
    case VAL_F32_GRID: {
      int64_t q = (int64_t)(u >> 40) - (1LL << 23);
      ((float*)vals)[pos] = (float)ldexp((double)q, -23);
      break;
    }
    case VAL_F64_GRID: {
      int64_t q = (int64_t)(u >> 11) - (1LL << 52);
      ((double*)vals)[pos] = ldexp((double)q, -52);
      break;
    }
    case VAL_INT_F32:
      ((float*)vals)[pos] = (float)((int)(((u >> 32) * 7ull) >> 32) - 3);
      break;
    case VAL_INT_F64:
      ((double*)vals)[pos] = (double)((int)(((u >> 32) * 7ull) >> 32) - 3);
      break;
    case VAL_NORMAL_F32: {
      double u1 = u01_open(u), u2 = u01_open(draw(key, 2 * ctr + 1));
      ((float*)vals)[pos] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
      break;
    }
    case VAL_POS_F32: {
      int64_t q = (int64_t)(u >> 41) + 1; /* 1..2^23 */
      ((float*)vals)[pos] = (float)ldexp((double)q, -23);
      break;
    }
    default:
      break;
  }
}

/* Poisson(lambda) by inversion of the CDF from one uniform; normal approximation for
 * large lambda where e^-lambda would underflow. */
static int64_t poisson(double lambda, uint64_t key) {
  if (lambda <= 0) return 0;
  if (lambda > 500.0) {
    double u1 = u01_open(draw(key, 0)), u2 = u01_open(draw(key, 1));
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double x = floor(lambda + sqrt(lambda) * z + 0.5);
    return x < 0 ? 0 : (int64_t)x;
  }
  double u = u01_open(draw(key, 0));
  double p = exp(-lambda), F = p;
  int64_t x = 0;
  while (u > F && x < (int64_t)(20 * lambda + 100)) {
    x++;
    p *= lambda / (double)x;
    F += p;
  }
  return x;
}

/* e^-lambda for 0 <= lambda <= 700 from basic arithmetic only: the alternating
 * Taylor series of e^-(lambda/1024), then ten squarings.  Every step is one IEEE
 * double operation in a fixed order, so a device copy of this routine (built without
 * contraction into fused multiply-adds) returns the same bits. */
static double exp_neg_series(double lambda) {
  const double x = lambda / 1024.0;
  double term = 1.0, sum = 1.0;
  for (int t = 1; t <= 20; t++) {
    term = term * x;
    term = term / (double)t;
    sum = (t & 1) ? sum - term : sum + term;
  }
  for (int s = 0; s < 10; s++) sum = sum * sum;
  return sum;
}

/* Poisson(lambda) by inversion of the CDF from one uniform, with e^-lambda from
 * exp_neg_series: the same count on the host and on the device (lambda <= 700;
 * larger means fall back to poisson()). */
static int64_t poisson_portable(double lambda, uint64_t key) {
  if (lambda <= 0) return 0;
  if (lambda > 700.0) return poisson(lambda, key);
  const double u = u01_open(draw(key, 0));
  double p = exp_neg_series(lambda), F = p;
  int64_t x = 0;
  const int64_t xmax = (int64_t)(20 * lambda + 100);
  while (u > F && x < xmax) {
    x++;
    const double r = lambda / (double)x;
    p = p * r;
    F = F + p;
  }
  return x;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

static void sort_i32(int32_t* v, int64_t n) {
  if (n <= 32) {
    for (int64_t i = 1; i < n; i++) {
      int32_t x = v[i];
      int64_t j = i - 1;
      while (j >= 0 && v[j] > x) {
        v[j + 1] = v[j];
        j--;
      }
      v[j + 1] = x;
    }
  } else {
    qsort(v, (size_t)n, sizeof(int32_t), cmp_i32);
  }
}

static int64_t uniq_sorted(int32_t* v, int64_t n) {
  if (n == 0) return 0;
  int64_t w = 1;
  for (int64_t i = 1; i < n; i++)
    if (v[i] != v[w - 1]) v[w++] = v[i];
  return w;
}

/* c distinct rows, uniform over [lo, lo+W), sorted ascending, into out[0..c).
 * Draw with replacement, sort, drop repeats, top up; the procedure is symmetric
 * under permutations of the row range, so the final set is a uniform c-subset. */
static void distinct_rows(int32_t* out, int64_t c, int64_t lo, int64_t W, uint64_t key) {
  if (c >= W) {
    for (int64_t t = 0; t < W; t++) out[t] = (int32_t)(lo + t);
    return;
  }
  uint64_t ctr = 0;
  int64_t have = 0;
  while (have < c) {
    for (int64_t t = have; t < c; t++) {
      uint64_t u = draw(key, ctr++);
      out[t] = (int32_t)(lo + (int64_t)(((u >> 32) * (uint64_t)W) >> 32));
    }
    sort_i32(out, c);
    have = uniq_sorted(out, c);
  }
}

/*
 * ER / tall-skinny counts.  count_mode 0: c ~ Poisson(mean); 1: c = round(mean);
 * 2: c ~ Poisson(mean) drawn by poisson_portable (the device generator's sampler).
 * Counts are clipped to the window width.  window > 0 draws each column's rows
 * from a window of `window` rows at a per-column seeded offset (same offset for
 * all k matrices); window <= 0 uses all m rows.
 * Fills colptr[i*(n+1) + j] for all i, j and nnz[i]; returns 0.
 */
int gen_er_counts(uint64_t seed, int64_t m, int64_t n, int32_t k, int32_t count_mode, double mean,
                  int64_t window, int32_t* colptr, int64_t* nnz) {
  int64_t W = (window > 0 && window < m) ? window : m;
  for (int32_t i = 0; i < k; i++) {
    int32_t* cp = colptr + (int64_t)i * (n + 1);
    cp[0] = 0;
    int64_t acc = 0;
    for (int64_t j = 0; j < n; j++) {
      const uint64_t ck = stream_key(seed, TAG_COUNT, (uint64_t)i, (uint64_t)j);
      int64_t c = count_mode == 0 ? poisson(mean, ck) : count_mode == 2 ? poisson_portable(mean, ck)
                                                                        : (int64_t)llround(mean);
      if (c > W) c = W;
      if (c < 0) c = 0;
      acc += c;
      if (acc > 0x7fffffffLL) return -1;
      cp[j + 1] = (int32_t)acc;
    }
    nnz[i] = acc;
  }
  return 0;
}

/* Rows and values for the counts written by gen_er_counts.  rowidx[i] / vals[i]
 * are per-matrix buffers of nnz[i] entries. */
int gen_er_fill(uint64_t seed, int64_t m, int64_t n, int32_t k, int64_t window, const int32_t* colptr,
                int32_t* const* rowidx, void* const* vals, int32_t value_kind) {
  int64_t W = (window > 0 && window < m) ? window : m;
  int fail = 0;
#pragma omp parallel
  {
    int64_t cap = 0;
    int32_t* buf = NULL;
#pragma omp for schedule(dynamic, 16) collapse(2)
    for (int32_t i = 0; i < k; i++) {
      for (int64_t j = 0; j < n; j++) {
        const int32_t* cp = colptr + (int64_t)i * (n + 1);
        int64_t c = cp[j + 1] - cp[j];
        if (c == 0) continue;
        if (c > cap) {
          free(buf);
          cap = c * 2;
          buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
          if (!buf) {
            fail = 1;
            cap = 0;
            continue;
          }
        }
        int64_t lo = 0;
        if (W < m) {
          uint64_t u = draw(stream_key(seed, TAG_OFFSET, 0, (uint64_t)j), 0);
          lo = (int64_t)(((u >> 32) * (uint64_t)(m - W + 1)) >> 32);
        }
        distinct_rows(buf, c, lo, W, stream_key(seed, TAG_ROWS, (uint64_t)i, (uint64_t)j));
        memcpy(rowidx[i] + cp[j], buf, sizeof(int32_t) * (size_t)c);
        if (vals && vals[i]) {
          uint64_t vk = stream_key(seed, TAG_VALS, (uint64_t)i, (uint64_t)j);
          for (int64_t t = 0; t < c; t++) write_value(vals[i], cp[j] + t, value_kind, vk, (uint64_t)t);
        }
      }
    }
    free(buf);
  }
  return fail ? -1 : 0;
}

/*
 * R-MAT: `edges` edges on a 2^scale x 2^scale matrix for each of k matrices.
 * Quadrant probabilities a (row 0, col 0), b (row 0, col 1), c (row 1, col 0),
 * d = 1-a-b-c.  Duplicate (row, col) pairs of one matrix are removed.
 * rowidx[i] / vals[i] must hold `edges` entries; nnz[i] receives the count kept.
 * colptr holds k*(2^scale+1) int32.
 */
int gen_rmat(uint64_t seed, int32_t scale, int64_t edges, double a, double b, double c, int32_t k,
             int32_t* colptr, int32_t* const* rowidx, void* const* vals, int32_t value_kind, int64_t* nnz) {
  const int64_t n = (int64_t)1 << scale;
  const uint64_t ta = (uint64_t)(a * 4294967296.0), tb = (uint64_t)((a + b) * 4294967296.0),
                 tc = (uint64_t)((a + b + c) * 4294967296.0);
  int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t i = 0; i < k; i++) {
    int32_t* er = (int32_t*)malloc(sizeof(int32_t) * (size_t)edges);
    int32_t* ec = (int32_t*)malloc(sizeof(int32_t) * (size_t)edges);
    int32_t* cp = colptr + (int64_t)i * (n + 1);
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!er || !ec || !fill) {
      fail = 1;
      free(er);
      free(ec);
      free(fill);
      continue;
    }
    uint64_t key = stream_key(seed, TAG_RMAT, (uint64_t)i, 0);
    for (int64_t e = 0; e < edges; e++) {
      int64_t r = 0, col = 0;
      for (int32_t lev = 0; lev < scale; lev += 2) {
        uint64_t u = draw(key, (uint64_t)e * (uint64_t)((scale + 1) / 2) + (uint64_t)(lev / 2));
        for (int32_t h = 0; h < 2 && lev + h < scale; h++) {
          uint64_t q = h == 0 ? (u & 0xffffffffull) : (u >> 32);
          int rb, cb;
          if (q < ta) { rb = 0; cb = 0; }
          else if (q < tb) { rb = 0; cb = 1; }
          else if (q < tc) { rb = 1; cb = 0; }
          else { rb = 1; cb = 1; }
          r = (r << 1) | rb;
          col = (col << 1) | cb;
        }
      }
      er[e] = (int32_t)r;
      ec[e] = (int32_t)col;
    }
    /* counting sort by column */
    for (int64_t e = 0; e < edges; e++) fill[ec[e] + 1]++;
    for (int64_t j = 0; j < n; j++) fill[j + 1] += fill[j];
    int32_t* rows = rowidx[i];
    {
      int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
      memcpy(pos, fill, sizeof(int64_t) * (size_t)n);
      for (int64_t e = 0; e < edges; e++) rows[pos[ec[e]]++] = er[e];
      free(pos);
    }
    /* sort rows within each column and drop repeats, compacting in place */
    int64_t w = 0;
    cp[0] = 0;
    for (int64_t j = 0; j < n; j++) {
      int64_t s = fill[j], len = fill[j + 1] - fill[j];
      sort_i32(rows + s, len);
      int64_t u = uniq_sorted(rows + s, len);
      memmove(rows + w, rows + s, sizeof(int32_t) * (size_t)u);
      w += u;
      cp[j + 1] = (int32_t)w;
    }
    nnz[i] = w;
    if (vals && vals[i]) {
      for (int64_t j = 0; j < n; j++) {
        uint64_t vk = stream_key(seed, TAG_VALS, (uint64_t)i, (uint64_t)j);
        for (int64_t t = cp[j]; t < cp[j + 1]; t++) write_value(vals[i], t, value_kind, vk, (uint64_t)(t - cp[j]));
      }
    }
    free(er);
    free(ec);
    free(fill);
  }
  return fail ? -1 : 0;
}

/* Counter-based uniform draws for host-side schedulers (arrival times, request
 * shapes): out[t] = U(0,1) for t in [0, count) of stream (seed, tag). */
void gen_uniform(uint64_t seed, uint64_t tag, int64_t count, double* out) {
  uint64_t key = stream_key(seed, tag, 0, 0);
  for (int64_t t = 0; t < count; t++) out[t] = u01_open(draw(key, (uint64_t)t));
}
