// Device copy of the ER generator of gen.c (count mode 2, no window): the same seeded
// matrices as the host generator, drawn on the GPU, for workloads whose inputs are
// too large to draw on the host (the served request stream).
//
// Like gen.c this only draws random sparsity patterns and values; it holds none of
// the arithmetic of the method.  Bit-identity with the host rests on: SplitMix64 and
// the stream keys (integer arithmetic), the portable Poisson sampler (IEEE double
// operations in a fixed order; this file is built with -ffp-contract=off so no
// multiply-add is fused), row draws by integer multiply-shift, and the same
// distinct-row procedure: rounds of (c - have) draws until c distinct rows are seen,
// the set being the distinct rows of all draws made (here kept in an LDS bitmap
// instead of a sorted buffer; the set, hence the sorted column, is the same).
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr int TAG_COUNT = 1, TAG_ROWS = 2, TAG_VALS = 3;
constexpr int KMAX = 64;       // matrices per call
constexpr int MMAX = 65536;    // rows (the LDS bitmap of one wavefront)
constexpr int WAVES = 4;

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t ctr) { return sm64_mix(key + (ctr + 1) * GOLDEN); }
__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j) {
  uint64_t h = sm64_mix(seed + GOLDEN);
  h = sm64_mix(h ^ (tag * 0xD1B54A32D192ED03ull));
  h = sm64_mix(h ^ (i * 0xABC98388FB8FAC03ull + 1));
  h = sm64_mix(h ^ (j * 0x8CB92BA72F3D8DD7ull + 2));
  return h;
}
__device__ __forceinline__ double u01_open(uint64_t u) {
  return ((double)(u >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ double exp_neg_series(double lambda) {
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

__device__ long long poisson_portable(double lambda, uint64_t key) {
  if (lambda <= 0) return 0;
  const double u = u01_open(draw(key, 0));
  double p = exp_neg_series(lambda), F = p;
  long long x = 0;
  const long long xmax = (long long)(20 * lambda + 100);
  while (u > F && x < xmax) {
    x++;
    const double r = lambda / (double)x;
    p = p * r;
    F = F + p;
  }
  return x;
}

__device__ void write_value(void* vals, long long pos, int kind, uint64_t key, uint64_t ctr) {
  const uint64_t u = draw(key, 2 * ctr);
  switch (kind) {
    case 0: {  // fp32 U(-1,1) on the 2^-23 grid
      const long long q = (long long)(u >> 40) - (1LL << 23);
      ((float*)vals)[pos] = (float)((double)q * 0x1p-23);
      break;
    }
    case 1: {  // fp64 U(-1,1) on the 2^-52 grid
      const long long q = (long long)(u >> 11) - (1LL << 52);
      ((double*)vals)[pos] = (double)q * 0x1p-52;
      break;
    }
    case 2:  // fp32 integers in {-3..3}
      ((float*)vals)[pos] = (float)((int)(((u >> 32) * 7ull) >> 32) - 3);
      break;
    case 4:  // fp64 integers in {-3..3}
      ((double*)vals)[pos] = (double)((int)(((u >> 32) * 7ull) >> 32) - 3);
      break;
    case 5: {  // fp32 U(0,1] on the 2^-23 grid
      const long long q = (long long)(u >> 41) + 1;
      ((float*)vals)[pos] = (float)((double)q * 0x1p-23);
      break;
    }
    default:
      break;
  }
}

struct GenArgs {
  uint64_t seed[KMAX];
  double mean[KMAX];
  int* colptr[KMAX];
  int* rows[KMAX];
  void* vals[KMAX];
  long long m, n;
  int k, kind;
};

// Column counts of every (matrix, column), into colptr_i[j + 1].
__global__ __launch_bounds__(256) void k_counts(GenArgs a) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.k * a.n) return;
  const int i = (int)(t / a.n);
  const long long j = t - (long long)i * a.n;
  long long c = poisson_portable(a.mean[i], stream_key(a.seed[i], TAG_COUNT, 0, (uint64_t)j));
  if (c > a.m) c = a.m;
  a.colptr[i][j + 1] = (int)c;
}

// Matrix blockIdx.x: inclusive scan of its counts in place (colptr), nnz into nnz[i];
// a total above INT32_MAX stores -1.
__global__ __launch_bounds__(1024) void k_scan(GenArgs a, long long* nnz) {
  __shared__ long long part[1024];
  int* cp = a.colptr[blockIdx.x];
  const long long n = a.n;
  const long long per = (n + 1023) / 1024;
  const long long lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
  long long s = 0;
  for (long long j = lo; j < hi; ++j) s += cp[j + 1];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  long long run = part[threadIdx.x] - s;
  const long long total = part[1023];
  if (total <= 0x7fffffffLL)
    for (long long j = lo; j < hi; ++j) {
      run += cp[j + 1];
      cp[j + 1] = (int)run;
    }
  if (threadIdx.x == 0) {
    cp[0] = 0;
    nnz[blockIdx.x] = total <= 0x7fffffffLL ? total : -1;
  }
}

// One wavefront per (matrix, column): c distinct rows by rounds of draws into an LDS
// bitmap, written out in ascending order, then the values.
__global__ __launch_bounds__(64 * WAVES) void k_fill(GenArgs a) {
  __shared__ unsigned bm_all[WAVES][MMAX / 32];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned* bm = bm_all[w];
  const long long units = a.k * a.n;
  const int nwords = (int)((a.m + 31) / 32);
  for (int q = lane; q < nwords; q += 64) bm[q] = 0u;
  __builtin_amdgcn_wave_barrier();
  for (long long unit = (long long)blockIdx.x * WAVES + w; unit < units; unit += (long long)gridDim.x * WAVES) {
    const int i = (int)(unit / a.n);
    const long long j = unit - (long long)i * a.n;
    const int* cp = a.colptr[i];
    const long long s = cp[j], c = cp[j + 1] - cp[j];
    if (c <= 0) continue;
    int* rows = a.rows[i] + s;
    if (c >= a.m) {
      for (long long t = lane; t < c; t += 64) rows[t] = (int)t;
    } else {
      const uint64_t key = stream_key(a.seed[i], TAG_ROWS, 0, (uint64_t)j);
      uint64_t ctr = 0;
      long long have = 0;
      while (have < c) {
        const long long need = c - have;
        int fresh = 0;
        for (long long t = lane; t < need; t += 64) {
          const uint64_t u = draw(key, ctr + (uint64_t)t);
          const unsigned r = (unsigned)(((u >> 32) * (uint64_t)a.m) >> 32);
          const unsigned bit = 1u << (r & 31);
          const unsigned old = atomicOr(&bm[r >> 5], bit);
          fresh += (old & bit) ? 0 : 1;
        }
        for (int off = 32; off > 0; off >>= 1) fresh += __shfl_xor(fresh, off, 64);
        have += fresh;
        ctr += (uint64_t)need;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // rows in ascending order: words in order, bits in order
      int base = 0;
      for (int q0 = 0; q0 < nwords; q0 += 64) {
        const int q = q0 + lane;
        unsigned word = q < nwords ? bm[q] : 0u;
        const int cnt = __popc(word);
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
          const int v = __shfl_up(incl, off, 64);
          if (lane >= off) incl += v;
        }
        int pos = base + incl - cnt;
        while (word) {
          const int b = __ffs(word) - 1;
          rows[pos++] = q * 32 + b;
          word &= word - 1;
        }
        base += __shfl(incl, 63, 64);
        if (q < nwords) bm[q] = 0u;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const uint64_t vk = stream_key(a.seed[i], TAG_VALS, 0, (uint64_t)j);
    for (long long t = lane; t < c; t += 64) write_value(a.vals[i], s + t, a.kind, vk, (uint64_t)t);
  }
}

GenArgs make_args(int k, long long m, long long n, const uint64_t* seeds, const double* means, int* const* colptr,
                  int* const* rows, void* const* vals, int kind) {
  GenArgs a{};
  for (int i = 0; i < k; ++i) {
    a.seed[i] = seeds[i];
    a.mean[i] = means ? means[i] : 0.0;
    a.colptr[i] = colptr[i];
    a.rows[i] = rows ? rows[i] : nullptr;
    a.vals[i] = vals ? vals[i] : nullptr;
  }
  a.m = m;
  a.n = n;
  a.k = k;
  a.kind = kind;
  return a;
}

}  // namespace

// Column pointers of k ER matrices m x n (matrix i: seed seeds[i], Poisson mean
// means[i] per column), each colptr[i] a DEVICE int32[n+1]; nnz: DEVICE int64[k]
// (-1 where a matrix exceeds INT32_MAX entries).  Returns 0, or -1 on bad arguments
// (k outside 1..64, m outside 1..65536, a mean outside [0, 700]), -2 on a launch error.
extern "C" int gendev_er_counts(int k, long long m, long long n, const uint64_t* seeds, const double* means,
                                int* const* colptr, long long* nnz, hipStream_t stream) {
  if (k < 1 || k > KMAX || m < 1 || m > MMAX || n < 0 || !seeds || !means || !colptr || !nnz) return -1;
  for (int i = 0; i < k; ++i)
    if (!(means[i] >= 0.0 && means[i] <= 700.0) || !colptr[i]) return -1;
  const GenArgs a = make_args(k, m, n, seeds, means, colptr, nullptr, nullptr, 0);
  const long long units = (long long)k * n;
  if (units > 0) k_counts<<<(unsigned)((units + 255) / 256), 256, 0, stream>>>(a);
  k_scan<<<k, 1024, 0, stream>>>(a, nnz);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Rows and values of the matrices whose column pointers gendev_er_counts wrote: rows[i]
// DEVICE int32[nnz_i], vals[i] DEVICE values of the kind (0 fp32 grid, 1 fp64 grid,
// 2 fp32 integers, 4 fp64 integers, 5 fp32 positive grid).  Same arguments otherwise.
extern "C" int gendev_er_fill(int k, long long m, long long n, const uint64_t* seeds, int* const* colptr,
                              int* const* rows, void* const* vals, int kind, hipStream_t stream) {
  if (k < 1 || k > KMAX || m < 1 || m > MMAX || n < 0 || !seeds || !colptr || !rows || !vals) return -1;
  if (kind != 0 && kind != 1 && kind != 2 && kind != 4 && kind != 5) return -1;
  const GenArgs a = make_args(k, m, n, seeds, nullptr, colptr, rows, vals, kind);
  const long long units = (long long)k * n;
  if (units > 0) {
    long long blocks = (units + WAVES - 1) / WAVES;
    if (blocks > 8192) blocks = 8192;
    k_fill<<<(unsigned)blocks, 64 * WAVES, 0, stream>>>(a);
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
