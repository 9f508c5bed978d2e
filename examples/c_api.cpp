// Minimal use of the C ABI (include/spkadd.h) without PyTorch: k random CSC matrices
// built on the host, copied to the device with hipMalloc/hipMemcpy, summed by
// spkadd_plan / spkadd_symbolic / spkadd_numeric, and checked against a dense sum on
// the host.  Prints "ok <nnz>" and exits 0 on success.
//
// Built by paper_2112_10223_amd/build.py (build_example) into examples/c_api.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "spkadd.h"

#define CHECK_HIP(x)                                                   \
  do {                                                                 \
    if ((x) != hipSuccess) {                                           \
      std::fprintf(stderr, "%s failed\n", #x);                         \
      return 1;                                                        \
    }                                                                  \
  } while (0)
#define CHECK_SPK(x)                                                               \
  do {                                                                             \
    spkadd_status st_ = (x);                                                       \
    if (st_ != SPKADD_OK) {                                                        \
      std::fprintf(stderr, "%s: status %d: %s\n", #x, (int)st_, spkadd_last_error()); \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

int main() {
  const int m = 3000, n = 500, k = 5;
  std::mt19937 rng(2112);
  std::vector<std::vector<int>> cp(k, std::vector<int>(n + 1, 0)), ri(k);
  std::vector<std::vector<float>> va(k);
  std::vector<double> dense((size_t)m * n, 0.0);
  std::vector<char> present((size_t)m * n, 0);
  for (int i = 0; i < k; ++i) {
    for (int j = 0; j < n; ++j) {
      const int c = (int)(rng() % 60);  // entries of column j of input i
      std::vector<char> used(m, 0);
      std::vector<int> rows;
      while ((int)rows.size() < c) {
        const int r = (int)(rng() % m);
        if (!used[r]) {
          used[r] = 1;
          rows.push_back(r);
        }
      }
      std::sort(rows.begin(), rows.end());
      for (int r : rows) {
        const float v = (float)((int)(rng() % 7) - 3);  // small integers: every sum is exact
        ri[i].push_back(r);
        va[i].push_back(v);
        dense[(size_t)j * m + r] += v;
        present[(size_t)j * m + r] = 1;
      }
      cp[i][j + 1] = (int)ri[i].size();
    }
  }
  // device copies; the ABI takes HOST arrays of k DEVICE pointers
  std::vector<int*> d_cp(k), d_ri(k);
  std::vector<float*> d_va(k);
  for (int i = 0; i < k; ++i) {
    CHECK_HIP(hipMalloc((void**)&d_cp[i], (n + 1) * sizeof(int)));
    CHECK_HIP(hipMalloc((void**)&d_ri[i], std::max<size_t>(ri[i].size(), 1) * sizeof(int)));
    CHECK_HIP(hipMalloc((void**)&d_va[i], std::max<size_t>(va[i].size(), 1) * sizeof(float)));
    CHECK_HIP(hipMemcpy(d_cp[i], cp[i].data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_ri[i], ri[i].data(), ri[i].size() * sizeof(int), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_va[i], va[i].data(), va[i].size() * sizeof(float), hipMemcpyHostToDevice));
  }
  hipStream_t s;
  CHECK_HIP(hipStreamCreate(&s));
  spkadd_plan_t plan = nullptr;
  CHECK_SPK(spkadd_plan(&plan, m, n, k, (const int32_t* const*)d_cp.data(), (const int32_t* const*)d_ri.data(),
                        SPKADD_F32, nullptr, s));
  int32_t* d_colptr_c = nullptr;
  CHECK_HIP(hipMalloc((void**)&d_colptr_c, (n + 1) * sizeof(int)));
  int64_t nnz = 0;
  CHECK_SPK(spkadd_symbolic(plan, d_colptr_c, &nnz, s));  // waits for nnz(B)
  int32_t* d_rowidx_c = nullptr;
  float* d_values_c = nullptr;
  CHECK_HIP(hipMalloc((void**)&d_rowidx_c, std::max<int64_t>(nnz, 1) * sizeof(int)));
  CHECK_HIP(hipMalloc((void**)&d_values_c, std::max<int64_t>(nnz, 1) * sizeof(float)));
  CHECK_SPK(spkadd_numeric(plan, (const void* const*)d_va.data(), d_rowidx_c, d_values_c, s));
  CHECK_HIP(hipStreamSynchronize(s));
  CHECK_SPK(spkadd_free(plan));
  std::vector<int> colptr_c(n + 1), rowidx_c(nnz);
  std::vector<float> values_c(nnz);
  CHECK_HIP(hipMemcpy(colptr_c.data(), d_colptr_c, (n + 1) * sizeof(int), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(rowidx_c.data(), d_rowidx_c, nnz * sizeof(int), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(values_c.data(), d_values_c, nnz * sizeof(float), hipMemcpyDeviceToHost));
  // the structural union, rows ascending, sums exact
  int64_t expect = 0;
  for (int j = 0; j < n; ++j) {
    int q = colptr_c[j];
    for (int r = 0; r < m; ++r) {
      if (!present[(size_t)j * m + r]) continue;
      ++expect;
      if (q >= colptr_c[j + 1] || rowidx_c[q] != r || values_c[q] != (float)dense[(size_t)j * m + r]) {
        std::fprintf(stderr, "mismatch in column %d at row %d\n", j, r);
        return 1;
      }
      ++q;
    }
    if (q != colptr_c[j + 1]) {
      std::fprintf(stderr, "column %d has extra entries\n", j);
      return 1;
    }
  }
  if (expect != nnz) {
    std::fprintf(stderr, "nnz %lld, expected %lld\n", (long long)nnz, (long long)expect);
    return 1;
  }
  for (int i = 0; i < k; ++i) {
    (void)hipFree(d_cp[i]);
    (void)hipFree(d_ri[i]);
    (void)hipFree(d_va[i]);
  }
  (void)hipFree(d_colptr_c);
  (void)hipFree(d_rowidx_c);
  (void)hipFree(d_values_c);
  (void)hipStreamDestroy(s);
  std::printf("ok %lld\n", (long long)nnz);
  return 0;
}
