// A C++ program that uses the solver through its C ABI only (include/ecg.h), with no Python
// and no PyTorch: it builds the 5-point Poisson operator on an N x N grid (Dirichlet
// walls), splits the grid into 2 x 4 boxes (t = 8), solves A x = b for b = 1 to a relative
// residual of 1e-8 with flexibly SRE-CG2 (one halving at switchTol 1e-4), and prints the
// report.  Exit status 0 when the solve converged.
//
// Build (from the repository root, after the library is built):
//   hipcc --offload-arch=gfx950 -O2 -I include paper_2305_19013_amd/examples/poisson_solve.cpp \
//         -L paper_2305_19013_amd -lecg -Wl,-rpath,$PWD/paper_2305_19013_amd -o poisson_solve
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ecg.h"

#define CHECK(call)                                                                    \
  do {                                                                                 \
    ecg_status st_ = (call);                                                           \
    if (st_ != ECG_OK && st_ != ECG_ENOTCONV) {                                        \
      std::fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, ecg_last_error()); \
      return 2;                                                                        \
    }                                                                                  \
  } while (0)

int main(int argc, char** argv) {
  const int N = argc > 1 ? std::atoi(argv[1]) : 64;
  if (N < 8 || N % 8) {
    std::fprintf(stderr, "grid size must be a positive multiple of 8\n");
    return 2;
  }
  const int64_t n = (int64_t)N * N;
  std::vector<int64_t> rowptr(n + 1, 0);
  std::vector<int32_t> col;
  std::vector<double> val;
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      const int64_t i = (int64_t)y * N + x;
      if (y > 0) { col.push_back((int32_t)(i - N)); val.push_back(-1.0); }
      if (x > 0) { col.push_back((int32_t)(i - 1)); val.push_back(-1.0); }
      col.push_back((int32_t)i); val.push_back(4.0);
      if (x < N - 1) { col.push_back((int32_t)(i + 1)); val.push_back(-1.0); }
      if (y < N - 1) { col.push_back((int32_t)(i + N)); val.push_back(-1.0); }
      rowptr[i + 1] = (int64_t)col.size();
    }
  // 2 x 4 boxes; box ids such that id >> 1 merges neighbouring boxes (2 x 2 after a halving)
  const int t = 8;
  std::vector<int32_t> part(n);
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      const int bx = x / (N / 2), by = y / (N / 4);  // bx in [0,2), by in [0,4)
      part[(int64_t)y * N + x] = (by & 1) | (bx << 1) | ((by >> 1) << 2);
    }

  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return 2;
  ecg_operator* A = nullptr;
  ecg_partition* P = nullptr;
  CHECK(ecg_operator_create_csr(n, (int64_t)col.size(), rowptr.data(), col.data(), val.data(), 0, s, &A));
  CHECK(ecg_partition_create(n, t, part.data(), 0, s, &P));

  ecg_options o;
  CHECK(ecg_options_default(&o));
  o.tol = 1e-8;
  o.reduce = ECG_REDUCE_SWITCHTOL_ONCE;
  o.switch_tol = 1e-4;
  o.q_budget_bytes = (int64_t)400 * t * n * 8;
  size_t ws_bytes = 0;
  CHECK(ecg_workspace_size(A, P, &o, &ws_bytes));

  double *b = nullptr, *x = nullptr;
  void* ws = nullptr;
  if (hipMalloc(&b, n * sizeof(double)) != hipSuccess || hipMalloc(&x, n * sizeof(double)) != hipSuccess ||
      hipMalloc(&ws, ws_bytes) != hipSuccess) {
    std::fprintf(stderr, "hipMalloc failed\n");
    return 2;
  }
  std::vector<double> ones(n, 1.0);
  (void)hipMemcpy(b, ones.data(), n * sizeof(double), hipMemcpyHostToDevice);
  (void)hipMemset(x, 0, n * sizeof(double));

  ecg_report rep;
  CHECK(ecg_solve(A, P, b, x, &o, ws, ws_bytes, s, &rep, nullptr));
  std::printf("poisson %dx%d t=%d: status=%d iters=%d switch=%d t_final=%d vectors=%lld relres_true=%.3e seconds=%.3f\n",
              N, N, t, (int)rep.status, rep.iters, rep.n_switch ? rep.switch_iters[0] : 0, rep.t_final,
              (long long)rep.vectors_stored, rep.relres_true, rep.seconds);

  (void)hipFree(b);
  (void)hipFree(x);
  (void)hipFree(ws);
  ecg_partition_destroy(P);
  ecg_operator_destroy(A);
  (void)hipStreamDestroy(s);
  return (rep.status == ECG_OK && rep.relres_true <= 1.01e-8) ? 0 : 1;
}
