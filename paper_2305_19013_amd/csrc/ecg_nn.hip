// Learned factorised preconditioner M^{-1} = G G^T: network forward/backward, loss and its
// gradient, Adam, and the CSR of G (C ABI in include/ecg_nn.h).
//
// The network is tiny (7 -> 32 -> 32 -> 3 per row), so it runs on the FP32 vector units
// with its weights in LDS; the stencil products of the loss run in FP64.  Every reduction
// is per-workgroup partials plus a fixed-order sum (bitwise reproducible).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "../../include/ecg_nn.h"
#include "ecg_internal.h"

namespace {

constexpr int kB = 256;
constexpr int NF = 7, NH = 32, NO = 3;
constexpr int NP = ECG_NN_NPARAM;
// offsets inside the flat parameter vector
constexpr int oW1 = 0, ob1 = oW1 + NH * NF, oW2 = ob1 + NH, ob2 = oW2 + NH * NH, oW3 = ob2 + NH,
              ob3 = oW3 + NO * NH;
static_assert(ob3 + NO == NP, "parameter layout");

ecg_status nn_fail(ecg_status s, const std::string& m) {
  ecg::set_last_error(m.c_str());
  return s;
}

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// --------------------------------------------------------------------- network per row
struct Row {
  float f[NF];
  float h1[NH];
  float h2[NH];
  float o[NO];
};

__device__ __forceinline__ void features(const double* __restrict__ a5, int nx, int n, int i, float* f) {
  const double d = a5[i];
  f[0] = (float)log(d);
  const double inv = 1.0 / d;
  f[1] = (float)(a5[n + i] * inv);
  f[2] = (float)(a5[2 * n + i] * inv);
  f[3] = (float)(a5[3 * n + i] * inv);
  f[4] = (float)(a5[4 * n + i] * inv);
  f[5] = (i % nx > 0) ? (float)log(a5[i - 1] * inv) : 0.f;
  f[6] = (i >= nx) ? (float)log(a5[i - nx] * inv) : 0.f;
}

__device__ __forceinline__ void forward_row(const float* __restrict__ P, Row& r) {
#pragma unroll 4
  for (int k = 0; k < NH; ++k) {
    float z = P[ob1 + k];
#pragma unroll
    for (int j = 0; j < NF; ++j) z += P[oW1 + k * NF + j] * r.f[j];
    r.h1[k] = tanhf(z);
  }
#pragma unroll 4
  for (int k = 0; k < NH; ++k) {
    float z = P[ob2 + k];
#pragma unroll 8
    for (int j = 0; j < NH; ++j) z += P[oW2 + k * NH + j] * r.h1[j];
    r.h2[k] = tanhf(z);
  }
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    float z = P[ob3 + k];
#pragma unroll 8
    for (int j = 0; j < NH; ++j) z += P[oW3 + k * NH + j] * r.h2[j];
    r.o[k] = z;
  }
}

__global__ void __launch_bounds__(kB)
k_nn_forward(int nx, int n, int nb, const double* __restrict__ a5, const float* __restrict__ params,
             double* __restrict__ g3) {
  __shared__ float P[NP];
  for (int e = threadIdx.x; e < NP; e += kB) P[e] = params[e];
  __syncthreads();
  const long long gid = (long long)blockIdx.x * kB + threadIdx.x;
  if (gid >= (long long)n * nb) return;
  const int s = (int)(gid / n), i = (int)(gid % n);
  const double* A = a5 + (size_t)s * 5 * n;
  Row r;
  features(A, nx, n, i, r.f);
  forward_row(P, r);
  const double sc = 1.0 / sqrt(A[i]);
  double* G = g3 + (size_t)s * 3 * n;
  G[i] = sc * exp((double)r.o[0]);
  G[n + i] = (i % nx > 0) ? sc * (double)r.o[1] : 0.0;
  G[2 * n + i] = (i >= nx) ? sc * (double)r.o[2] : 0.0;
}

// --------------------------------------------------------------------- stencil products
// out = G v (which 0), G^T v (which 1), A v (which 2); optional: out -= sub.
__global__ void __launch_bounds__(kB)
k_apply(int which, int nx, int n, int nb, const double* __restrict__ a5, const double* __restrict__ g3,
        const double* __restrict__ v, const double* __restrict__ sub, double* __restrict__ out) {
  const long long gid = (long long)blockIdx.x * kB + threadIdx.x;
  if (gid >= (long long)n * nb) return;
  const int s = (int)(gid / n), i = (int)(gid % n);
  const double* V = v + (size_t)s * n;
  const bool w = i % nx > 0, e = i % nx < nx - 1, so = i >= nx, no = i < n - nx;
  double y;
  if (which == 0) {
    const double* G = g3 + (size_t)s * 3 * n;
    y = G[i] * V[i];
    if (w) y += G[n + i] * V[i - 1];
    if (so) y += G[2 * n + i] * V[i - nx];
  } else if (which == 1) {
    const double* G = g3 + (size_t)s * 3 * n;
    y = G[i] * V[i];
    if (e) y += G[n + i + 1] * V[i + 1];
    if (no) y += G[2 * n + i + nx] * V[i + nx];
  } else {
    const double* A = a5 + (size_t)s * 5 * n;
    y = A[i] * V[i];
    if (w) y += A[n + i] * V[i - 1];
    if (e) y += A[2 * n + i] * V[i + 1];
    if (so) y += A[3 * n + i] * V[i - nx];
    if (no) y += A[4 * n + i] * V[i + nx];
  }
  if (sub) y -= sub[(size_t)s * n + i];
  out[(size_t)s * n + i] = y;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = kB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  return red[0];
}

// per operator (blockIdx.y) and row block (blockIdx.x): partial sums of p.q and r.t
__global__ void __launch_bounds__(kB)
k_dots(int n, const double* __restrict__ p, const double* __restrict__ q, const double* __restrict__ r,
       const double* __restrict__ t, double* __restrict__ part) {
  __shared__ double red[kB];
  const int s = blockIdx.y;
  const int i = blockIdx.x * kB + threadIdx.x;
  double a = 0.0, b = 0.0;
  if (i < n) {
    const size_t k = (size_t)s * n + i;
    a = p[k] * q[k];
    b = r[k] * t[k];
  }
  const double sa = block_sum(a, red);
  __syncthreads();
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    part[((size_t)s * gridDim.x + blockIdx.x) * 2] = sa;
    part[((size_t)s * gridDim.x + blockIdx.x) * 2 + 1] = sb;
  }
}

// loss[s] = (e^T A e) / (x^T A x); kfac[s] = 2 / (x^T A x)
__global__ void __launch_bounds__(kB)
k_loss(int nblk, const double* __restrict__ part, double* __restrict__ loss, double* __restrict__ kfac) {
  __shared__ double red[kB];
  const int s = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int j = threadIdx.x; j < nblk; j += kB) {
    a += part[((size_t)s * nblk + j) * 2];
    b += part[((size_t)s * nblk + j) * 2 + 1];
  }
  const double sa = block_sum(a, red);
  __syncthreads();
  const double sb = block_sum(b, red);
  if (threadIdx.x == 0) {
    loss[s] = sa / sb;
    kfac[s] = 2.0 / sb;
  }
}

// dG_ij = kfac ((A e)_i u_j + b_i w_j) on the pattern
__global__ void __launch_bounds__(kB)
k_dg(int nx, int n, int nb, const double* __restrict__ Ae, const double* __restrict__ u,
     const double* __restrict__ b, const double* __restrict__ w, const double* __restrict__ kfac,
     double* __restrict__ dg3) {
  const long long gid = (long long)blockIdx.x * kB + threadIdx.x;
  if (gid >= (long long)n * nb) return;
  const int s = (int)(gid / n), i = (int)(gid % n);
  const size_t o = (size_t)s * n;
  const double k = kfac[s];
  const double ae = Ae[o + i], bi = b[o + i];
  double* D = dg3 + (size_t)s * 3 * n;
  D[i] = k * (ae * u[o + i] + bi * w[o + i]);
  D[n + i] = (i % nx > 0) ? k * (ae * u[o + i - 1] + bi * w[o + i - 1]) : 0.0;
  D[2 * n + i] = (i >= nx) ? k * (ae * u[o + i - nx] + bi * w[o + i - nx]) : 0.0;
}

// --------------------------------------------------------------------- backward
// A workgroup walks `rows_per_wg` consecutive global rows in tiles of 64: 64 threads
// backpropagate one row each into LDS, then all threads add the tile's outer products to
// the parameters they own (p = tid + 256 q), in FP64.
constexpr int kTile = 64;
constexpr int kPerThread = (NP + kB - 1) / kB;

__global__ void __launch_bounds__(kB)
k_nn_backward(int nx, int n, int nb, int rows_per_wg, const double* __restrict__ a5,
              const float* __restrict__ params, const double* __restrict__ dg3, double scale,
              double* __restrict__ part) {
  __shared__ float P[NP];
  __shared__ float sf[kTile][NF];
  __shared__ float sh1[kTile][NH];
  __shared__ float sh2[kTile][NH];
  __shared__ float sd1[kTile][NH];
  __shared__ float sd2[kTile][NH];
  __shared__ float sd3[kTile][NO];
  for (int e = threadIdx.x; e < NP; e += kB) P[e] = params[e];
  __syncthreads();
  const long long total = (long long)n * nb;
  const long long r0 = (long long)blockIdx.x * rows_per_wg;
  const long long r1 = r0 + rows_per_wg < total ? r0 + rows_per_wg : total;
  double acc[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) acc[q] = 0.0;
  for (long long t0 = r0; t0 < r1; t0 += kTile) {
    if (threadIdx.x < kTile) {
      const long long gid = t0 + threadIdx.x;
      const int tr = threadIdx.x;
      if (gid < r1) {
        const int s = (int)(gid / n), i = (int)(gid % n);
        const double* A = a5 + (size_t)s * 5 * n;
        Row r;
        features(A, nx, n, i, r.f);
        forward_row(P, r);
        const double sc = 1.0 / sqrt(A[i]);
        const double* D = dg3 + (size_t)s * 3 * n;
        const double gd = sc * exp((double)r.o[0]);
        float d3[NO];
        d3[0] = (float)(scale * D[i] * gd);
        d3[1] = (i % nx > 0) ? (float)(scale * D[n + i] * sc) : 0.f;
        d3[2] = (i >= nx) ? (float)(scale * D[2 * n + i] * sc) : 0.f;
        float d2[NH];
#pragma unroll 4
        for (int j = 0; j < NH; ++j) {
          float z = 0.f;
#pragma unroll
          for (int k = 0; k < NO; ++k) z += P[oW3 + k * NH + j] * d3[k];
          d2[j] = z * (1.f - r.h2[j] * r.h2[j]);
        }
#pragma unroll 4
        for (int j = 0; j < NH; ++j) {
          float z = 0.f;
#pragma unroll 8
          for (int k = 0; k < NH; ++k) z += P[oW2 + k * NH + j] * d2[k];
          sd1[tr][j] = z * (1.f - r.h1[j] * r.h1[j]);
          sd2[tr][j] = d2[j];
          sh1[tr][j] = r.h1[j];
          sh2[tr][j] = r.h2[j];
        }
#pragma unroll
        for (int j = 0; j < NF; ++j) sf[tr][j] = r.f[j];
#pragma unroll
        for (int k = 0; k < NO; ++k) sd3[tr][k] = d3[k];
      } else {  // past the end: contributes nothing
        for (int j = 0; j < NH; ++j) sd1[tr][j] = sd2[tr][j] = sh1[tr][j] = sh2[tr][j] = 0.f;
        for (int j = 0; j < NF; ++j) sf[tr][j] = 0.f;
        for (int k = 0; k < NO; ++k) sd3[tr][k] = 0.f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int p = (int)threadIdx.x + q * kB;
      if (p >= NP) continue;
      double s = 0.0;
      if (p < ob1) {
        const int a = (p - oW1) / NF, b = (p - oW1) % NF;
        for (int t = 0; t < kTile; ++t) s += (double)sd1[t][a] * (double)sf[t][b];
      } else if (p < oW2) {
        const int a = p - ob1;
        for (int t = 0; t < kTile; ++t) s += (double)sd1[t][a];
      } else if (p < ob2) {
        const int a = (p - oW2) / NH, b = (p - oW2) % NH;
        for (int t = 0; t < kTile; ++t) s += (double)sd2[t][a] * (double)sh1[t][b];
      } else if (p < oW3) {
        const int a = p - ob2;
        for (int t = 0; t < kTile; ++t) s += (double)sd2[t][a];
      } else if (p < ob3) {
        const int a = (p - oW3) / NH, b = (p - oW3) % NH;
        for (int t = 0; t < kTile; ++t) s += (double)sd3[t][a] * (double)sh2[t][b];
      } else {
        const int a = p - ob3;
        for (int t = 0; t < kTile; ++t) s += (double)sd3[t][a];
      }
      acc[q] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int p = (int)threadIdx.x + q * kB;
    if (p < NP) part[(size_t)blockIdx.x * NP + p] = acc[q];
  }
}

__global__ void __launch_bounds__(kB) k_sum_params(int nwg, const double* __restrict__ part, double* __restrict__ grad) {
  const int p = blockIdx.x * kB + threadIdx.x;
  if (p >= NP) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += part[(size_t)w * NP + p];
  grad[p] = s;
}

__global__ void __launch_bounds__(kB)
k_adam(int np, float* __restrict__ params, const double* __restrict__ grad, double* __restrict__ m,
       double* __restrict__ v, double lr, double b1, double b2, double eps, double c1, double c2) {
  const int p = blockIdx.x * kB + threadIdx.x;
  if (p >= np) return;
  const double g = grad[p];
  const double mm = b1 * m[p] + (1.0 - b1) * g;
  const double vv = b2 * v[p] + (1.0 - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const double mh = mm / c1, vh = vv / c2;
  params[p] = (float)((double)params[p] - lr * mh / (sqrt(vh) + eps));
}

__global__ void __launch_bounds__(kB)
k_factor_csr(int nx, int n, const double* __restrict__ g3, long long* __restrict__ rowptr, int* __restrict__ col,
             double* __restrict__ val) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i > n) return;
  // entries before row i: i diagonals, i - ceil(i/nx) west, max(0, i - nx) south
  const long long start = (long long)i + (i - (i + nx - 1) / nx) + (i > nx ? i - nx : 0);
  rowptr[i] = start;
  if (i == n) return;
  long long k = start;
  if (i >= nx) {
    col[k] = i - nx;
    val[k++] = g3[2 * n + i];
  }
  if (i % nx > 0) {
    col[k] = i - 1;
    val[k++] = g3[n + i];
  }
  col[k] = i;
  val[k] = g3[i];
}

// Factorised sparse approximate inverse on the same pattern (Kolotilina and Yeremin): column
// j of G, with rows {j, j+1 (east), j+nx (north)}, is A_C^{-1} e_1 scaled to unit A-norm, C
// those rows.  For a 5-point operator the east and north neighbours do not couple, so
// A_C^{-1} e_1 = (1, -a_jE / a_EE, -a_jN / a_NN) / s_j with the Schur complement
// s_j = a_jj - a_jE^2 / a_EE - a_jN^2 / a_NN, and the column is that vector times sqrt(s_j).
// Row i of G then holds 1/sqrt(s_i) (diagonal), -a_{i-1,i} / (a_ii sqrt(s_{i-1})) (west) and
// -a_{i-nx,i} / (a_ii sqrt(s_{i-nx})) (south), with a_{i-1,i} = a_iW and a_{i-nx,i} = a_iS by
// symmetry.  The minimiser of the Kaporin condition number of G^T A G over the pattern.
__device__ __forceinline__ double fsai_schur(const double* __restrict__ a5, int n, int nx, int j) {
  double s = a5[j];
  if (j % nx < nx - 1) s -= a5[2 * n + j] * a5[2 * n + j] / a5[j + 1];
  if (j + nx < n) s -= a5[4 * n + j] * a5[4 * n + j] / a5[j + nx];
  return s;
}

__global__ void __launch_bounds__(kB)
k_fsai(int nx, int n, int nb, const double* __restrict__ a5, double* __restrict__ g3) {
  const long long e = (long long)blockIdx.x * kB + threadIdx.x;
  if (e >= (long long)nb * n) return;
  const int op = (int)(e / n), i = (int)(e % n);
  const double* A = a5 + (size_t)op * 5 * n;
  double* G = g3 + (size_t)op * 3 * n;
  const double aii = A[i];
  G[i] = 1.0 / sqrt(fsai_schur(A, n, nx, i));
  G[n + i] = (i % nx > 0) ? -A[n + i] / (aii * sqrt(fsai_schur(A, n, nx, i - 1))) : 0.0;
  G[2 * n + i] = (i >= nx) ? -A[3 * n + i] / (aii * sqrt(fsai_schur(A, n, nx, i - nx))) : 0.0;
}

// workspace layout of loss_grad/backward: u, e, Ae, w, Ax (5 nb n doubles), dot partials,
// loss factors, backward partials
struct NnPlan {
  size_t u, e, ae, w, ax, dots, kfac, bpart, total;
  int nblk, nwg, rows_per_wg;
};

NnPlan nn_plan(int nx, int ny, int nb) {
  NnPlan p;
  const size_t n = (size_t)nx * ny;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~size_t(255);
    return at;
  };
  p.u = take(n * nb * 8);
  p.e = take(n * nb * 8);
  p.ae = take(n * nb * 8);
  p.w = take(n * nb * 8);
  p.ax = take(n * nb * 8);
  p.nblk = cdiv((long long)n, kB);
  p.dots = take((size_t)nb * p.nblk * 2 * 8);
  p.kfac = take((size_t)nb * 8);
  p.rows_per_wg = 4096;
  p.nwg = cdiv((long long)n * nb, p.rows_per_wg);
  p.bpart = take((size_t)p.nwg * NP * 8);
  p.total = off;
  return p;
}

ecg_status check_dims(int nx, int ny, int nb) {
  if (nx < 2 || ny < 2 || nb < 1) return nn_fail(ECG_EINVAL, "need nx, ny >= 2 and nb >= 1");
  if ((long long)nx * ny * nb >= 0x7fffffffLL) return nn_fail(ECG_EINVAL, "nx*ny*nb must be < 2^31");
  return ECG_OK;
}

#define NNCHK(expr)                                                                            \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return nn_fail(ECG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

extern "C" {

ecg_status ecg_nn_forward(int32_t nx, int32_t ny, int32_t nb, const double* a5, const float* params, double* g3,
                          void* hip_stream) {
  if (!a5 || !params || !g3) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, nb);
  if (st != ECG_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const int n = nx * ny;
  hipLaunchKernelGGL(k_nn_forward, dim3(cdiv((long long)n * nb, kB)), dim3(kB), 0, s, nx, n, nb, a5, params, g3);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_nn_workspace_size(int32_t nx, int32_t ny, int32_t nb, size_t* bytes) {
  if (!bytes) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, nb);
  if (st != ECG_OK) return st;
  *bytes = nn_plan(nx, ny, nb).total;
  return ECG_OK;
}

ecg_status ecg_nn_loss_grad(int32_t nx, int32_t ny, int32_t nb, const double* a5, const double* g3, const double* b,
                            const double* x, double* loss, double* dg3, void* workspace, size_t ws_bytes,
                            void* hip_stream) {
  if (!a5 || !g3 || !b || !x || !loss || !dg3 || !workspace) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, nb);
  if (st != ECG_OK) return st;
  const NnPlan pl = nn_plan(nx, ny, nb);
  if (ws_bytes < pl.total) return nn_fail(ECG_ENOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)hip_stream;
  char* ws = static_cast<char*>(workspace);
  double* u = reinterpret_cast<double*>(ws + pl.u);
  double* e = reinterpret_cast<double*>(ws + pl.e);
  double* ae = reinterpret_cast<double*>(ws + pl.ae);
  double* w = reinterpret_cast<double*>(ws + pl.w);
  double* ax = reinterpret_cast<double*>(ws + pl.ax);
  double* dots = reinterpret_cast<double*>(ws + pl.dots);
  double* kfac = reinterpret_cast<double*>(ws + pl.kfac);
  const int n = nx * ny;
  const dim3 grid(cdiv((long long)n * nb, kB));
  hipLaunchKernelGGL(k_apply, grid, dim3(kB), 0, s, 1, nx, n, nb, a5, g3, b, nullptr, u);    // u = G^T b
  hipLaunchKernelGGL(k_apply, grid, dim3(kB), 0, s, 0, nx, n, nb, a5, g3, u, x, e);          // e = G u - x
  hipLaunchKernelGGL(k_apply, grid, dim3(kB), 0, s, 2, nx, n, nb, a5, g3, e, nullptr, ae);   // A e
  hipLaunchKernelGGL(k_apply, grid, dim3(kB), 0, s, 1, nx, n, nb, a5, g3, ae, nullptr, w);   // w = G^T A e
  hipLaunchKernelGGL(k_apply, grid, dim3(kB), 0, s, 2, nx, n, nb, a5, g3, x, nullptr, ax);   // A x
  hipLaunchKernelGGL(k_dots, dim3(pl.nblk, nb), dim3(kB), 0, s, n, e, ae, x, ax, dots);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(kB), 0, s, pl.nblk, dots, loss, kfac);
  hipLaunchKernelGGL(k_dg, grid, dim3(kB), 0, s, nx, n, nb, ae, u, b, w, kfac, dg3);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_nn_backward(int32_t nx, int32_t ny, int32_t nb, const double* a5, const float* params,
                           const double* dg3, double scale, double* grad, void* workspace, size_t ws_bytes,
                           void* hip_stream) {
  if (!a5 || !params || !dg3 || !grad || !workspace) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, nb);
  if (st != ECG_OK) return st;
  const NnPlan pl = nn_plan(nx, ny, nb);
  if (ws_bytes < pl.total) return nn_fail(ECG_ENOMEM, "workspace too small");
  hipStream_t s = (hipStream_t)hip_stream;
  double* part = reinterpret_cast<double*>(static_cast<char*>(workspace) + pl.bpart);
  const int n = nx * ny;
  hipLaunchKernelGGL(k_nn_backward, dim3(pl.nwg), dim3(kB), 0, s, nx, n, nb, pl.rows_per_wg, a5, params, dg3, scale,
                     part);
  hipLaunchKernelGGL(k_sum_params, dim3(cdiv(NP, kB)), dim3(kB), 0, s, pl.nwg, part, grad);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_nn_adam(int32_t nparam, float* params, const double* grad, double* m, double* v, int32_t step,
                       double lr, double beta1, double beta2, double eps, void* hip_stream) {
  if (!params || !grad || !m || !v || nparam < 1 || step < 1) return nn_fail(ECG_EINVAL, "bad argument");
  hipStream_t s = (hipStream_t)hip_stream;
  const double c1 = 1.0 - std::pow(beta1, step), c2 = 1.0 - std::pow(beta2, step);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(nparam, kB)), dim3(kB), 0, s, nparam, params, grad, m, v, lr, beta1, beta2,
                     eps, c1, c2);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_nn_fsai(int32_t nx, int32_t ny, int32_t nb, const double* a5, double* g3, void* hip_stream) {
  if (!a5 || !g3) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, nb);
  if (st != ECG_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const int n = nx * ny;
  hipLaunchKernelGGL(k_fsai, dim3(cdiv((long long)nb * n, kB)), dim3(kB), 0, s, nx, n, nb, a5, g3);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

ecg_status ecg_nn_factor_csr(int32_t nx, int32_t ny, const double* g3, int64_t* rowptr, int32_t* colind,
                             double* vals, void* hip_stream) {
  if (!g3 || !rowptr || !colind || !vals) return nn_fail(ECG_EINVAL, "NULL argument");
  ecg_status st = check_dims(nx, ny, 1);
  if (st != ECG_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  const int n = nx * ny;
  hipLaunchKernelGGL(k_factor_csr, dim3(cdiv(n + 1, kB)), dim3(kB), 0, s, nx, n, g3,
                     reinterpret_cast<long long*>(rowptr), colind, vals);
  NNCHK(hipGetLastError());
  NNCHK(hipStreamSynchronize(s));
  return ECG_OK;
}

}  // extern "C"
