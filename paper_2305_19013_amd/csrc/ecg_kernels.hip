// HIP kernels for gfx950 (CDNA4): the streaming steps of flexibly enlarged CG.
//
// Every reduction runs in a fixed order (per-workgroup partials, then a fixed-order
// sum), so results are bitwise reproducible run to run.  No floating-point atomics.
//
// Grids that stream rows are launched with a workgroup count padded to a multiple of 8
// and remapped so that each of the 8 XCDs (which receive workgroups round-robin) owns
// one contiguous range of rows; neighbouring rows of the stencil then share an L2.

#include "ecg_internal.h"

namespace ecg {

namespace {

inline int pad8(int g) { return (g + 7) / 8 * 8; }
inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Logical workgroup index under the XCD-contiguous remapping (grid padded to 8).
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

// Deterministic tree sum of one value per thread (256 threads); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

template <typename T>
__device__ __forceinline__ const T* csr_vals(const DevCsr& A);
template <>
__device__ __forceinline__ const double* csr_vals<double>(const DevCsr& A) { return A.val; }
template <>
__device__ __forceinline__ const float* csr_vals<float>(const DevCsr& A) { return A.valf; }

// ------------------------------------------------------------------ vectors
__global__ void __launch_bounds__(kBlock)
k_residual(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
           const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ y,
           double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    const double yi = b[i] - s;
    y[i] = yi;
    acc = yi * yi;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock)
k_residual_f(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
             const double* __restrict__ b, const double* __restrict__ x, float* __restrict__ y,
             double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    const double yi = b[i] - s;
    y[i] = (float)yi;
    acc = yi * yi;
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock)
k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
       const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
  y[i] = s;
}

__global__ void __launch_bounds__(kBlock) k_sum(const double* __restrict__ part, int m, double* __restrict__ out) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += kBlock) acc += part[i];
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) *out = tot;
}

__global__ void __launch_bounds__(kBlock) k_cast_d2f(int n, const double* __restrict__ in, float* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void __launch_bounds__(kBlock) k_axpy_f2d(int n, const float* __restrict__ d, double* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += (double)d[i];
}

__global__ void __launch_bounds__(kBlock) k_axpy_d(int n, const double* __restrict__ d, double* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += d[i];
}

__global__ void __launch_bounds__(kBlock)
k_gather(int nnz, const double* __restrict__ src, const int* __restrict__ perm, double* __restrict__ dst) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nnz) dst[i] = src[perm[i]];
}

// ------------------------------------------------------------------ SpMM
// Y = A X, row-major n x TC blocks.  TC lanes per row: lane c accumulates column c, so a
// wavefront reads TC contiguous values of X per nonzero (coalesced block rows).
template <typename T, int TC>
__global__ void __launch_bounds__(kBlock)
k_spmm(int n, int nwg, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v,
       const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int RPB = kBlock / TC;
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int row = blk * RPB + (int)threadIdx.x / TC;
  const int c = (int)threadIdx.x % TC;
  if (row >= n) return;
  T acc = T(0);
  const int k1 = rp[row + 1];
  for (int k = rp[row]; k < k1; ++k) acc += v[k] * X[(size_t)ci[k] * TC + c];
  Y[(size_t)row * TC + c] = acc;
}

// ------------------------------------------------------------------ split T^t
template <typename T, typename TV, int TC>
__global__ void __launch_bounds__(kBlock)
k_split(int n, const int* __restrict__ part, int level, const TV* __restrict__ v, T* __restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (long long)n * TC) return;
  const int row = (int)(e / TC);
  const int c = (int)(e % TC);
  out[e] = ((part[row] >> level) == c) ? (T)v[row] : T(0);
}

// ------------------------------------------------------------------ CGS2 Gram G = Q^T Y
// One workgroup = one stored block j of the span x one chunk of rows.  It writes the
// WQ x TC partial product of that chunk; a second kernel sums the chunks in order.
template <typename T, int WQ, int TC>
__global__ void __launch_bounds__(kBlock)
k_gram(int n, Span<T> sp, int rows_per_chunk, const T* __restrict__ Y, T* __restrict__ part, int m) {
  constexpr int OUT = WQ * TC;
  constexpr int NA = OUT >= kBlock ? OUT / kBlock : 1;  // outputs (a values) per thread
  constexpr int AG = WQ / NA;
  constexpr int RS = kBlock / (TC * AG);  // row slices reduced at the end
  static_assert(RS >= 1 && TC * AG * RS == kBlock, "thread mapping");
  __shared__ T red[RS > 1 ? kBlock : 1];
  const int j = blockIdx.x;
  const int chunk = blockIdx.y;
  const int b = (int)threadIdx.x % TC;
  const int ag = ((int)threadIdx.x / TC) % AG;
  const int rs = (int)threadIdx.x / (TC * AG);
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  const T* __restrict__ Q = sp.base + (size_t)j * sp.stride;
  T acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = T(0);
  for (int row = r0 + rs; row < r1; row += RS) {
    const T yv = Y[(size_t)row * TC + b];
    const T* __restrict__ q = Q + (size_t)row * WQ + ag * NA;
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] += q[i] * yv;
  }
  if constexpr (RS > 1) {
    red[threadIdx.x] = acc[0];
    __syncthreads();
    if (rs == 0) {
      T s = T(0);
      for (int q = 0; q < RS; ++q) s += red[threadIdx.x + q * TC * AG];
      acc[0] = s;
    }
  }
  if (rs == 0) {
    const size_t base = ((size_t)chunk * m + sp.goff + (size_t)j * WQ + ag * NA) * TC + b;
#pragma unroll
    for (int i = 0; i < NA; ++i) part[base + (size_t)i * TC] = acc[i];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_reduce_chunks(long long len, int nchunks, const T* __restrict__ part, T* __restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  T s = T(0);
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * len + e];
  out[e] = s;
}

// ------------------------------------------------------------------ CGS2 update W -= Q G
template <typename T, int WQ, int TC>
__global__ void __launch_bounds__(kBlock)
k_update(int n, int nwg, Span<T> sp, const T* __restrict__ G, T* __restrict__ W) {
  constexpr int RPB = kBlock / TC;
  __shared__ T Gs[WQ * TC];
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int row = blk * RPB + (int)threadIdx.x / TC;
  const int b = (int)threadIdx.x % TC;
  T acc = T(0);
  for (int j = 0; j < sp.nblk; ++j) {
    __syncthreads();
    for (int e = threadIdx.x; e < WQ * TC; e += kBlock) Gs[e] = G[(size_t)(sp.goff + j * WQ) * TC + e];
    __syncthreads();
    if (row < n) {
      const T* __restrict__ q = sp.base + (size_t)j * sp.stride + (size_t)row * WQ;
#pragma unroll 8
      for (int a = 0; a < WQ; ++a) acc += q[a] * Gs[a * TC + b];
    }
  }
  if (row < n) W[(size_t)row * TC + b] -= acc;
}

// ------------------------------------------------------------------ t x t Grams (FP64)
template <typename T, int TC, bool WITH_R>
__global__ void __launch_bounds__(kBlock)
k_small_gram(int n, int rows_per_chunk, const T* __restrict__ X, const T* __restrict__ Y,
             const T* __restrict__ r, double* __restrict__ part) {
  constexpr int NOUT = TC * TC + (WITH_R ? TC : 0);
  constexpr int NPT = (NOUT + kBlock - 1) / kBlock;
  const int chunk = blockIdx.x;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  double acc[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) acc[i] = 0.0;
  for (int row = r0; row < r1; ++row) {
    const T* __restrict__ xr = X + (size_t)row * TC;
    const T* __restrict__ yr = Y + (size_t)row * TC;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int e = (int)threadIdx.x + i * kBlock;
      if (e < TC * TC) {
        acc[i] += (double)xr[e / TC] * (double)yr[e % TC];
      } else if (WITH_R && e < NOUT) {
        acc[i] += (double)xr[e - TC * TC] * (double)r[row];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int e = (int)threadIdx.x + i * kBlock;
    if (e < NOUT) part[(size_t)chunk * NOUT + e] = acc[i];
  }
}

__global__ void __launch_bounds__(kBlock)
k_reduce_small(int len, int nchunks, const double* __restrict__ part, double* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * len + e];
  out[e] = s;
}

// ------------------------------------------------------------------ t x t factor (FP64)
// Right-looking Cholesky of a tc x tc Gram with left-to-right column deflation, then the
// inverse of the (upper triangular) factor.  One workgroup; tc <= 64.
// The factor R lives in the upper triangle of A (row j = R[j][.]); the strictly upper part
// of X = R^{-1} is kept transposed in the strictly lower triangle of A and diag(X) in xd.
__global__ void __launch_bounds__(kBlock)
k_factor(int mode, int tc, int tc_live, const double* __restrict__ in, double tau,
         double* __restrict__ inv, double* __restrict__ beta, IterStatus* __restrict__ st) {
  __shared__ double A[kMaxT * kMaxT];
  __shared__ double d0[kMaxT];
  __shared__ double xd[kMaxT];
  __shared__ double u[kMaxT];
  __shared__ double al[kMaxT];
  __shared__ int keep[kMaxT];
  __shared__ int brk;
  const int tid = threadIdx.x;
  for (int e = tid; e < tc * tc; e += kBlock) A[(e / tc) * kMaxT + (e % tc)] = in[e];
  if (tid == 0) brk = 0;
  __syncthreads();
  if (tid < tc) {
    d0[tid] = A[tid * kMaxT + tid];
    u[tid] = (mode == 1) ? in[tc * tc + tid] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < tc; ++j) {
    if (tid == 0) {
      const double piv = A[j * kMaxT + j];
      bool ok;
      if (j >= tc_live) {
        ok = false;
      } else if (tau >= 0.0) {
        ok = (d0[j] > 0.0) && (piv > tau * d0[j]);
      } else {
        ok = piv > 0.0;
        if (!ok) brk = 1;
      }
      keep[j] = ok ? 1 : 0;
      A[j * kMaxT + j] = ok ? sqrt(piv) : 0.0;
    }
    __syncthreads();
    const bool kj = keep[j] != 0;
    const double rjj = A[j * kMaxT + j];
    for (int i = j + 1 + tid; i < tc; i += kBlock) A[j * kMaxT + i] = kj ? A[j * kMaxT + i] / rjj : 0.0;
    __syncthreads();
    if (kj) {
      const int w = tc - j - 1;  // trailing size
      for (int e = tid; e < w * w; e += kBlock) {
        const int i = j + 1 + e / w;
        const int k = j + 1 + e % w;
        if (k >= i) A[i * kMaxT + k] -= A[j * kMaxT + i] * A[j * kMaxT + k];
      }
    }
    __syncthreads();
  }
  // X = R^{-1}: thread c builds column c by back substitution.
  if (tid < tc) {
    const int c = tid;
    if (keep[c]) {
      xd[c] = 1.0 / A[c * kMaxT + c];
      for (int i = c - 1; i >= 0; --i) {
        double x = 0.0;
        if (keep[i]) {
          double s = A[i * kMaxT + c] * xd[c];
          for (int k = i + 1; k < c; ++k) s += A[i * kMaxT + k] * A[c * kMaxT + k];
          x = -s / A[i * kMaxT + i];
        }
        A[c * kMaxT + i] = x;  // X[i][c]
      }
    } else {
      xd[c] = 0.0;
      for (int i = 0; i < c; ++i) A[c * kMaxT + i] = 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < tc * tc; e += kBlock) {
    const int i = e / tc, c = e % tc;
    double x = 0.0;
    if (i == c) x = xd[c];
    else if (i < c) x = A[c * kMaxT + i];
    inv[e] = x;
  }
  if (mode == 1) {
    // alpha = X^T u, beta = X alpha
    if (tid < tc) {
      const int b = tid;
      double s = xd[b] * u[b];
      for (int a = 0; a < b; ++a) s += A[b * kMaxT + a] * u[a];
      al[b] = s;
    }
    __syncthreads();
    if (tid < tc) {
      const int a = tid;
      double s = xd[a] * al[a];
      for (int b = a + 1; b < tc; ++b) s += A[b * kMaxT + a] * al[b];
      beta[a] = s;
    }
  }
  if (tid == 0) {
    int cnt = 0;
    for (int j = 0; j < tc_live; ++j) cnt += keep[j];
    if (mode == 0) st->keep_e = cnt;
    else st->keep_a = cnt;
    if (brk) st->breakdown = 1;
  }
}

// ------------------------------------------------------------------ out = X M (t x t)
template <typename T, int TC>
__global__ void __launch_bounds__(kBlock)
k_times_small(int n, int nwg, const T* __restrict__ X, const double* __restrict__ M, T* __restrict__ out) {
  constexpr int RPB = kBlock / TC;
  __shared__ T Ms[TC * TC];
  for (int e = threadIdx.x; e < TC * TC; e += kBlock) Ms[e] = (T)M[e];
  __syncthreads();
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int row = blk * RPB + (int)threadIdx.x / TC;
  const int b = (int)threadIdx.x % TC;
  if (row >= n) return;
  const T* __restrict__ xr = X + (size_t)row * TC;
  T acc = T(0);
#pragma unroll 8
  for (int a = 0; a < TC; ++a) acc += xr[a] * Ms[a * TC + b];
  out[(size_t)row * TC + b] = acc;
}

// ------------------------------------------------------------------ fused final update
template <typename T, typename TX, int TC>
__global__ void __launch_bounds__(kBlock)
k_final_update(int n, int nwg, const T* __restrict__ H, const T* __restrict__ Y, const double* __restrict__ Cinv,
               const double* __restrict__ beta, T* __restrict__ Wq, T* __restrict__ Zn, TX* __restrict__ x,
               T* __restrict__ r, double* __restrict__ part) {
  constexpr int RPB = kBlock / TC;
  __shared__ T Cs[TC * TC];
  __shared__ T bs[TC];
  __shared__ double red[kBlock];
  for (int e = threadIdx.x; e < TC * TC; e += kBlock) Cs[e] = (T)Cinv[e];
  if ((int)threadIdx.x < TC) bs[threadIdx.x] = (T)beta[threadIdx.x];
  __syncthreads();
  const int blk = xcd_block();
  if (blk >= nwg) return;  // whole workgroup leaves; no later barrier is skipped by a subset
  const int row = blk * RPB + (int)threadIdx.x / TC;
  const int b = (int)threadIdx.x % TC;
  double rr = 0.0;
  T hx = T(0), yr = T(0);
  if (row < n) {
    const T* __restrict__ hrow = H + (size_t)row * TC;
    const T* __restrict__ yrow = Y + (size_t)row * TC;
    T w = T(0), z = T(0);
#pragma unroll 8
    for (int a = 0; a < TC; ++a) {
      const T c = Cs[a * TC + b];
      w += hrow[a] * c;
      z += yrow[a] * c;
    }
    Wq[(size_t)row * TC + b] = w;
    Zn[(size_t)row * TC + b] = z;
    hx = hrow[b] * bs[b];
    yr = yrow[b] * bs[b];
  }
  // sum over the TC lanes of this row (rows never straddle a wavefront: TC divides 64)
#pragma unroll
  for (int off = TC / 2; off > 0; off >>= 1) {
    hx += __shfl_xor(hx, off, 64);
    yr += __shfl_xor(yr, off, 64);
  }
  if (row < n && b == 0) {
    x[row] += (TX)hx;
    const T rn = r[row] - yr;
    r[row] = rn;
    rr = (double)rn * (double)rn;
  }
  const double tot = block_sum(rr, red);
  if (threadIdx.x == 0) part[blk] = tot;
}

// ------------------------------------------------------------------ triangular solves
// One workgroup per independent group (subdomain); levels processed in order with a
// workgroup barrier in between.  which = 0: forward (L, diagonal last in each row);
// which = 1: backward with U = L^T (diagonal first in each row).
template <typename T, int TC>
__global__ void __launch_bounds__(kBlock)
k_trisolve(int which, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v,
           const int* __restrict__ lptr, const int* __restrict__ lrows, int maxlev,
           const T* __restrict__ X, T* __restrict__ Y) {
  const int g = blockIdx.x;
  for (int l = 0; l < maxlev; ++l) {
    const int p0 = lptr[g * (maxlev + 1) + l];
    const int p1 = lptr[g * (maxlev + 1) + l + 1];
    const int cnt = (p1 - p0) * TC;
    for (int e = threadIdx.x; e < cnt; e += kBlock) {
      const int row = lrows[p0 + e / TC];
      const int c = e % TC;
      const int k0 = rp[row], k1 = rp[row + 1];
      T s = X[(size_t)row * TC + c];
      T d;
      if (which == 0) {
        for (int k = k0; k < k1 - 1; ++k) s -= v[k] * Y[(size_t)ci[k] * TC + c];
        d = v[k1 - 1];
      } else {
        for (int k = k0 + 1; k < k1; ++k) s -= v[k] * Y[(size_t)ci[k] * TC + c];
        d = v[k0];
      }
      Y[(size_t)row * TC + c] = s / d;
    }
    __syncthreads();
  }
}

// IC(0): rows of one group, level by level.  L's pattern is the lower triangle of A within
// the group (diagonal last); apos[k] = position in A of L entry k.
__global__ void __launch_bounds__(kBlock)
k_ic0(const int* __restrict__ rp, const int* __restrict__ ci, double* __restrict__ lv,
      const int* __restrict__ apos, const double* __restrict__ av, const int* __restrict__ lptr,
      const int* __restrict__ lrows, int maxlev, int* __restrict__ fail) {
  const int g = blockIdx.x;
  for (int l = 0; l < maxlev; ++l) {
    const int p0 = lptr[g * (maxlev + 1) + l];
    const int p1 = lptr[g * (maxlev + 1) + l + 1];
    for (int p = p0 + threadIdx.x; p < p1; p += kBlock) {
      const int row = lrows[p];
      const int k0 = rp[row], k1 = rp[row + 1];
      double dsum = 0.0;
      for (int k = k0; k < k1 - 1; ++k) {
        const int c = ci[k];
        double s = av[apos[k]];
        // subtract sum_{j < c} L[row][j] L[c][j] over the common pattern
        int kr = k0;
        int kc = rp[c];
        const int kc1 = rp[c + 1] - 1;  // exclude c's diagonal
        while (kr < k && kc < kc1) {
          const int jr = ci[kr], jc = ci[kc];
          if (jr == jc) {
            s -= lv[kr] * lv[kc];
            ++kr;
            ++kc;
          } else if (jr < jc) {
            ++kr;
          } else {
            ++kc;
          }
        }
        const double lval = s / lv[rp[c + 1] - 1];
        lv[k] = lval;
        dsum += lval * lval;
      }
      const double dd = av[apos[k1 - 1]] - dsum;
      if (!(dd > 0.0)) {
        fail[0] = 1;
        lv[k1 - 1] = 1.0;
      } else {
        lv[k1 - 1] = sqrt(dd);
      }
    }
    __syncthreads();
  }
}

}  // namespace

// ====================================================================== launchers

int launch_residual(const DevCsr& A, const double* b, const double* x, double* y, double* part,
                    hipStream_t s) {
  const int g = cdiv(A.n, kBlock);
  stat_begin(s);
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(kBlock), 0, s, A.n, A.rowptr, A.col, A.val, b, x, y, part);
  stat_end(kStatVector, A.nnz * 12.0 + 4.0 * (A.n + 1) + 24.0 * A.n, 2.0 * A.nnz, s);
  return g;
}

int launch_residual_f(const DevCsr& A, const double* b, const double* x, float* r, double* part,
                      hipStream_t s) {
  const int g = cdiv(A.n, kBlock);
  stat_begin(s);
  hipLaunchKernelGGL(k_residual_f, dim3(g), dim3(kBlock), 0, s, A.n, A.rowptr, A.col, A.val, b, x, r, part);
  stat_end(kStatVector, A.nnz * 12.0 + 4.0 * (A.n + 1) + 20.0 * A.n, 2.0 * A.nnz, s);
  return g;
}

void launch_spmv(const DevCsr& A, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(cdiv(A.n, kBlock)), dim3(kBlock), 0, s, A.n, A.rowptr, A.col, A.val, x, y);
}

void launch_sum(const double* part, int m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, s, part, m, out);
}

void launch_cast_d2f(int n, const double* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, in, out);
}
void launch_axpy_f2d(int n, const float* d, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_f2d, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, d, x);
}
void launch_axpy_d(int n, const double* d, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_d, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, d, x);
}
void launch_cast_val(int nnz, const double* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(cdiv(nnz, kBlock)), dim3(kBlock), 0, s, nnz, in, out);
}
void launch_gather(int nnz, const double* src, const int* perm, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(cdiv(nnz, kBlock)), dim3(kBlock), 0, s, nnz, src, perm, dst);
}

#define ECG_TC_CASES(MACRO) MACRO(1) MACRO(2) MACRO(4) MACRO(8) MACRO(16) MACRO(32) MACRO(64)

template <typename T>
static const T* vals_of(const DevCsr& A);
template <>
const double* vals_of<double>(const DevCsr& A) { return A.val; }
template <>
const float* vals_of<float>(const DevCsr& A) { return A.valf; }

template <typename T>
void launch_spmm(const DevCsr& A, int tc, const T* X, T* Y, hipStream_t s) {
  switch (tc) {
#define C(TC)                                                                                    \
  case TC: {                                                                                     \
    const int nwg = cdiv(A.n, kBlock / TC);                                                      \
    stat_begin(s);                                                                               \
    hipLaunchKernelGGL((k_spmm<T, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, A.rowptr, \
                       A.col, vals_of<T>(A), X, Y);                                              \
    stat_end(kStatSpmm, (double)A.nnz * (sizeof(T) + 4) + 4.0 * (A.n + 1) + 2.0 * sizeof(T) * A.n * TC, \
             2.0 * A.nnz * TC, s);                                                               \
    break;                                                                                       \
  }
    ECG_TC_CASES(C)
#undef C
  }
}

template <typename T>
void launch_split(int n, const int* part, int level, int tc, const double* v, T* out, hipStream_t s) {
  const int g = cdiv((long long)n * tc, kBlock);
  switch (tc) {
#define C(TC)                                                                                    \
  case TC:                                                                                       \
    stat_begin(s);                                                                               \
    hipLaunchKernelGGL((k_split<T, double, TC>), dim3(g), dim3(kBlock), 0, s, n, part, level, v, out); \
    stat_end(kStatSplit, (double)n * (4 + 8) + (double)n * TC * sizeof(T), 0.0, s);              \
    break;
    ECG_TC_CASES(C)
#undef C
  }
}

template <typename T>
void launch_split_t(int n, const int* part, int level, int tc, const T* v, T* out, hipStream_t s) {
  const int g = cdiv((long long)n * tc, kBlock);
  switch (tc) {
#define C(TC)                                                                                    \
  case TC:                                                                                       \
    stat_begin(s);                                                                               \
    hipLaunchKernelGGL((k_split<T, T, TC>), dim3(g), dim3(kBlock), 0, s, n, part, level, v, out); \
    stat_end(kStatSplit, (double)n * (4 + sizeof(T)) + (double)n * TC * sizeof(T), 0.0, s);      \
    break;
    ECG_TC_CASES(C)
#undef C
  }
}

// Chunk count for the CGS2 Gram: enough workgroups to fill 256 CUs several times over,
// but at least 256 rows per chunk.
static int gram_chunks(int n, int nblk_total, size_t part_cap, int m, int tc) {
  int nch = 2048 / (nblk_total > 0 ? nblk_total : 1);
  nch = nch < 1 ? 1 : nch;
  const int maxc = cdiv(n, 256);
  if (nch > maxc) nch = maxc;
  while (nch > 1 && (size_t)nch * m * tc > part_cap) --nch;
  return nch;
}

template <typename T, int WQ, int TC>
static void gram_span(int n, const Span<T>& sp, int rpc, int nch, const T* Y, T* part, int m, hipStream_t s) {
  stat_begin(s);
  hipLaunchKernelGGL((k_gram<T, WQ, TC>), dim3(sp.nblk, nch), dim3(kBlock), 0, s, n, sp, rpc, Y, part, m);
  stat_end(kStatGram, (double)sizeof(T) * n * ((double)sp.nblk * WQ + TC), 2.0 * n * sp.nblk * WQ * TC, s);
}

template <typename T, int TC>
static void gram_span_wq(int n, const Span<T>& sp, int rpc, int nch, const T* Y, T* part, int m, hipStream_t s) {
  switch (sp.width) {
#define C(WQ)                                                        \
  case WQ:                                                           \
    gram_span<T, WQ, TC>(n, sp, rpc, nch, Y, part, m, s);            \
    break;
    ECG_TC_CASES(C)
#undef C
  }
}

template <typename T>
void launch_gram(int n, const Span<T>* spans, int nspan, int m, int tc, const T* Y, T* G, T* part_buf,
                 size_t part_cap, hipStream_t s) {
  int nblk = 0;
  for (int i = 0; i < nspan; ++i) nblk += spans[i].nblk;
  const int nch = gram_chunks(n, nblk, part_cap, m, tc);
  const int rpc = cdiv(n, nch);
  T* dst = (nch == 1) ? G : part_buf;
  for (int i = 0; i < nspan; ++i) {
    switch (tc) {
#define C(TC)                                                              \
  case TC:                                                                 \
    gram_span_wq<T, TC>(n, spans[i], rpc, nch, Y, dst, m, s);              \
    break;
      ECG_TC_CASES(C)
#undef C
    }
  }
  if (nch > 1) {
    const long long len = (long long)m * tc;
    stat_begin(s);
    hipLaunchKernelGGL((k_reduce_chunks<T>), dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, len, nch, part_buf, G);
    stat_end(kStatGramReduce, (double)sizeof(T) * (nch + 1) * len, (double)nch * len, s);
  }
}

template <typename T, int TC>
static void update_span(int n, const Span<T>& sp, const T* G, T* W, hipStream_t s) {
  const int nwg = cdiv(n, kBlock / TC);
  switch (sp.width) {
#define C(WQ)                                                                                     \
  case WQ:                                                                                        \
    stat_begin(s);                                                                               \
    hipLaunchKernelGGL((k_update<T, WQ, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, sp, G, W); \
    stat_end(kStatUpdate, (double)sizeof(T) * n * ((double)sp.nblk * WQ + 2.0 * TC),             \
             2.0 * n * sp.nblk * WQ * TC, s);                                                    \
    break;
    ECG_TC_CASES(C)
#undef C
  }
}

template <typename T>
void launch_update(int n, const Span<T>* spans, int nspan, int tc, const T* G, T* W, hipStream_t s) {
  for (int i = 0; i < nspan; ++i) {
    switch (tc) {
#define C(TC)                                   \
  case TC:                                      \
    update_span<T, TC>(n, spans[i], G, W, s);   \
    break;
      ECG_TC_CASES(C)
#undef C
    }
  }
}

template <typename T>
void launch_small_gram(int n, int tc, const T* X, const T* Y, const T* r, double* part, double* out,
                       hipStream_t s) {
  int nch = cdiv(n, 256);
  if (nch > kSmallChunks) nch = kSmallChunks;
  const int rpc = cdiv(n, nch);
  const int nout = tc * tc + (r ? tc : 0);
  switch (tc) {
#define C(TC)                                                                                        \
  case TC:                                                                                           \
    if (r)                                                                                           \
      hipLaunchKernelGGL((k_small_gram<T, TC, true>), dim3(nch), dim3(kBlock), 0, s, n, rpc, X, Y, r, part); \
    else                                                                                             \
      hipLaunchKernelGGL((k_small_gram<T, TC, false>), dim3(nch), dim3(kBlock), 0, s, n, rpc, X, Y, r, part); \
    break;
    ECG_TC_CASES(C)
#undef C
  }
  hipLaunchKernelGGL(k_reduce_small, dim3(cdiv(nout, kBlock)), dim3(kBlock), 0, s, nout, nch, part, out);
}

void launch_factor(int mode, int tc, int tc_live, const double* in, double tau, double* inv, double* beta,
                   IterStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_factor, dim3(1), dim3(kBlock), 0, s, mode, tc, tc_live, in, tau, inv, beta, st);
}

template <typename T>
void launch_times_small(int n, int tc, const T* X, const double* M, T* out, hipStream_t s) {
  switch (tc) {
#define C(TC)                                                                                         \
  case TC: {                                                                                          \
    const int nwg = cdiv(n, kBlock / TC);                                                             \
    hipLaunchKernelGGL((k_times_small<T, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, X, M, out); \
    break;                                                                                            \
  }
    ECG_TC_CASES(C)
#undef C
  }
}

template <typename T, typename TX>
int launch_final_update(int n, int tc, const T* H, const T* Y, const double* Cinv, const double* beta, T* Wq,
                        T* Zn, TX* x, T* r, double* part, hipStream_t s) {
  int nwg = 0;
  switch (tc) {
#define C(TC)                                                                                          \
  case TC:                                                                                             \
    nwg = cdiv(n, kBlock / TC);                                                                        \
    stat_begin(s);                                                                                     \
    hipLaunchKernelGGL((k_final_update<T, TX, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, H, Y, Cinv, \
                       beta, Wq, Zn, x, r, part);                                                      \
    stat_end(kStatFinal, 4.0 * sizeof(T) * n * TC + (double)n * (2 * sizeof(TX) + 2 * sizeof(T)),      \
             4.0 * n * TC * TC + 4.0 * n * TC, s);                                                     \
    break;
    ECG_TC_CASES(C)
#undef C
  }
  return nwg;
}

template <typename T>
void launch_trisolve(const DevTri& M, int which, int tc, const T* X, T* Y, hipStream_t s) {
  const DevCsr& F = which == 0 ? M.L : M.U;
  const int* lp = which == 0 ? M.lvl_ptr_L : M.lvl_ptr_U;
  const int* lr = which == 0 ? M.lvl_rows_L : M.lvl_rows_U;
  switch (tc) {
#define C(TC)                                                                                        \
  case TC:                                                                                           \
    stat_begin(s);                                                                               \
    hipLaunchKernelGGL((k_trisolve<T, TC>), dim3(M.ngroups), dim3(kBlock), 0, s, which, F.rowptr, F.col, \
                       vals_of<T>(F), lp, lr, M.maxlev, X, Y);                                       \
    stat_end(kStatSplit, (double)F.nnz * (sizeof(T) + 4) + 4.0 * (F.n + 1) + 2.0 * sizeof(T) * F.n * TC, \
             2.0 * F.nnz * TC, s);                                                               \
    break;
    ECG_TC_CASES(C)
#undef C
  }
}

void launch_ic0(const DevCsr& A, DevTri& M, const int* apos, int* fail, hipStream_t s) {
  hipLaunchKernelGGL(k_ic0, dim3(M.ngroups), dim3(kBlock), 0, s, M.L.rowptr, M.L.col, M.L.val, apos, A.val,
                     M.lvl_ptr_L, M.lvl_rows_L, M.maxlev, fail);
}

// explicit instantiations
#define INST(T)                                                                                          \
  template void launch_spmm<T>(const DevCsr&, int, const T*, T*, hipStream_t);                           \
  template void launch_split<T>(int, const int*, int, int, const double*, T*, hipStream_t);             \
  template void launch_split_t<T>(int, const int*, int, int, const T*, T*, hipStream_t);                \
  template void launch_gram<T>(int, const Span<T>*, int, int, int, const T*, T*, T*, size_t, hipStream_t); \
  template void launch_update<T>(int, const Span<T>*, int, int, const T*, T*, hipStream_t);             \
  template void launch_small_gram<T>(int, int, const T*, const T*, const T*, double*, double*, hipStream_t); \
  template void launch_times_small<T>(int, int, const T*, const double*, T*, hipStream_t);              \
  template void launch_trisolve<T>(const DevTri&, int, int, const T*, T*, hipStream_t);
INST(double)
INST(float)
#undef INST
template int launch_final_update<double, double>(int, int, const double*, const double*, const double*,
                                                 const double*, double*, double*, double*, double*, double*,
                                                 hipStream_t);
template int launch_final_update<float, double>(int, int, const float*, const float*, const double*,
                                                const double*, float*, float*, double*, float*, double*,
                                                hipStream_t);

}  // namespace ecg
