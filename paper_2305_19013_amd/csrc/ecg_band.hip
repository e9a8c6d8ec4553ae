// Block-Jacobi exact Cholesky preconditioner (Section 5.3, eq. (cholprec)): every diagonal
// block A_g of A is factored A_g = L_g L_g^T with fill, and L^{-1}, L^{-T} are applied
// blockwise.  Blocks are independent of the ECG partition (the paper uses 64 or 128 of
// them for every t).
//
// Storage.  Within a block the rows keep the matrix order; the band W of a block is the
// largest distance, in that local order, between a row and a column of A it couples to
// (rounded up to 32, 64 or 128).  A 2D grid block of w cells per
// grid row has W = w.  The factor is kept in column band form during the factorisation,
// ab[j*(W+1) + d] = L[j+d][j], and then re-packed per panel of kPanel rows:
//   [ Dinv | F | Dinv^T | B ]      Dinv = (L_pp)^{-1}                  (P x P)
//                                  F    = Dinv L[p rows, W rows before] (P x W)
//                                  B    = Dinv^T L[W rows after, p rows]^T (P x W)
// so that a forward sweep is  Y_p = Dinv X_p - F Y_prev  and a backward sweep is
// Y_p = Dinv^T X_p - B Y_next: one small dense product per panel, with the W neighbouring
// rows of Y kept in LDS.  Rows past the end of a block are identity rows.
#include <hip/hip_runtime.h>

#include "ecg_internal.h"

namespace ecg {

namespace {

// Entry L[i][j] of a block's band factor (ng rows); identity past the end.
__device__ inline double band_get(const double* ab, int ng, int W, int i, int j) {
  if (i >= ng || j >= ng) return i == j ? 1.0 : 0.0;
  if (j < 0 || i < j || i - j > W) return 0.0;
  return ab[(size_t)j * (W + 1) + (i - j)];
}

// Right-looking band Cholesky, one workgroup per block.  The W+1 active columns
// j..j+W live in LDS (column j+c in slot (j+c) mod (W+1)); a finished column is
// written back and the slot takes column j+W+1.
__global__ void __launch_bounds__(kBlock)
k_band_chol(int W, const int* __restrict__ row_off, const long long* __restrict__ ab_off, double* __restrict__ ab,
            int* __restrict__ fail) {
  extern __shared__ double win[];  // (W+1) x (W+1)
  const int g = blockIdx.x;
  const int ng = row_off[g + 1] - row_off[g];
  double* a = ab + ab_off[g];
  const int ld = W + 1;
  const int tid = threadIdx.x;
  for (int e = tid; e < ld * ld; e += blockDim.x) {
    const int c = e / ld, d = e % ld;
    win[e] = (c < ng) ? a[(size_t)c * ld + d] : 0.0;
  }
  __syncthreads();
  __shared__ double piv_s;
  for (int j = 0; j < ng; ++j) {
    double* cj = win + (size_t)(j % ld) * ld;
    if (tid == 0) {
      double piv = cj[0];
      if (!(piv > 0.0)) {
        atomicOr(fail, 1);
        piv = 1.0;
      }
      piv_s = sqrt(piv);
    }
    __syncthreads();
    const double ljj = piv_s;
    for (int d = tid; d <= W; d += blockDim.x) {
      const double v = (d == 0) ? ljj : ((j + d < ng) ? cj[d] / ljj : 0.0);
      cj[d] = v;
      a[(size_t)j * ld + d] = v;
    }
    __syncthreads();
    // trailing update of columns j+1..j+W: L[j+d][j+c] -= L[j+d][j] L[j+c][j], d >= c
    for (int e = tid; e < W * W; e += blockDim.x) {
      const int c = e / W + 1, d = e % W + 1;
      if (d >= c && j + d < ng) win[(size_t)((j + c) % ld) * ld + (d - c)] -= cj[d] * cj[c];
    }
    __syncthreads();
    // slot of column j takes column j+W+1
    const int nc = j + W + 1;
    for (int d = tid; d <= W; d += blockDim.x) cj[d] = (nc < ng) ? a[(size_t)nc * ld + d] : 0.0;
    __syncthreads();
  }
}

// One workgroup per panel: invert the P x P diagonal block and form F and B.
__global__ void __launch_bounds__(kBlock)
k_band_panels(int W, int nblocks, const int* __restrict__ row_off, const long long* __restrict__ ab_off,
              const double* __restrict__ ab, const long long* __restrict__ panel_off, double* __restrict__ panels) {
  constexpr int P = kPanel;
  __shared__ double D[P][P + 1];
  __shared__ double Di[P][P + 1];
  const long long gp = blockIdx.x;
  int lo = 0, hi = nblocks - 1;  // block of this panel: panel_off[g] <= gp < panel_off[g+1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (panel_off[mid] <= gp) lo = mid; else hi = mid - 1;
  }
  const int g = lo;
  const int ng = row_off[g + 1] - row_off[g];
  const double* a = ab + ab_off[g];
  const int i0 = (int)(gp - panel_off[g]) * P;
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += blockDim.x) {
    const int r = e / P, c = e % P;
    D[r][c] = band_get(a, ng, W, i0 + r, i0 + c);
  }
  __syncthreads();
  // Di = D^{-1}: thread c solves D x = e_c by forward substitution
  if (tid < P) {
    const int c = tid;
    for (int r = 0; r < P; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) s -= D[r][k] * Di[k][c];
      Di[r][c] = (r < c) ? 0.0 : s / D[r][r];
    }
  }
  __syncthreads();
  const long long PS = 2LL * P * P + 2LL * P * W;
  double* out = panels + gp * PS;
  double* oDi = out;
  double* oF = out + P * P;
  double* oDt = oF + (size_t)P * W;
  double* oB = oDt + P * P;
  for (int e = tid; e < P * P; e += blockDim.x) {
    const int r = e / P, c = e % P;
    oDi[e] = Di[r][c];
    oDt[e] = Di[c][r];
  }
  for (int e = tid; e < P * W; e += blockDim.x) {
    const int r = e / W, c = e % W;
    // F[r][c] = sum_k Di[r][k] L[i0+k][i0-W+c]
    double f = 0.0;
    for (int k = 0; k <= r; ++k) f += Di[r][k] * band_get(a, ng, W, i0 + k, i0 - W + c);
    oF[e] = f;
    // B[r][c] = sum_k Di[k][r] L[i0+P+c][i0+k]
    double b = 0.0;
    for (int k = r; k < P; ++k) b += Di[k][r] * band_get(a, ng, W, i0 + P + c, i0 + k);
    oB[e] = b;
  }
}

// Y = L^{-1} X (FWD) or L^{-T} X for row-major n x ldx blocks; grid (nblocks, ldx / CW),
// CW dividing ldx; the band W is a power of two (32, 64 or 128), so the ring of the last W
// rows of Y is indexed with a mask.
// Thread (r, c) < P*CW computes row r, column c of a panel; all kBlock threads stage the
// panel matrices, those of the next two steps (and their right-hand side rows) held in
// registers while the current one is used: a step is shorter than one round trip to
// memory, so one step of look-ahead left the sweep waiting on its loads.  In LDS the matrix rows are padded by one double so the
// rows read by one wavefront fall on different banks.
template <typename T, int CW, int W, bool FWD>
__global__ void __launch_bounds__(kBlock)
k_band_solve(const int* __restrict__ row_off, const int* __restrict__ rows, const long long* __restrict__ panel_off,
             const double* __restrict__ panels, int ldx, const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int P = kPanel;
  constexpr int LDD = P + 1, LDF = W + 1;          // padded LDS row strides of Dinv and F
  constexpr int MS = P * LDD + P * LDF;            // LDS doubles of one staged panel
  constexpr int ME = P * (P + W);                  // doubles of one sweep's half of a record
  constexpr int NPF = (ME + kBlock - 1) / kBlock;
  constexpr long long PS = 2LL * P * P + 2LL * P * W;
  __shared__ double mat[2][MS];
  __shared__ double xs[P][CW];
  __shared__ double yw[W][CW];
  const int g = blockIdx.x;
  const int c0 = blockIdx.y * CW;
  const int ng = row_off[g + 1] - row_off[g];
  const int* rw = rows + row_off[g];
  const long long p0 = panel_off[g];
  const int npan = (int)(panel_off[g + 1] - p0);
  const long long half = FWD ? 0 : (long long)P * (P + W);
  const int tid = threadIdx.x;
  const int r = tid / CW, c = tid % CW;
  const bool worker = tid < P * CW;
  for (int e = tid; e < W * CW; e += kBlock) yw[e / CW][e % CW] = 0.0;
  // the matrices (and right-hand side rows) of a step are requested two steps ahead, into
  // one of two register buffers: even steps use pfa / xa, odd steps pfb / xb
  double pfa[NPF], pfb[NPF];
  auto fetch = [&](double (&pf)[NPF], int step) {
    const int p = FWD ? step : npan - 1 - step;
    const double* src = panels + (p0 + p) * PS + half;
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int e = tid + q * kBlock;
      pf[q] = (e < ME) ? src[e] : 0.0;
    }
  };
  auto stash = [&](const double (&pf)[NPF], int buf) {
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
      const int e = tid + q * kBlock;
      if (e < P * P) {
        mat[buf][(e / P) * LDD + e % P] = pf[q];
      } else if (e < ME) {
        const int f = e - P * P;
        mat[buf][P * LDD + (f / W) * LDF + f % W] = pf[q];
      }
    }
  };
  // the right-hand side value of row i0 + r and that row's global index, which the step
  // also needs for its store of Y
  auto load_x = [&](int step, double& xv, int& gi) {
    const int i = (FWD ? step : npan - 1 - step) * P + r;
    gi = (worker && i < ng) ? rw[i] : -1;
    xv = gi >= 0 ? (double)X[(size_t)gi * ldx + c0 + c] : 0.0;
  };
  double xa = 0.0, xb = 0.0;
  int ga = -1, gb = -1;
  if (npan > 0) {
    fetch(pfa, 0);
    load_x(0, xa, ga);
    stash(pfa, 0);
  }
  if (npan > 1) {
    fetch(pfb, 1);
    load_x(1, xb, gb);
  }
  // one step: its matrices are in mat[step & 1] and its right-hand side in x_mine; the
  // buffers pf_mine / x_mine are free again and take step + 2, and pf_next (step + 1) is
  // staged at the end
  auto body = [&](int step, double (&pf_mine)[NPF], double& x_mine, int& g_mine, const double (&pf_next)[NPF]) {
    const int buf = step & 1;
    const int p = FWD ? step : npan - 1 - step;
    const int i0 = p * P;
    const double xcur = x_mine;
    const int gcur = g_mine;
    if (step + 2 < npan) {
      fetch(pf_mine, step + 2);
      load_x(step + 2, x_mine, g_mine);
    }
    if (worker) xs[r][c] = xcur;
    __syncthreads();  // xs, mat[buf] ready
    double acc = 0.0;
    if (worker) {
      const double* mD = mat[buf] + r * LDD;             // row r of Dinv (Dinv^T)
      const double* mF = mat[buf] + P * LDD + r * LDF;   // row r of F (B)
#pragma unroll 8
      for (int k = 0; k < P; ++k) acc += mD[k] * xs[k][c];
      // coupling rows: FWD row i0-W+k, BWD row i0+P+k; both sit in slot (i0 [+P] + k) mod W
      const int base = FWD ? i0 : i0 + P;
#pragma unroll 8
      for (int k = 0; k < W; ++k) acc -= mF[k] * yw[(base + k) & (W - 1)][c];
    }
    __syncthreads();  // window reads done before the slots of the oldest rows are reused
    if (worker) {
      yw[(i0 + r) & (W - 1)][c] = acc;
      if (gcur >= 0) Y[(size_t)gcur * ldx + c0 + c] = (T)acc;
    }
    if (step + 1 < npan) stash(pf_next, buf ^ 1);  // mat[buf ^ 1] was last read before the first barrier
  };
  for (int step = 0; step < npan; step += 2) {
    body(step, pfa, xa, ga, pfb);
    if (step + 1 < npan) body(step + 1, pfb, xb, gb, pfa);
  }
}

template <typename T, int CW, int W>
void band_launch(const DevBand& B, int which, int tc, const T* X, T* Y, hipStream_t s) {
  dim3 grid(B.nblocks, tc / CW);
  if (which == 0)
    hipLaunchKernelGGL((k_band_solve<T, CW, W, true>), grid, dim3(kBlock), 0, s, B.row_off, B.rows, B.panel_off,
                       B.panels, tc, X, Y);
  else
    hipLaunchKernelGGL((k_band_solve<T, CW, W, false>), grid, dim3(kBlock), 0, s, B.row_off, B.rows, B.panel_off,
                       B.panels, tc, X, Y);
}

template <typename T, int W>
void band_dispatch_cw(const DevBand& B, int which, int tc, const T* X, T* Y, hipStream_t s) {
  // columns per workgroup: the largest of 8, 4, 2, 1 that divides tc
  if (tc % 8 == 0)
    band_launch<T, 8, W>(B, which, tc, X, Y, s);
  else if (tc % 4 == 0)
    band_launch<T, 4, W>(B, which, tc, X, Y, s);
  else if (tc % 2 == 0)
    band_launch<T, 2, W>(B, which, tc, X, Y, s);
  else
    band_launch<T, 1, W>(B, which, tc, X, Y, s);
}

}  // namespace

void launch_band_chol(const DevBand& B, const int* row_off, const long long* ab_off, double* ab, int* fail,
                      hipStream_t s) {
  const size_t lds = (size_t)(B.W + 1) * (B.W + 1) * sizeof(double);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_band_chol), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(k_band_chol, dim3(B.nblocks), dim3(kBlock), lds, s, B.W, row_off, ab_off, ab, fail);
}

void launch_band_panels(const DevBand& B, const long long* ab_off, const double* ab, hipStream_t s) {
  hipLaunchKernelGGL(k_band_panels, dim3((unsigned)B.npanels), dim3(kBlock), 0, s, B.W, B.nblocks, B.row_off,
                     ab_off, ab, B.panel_off, B.panels);
}

template <typename T>
void launch_band_solve(const DevBand& B, int which, int tc, const T* X, T* Y, hipStream_t s) {
  stat_begin(s);
  if (B.W == 32)
    band_dispatch_cw<T, 32>(B, which, tc, X, Y, s);
  else if (B.W == 64)
    band_dispatch_cw<T, 64>(B, which, tc, X, Y, s);
  else
    band_dispatch_cw<T, kBandMax>(B, which, tc, X, Y, s);
  // algorithmic bytes: one half of every panel record, X and Y once
  stat_end(kStatSplit, 8.0 * (double)B.npanels * kPanel * (kPanel + B.W) * (tc > 8 ? tc / 8 : 1) +
                           2.0 * sizeof(T) * B.n * tc + 4.0 * B.n,
           2.0 * (double)B.npanels * kPanel * (kPanel + B.W) * tc, s);
}

template void launch_band_solve<double>(const DevBand&, int, int, const double*, double*, hipStream_t);
template void launch_band_solve<float>(const DevBand&, int, int, const float*, float*, hipStream_t);

}  // namespace ecg
