// Internal declarations shared by the kernel and driver translation units.
// Not part of the public ABI (include/ecg.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ecg {

constexpr int kBlock = 256;      // threads per workgroup for streaming kernels
constexpr int kMaxT = 64;        // widest block (t x t factor runs in one workgroup)
constexpr int kSmallChunks = 4096;  // partial sums of the t x t Grams (one wavefront each)

// Device copy of a sparse matrix in CSR form (int32 row pointers).
constexpr int kMaxDiag = 16;  // diagonal (DIA) form kept for matrices with at most this many
struct DiaOffsets {
  int off[kMaxDiag];  // distinct column - row offsets, ascending
};
struct DevCsr {
  int n = 0;
  int nnz = 0;
  int* rowptr = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;  // FP32 copy of val
  // diagonal form of the same matrix (ndiag = 0 when not kept): dval[d*n + i] = a(i, i+off[d]),
  // 0 where that entry is absent or outside the matrix
  int ndiag = 0;
  DiaOffsets dia{};
  double* dval = nullptr;
  float* dvalf = nullptr;
  // grid stencil (gnx = 0 when not one): the diagonal form has the offsets
  // -c, -b, -a, 0, a, b, c (7 diagonals) or -c, -a, 0, a, c (5, then b = c) with
  // b = gnx, c = gnx * gny and n = gnz * c, so that row z*c + y*b + x has its +-b and +-c
  // neighbours at (x, y +- 1, z) and (x, y, z +- 1); a = ga is any remaining offset.
  int gnx = 0, gny = 0, gnz = 0, ga = 0;
  // SELL-C-sigma form of a general matrix (kept when there is no diagonal form; nslice = 0
  // otherwise): rows sorted by length, longest first, within windows of kSellSigma rows, cut
  // into slices of kSellC consecutive sorted rows; slice s holds sell_len[s] entries per row
  // (its longest row), stored entry-major from sell_ptr[s]: entry k of the slice's row i at
  // sell_ptr[s] + k * kSellC + i.  Rows shorter than the slice are padded with weight 0 on
  // their own column.  sell_row[p] is the original row at sorted position p (-1 past n).
  int nslice = 0;
  int* sell_ptr = nullptr;
  int* sell_len = nullptr;
  int* sell_row = nullptr;
  int* sell_col = nullptr;
  double* sell_val = nullptr;
  float* sell_valf = nullptr;
};
constexpr int kSellC = 64;      // rows per SELL slice
constexpr int kSellSigma = 1024;  // sorting window of the SELL form

// Which product kernel launch_spmm uses (the automatic choice takes the most specific one
// the matrix has).
enum SpmmKernel { kSpmmAuto = -1, kSpmmCsr = 0, kSpmmDia = 1, kSpmmGrid = 2, kSpmmGridLds = 3, kSpmmGridDma = 4,
                  kSpmmSell = 5 };
// whether the LDS-staged grid kernels apply to A at block width tc, elt bytes per value
bool spmm_grid_lds_ok(const DevCsr& A, int tc, int elt);
bool spmm_grid_dma_ok(const DevCsr& A, int tc, int elt);

// One contiguous run of stored blocks of equal width: block j of the span starts at
// base + j * stride (elements); its Gram rows start at goff + j * width.
template <typename T>
struct Span {
  const T* base;
  long long stride;
  int nblk;
  int width;
  int goff;
};

// Per-iteration values read back by the host (one small D2H copy per iteration).
struct IterStatus {
  double rr;          // ||r||^2 after the update
  int keep_e;         // columns kept by the Euclidean QR step
  int keep_a;         // columns kept by the A-step
  int breakdown;      // non-positive pivot with deflation disabled
  int pad;
};

// ------------------------------------------------------------------ kernel timing
// Classes as documented for ecg_kernel_stats in include/ecg.h.
enum StatClass {
  kStatSpmm = 0, kStatGram = 1, kStatGramReduce = 2, kStatUpdate = 3, kStatSmallGram = 4,
  kStatFactor = 5, kStatTimesSmall = 6, kStatFinal = 7, kStatSplit = 8, kStatVector = 9, kNumStat = 10
};
extern bool g_stats_on;
// Message returned by ecg_last_error() (thread-local), for translation units other than
// the driver.
void set_last_error(const char* msg);
// Record an event before a launch / after it (no-ops unless timing is enabled).
void stat_begin(hipStream_t s);
void stat_end(int cls, double bytes, double flops, hipStream_t s);

// ------------------------------------------------------------------ launchers
// All launchers enqueue on `s` and do not synchronise.

// y = b - A x (FP64); per-workgroup partial sums of y_i^2 into part[grid]; returns grid.
int launch_residual(const DevCsr& A, const double* b, const double* x, double* y, double* part,
                    hipStream_t s);
// y = A x (FP64 vector).
void launch_spmv(const DevCsr& A, const double* x, double* y, hipStream_t s);
// out = sum of part[0..m) in a fixed order (single workgroup); out is device double.
void launch_sum(const double* part, int m, double* out, hipStream_t s);

// Y = A X for row-major n x tc blocks.
template <typename T>
void launch_spmm(const DevCsr& A, int tc, const T* X, T* Y, hipStream_t s, int kernel = kSpmmAuto);

// out = [T^{tc}(v)] with the map (part >> level); row-major n x tc (tc >= subdomain count).
template <typename T>
void launch_split(int n, const int* part, int level, int tc, const double* v, T* out, hipStream_t s);
template <typename T>
void launch_split_t(int n, const int* part, int level, int tc, const T* v, T* out, hipStream_t s);

// CGS2 Gram G = Q^T Y for a list of spans; G is (sum of span widths*nblk) x tc, in T.
// part_buf must hold nchunks * m * tc values; returns after enqueueing partials + reduce.
template <typename T>
void launch_gram(int n, const Span<T>* spans, int nspan, int m, int tc, const T* Y, T* G,
                 T* part_buf, size_t part_cap, hipStream_t s);

// W -= Q G for the same spans.
template <typename T>
void launch_update(int n, const Span<T>* spans, int nspan, int tc, const T* G, T* W, hipStream_t s);

// t x t Grams in FP64: out[0 .. tc*tc) = X^T Y (row a, col b), and if r != nullptr
// out[tc*tc .. tc*tc+tc) = X^T r.  part must hold kSmallChunks*(tc*tc+tc) doubles.
template <typename T>
void launch_small_gram(int n, int tc, const T* X, const T* Y, const T* r, double* part, double* out,
                       hipStream_t s);

// Cholesky with column deflation of a tc x tc SPD matrix (FP64), single workgroup.
// mode 0 (Euclidean step): in = E; writes Rinv (tc x tc, upper, zero rows/cols for dropped
//   columns) and st->keep_e.
// mode 1 (A step): in = S followed by u (tc); writes Cinv, beta = Cinv Cinv^T u (tc) and
//   st->keep_a.
// tc_live: columns >= tc_live are padding (always dropped, not counted as deflated).
// ref (nullable): a tc x tc matrix whose diagonal is the pivot-test reference (mode 0).
void launch_factor(int mode, int tc, int tc_live, const double* in, const double* ref, double tau, double* inv,
                   double* beta, IterStatus* st, hipStream_t s);
// MSDO-CG candidate: out = S + P diag(-u) for row-major n x tc blocks (u: tc values).
template <typename T>
void launch_msdo_combine(int n, int tc, const T* S, const T* P, const double* u, T* out, hipStream_t s);

// out = X M for row-major n x tc X and a tc x tc matrix M (FP64, converted to T).
template <typename T>
void launch_times_small(int n, int tc, const T* X, const double* M, T* out, hipStream_t s);

// Final fused update: Wq = H Cinv (stored block), Zn = Y Cinv (next candidate),
// x += H beta, r -= Y beta, per-workgroup partial sums of r^2 (returns grid size).
template <typename T, typename TX>
int launch_final_update(int n, int tc, const T* H, const T* Y, const double* Cinv,
                        const double* beta, T* Wq, T* Zn, TX* x, T* r, double* part, hipStream_t s);

// Zero the first bytes (rounded up to 8) of p; p 8-byte aligned.
void launch_zero(void* p, size_t bytes, hipStream_t s);
// Precision conversion helpers.
void launch_cast_d2f(int n, const double* in, float* out, hipStream_t s);
void launch_axpy_f2d(int n, const float* d, double* x, hipStream_t s, double alpha = 1.0);  // x += alpha d
void launch_axpy_d(int n, const double* d, double* x, hipStream_t s);    // x += d
void launch_cast_val(int nnz, const double* in, float* out, hipStream_t s);
// r = (float)(b - A x) computed in FP64; partial sums of the FP64 residual squared.
int launch_residual_f(const DevCsr& A, const double* b, const double* x, float* r, double* part,
                      hipStream_t s);

// ---- block-Jacobi IC(0) and sparse triangular solves -------------------------
struct DevTri {
  // Lower factor L (CSR, diagonal last in each row) and L^T (CSR, diagonal first),
  // rows grouped by independent group (subdomain) and level.
  DevCsr L, U;
  int ngroups = 0;
  int* lvl_ptr_L = nullptr;   // [ngroups*(maxlev+1)] row-list offsets per (group, level)
  int* lvl_rows_L = nullptr;  // row ids ordered by (group, level)
  int* lvl_ptr_U = nullptr;
  int* lvl_rows_U = nullptr;
  int maxlev = 0;
  int* loc = nullptr;  // [n] index of each row within its group (rows of a group in order)
  int maxrows = 0;     // rows of the largest group
  // for the LDS sweeps, per factor (L, U): the row range of the p-th row in level order
  // (kr[2p], kr[2p+1]) and the group-local column of every entry
  int* kr_L = nullptr;
  int* kr_U = nullptr;
  int* lcol_L = nullptr;
  int* lcol_U = nullptr;
};
// Y = L^{-1} X (which = 0) or Y = L^{-T} X (which = 1) for row-major n x tc blocks.
template <typename T>
void launch_trisolve(const DevTri& M, int which, int tc, const T* X, T* Y, hipStream_t s);

// Block-Jacobi exact Cholesky in panel form (see ecg_band.hip for the layout).
constexpr int kPanel = 32;    // rows per panel
constexpr int kBandMax = 128; // widest band (multiple of kPanel)
struct DevBand {
  int n = 0;
  int nblocks = 0;
  int W = 0;                      // band: 32, 64 or 128 (kBandMax)
  long long npanels = 0;
  int* row_off = nullptr;         // [nblocks+1] offsets into rows
  int* rows = nullptr;            // global row of every local row, block by block
  long long* panel_off = nullptr; // [nblocks+1] first panel of each block
  double* panels = nullptr;       // npanels records of 2 P^2 + 2 P W doubles
};
void launch_band_chol(const DevBand& B, const int* row_off, const long long* ab_off, double* ab, int* fail,
                      hipStream_t s);
void launch_band_panels(const DevBand& B, const long long* ab_off, const double* ab, hipStream_t s);
template <typename T>
void launch_band_solve(const DevBand& B, int which, int tc, const T* X, T* Y, hipStream_t s);
// IC(0) numeric factorisation into M.L.val (pattern already set), FP64; sets *fail.
void launch_ic0(const DevCsr& A, DevTri& M, const int* diag_pos_A, int* fail, hipStream_t s);
// Copy L values into U (transpose) using a precomputed permutation U.val[k] = L.val[perm[k]].
void launch_gather(int nnz, const double* src, const int* perm, double* dst, hipStream_t s);

}  // namespace ecg
