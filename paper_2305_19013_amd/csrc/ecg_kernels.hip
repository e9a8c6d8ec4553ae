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

// First stage of a long sum: workgroup b adds the fixed slice [b*per, (b+1)*per).
__global__ void __launch_bounds__(kBlock)
k_sum_stage(const double* __restrict__ part, int m, int per, double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int lo = blockIdx.x * per;
  const int hi = min(m, lo + per);
  double acc = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kBlock) acc += part[i];
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_cast_d2f(int n, const double* __restrict__ in, float* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void __launch_bounds__(kBlock) k_axpy_f2d(int n, double alpha, const float* __restrict__ d,
                                                     double* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += alpha * (double)d[i];
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
// Y is written with non-temporal stores in all three product kernels: the next kernel (the
// CGS2 Gram) streams the stored basis, and Y lines left dirty in the caches cost it
// write-backs in the middle of that stream (measured: the Gram and the t x t Grams after it
// run 3-5% faster).
// Y = A X, row-major n x TC blocks.  Each lane owns VL consecutive columns of one row
// (one 16-byte load of X per nonzero), so TC / VL lanes share a row and a wavefront reads
// whole contiguous block rows of X.  The nonzeros of a row are taken eight at a time: the
// column indices and values first, then the eight block-row loads of X back to back, so
// the gathers of a stencil row are all in flight together; a slot past the end of the row
// re-reads the row's own block row with weight zero (the diagonal is always present).
// Products are summed in the stored order of the row, one FMA each.
// acc += a * x, one fused multiply-add per component: all three product kernels build a row
// as the same chain of correctly rounded FMAs in ascending column order, whatever the
// compiler would contract on its own.
__device__ __forceinline__ double fmac(double a, double x, double acc) { return __builtin_fma(a, x, acc); }
__device__ __forceinline__ float fmac(float a, float x, float acc) { return __builtin_fmaf(a, x, acc); }
template <typename T, typename V, int VL>
__device__ __forceinline__ void fma_row(V& acc, T a, const V& x) {
#pragma unroll
  for (int e = 0; e < VL; ++e) acc[e] = fmac(a, x[e], acc[e]);
}

template <typename T, int TC>
struct SpmmShape {
  static constexpr int VL = (16 / (int)sizeof(T)) < TC ? (16 / (int)sizeof(T)) : TC;  // columns per lane
  static constexpr int LPR = TC / VL;                                                   // lanes per row
  static constexpr int RPB = kBlock / LPR;                                              // rows per workgroup
};

template <typename T, int TC>
__global__ void __launch_bounds__(kBlock)
k_spmm(int n, int nwg, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v,
       const T* __restrict__ X, T* __restrict__ Y) {
  using S = SpmmShape<T, TC>;
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  constexpr int KB = 8;
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int row = blk * S::RPB + (int)threadIdx.x / S::LPR;
  const int c = ((int)threadIdx.x % S::LPR) * S::VL;
  if (row >= n) return;
  const T* __restrict__ Xc = X + c;
  Vec acc = Vec(0);
  const int k0 = rp[row], k1 = rp[row + 1];
  for (int kb = k0; kb < k1; kb += KB) {
    int col[KB];
    T val[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const bool ok = kb + u < k1;
      col[u] = ok ? ci[kb + u] : row;
      val[u] = ok ? v[kb + u] : T(0);
    }
    Vec xv[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) xv[u] = *reinterpret_cast<const Vec*>(Xc + (size_t)col[u] * TC);
#pragma unroll
    for (int u = 0; u < KB; ++u) fma_row<T, Vec, S::VL>(acc, val[u], xv[u]);
  }
  __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Y + (size_t)row * TC + c));
}

// The same product for a matrix in SELL-C-sigma form (DevCsr): positions in the sorted row
// order; the LPR lanes of a position read its entries from the slice entry-major, so the
// rows of a wavefront read consecutive words for each entry, and write the result to the
// position's original row.  A row's entries come in the CSR order and the slice padding adds
// weight-zero terms on the row's own block row, so the result equals the CSR kernel's.
template <typename T, int TC>
__global__ void __launch_bounds__(kBlock)
k_spmm_sell(int npos, int nwg, const int* __restrict__ sptr, const int* __restrict__ slen,
            const int* __restrict__ srow, const int* __restrict__ scol, const T* __restrict__ sval,
            const T* __restrict__ X, T* __restrict__ Y) {
  using S = SpmmShape<T, TC>;
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  constexpr int KB = 8;
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int pos = blk * S::RPB + (int)threadIdx.x / S::LPR;
  if (pos >= npos) return;
  const int row = srow[pos];
  if (row < 0) return;  // padding position of the last slice
  const int c = ((int)threadIdx.x % S::LPR) * S::VL;
  const int sl = pos / kSellC, i = pos % kSellC;
  const int base = sptr[sl] + i, len = slen[sl];
  const T* __restrict__ Xc = X + c;
  Vec acc = Vec(0);
  for (int kb = 0; kb < len; kb += KB) {
    int col[KB];
    T val[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const bool ok = kb + u < len;
      col[u] = ok ? scol[base + (kb + u) * kSellC] : row;
      val[u] = ok ? sval[base + (kb + u) * kSellC] : T(0);
    }
    Vec xv[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) xv[u] = *reinterpret_cast<const Vec*>(Xc + (size_t)col[u] * TC);
#pragma unroll
    for (int u = 0; u < KB; ++u) fma_row<T, Vec, S::VL>(acc, val[u], xv[u]);
  }
  __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Y + (size_t)row * TC + c));
}

// Coefficients of a row of the diagonal form with few instructions: of the LPR lanes that
// share a row, lane li loads diagonals li, li + LPR, ... (coalesced along the rows) and
// the others read them across lanes.  Each wavefront load instruction costs the memory
// pipeline about as much for 64 broadcast values as for a 1 KB block row, so one load per
// NL diagonals instead of one per diagonal takes most of that cost away.  Rows with fewer
// than 4 lanes load their coefficients directly.
template <typename T, int LPR, int MAXD>
struct RowCoef {
  static constexpr bool kShuffle = LPR >= 4;
  static constexpr int NL = kShuffle ? (MAXD + LPR - 1) / LPR : MAXD;
  T v[NL];
  int lb;  // first lane of the row in the wavefront
  __device__ __forceinline__ void load(const T* __restrict__ dv, int n, int nd, int row) {
    const int li = (int)threadIdx.x % LPR;
    lb = ((int)threadIdx.x & 63) - li;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int d = kShuffle ? li + j * LPR : j;
      v[j] = d < nd ? dv[(size_t)d * n + row] : T(0);
    }
  }
  __device__ __forceinline__ T get(int d) const {
    if constexpr (kShuffle) return __shfl(v[d / LPR], lb + d % LPR);
    else return v[d];
  }
};

// The same product for a matrix kept in diagonal form: no index loads, the ND block-row
// gathers of a row issued together, the diagonal values read coalesced along the rows.
// Diagonals are summed in ascending offset order, the column order of the CSR rows, and an
// absent entry contributes 0 * x, so the result equals the CSR kernel's.
template <typename T, int TC, int MAXD>
__global__ void __launch_bounds__(kBlock)
k_spmm_dia(int n, int nwg, int nd, DiaOffsets dia, const T* __restrict__ dv, const T* __restrict__ X,
           T* __restrict__ Y) {
  using S = SpmmShape<T, TC>;
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  const int blk = xcd_block();
  if (blk >= nwg) return;
  const int row = blk * S::RPB + (int)threadIdx.x / S::LPR;
  const int c = ((int)threadIdx.x % S::LPR) * S::VL;
  if (row >= n) return;  // every lane of a row leaves together
  const T* __restrict__ Xc = X + c;
  RowCoef<T, S::LPR, MAXD> coef;
  coef.load(dv, n, nd, row);
  T val[MAXD];
  Vec xv[MAXD];
#pragma unroll
  for (int d = 0; d < MAXD; ++d) {
    const int j = row + dia.off[d];
    const bool ok = d < nd && j >= 0 && j < n;
    const T a = coef.get(d);
    val[d] = ok ? a : T(0);
    xv[d] = ok ? *reinterpret_cast<const Vec*>(Xc + (size_t)j * TC) : Vec(0);
  }
  Vec acc = Vec(0);
#pragma unroll
  for (int d = 0; d < MAXD; ++d)
    if (d < nd) fma_row<T, Vec, S::VL>(acc, val[d], xv[d]);
  __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Y + (size_t)row * TC + c));
}

// The diagonal-form product for a grid stencil (DevCsr::gnx > 0): rows are walked as a box,
// r = z*c + y*b + x.  A lane owns VL columns of K rows (x, y0..y0+K-1) and marches z
// through a segment of zseg planes, keeping the block rows of planes z-1, z, z+1 in
// registers: the +-c neighbours and, inside the K rows, the +-b ones are reused instead of
// re-read, so a row costs about 3 + 2/K block-row loads instead of 7.  Every term is the
// diagonal kernel's (same linear neighbour, same range test, same ascending order), so the
// result is bitwise that of k_spmm_dia.  ND = 7 (3-D) or 5 (2-D: b = c, gny = 1, K = 1).
template <typename T, int TC, int ND, int K>
__global__ void __launch_bounds__(kBlock)
k_spmm_grid(int n, int gnx, int gny, int gnz, int ga, int zseg, int nxb, int nyb, int nwork,
            const T* __restrict__ dv, const T* __restrict__ X, T* __restrict__ Y) {
  static_assert(ND == 7 || (ND == 5 && K == 1), "grid stencil shape");
  using S = SpmmShape<T, TC>;
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  const int w = xcd_block();
  if (w >= nwork) return;
  // x blocks fastest: the workgroups that share halo rows run together on one XCD
  const int bx = w % nxb, by = (w / nxb) % nyb, bz = w / (nxb * nyb);
  const int x = bx * S::RPB + (int)threadIdx.x / S::LPR;
  if (x >= gnx) return;  // every lane of a row leaves together
  const T* __restrict__ Xc = X + ((int)threadIdx.x % S::LPR) * S::VL;
  T* __restrict__ Yc = Y + ((int)threadIdx.x % S::LPR) * S::VL;
  const int b = gnx, c = gnx * gny;
  const int y0 = by * K;
  const int z0 = bz * zseg, z1 = min(gnz, z0 + zseg);
  const int rb = y0 * b + x;
  auto ld = [&](int r) -> Vec {
    return (r >= 0 && r < n) ? *reinterpret_cast<const Vec*>(Xc + (size_t)r * TC) : Vec(0);
  };
  Vec prev[K], cur[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    prev[k] = ld((z0 - 1) * c + rb + k * b);
    cur[k] = ld(z0 * c + rb + k * b);
  }
  for (int z = z0; z < z1; ++z) {
    const int r0 = z * c + rb;
    Vec nxt[K], xm[K], xp[K], ym, yp;
#pragma unroll
    for (int k = 0; k < K; ++k) nxt[k] = ld(r0 + k * b + c);
    if constexpr (ND == 7) {
      ym = ld(r0 - b);
      yp = ld(r0 + K * b);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      xm[k] = ld(r0 + k * b - ga);
      xp[k] = ld(r0 + k * b + ga);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (y0 + k >= gny) break;  // the same for the whole workgroup
      const int r = r0 + k * b;
      RowCoef<T, S::LPR, ND> coef;
      coef.load(dv, n, ND, r);
      auto term = [&](int d, int j, const Vec& xv, Vec& acc) {
        const T a = coef.get(d);
        fma_row<T, Vec, S::VL>(acc, (j >= 0 && j < n) ? a : T(0), xv);
      };
      Vec acc = Vec(0);
      if constexpr (ND == 7) {
        term(0, r - c, prev[k], acc);
        term(1, r - b, k > 0 ? cur[k > 0 ? k - 1 : 0] : ym, acc);
        term(2, r - ga, xm[k], acc);
        term(3, r, cur[k], acc);
        term(4, r + ga, xp[k], acc);
        term(5, r + b, k < K - 1 ? cur[k < K - 1 ? k + 1 : k] : yp, acc);
        term(6, r + c, nxt[k], acc);
      } else {
        term(0, r - c, prev[k], acc);
        term(1, r - ga, xm[k], acc);
        term(2, r, cur[k], acc);
        term(3, r + ga, xp[k], acc);
        term(4, r + c, nxt[k], acc);
      }
      __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Yc + (size_t)r * TC));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      prev[k] = cur[k];
      cur[k] = nxt[k];
    }
  }
}

// The grid-stencil product with each plane of block rows staged in LDS (3-D 7-point
// operators with unit x stride).  A workgroup owns a tile of RX x-rows by K y-rows and
// marches z through zseg planes.  For every plane it reads the tile with a one-row halo in
// x and y, (RX+2) x (K+2) block rows, once per workgroup (16 bytes per lane, contiguous
// along x), and the tile's seven coefficient rows, into LDS; a lane then takes its x and y
// neighbours and its coefficients from LDS and its z neighbours from registers (planes
// z-1, z, z+1 of its own rows).  The loads run two planes ahead: while plane z is
// computed, plane z+1 (already loaded) waits in registers to be written to LDS and plane
// z+2 is in flight, so a wavefront never waits for memory it asked for in the same plane.
// Loads go through buffer descriptors: a row outside [0, n) reads as zero with no branch,
// so every plane issues the same loads and each wait covers only the plane it needs.  Each
// LDS slot holds X at the linear index of its tile position (zero outside [0, n)), and
// every term has the diagonal kernel's neighbour, range test and place in the ascending
// chain of FMAs, so the result is bitwise that of k_spmm_dia and k_spmm_grid.
template <typename T, int TC, int K>
struct GridLds {
  using S = SpmmShape<T, TC>;
  static constexpr int RX = S::RPB;              // x rows of a tile
  static constexpr int TX = RX + 2, TY = K + 2;  // with the halo
  static constexpr int CPR = S::LPR;             // 16-byte chunks per block row
  static constexpr int HALO = 2 * TX + 2 * K;    // halo rows per plane
  static constexpr int HCH = (HALO * CPR + kBlock - 1) / kBlock;  // halo chunks per thread
  static constexpr int CE = 16 / (int)sizeof(T);                  // coefficients per chunk
  static constexpr int CCH = 7 * K * RX / CE;                     // coefficient chunks per plane
  static constexpr int CPT = (CCH + kBlock - 1) / kBlock;         // ... per thread
  static constexpr size_t kRowBytes = (size_t)TY * TX * CPR * 16;
  static constexpr size_t kCoefBytes = (size_t)K * RX * 8 * sizeof(T);
  static constexpr size_t kLds = 2 * (kRowBytes + kCoefBytes);
};

// CW: columns of the block one workgroup takes (CW < TC splits wide blocks into column
// groups, so that a tile of 512-byte FP64 rows keeps the x extent of a 256-byte one).
// Needs n * TC * sizeof(T) and 7 * n * sizeof(T) below 4 GiB (32-bit buffer offsets).
template <typename T, int TC, int CW, int K>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_spmm_grid_lds(int n, int gnx, int gny, int gnz, int zseg, int nxb, int nyb, int nwork,
                const T* __restrict__ dv, const T* __restrict__ X, T* __restrict__ Y) {
  static_assert(TC % CW == 0, "column groups");
  using G = GridLds<T, CW, K>;
  using S = typename G::S;
  static_assert(S::VL * (int)sizeof(T) == 16, "16-byte lane chunks");
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Vec* rows_lds = reinterpret_cast<Vec*>(lds_raw);                        // [2][TY][TX][CPR]
  T* coef_lds = reinterpret_cast<T*>(lds_raw + 2 * G::kRowBytes);         // [2][K][RX][8]
  const int w = xcd_block();
  if (w >= nwork) return;  // the whole workgroup leaves together
  const int tiles = nwork / (TC / CW);
  const int cg = w / tiles, wt = w % tiles;  // column group slowest: neighbouring tiles adjacent
  const int bx = wt % nxb, by = (wt / nxb) % nyb, bz = wt / (nxb * nyb);
  const int tid = (int)threadIdx.x;
  const int li = tid % G::CPR, xl = tid / G::CPR;
  const int b = gnx, c = gnx * gny;
  const int x0 = bx * G::RX, y0 = by * K;
  const int z0 = bz * zseg, z1 = min(gnz, z0 + zseg);
  const int x = x0 + xl;
  T* __restrict__ Yg = Y + cg * CW;
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, 0, (int)((size_t)n * TC * sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t cr =
      __builtin_amdgcn_make_buffer_rsrc((void*)dv, 0, (int)((size_t)7 * n * sizeof(T)), 0x00020000);
  constexpr unsigned kOut = 0xFFFFFFF0u;  // past the end of either buffer: reads as zero
  // linear index of tile position (yi, xi) of plane zz (halo included); 32-bit, since
  // n * TC * sizeof(T) < 4 GiB
  auto lin = [&](int zz, int yi, int xi) -> int { return zz * c + (y0 + yi - 1) * b + (x0 + xi - 1); };
  auto ldx = [&](int r, int chunk) -> Vec {
    const unsigned off = (r >= 0 && r < n) ? (unsigned)r * (unsigned)(TC * sizeof(T)) +
                                                 (unsigned)((cg * CW + chunk * S::VL) * sizeof(T))
                                           : kOut;
    return __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)off, 0, 0));
  };
  auto halo_pos = [&](int h, int& yi, int& xi) {
    if (h < G::TX) {
      yi = 0, xi = h;
    } else if (h < 2 * G::TX) {
      yi = G::TY - 1, xi = h - G::TX;
    } else {
      const int h2 = h - 2 * G::TX;
      yi = 1 + h2 / 2, xi = (h2 & 1) ? G::TX - 1 : 0;
    }
  };
  auto slot = [&](int buf, int yi, int xi, int chunk) -> Vec& {
    return rows_lds[(((size_t)buf * G::TY + yi) * G::TX + xi) * G::CPR + chunk];
  };
  // coefficient chunk q of plane zz -> (d, k, x .. x + CE - 1) of dv[d][row]; rows outside
  // [0, n) read as zero, and rows past the grid in x or y are never used
  auto ldc = [&](int zz, int q) -> Vec {
    const int per = G::RX / G::CE;
    const int xc = (q % per) * G::CE, dk = q / per, d = dk / K, k = dk % K;
    const int r = zz * c + (y0 + k) * b + x0 + xc;
    const unsigned off = (q < G::CCH && r >= 0 && r < n) ? ((unsigned)d * (unsigned)n + (unsigned)r) * (unsigned)sizeof(T) : kOut;
    return __builtin_bit_cast(Vec, __builtin_amdgcn_raw_buffer_load_b128(cr, (int)off, 0, 0));
  };
  auto stc = [&](int buf, int q, const Vec& v) {
    const int per = G::RX / G::CE;
    const int xc = (q % per) * G::CE, dk = q / per, d = dk / K, k = dk % K;
#pragma unroll
    for (int e = 0; e < G::CE; ++e) coef_lds[(((size_t)buf * K + k) * G::RX + xc + e) * 8 + d] = v[e];
  };
  auto load_own = [&](Vec (&o)[K], int zz) {
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = ldx(lin(zz, k + 1, xl + 1), li);
  };
  auto load_rest = [&](Vec (&h)[G::HCH], Vec (&cv)[G::CPT], int zz) {
#pragma unroll
    for (int i = 0; i < G::HCH; ++i) {
      const int q = tid + i * kBlock;
      int yi = 0, xi = 0;
      halo_pos(q / G::CPR, yi, xi);
      h[i] = ldx(q < G::HALO * G::CPR ? lin(zz, yi, xi) : -1, q % G::CPR);
    }
#pragma unroll
    for (int i = 0; i < G::CPT; ++i) cv[i] = ldc(zz, tid + i * kBlock);
  };
  auto store_plane = [&](int buf, const Vec (&o)[K], const Vec (&h)[G::HCH], const Vec (&cv)[G::CPT]) {
#pragma unroll
    for (int k = 0; k < K; ++k) slot(buf, k + 1, xl + 1, li) = o[k];
#pragma unroll
    for (int i = 0; i < G::HCH; ++i) {
      const int q = tid + i * kBlock;
      if (q < G::HALO * G::CPR) {
        int yi, xi;
        halo_pos(q / G::CPR, yi, xi);
        slot(buf, yi, xi, q % G::CPR) = h[i];
      }
    }
#pragma unroll
    for (int i = 0; i < G::CPT; ++i)
      if (tid + i * kBlock < G::CCH) stc(buf, tid + i * kBlock, cv[i]);
  };
  auto compute = [&](int z, int buf, const Vec (&prev)[K], const Vec (&cur)[K], const Vec (&nxt)[K]) {
    if (x >= gnx) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (y0 + k >= gny) break;  // the same for the whole workgroup
      const long long r = (long long)z * c + (long long)(y0 + k) * b + x;
      const T* cf = coef_lds + (((size_t)buf * K + k) * G::RX + xl) * 8;
      auto term = [&](int d, long long j, const Vec& xv, Vec& acc) {
        fma_row<T, Vec, S::VL>(acc, (j >= 0 && j < n) ? cf[d] : T(0), xv);
      };
      Vec acc = Vec(0);
      term(0, r - c, prev[k], acc);
      term(1, r - b, slot(buf, k, xl + 1, li), acc);
      term(2, r - 1, slot(buf, k + 1, xl, li), acc);
      term(3, r, cur[k], acc);
      term(4, r + 1, slot(buf, k + 1, xl + 2, li), acc);
      term(5, r + b, slot(buf, k + 2, xl + 1, li), acc);
      term(6, r + c, nxt[k], acc);
      __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Yg + (size_t)r * TC + li * S::VL));
    }
  };

  // Own rows rotate through four register sets (planes z-1, z, z+1 and the one in flight)
  // and the halo and coefficients through two, by unrolling the plane loop four times
  // rather than by copies: a copy of registers still being loaded would wait for them.
  Vec o0[K], o1[K], o2[K], o3[K];
  Vec ha[G::HCH], hb[G::HCH], ca[G::CPT], cb[G::CPT];
  // plane z0 into buffer 0; planes z0 - 1 and z0 + 1 of the own rows and the halo and
  // coefficients of z0 + 1 into registers
  load_own(o0, z0 - 1);
  load_own(o1, z0);
  load_rest(ha, ca, z0);
  store_plane(0, o1, ha, ca);
  load_own(o2, z0 + 1);
  load_rest(ha, ca, z0 + 1);
  __syncthreads();
  // plane z: plane z + 2 is requested (own rows while z + 2 <= z1, halo and coefficients
  // while z + 2 < z1), plane z is computed from planes z - 1, z, z + 1 of the own rows,
  // and plane z + 1 goes to the other LDS buffer
  auto step = [&](int z, const Vec (&pv)[K], const Vec (&cu)[K], const Vec (&n1)[K], Vec (&n2)[K],
                  const Vec (&h1)[G::HCH], Vec (&h2)[G::HCH], const Vec (&k1)[G::CPT], Vec (&k2)[G::CPT],
                  bool own2, bool rest2) {
    const int buf = (z - z0) & 1;
    if (own2) load_own(n2, z + 2);
    if (rest2) load_rest(h2, k2, z + 2);
    compute(z, buf, pv, cu, n1);
    store_plane(buf ^ 1, n1, h1, k1);  // that buffer was last read before the previous barrier
    __syncthreads();
  };
  int z = z0;
  for (; z + 5 < z1; z += 4) {
    step(z, o0, o1, o2, o3, ha, hb, ca, cb, true, true);
    step(z + 1, o1, o2, o3, o0, hb, ha, cb, ca, true, true);
    step(z + 2, o2, o3, o0, o1, ha, hb, ca, cb, true, true);
    step(z + 3, o3, o0, o1, o2, hb, ha, cb, ca, true, true);
  }
  // at most five planes are left, starting again with the first register arrangement
  if (z < z1) step(z, o0, o1, o2, o3, ha, hb, ca, cb, z + 2 <= z1, z + 2 < z1);
  if (z + 1 < z1) step(z + 1, o1, o2, o3, o0, hb, ha, cb, ca, z + 3 <= z1, z + 3 < z1);
  if (z + 2 < z1) step(z + 2, o2, o3, o0, o1, ha, hb, ca, cb, z + 4 <= z1, z + 4 < z1);
  if (z + 3 < z1) step(z + 3, o3, o0, o1, o2, hb, ha, cb, ca, z + 5 <= z1, z + 5 < z1);
  if (z + 4 < z1) step(z + 4, o0, o1, o2, o3, ha, hb, ca, cb, z + 6 <= z1, z + 6 < z1);
}

// The same product with the plane tiles brought into LDS by direct buffer loads (no
// registers in between): each lane's 16 bytes go straight to the lane's slot of a 1 KB
// stretch of the tile, and rows outside [0, n) read as zero through the buffer's range
// check.  Four tile planes rotate in LDS: plane z+2 is loaded while plane z is computed
// from planes z-1, z and z+1, so the z neighbours need no registers either.
template <typename T, int TC, int K>
struct GridDma {
  using S = SpmmShape<T, TC>;
  static constexpr int RX = S::RPB;
  static constexpr int TX = RX + 2, TY = K + 2;
  static constexpr int CPR = S::LPR;
  static constexpr int CH = TY * TX * CPR;              // 16-byte chunks of a tile plane
  static constexpr int NJ = (CH + 63) / 64;             // wave loads per plane
  static constexpr int CE = 16 / (int)sizeof(T);
  static constexpr int CCH = 7 * K * RX / CE;           // coefficient chunks per plane
  static constexpr int NCJ = (CCH + 63) / 64;
  static constexpr int R = 4;                           // planes in the ring
  static constexpr size_t kPlane = (size_t)NJ * 1024;
  static constexpr size_t kCoef = (size_t)NCJ * 1024;
  static constexpr size_t kLds = R * (kPlane + kCoef);
};

// s_waitcnt vmcnt(0) with the other counters left alone (gfx9 encoding)
__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <typename T, int TC, int K>
__global__ void __launch_bounds__(kBlock)
k_spmm_grid_dma(int n, int gnx, int gny, int gnz, int zseg, int nxb, int nyb, int nwork,
                const T* __restrict__ dv, const T* __restrict__ X, T* __restrict__ Y) {
  using G = GridDma<T, TC, K>;
  using S = typename G::S;
  typedef T Vec __attribute__((ext_vector_type(S::VL)));
  extern __shared__ __align__(1024) unsigned char lds_raw[];
  const int w = xcd_block();
  if (w >= nwork) return;  // the whole workgroup leaves together
  const int bx = w % nxb, by = (w / nxb) % nyb, bz = w / (nxb * nyb);
  const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = tid % G::CPR, xl = tid / G::CPR;
  const int b = gnx, c = gnx * gny;
  const int x0 = bx * G::RX, y0 = by * K;
  const int z0 = bz * zseg, z1 = min(gnz, z0 + zseg);
  const int x = x0 + xl;
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc((void*)X, 0, (int)((size_t)n * TC * sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t cr =
      __builtin_amdgcn_make_buffer_rsrc((void*)dv, 0, (int)((size_t)7 * n * sizeof(T)), 0x00020000);
  constexpr unsigned kOut = 0xFFFFFFF0u;  // past the end of either buffer: reads as zero
  auto plane_at = [&](int zz) -> unsigned char* {
    return lds_raw + (size_t)((zz - z0 + 1) & (G::R - 1)) * (G::kPlane + G::kCoef);
  };
  // enqueue plane zz (tile with halo, then the coefficients of the tile's own rows)
  auto load_plane = [&](int zz) {
    unsigned char* base = plane_at(zz);
    for (int j = wave; j < G::NJ; j += 4) {
      const int f = j * 64 + lane;
      unsigned off = kOut;
      if (f < G::CH) {
        const int pos = f / G::CPR, ch = f % G::CPR;
        const int yi = pos / G::TX, xi = pos % G::TX;
        const long long r = (long long)zz * c + (long long)(y0 + yi - 1) * b + (x0 + xi - 1);
        if (r >= 0 && r < n) off = (unsigned)((r * TC + ch * S::VL) * (long long)sizeof(T));
      }
      __builtin_amdgcn_raw_ptr_buffer_load_lds(xr, (__attribute__((address_space(3))) void*)(base + (size_t)j * 1024),
                                               16, off, 0, 0, 0);
    }
    for (int j = wave; j < G::NCJ; j += 4) {
      const int q = j * 64 + lane;
      unsigned off = kOut;
      if (q < G::CCH) {
        constexpr int per = G::RX / G::CE;
        const int xc = (q % per) * G::CE, dk = q / per, d = dk / K, k = dk % K;
        if (zz < gnz && y0 + k < gny && x0 + xc < gnx) {
          const long long r = (long long)zz * c + (long long)(y0 + k) * b + x0 + xc;
          off = (unsigned)(((long long)d * n + r) * (long long)sizeof(T));
        }
      }
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          cr, (__attribute__((address_space(3))) void*)(base + G::kPlane + (size_t)j * 1024), 16, off, 0, 0, 0);
    }
  };
  auto row_at = [&](int zz, int yi, int xi) -> Vec {
    const Vec* p = reinterpret_cast<const Vec*>(plane_at(zz));
    return p[(yi * G::TX + xi) * G::CPR + li];
  };
  load_plane(z0 - 1);
  load_plane(z0);
  load_plane(z0 + 1);
  for (int z = z0; z < z1; ++z) {
    wait_vm0();  // this wave's loads of plane z + 1 (and of the planes before) have landed
    __syncthreads();  // ... and every wave's; the slot of plane z + 2 is no longer read
    if (z + 2 <= z1) load_plane(z + 2);
    if (x < gnx) {
      const T* cf = reinterpret_cast<const T*>(plane_at(z) + G::kPlane);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (y0 + k >= gny) break;  // the same for the whole workgroup
        const long long r = (long long)z * c + (long long)(y0 + k) * b + x;
        auto coef = [&](int d) { return cf[(d * K + k) * G::RX + xl]; };
        auto term = [&](int d, long long j, const Vec& xv, Vec& acc) {
          fma_row<T, Vec, S::VL>(acc, (j >= 0 && j < n) ? coef(d) : T(0), xv);
        };
        Vec acc = Vec(0);
        term(0, r - c, row_at(z - 1, k + 1, xl + 1), acc);
        term(1, r - b, row_at(z, k, xl + 1), acc);
        term(2, r - 1, row_at(z, k + 1, xl), acc);
        term(3, r, row_at(z, k + 1, xl + 1), acc);
        term(4, r + 1, row_at(z, k + 1, xl + 2), acc);
        term(5, r + b, row_at(z, k + 2, xl + 1), acc);
        term(6, r + c, row_at(z + 1, k + 1, xl + 1), acc);
        __builtin_nontemporal_store(acc, reinterpret_cast<Vec*>(Y + (size_t)r * TC + li * S::VL));
      }
    }
  }
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

constexpr int kGramSplit = 32;  // first-stage sums of the Gram chunk reduction

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_reduce_chunks(long long len, int nchunks, const T* __restrict__ part, T* __restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  T s = T(0);
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * len + e];
  out[e] = s;
}

// First stage of the chunk sum: chunks [y*per, (y+1)*per) summed in order into mid[y][e]
// (grid y = blockIdx.y), so a long chunk list is summed by many workgroups in a fixed order.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_reduce_chunks_stage(long long len, int nchunks, int per, const T* __restrict__ part, T* __restrict__ mid) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  const int c0 = blockIdx.y * per;
  const int c1 = min(nchunks, c0 + per);
  T s = T(0);
  for (int c = c0; c < c1; ++c) s += part[(size_t)c * len + e];
  mid[(size_t)blockIdx.y * len + e] = s;
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

// ------------------------------------------------------------------ MFMA tall-skinny products
// 16x16x4 matrix-core tiles (FP64: v_mfma_f64_16x16x4f64, FP32: v_mfma_f32_16x16x4f32).
// Operand layout of one wavefront: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the 16x16 result sits in 4 values per lane v = 0..3 at column l%16 and row
// 4*(l/16)+v for FP32 but (l/16)+4*v for FP64 (checked on gfx950 with a lane probe).
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using V = mf_d4;
  __device__ __forceinline__ static V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int g, int v) { return g + 4 * v; }
};
template <>
struct Mfma<float> {
  using V = mf_f4;
  __device__ __forceinline__ static V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int g, int v) { return 4 * g + v; }
};

// Q columns handled by one Gram wavefront (more columns = fewer re-reads of Y).  A lane
// reads TA >= 16/sizeof(T) consecutive values of a row (at least one 16-byte load); when a
// stored block is narrower than 16*TA columns, BPG consecutive blocks form one "virtual
// block" of 16*TA columns, lane c reading block (TA*c)/WQ of the group.
template <typename T, int WQ, int TC>
struct GramTile {
  static constexpr int QC = (TC >= 64 || sizeof(T) == 8) ? 64 : 128;
  static constexpr int VPL = 16 / (int)sizeof(T);            // values per 16-byte load
  static constexpr int TA = (WQ / 16 > VPL) ? WQ / 16 : VPL;  // values per lane per row
  static constexpr int VW = 16 * TA;                          // virtual block width
  static constexpr int BPG = VW / WQ;                         // stored blocks per virtual block
  static constexpr int JB = QC >= VW ? QC / VW : 1;           // virtual blocks per wavefront
  static constexpr int NB = JB * BPG;                         // stored blocks per wavefront
  // FP64 at t = 32 is close to the matrix cores' rate (8 flop/B), so it trades operand
  // lookahead for occupancy: two row quads ahead instead of four lets the accumulators sit
  // in ordinary VGPRs at four wavefronts per SIMD (two otherwise); 10% faster per sweep.
  // At t = 16 the same trade was 2-5% slower.
  static constexpr bool WIDE64 = sizeof(T) == 8 && TC == 32;
  static constexpr int RQ = WIDE64 ? 2 : 4;     // row quads loaded ahead
  static constexpr int WAVES = WIDE64 ? 4 : 1;  // minimum wavefronts per SIMD asked of the compiler
};

// CGS2 Gram on matrix cores: one wavefront = JB stored blocks x one chunk of rows.
// K of the 16x16x4 product runs over rows (4 rows per instruction, lane group g = l/16
// takes row r+g).  M and N are interleaved so that each lane reads TA (TB) consecutive
// values of a row with one vector load: tile ta pairs M-index i with Q column TA*i+ta,
// tile tb pairs N-index j with Y column TB*j+tb.  A candidate narrower than 16 columns
// (TC = 8 after halvings) fills the N lanes past TC with zeros and writes only its own
// columns.  Sixteen rows are loaded before the products of the first four start, to keep
// enough loads in flight.
template <typename T, int WQ, int TC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(GramTile<T, WQ, TC>::WAVES)))
k_gram_mfma(int n, Span<T> sp, int rows_per_chunk, int units, int nwork, const T* __restrict__ Y,
            T* __restrict__ part, int m) {
  using V = typename Mfma<T>::V;
  using GT = GramTile<T, WQ, TC>;
  constexpr int JB = GT::JB, BPG = GT::BPG;
  constexpr bool NARROW = TC < 16;
  constexpr int TA = GT::TA, TB = NARROW ? 1 : TC / 16;
  typedef T TAv __attribute__((ext_vector_type(TA)));
  typedef T TBv __attribute__((ext_vector_type(TB)));
  constexpr int RQ = GT::RQ;  // row quads loaded ahead
  const int lane = threadIdx.x;
  const int g = lane >> 4, c = lane & 15;
  // chunk-major order, one contiguous range per XCD: the workgroups that share a chunk
  // of Y run together on one XCD and read it from that XCD's L2
  const int w = xcd_block();
  if (w >= nwork) return;
  const int chunk = w / units;
  const int j0 = (w % units) * GT::NB;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  V acc[JB][TA][TB];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int ta = 0; ta < TA; ++ta)
#pragma unroll
      for (int tb = 0; tb < TB; ++tb) acc[jb][ta][tb] = V{0, 0, 0, 0};
  const T* __restrict__ Qb[JB];
  bool jv[JB];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int blk = j0 + jb * BPG + (TA * c) / WQ;  // stored block this lane reads
    jv[jb] = blk < sp.nblk;
    Qb[jb] = sp.base + (size_t)(jv[jb] ? blk : j0) * sp.stride + (TA * c) % WQ;
  }
  const T* __restrict__ Yc = Y + (NARROW ? (c < TC ? c : 0) : TB * c);
  const bool cy = !NARROW || c < TC;  // this lane's N column is one of Y's
  // operands of 4*RQ rows, double-buffered: the next batch is requested before the
  // products of the current one are issued
  TAv qa0[RQ][JB], qa1[RQ][JB];
  TBv yb0[RQ], yb1[RQ];
  auto load = [&](TAv (&qa)[RQ][JB], TBv (&yb)[RQ], int row) {
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int rr = row + 4 * q + g;
      const bool ok = rr < r1;
      yb[q] = (ok && cy) ? *reinterpret_cast<const TBv*>(Yc + (size_t)rr * TC) : TBv(0);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)  // Q is streamed once: keep it out of the caches
        qa[q][jb] = (ok && jv[jb]) ? __builtin_nontemporal_load(reinterpret_cast<const TAv*>(Qb[jb] + (size_t)rr * WQ))
                                   : TAv(0);
    }
  };
  auto product = [&](const TAv (&qa)[RQ][JB], const TBv (&yb)[RQ]) {
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int ta = 0; ta < TA; ++ta)
#pragma unroll
          for (int tb = 0; tb < TB; ++tb)
            acc[jb][ta][tb] = Mfma<T>::run(qa[q][jb][ta], yb[q][tb], acc[jb][ta][tb]);
  };
  load(qa0, yb0, r0);
  int row = r0;
  for (; row + 4 * RQ < r1; row += 8 * RQ) {
    load(qa1, yb1, row + 4 * RQ);
    product(qa0, yb0);
    load(qa0, yb0, row + 8 * RQ);  // past the chunk: zeros, no memory access
    product(qa1, yb1);
  }
  if (row < r1) product(qa0, yb0);
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const size_t rowbase = (size_t)chunk * m + sp.goff + (size_t)(j0 + jb * BPG) * WQ;
#pragma unroll
    for (int ta = 0; ta < TA; ++ta)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int vc = TA * Mfma<T>::row(g, v) + ta;  // column of the virtual block
        if (j0 + jb * BPG + vc / WQ >= sp.nblk) continue;
        const size_t a = rowbase + vc;
        if (!cy) continue;
#pragma unroll
        for (int tb = 0; tb < TB; ++tb) part[a * TC + (NARROW ? c : TB * c + tb)] = acc[jb][ta][tb][v];
      }
  }
}

// CGS2 update W -= Q G on matrix cores.  A workgroup owns 256 rows (4 wavefronts x 4 row
// tiles of 16); K runs over the stored columns of the span in order.  Matrix-core operand
// layout wants a lane to hold four consecutive columns of one row (instruction s of a
// 16-column chunk pairs lane group g with column 4g+s; the matching rows of G come from
// LDS), but read that way straight from memory every load instruction touches sixteen
// 128-byte lines and uses half of each.  So Q goes through LDS: a wavefront reads its 64
// rows x SC columns (SC x sizeof(T) = 128 bytes, one whole line per row) with 16-byte
// non-temporal lane loads that use every byte of the lines they touch, writes them to its
// own LDS tile, and reads them back in the operand layout.  Two such stages are in flight
// in registers while the third is multiplied.  G is staged KS stored columns at a time in
// two LDS buffers: the next stage is fetched into registers while the current one is
// multiplied, so each G stage costs one barrier.  Narrow shapes after halvings: columns
// of 8-column stored blocks follow each other in K like any others, and a candidate of 8
// columns fills the N lanes past TC with zero rows of G and writes only its own columns.
template <typename T, int WQ, int TC>
struct UpdateTile {
  static constexpr int VQ = WQ >= 16 ? WQ : 16;
  static constexpr int LINE = 128 / (int)sizeof(T);
  static constexpr int SC = LINE < VQ ? LINE : VQ;  // stored columns of a Q stage
  static constexpr int VL = 16 / (int)sizeof(T);    // values per 16-byte lane load
  static constexpr int NL = SC / VL;                // lane loads per Q stage (64 rows)
  static constexpr int LDQ = SC + VL;               // LDS row pitch of a Q tile (padded)
  static constexpr int KS = TC >= 64 && SC <= 16 ? 32 : 64;  // stored columns per G stage
  static constexpr int NE = KS * TC;                // G values per stage
  static constexpr int PER = NE / kBlock;           // per thread
  static constexpr int QPS = KS / SC;              // Q stages per G stage (even)
  static_assert(KS % (2 * SC) == 0 && SC % 16 == 0 && NE % kBlock == 0, "stages");
};

template <typename T, int WQ, int TC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TC <= 32 ? 2 : 1)))
k_update_mfma(int n, int nwg, Span<T> sp, const T* __restrict__ G, T* __restrict__ W) {
  using V = typename Mfma<T>::V;
  using U = UpdateTile<T, WQ, TC>;
  typedef T T4 __attribute__((ext_vector_type(4)));
  typedef T L16 __attribute__((ext_vector_type(U::VL)));  // one 16-byte lane load
  constexpr bool NARROW = TC < 16;
  constexpr int TB = NARROW ? 1 : TC / 16, RT = 4;
  constexpr int SC = U::SC, NL = U::NL, LDQ = U::LDQ, KS = U::KS;
  __shared__ T Gs[2][U::NE];
  __shared__ __align__(16) T Qs[4][64 * LDQ];
  const int blk = xcd_block();
  if (blk >= nwg || sp.nblk <= 0) return;  // the whole workgroup leaves together
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int rowbase = blk * 256 + wave * 64;
  const int ncol = sp.nblk * WQ;            // stored columns of the span
  const int nq = (ncol + SC - 1) / SC;      // Q stages
  const int nst = (ncol + KS - 1) / KS;     // G stages
  const T* __restrict__ Gspan = G + (size_t)sp.goff * TC;
  const int total = ncol * TC;  // G values of this span
  T* __restrict__ Qw = Qs[wave];
  V acc[RT][TB];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int tb = 0; tb < TB; ++tb) acc[rt][tb] = V{0, 0, 0, 0};
  // Loads are unconditional, so that nothing branches around them and the wait for a stage
  // does not also wait for the loads issued after it.  G values past the span are loaded
  // from its last one and replaced by zero when staged.  Q rows past n are loaded from row
  // n - 1: a row of the product depends on its own row of Q only, and rows past n are not
  // stored.  Columns past the last stored block (odd counts of 8-column blocks) are loaded
  // from that block and meet zero rows of G.
  T pre[U::PER];
  auto fetch = [&](int st) {
#pragma unroll
    for (int i = 0; i < U::PER; ++i) pre[i] = Gspan[min(st * U::NE + (int)threadIdx.x + i * kBlock, total - 1)];
  };
  auto stash = [&](int buf, int st) {
#pragma unroll
    for (int i = 0; i < U::PER; ++i) {
      const int e = (int)threadIdx.x + i * kBlock;
      Gs[buf][e] = st * U::NE + e < total ? pre[i] : T(0);
    }
  };
  // stage q: columns q*SC .. q*SC+SC-1 of the span for this wavefront's 64 rows; lane load
  // i covers rows 64 / NL * i .. of the tile, SC / VL lanes per row
  constexpr int LPR = SC / U::VL, RPL = 64 / LPR;  // lanes per tile row, tile rows per load
  const int lr = lane / LPR, col = (lane % LPR) * U::VL;
  auto loadq = [&](L16 (&v)[NL], int q) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int rl = i * RPL + lr;
      const int k = q * SC + col;
      const int bj = min(k / WQ, sp.nblk - 1), row = min(rowbase + rl, n - 1);
      v[i] = __builtin_nontemporal_load(
          reinterpret_cast<const L16*>(sp.base + (size_t)bj * sp.stride + (size_t)row * WQ + k % WQ));
    }
  };
  auto put = [&](const L16 (&v)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; ++i) *reinterpret_cast<L16*>(Qw + (i * RPL + lr) * LDQ + col) = v[i];
  };
  // the LDS tile is private to the wavefront, whose LDS instructions complete in order:
  // these only keep the compiler from moving tile accesses across each other
  auto tile_order = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // consecutive products go to different accumulators (RT x TB of them)
  auto compute = [&](int cur, int kb) {
#pragma unroll
    for (int kc = 0; kc < SC / 16; ++kc) {
      T4 qv[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const T* p = Qw + (rt * 16 + c) * LDQ + kc * 16 + 4 * g;
        if constexpr (sizeof(T) == 8) {
          const L16 a = *reinterpret_cast<const L16*>(p), b = *reinterpret_cast<const L16*>(p + 2);
          qv[rt] = T4{a[0], a[1], b[0], b[1]};
        } else {
          qv[rt] = *reinterpret_cast<const T4*>(p);
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kk = kb + kc * 16 + 4 * g + s4;
        T gv[TB];
#pragma unroll
        for (int tb = 0; tb < TB; ++tb)
          gv[tb] = (NARROW && c >= TC) ? T(0) : Gs[cur][kk * TC + (NARROW ? c : tb * 16 + c)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int tb = 0; tb < TB; ++tb) acc[rt][tb] = Mfma<T>::run(qv[rt][s4], gv[tb], acc[rt][tb]);
      }
    }
  };
  // Every G stage takes QPS Q stages, also past the last one (their loads repeat the last
  // stage and meet zero rows of G), so that the loop issues the same loads on every path
  // and each stage waits only for its own: into LDS, the stage two ahead into the freed
  // registers, then the products.
  L16 v0[NL], v1[NL];
  fetch(0);
  stash(0, 0);
  loadq(v0, 0);
  __builtin_amdgcn_sched_barrier(0);  // stage 0's loads strictly before stage 1's
  loadq(v1, min(1, nq - 1));
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    fetch(min(st + 1, nst - 1));
#pragma unroll
    for (int qq = 0; qq < U::QPS; qq += 2) {
      const int q = st * U::QPS + qq;
      put(v0);
      tile_order();
      loadq(v0, min(q + 2, nq - 1));
      compute(cur, qq * SC);
      tile_order();
      put(v1);
      tile_order();
      loadq(v1, min(q + 3, nq - 1));
      compute(cur, (qq + 1) * SC);
      tile_order();
    }
    stash(cur ^ 1, st + 1);  // that buffer was last read before the previous barrier
    __syncthreads();
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rowbase + rt * 16 + Mfma<T>::row(g, v);
      if (row < n) {
        if (NARROW && c >= TC) continue;
#pragma unroll
        for (int tb = 0; tb < TB; ++tb) W[(size_t)row * TC + (NARROW ? c : tb * 16 + c)] -= acc[rt][tb][v];
      }
    }
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

// t x t Grams on FP64 matrix cores (FP32 data is widened on load, so these Grams are
// accumulated in FP64 in both precisions).  One wavefront per chunk of rows; K runs over
// rows.  Tile ta pairs M-index i with column TA*i+ta of X, tile tb < TB pairs N-index j with
// column TB*j+tb of Y; with WITH_R one more tile carries r in its column 0 (u = X^T r).
template <typename T, int TC, bool WITH_R>
__global__ void __launch_bounds__(64)
k_small_gram_mfma(int n, int rows_per_chunk, const T* __restrict__ X, const T* __restrict__ Y,
                  const T* __restrict__ r, double* __restrict__ part) {
  using V = Mfma<double>::V;
  constexpr int TA = TC / 16, TB = TC / 16, TR = TB + (WITH_R ? 1 : 0);
  constexpr int NOUT = TC * TC + (WITH_R ? TC : 0);
  typedef T Tv __attribute__((ext_vector_type(TA)));
  const int lane = threadIdx.x;
  const int g = lane >> 4, c = lane & 15;
  const int chunk = blockIdx.x;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(n, r0 + rows_per_chunk);
  V acc[TA][TR];
#pragma unroll
  for (int ta = 0; ta < TA; ++ta)
#pragma unroll
    for (int tb = 0; tb < TR; ++tb) acc[ta][tb] = V{0, 0, 0, 0};
  for (int row = r0; row < r1; row += 16) {
    Tv xa[4], yb[4];
    double rv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = row + 4 * q + g;
      const bool ok = rr < r1;
      xa[q] = ok ? *reinterpret_cast<const Tv*>(X + (size_t)rr * TC + TA * c) : Tv(0);
      yb[q] = ok ? *reinterpret_cast<const Tv*>(Y + (size_t)rr * TC + TB * c) : Tv(0);
      rv[q] = (WITH_R && ok && c == 0) ? (double)r[rr] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ta = 0; ta < TA; ++ta) {
#pragma unroll
        for (int tb = 0; tb < TB; ++tb)
          acc[ta][tb] = Mfma<double>::run((double)xa[q][ta], (double)yb[q][tb], acc[ta][tb]);
        if constexpr (WITH_R) acc[ta][TB] = Mfma<double>::run((double)xa[q][ta], rv[q], acc[ta][TB]);
      }
  }
  double* __restrict__ out = part + (size_t)chunk * NOUT;
#pragma unroll
  for (int ta = 0; ta < TA; ++ta)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = TA * Mfma<double>::row(g, v) + ta;
#pragma unroll
      for (int tb = 0; tb < TB; ++tb) out[a * TC + TB * c + tb] = acc[ta][tb][v];
      if constexpr (WITH_R) {
        if (c == 0) out[TC * TC + a] = acc[ta][TB][v];
      }
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

// First stage: split y of the chunks [y*per, (y+1)*per) summed in order into mid[y][e].
__global__ void __launch_bounds__(kBlock)
k_reduce_small_stage(int len, int nchunks, int per, const double* __restrict__ part, double* __restrict__ mid) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  const int c0 = blockIdx.y * per;
  const int c1 = min(nchunks, c0 + per);
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += part[(size_t)c * len + e];
  mid[(size_t)blockIdx.y * len + e] = s;
}

// ------------------------------------------------------------------ t x t factor (FP64)
// Right-looking Cholesky of a tc x tc Gram with left-to-right column deflation, then the
// inverse of the (upper triangular) factor.  One workgroup; tc <= 64.
// The factor R lives in the upper triangle of A (row j = R[j][.]); the strictly upper part
// of X = R^{-1} is kept transposed in the strictly lower triangle of A and diag(X) in xd.
__global__ void __launch_bounds__(kBlock)
k_factor(int mode, int tc, int tc_live, const double* __restrict__ in, const double* __restrict__ ref, double tau,
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
    // reference of the pivot test: the column's squared norm before CGS2 when given
    d0[tid] = ref ? ref[tid * tc + tid] : A[tid * kMaxT + tid];
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

// ------------------------------------------------------------------ n x t block times t x t (MFMA)
// Out = X M for a row-major n x TC block X and a TC x TC matrix M (FP64 on input), on
// matrix cores, TC >= 16.  A wavefront owns RT tiles of 16 rows; K runs over the TC
// columns of X, 16 at a time: each lane reads four consecutive values of one row with one
// vector load and instruction s pairs lane group g with column 4g+s (the same
// permutation of K is applied to the rows of M, staged in LDS).
// FINAL: the fused update of the block iteration.  The same M (= C^{-1}) multiplies H
// and Y (W = H C^{-1} into the stored-block slot, Z = Y C^{-1} the next candidate) on
// matrix cores, and the row products H beta and Y beta are formed from the same loaded
// values with vector FMAs (each lane takes its four columns, then the four lane groups of
// a row are summed by two cross-lane exchanges): x += H beta, r -= Y beta, and the squared
// norm of the new r is reduced per workgroup.
template <int TC, bool FINAL = false>
struct SmallTile {
  // row tiles per wavefront; the fused update carries two products, so half as many
  static constexpr int RT0 = TC >= 64 ? 1 : (TC == 32 ? 2 : 4);
  static constexpr int RT = FINAL ? (RT0 > 1 ? RT0 / 2 : 1) : RT0;
  static constexpr int ROWS = 4 * 16 * RT;  // rows per workgroup
};

template <typename T, typename TX, int TC, bool FINAL>
__global__ void __launch_bounds__(kBlock)
k_small_mfma(int n, int nwg, int ntiles, const T* __restrict__ H, const T* __restrict__ Yin, const double* __restrict__ M,
             const double* __restrict__ beta, T* __restrict__ Wout, T* __restrict__ Zout, TX* __restrict__ x,
             T* __restrict__ r, double* __restrict__ part) {
  using V = typename Mfma<T>::V;
  typedef T T4 __attribute__((ext_vector_type(4)));
  constexpr int TB = TC / 16;
  constexpr int NT = TB;  // output column tiles
  constexpr int LD = NT * 16;
  constexpr int RT = SmallTile<TC, FINAL>::RT;
  __shared__ T Ms[TC * LD];
  __shared__ __align__(32) T Bs[FINAL ? TC : 1];
  __shared__ double red[FINAL ? kBlock : 1];
  for (int e = threadIdx.x; e < TC * LD; e += kBlock) Ms[e] = (T)M[e];
  if constexpr (FINAL)
    for (int e = threadIdx.x; e < TC; e += kBlock) Bs[e] = (T)beta[e];
  __syncthreads();
  const int blk = xcd_block();
  if (blk >= nwg) return;  // uniform over the workgroup: no later barrier is split
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  double rr = 0.0;
  // row tiles blk, blk + nwg, ...: M is staged once per workgroup, and the partial norm of
  // a workgroup sums its tiles in that fixed order
  for (int tile = blk; tile < ntiles; tile += nwg) {
    const int rowbase = tile * SmallTile<TC, FINAL>::ROWS + wave * 16 * RT;
    V aw[RT][NT], az[FINAL ? RT : 1][FINAL ? NT : 1];
    T hb[RT], yb[RT];  // FINAL: this lane's part of (H beta)_row and (Y beta)_row
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      hb[rt] = T(0), yb[rt] = T(0);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        aw[rt][nt] = V{0, 0, 0, 0};
        if constexpr (FINAL) az[rt][nt] = V{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int kc = 0; kc < TC / 16; ++kc) {
      T4 qh[RT], qy[FINAL ? RT : 1];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int row = rowbase + rt * 16 + c;
        const size_t off = (size_t)row * TC + kc * 16 + 4 * g;
        qh[rt] = row < n ? *reinterpret_cast<const T4*>(H + off) : T4{0, 0, 0, 0};
        if constexpr (FINAL) qy[rt] = row < n ? *reinterpret_cast<const T4*>(Yin + off) : T4{0, 0, 0, 0};
      }
      if constexpr (FINAL) {
        const T4 bq = *reinterpret_cast<const T4*>(Bs + kc * 16 + 4 * g);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            hb[rt] = fmac(qh[rt][s4], bq[s4], hb[rt]);
            yb[rt] = fmac(qy[rt][s4], bq[s4], yb[rt]);
          }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kk = kc * 16 + 4 * g + s4;
        T gv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) gv[nt] = Ms[kk * LD + nt * 16 + c];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            aw[rt][nt] = Mfma<T>::run(qh[rt][s4], gv[nt], aw[rt][nt]);
            if constexpr (FINAL) az[rt][nt] = Mfma<T>::run(qy[rt][s4], gv[nt], az[rt][nt]);
          }
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rowbase + rt * 16 + Mfma<T>::row(g, v);
        if (row < n) {
#pragma unroll
          for (int tb = 0; tb < TB; ++tb) {
            Wout[(size_t)row * TC + tb * 16 + c] = aw[rt][tb][v];
            if constexpr (FINAL) Zout[(size_t)row * TC + tb * 16 + c] = az[rt][tb][v];
          }
        }
      }
    if constexpr (FINAL) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        // lanes c, c + 16, c + 32, c + 48 hold the four column groups of row c
        T h = hb[rt] + __shfl_xor(hb[rt], 16, 64);
        T y = yb[rt] + __shfl_xor(yb[rt], 16, 64);
        h += __shfl_xor(h, 32, 64);
        y += __shfl_xor(y, 32, 64);
        const int row = rowbase + rt * 16 + c;
        if (g == 0 && row < n) {
          x[row] += (TX)h;
          const T rn = r[row] - y;
          r[row] = rn;
          rr += (double)rn * (double)rn;
        }
      }
    }
  }
  if constexpr (FINAL) {
    const double tot = block_sum(rr, red);
    if (threadIdx.x == 0) part[blk] = tot;
  }
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

// The same sweeps with the group's solution held in LDS: grid (groups, tc / CW), a workgroup
// owns CW columns of one group, so every dependency of a row (earlier levels of the same
// group, the factor being block diagonal) is read from LDS instead of through L2.  Same
// operations in the same order as k_trisolve.
template <typename T, int CW>
__global__ void __launch_bounds__(kBlock)
k_trisolve_lds(int which, int tc, const int* __restrict__ kr, const int* __restrict__ lcol, const T* __restrict__ v,
               const int* __restrict__ lptr, const int* __restrict__ lrows, int maxlev, const int* __restrict__ loc,
               const T* __restrict__ X, T* __restrict__ Y) {
  extern __shared__ unsigned char tri_smem[];
  T* ys = reinterpret_cast<T*>(tri_smem);  // [rows of the group][CW]
  const int g = blockIdx.x;
  const int c0 = blockIdx.y * CW;
  for (int l = 0; l < maxlev; ++l) {
    const int p0 = lptr[g * (maxlev + 1) + l];
    const int p1 = lptr[g * (maxlev + 1) + l + 1];
    const int cnt = (p1 - p0) * CW;
    for (int e = threadIdx.x; e < cnt; e += kBlock) {
      const int p = p0 + e / CW;
      const int c = e % CW;
      const int row = lrows[p];
      const int k0 = kr[2 * p], k1 = kr[2 * p + 1];
      T s = X[(size_t)row * tc + c0 + c];
      T d;
      if (which == 0) {
        for (int k = k0; k < k1 - 1; ++k) s -= v[k] * ys[lcol[k] * CW + c];
        d = v[k1 - 1];
      } else {
        for (int k = k0 + 1; k < k1; ++k) s -= v[k] * ys[lcol[k] * CW + c];
        d = v[k0];
      }
      const T y = s / d;
      ys[loc[row] * CW + c] = y;
      Y[(size_t)row * tc + c0 + c] = y;
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
  if (m <= 8192) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, s, part, m, out);
    return;
  }
  // two stages: 128 slices, then their sum; the slices live past the end of `part`
  const int nb = 128;
  const int per = cdiv(m, nb);
  double* mid = const_cast<double*>(part) + m;
  hipLaunchKernelGGL(k_sum_stage, dim3(nb), dim3(kBlock), 0, s, part, m, per, mid);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, s, mid, nb, out);
}

// Zero `words` 8-byte words (a kernel rather than hipMemsetAsync, so that the solve's
// clears are ordinary kernel launches on the caller's stream).
__global__ void __launch_bounds__(kBlock) k_zero_words(long long words, unsigned long long* __restrict__ p) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < words) p[i] = 0ull;
}
void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long words = (long long)((bytes + 7) / 8);
  if (words > 0)
    hipLaunchKernelGGL(k_zero_words, dim3(cdiv(words, kBlock)), dim3(kBlock), 0, s, words,
                       static_cast<unsigned long long*>(p));
}
void launch_cast_d2f(int n, const double* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, in, out);
}
void launch_axpy_f2d(int n, const float* d, double* x, hipStream_t s, double alpha) {
  hipLaunchKernelGGL(k_axpy_f2d, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, n, alpha, d, x);
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
static const T* dia_vals_of(const DevCsr& A);
template <>
const double* dia_vals_of<double>(const DevCsr& A) { return A.dval; }
template <>
const float* dia_vals_of<float>(const DevCsr& A) { return A.dvalf; }
template <typename T>
static const T* sell_vals_of(const DevCsr& A);
template <>
const double* sell_vals_of<double>(const DevCsr& A) { return A.sell_val; }
template <>
const float* sell_vals_of<float>(const DevCsr& A) { return A.sell_valf; }

constexpr int kGridK = 2;     // rows (y) per lane of the 3-D grid-stencil product
constexpr int kGridZseg = 16;  // planes per workgroup of the grid-stencil product
constexpr int kGridLdsK = 4;   // y rows per tile of the LDS-staged grid-stencil product
constexpr int kGridDmaK = 2;   // y rows per tile of the product fed by direct loads to LDS

// The automatic choice.  The grid kernel pays off on 3-D stencils once a row spans at least
// 4 lanes (so that its coefficients take one load per lane); on 2-D operators of the sizes
// here the diagonal kernel is as fast or faster (the 2-D grid walk has too few workgroups).

// The LDS-staged grid kernel needs a 3-D 7-point grid stencil with unit x stride, at least 4
// lanes per block row and rows of whole 16-byte coefficient chunks.
// Both LDS-staged kernels read X and the coefficients through 32-bit buffer offsets.
bool spmm_grid_lds_ok(const DevCsr& A, int tc, int elt) {
  const int vl = std::min(16 / elt, tc);
  return A.gnx > 0 && A.ndiag == 7 && A.ga == 1 && tc / vl >= 4 && A.gnx % (16 / elt) == 0 &&
         (double)A.n * tc * elt <= 4294967040.0 && (double)A.n * 7 * elt <= 4294967040.0;
}

bool spmm_grid_dma_ok(const DevCsr& A, int tc, int elt) { return spmm_grid_lds_ok(A, tc, elt); }

// The automatic choice: the most specific form the matrix has; among the 3-D grid-stencil
// kernels the one measured fastest at this width and precision on the 128^3 and 160^3
// operators: LDS-staged for FP64 t >= 16 and FP32 t >= 32, register planes otherwise (the
// kernel fed by direct loads is slower at every width since the LDS-staged one loads two
// planes ahead).
inline int spmm_choice(const DevCsr& A, int tc, int elt) {
  const int lpr = tc / std::min(16 / elt, tc);
  if (A.gnx > 0 && A.ndiag == 7 && lpr >= 4) {
    if (tc >= (elt == 8 ? 16 : 32) && spmm_grid_lds_ok(A, tc, elt)) return kSpmmGridLds;
    return kSpmmGrid;
  }
  if (A.ndiag > 0) return kSpmmDia;
  return A.nslice > 0 ? kSpmmSell : kSpmmCsr;
}

template <typename T>
void launch_spmm(const DevCsr& A, int tc, const T* X, T* Y, hipStream_t s, int kernel) {
  switch (tc) {
#define C(TC)                                                                                    \
  case TC: {                                                                                     \
    using Sh = SpmmShape<T, TC>;                                                                 \
    const int nwg = cdiv(A.n, Sh::RPB);                                                          \
    if (kernel == kSpmmAuto) kernel = spmm_choice(A, TC, (int)sizeof(T));                        \
    stat_begin(s);                                                                               \
    if (kernel == kSpmmGridLds) {                                                                \
      if constexpr (Sh::LPR >= 4) {                                                              \
        constexpr int CW = (sizeof(T) == 8 && TC > 32) ? 32 : TC;                                \
        using GL = GridLds<T, CW, kGridLdsK>;                                                    \
        const int nxb = cdiv(A.gnx, GL::RX), nyb = cdiv(A.gny, kGridLdsK);                       \
        const int nwork = nxb * nyb * cdiv(A.gnz, kGridZseg) * (TC / CW);                        \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_spmm_grid_lds<T, TC, CW, kGridLdsK>), \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)GL::kLds);    \
        hipLaunchKernelGGL((k_spmm_grid_lds<T, TC, CW, kGridLdsK>), dim3(pad8(nwork)), dim3(kBlock), GL::kLds, \
                           s, A.n, A.gnx, A.gny, A.gnz, kGridZseg, nxb, nyb, nwork, dia_vals_of<T>(A), X, Y); \
      }                                                                                          \
    } else if (kernel == kSpmmGridDma) {                                                         \
      if constexpr (Sh::LPR >= 4) {                                                              \
        using GD = GridDma<T, TC, kGridDmaK>;                                                    \
        const int nxb = cdiv(A.gnx, GD::RX), nyb = cdiv(A.gny, kGridDmaK);                       \
        const int nwork = nxb * nyb * cdiv(A.gnz, kGridZseg);                                    \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_spmm_grid_dma<T, TC, kGridDmaK>), \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)GD::kLds);    \
        hipLaunchKernelGGL((k_spmm_grid_dma<T, TC, kGridDmaK>), dim3(pad8(nwork)), dim3(kBlock), GD::kLds, s, \
                           A.n, A.gnx, A.gny, A.gnz, kGridZseg, nxb, nyb, nwork, dia_vals_of<T>(A), X, Y); \
      }                                                                                          \
    } else if (kernel == kSpmmGrid) {                                                            \
      const int K = A.ndiag == 7 ? kGridK : 1;                                                   \
      const int nxb = cdiv(A.gnx, Sh::RPB), nyb = cdiv(A.gny, K), nzb = cdiv(A.gnz, kGridZseg);  \
      const int nwork = nxb * nyb * nzb;                                                         \
      if (A.ndiag == 7)                                                                          \
        hipLaunchKernelGGL((k_spmm_grid<T, TC, 7, kGridK>), dim3(pad8(nwork)), dim3(kBlock), 0, s, A.n, \
                           A.gnx, A.gny, A.gnz, A.ga, kGridZseg, nxb, nyb, nwork, dia_vals_of<T>(A), X, Y); \
      else                                                                                       \
        hipLaunchKernelGGL((k_spmm_grid<T, TC, 5, 1>), dim3(pad8(nwork)), dim3(kBlock), 0, s, A.n, \
                           A.gnx, A.gny, A.gnz, A.ga, kGridZseg, nxb, nyb, nwork, dia_vals_of<T>(A), X, Y); \
    } else if (kernel == kSpmmDia && A.ndiag == 5)                                               \
      hipLaunchKernelGGL((k_spmm_dia<T, TC, 5>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, A.ndiag, \
                         A.dia, dia_vals_of<T>(A), X, Y);                                        \
    else if (kernel == kSpmmDia && A.ndiag == 7)                                                 \
      hipLaunchKernelGGL((k_spmm_dia<T, TC, 7>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, A.ndiag, \
                         A.dia, dia_vals_of<T>(A), X, Y);                                        \
    else if (kernel == kSpmmDia && A.ndiag <= 8)                                                 \
      hipLaunchKernelGGL((k_spmm_dia<T, TC, 8>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, A.ndiag, \
                         A.dia, dia_vals_of<T>(A), X, Y);                                        \
    else if (kernel == kSpmmDia)                                                                 \
      hipLaunchKernelGGL((k_spmm_dia<T, TC, kMaxDiag>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, \
                         A.ndiag, A.dia, dia_vals_of<T>(A), X, Y);                               \
    else if (kernel == kSpmmSell) {                                                              \
      const int npos = A.nslice * kSellC, nws = cdiv(npos, Sh::RPB);                             \
      hipLaunchKernelGGL((k_spmm_sell<T, TC>), dim3(pad8(nws)), dim3(kBlock), 0, s, npos, nws, A.sell_ptr, \
                         A.sell_len, A.sell_row, A.sell_col, sell_vals_of<T>(A), X, Y);          \
    } else                                                                                       \
      hipLaunchKernelGGL((k_spmm<T, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, A.n, nwg, A.rowptr, \
                         A.col, vals_of<T>(A), X, Y);                                            \
    stat_end(kStatSpmm, (kernel != kSpmmCsr && kernel != kSpmmSell ? (double)A.ndiag * A.n * sizeof(T) \
                                            : (double)A.nnz * (sizeof(T) + 4) + 4.0 * (A.n + 1)) + \
                            2.0 * sizeof(T) * A.n * TC,                                          \
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

// Work units of one span: Gram wavefronts/workgroups along the block axis.
template <typename T>
static int gram_units(const Span<T>& sp, int tc) {
  if (sp.width >= 8 && tc >= 8) {
    const int jb = ((tc >= 64 || sizeof(T) == 8) ? 64 : 128) / sp.width;
    const int JB = jb < 1 ? 1 : jb;
    return (sp.nblk + JB - 1) / JB;
  }
  return sp.nblk;
}

// Row chunks of the CGS2 Gram: a chunk of Y is at most 1 MiB (it is re-read by every
// block group, from L2), there are enough work units to fill 256 CUs many times over, at
// least 256 rows per chunk, and the partial sums fit the workspace.
static int gram_chunks(int n, int units, size_t part_cap, int m, int tc, int elt) {
  units = units > 0 ? units : 1;
  int nch = cdiv((long long)n * tc * elt, 1 << 20);
  const int want = cdiv(4096, units);
  if (nch < want) nch = want;
  const int maxc = cdiv(n, 256);
  if (nch > maxc) nch = maxc;
  // the partials and the first-stage sums of the reduction share the buffer
  while (nch > 1 && (size_t)(nch + kGramSplit) * m * tc > part_cap) nch = (nch + 1) / 2 < nch ? (nch + 1) / 2 : nch - 1;
  return nch < 1 ? 1 : nch;
}

template <typename T, int WQ, int TC>
static void gram_span(int n, const Span<T>& sp, int rpc, int nch, const T* Y, T* part, int m, hipStream_t s) {
  stat_begin(s);
  if constexpr (WQ >= 8 && TC >= 8) {
    constexpr int NB = GramTile<T, WQ, TC>::NB;
    const int units = (sp.nblk + NB - 1) / NB;
    const int nwork = units * nch;
    hipLaunchKernelGGL((k_gram_mfma<T, WQ, TC>), dim3(pad8(nwork)), dim3(64), 0, s, n, sp, rpc, units, nwork, Y,
                       part, m);
  } else {
    hipLaunchKernelGGL((k_gram<T, WQ, TC>), dim3(sp.nblk, nch), dim3(kBlock), 0, s, n, sp, rpc, Y, part, m);
  }
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
  int units = 0;
  for (int i = 0; i < nspan; ++i) units += gram_units(spans[i], tc);
  int nch = gram_chunks(n, units, part_cap, m, tc, (int)sizeof(T));
  const int rpc = (cdiv(n, nch) + 15) / 16 * 16;  // multiple of 16 rows (one load batch)
  nch = cdiv(n, rpc);
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
    if (nch > kGramSplit) {
      // two fixed-order stages: kGramSplit partial sums of consecutive chunks, then their sum
      const int per = cdiv(nch, kGramSplit);
      const int nsplit = cdiv(nch, per);
      T* mid = part_buf + (size_t)nch * len;
      hipLaunchKernelGGL((k_reduce_chunks_stage<T>), dim3(cdiv(len, kBlock), nsplit), dim3(kBlock), 0, s, len, nch,
                         per, part_buf, mid);
      hipLaunchKernelGGL((k_reduce_chunks<T>), dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, len, nsplit, mid, G);
    } else {
      hipLaunchKernelGGL((k_reduce_chunks<T>), dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, len, nch, part_buf, G);
    }
    stat_end(kStatGramReduce, (double)sizeof(T) * (nch + 1) * len, (double)nch * len, s);
  }
}

template <typename T, int TC>
static void update_span(int n, const Span<T>& sp, const T* G, T* W, hipStream_t s) {
  switch (sp.width) {
#define C(WQ)                                                                                          \
  case WQ: {                                                                                           \
    stat_begin(s);                                                                                     \
    if constexpr (WQ >= 8 && TC >= 8) {                                                                \
      const int nwg = cdiv(n, 256);                                                                    \
      hipLaunchKernelGGL((k_update_mfma<T, WQ, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, sp, G, W); \
    } else {                                                                                           \
      const int nwg = cdiv(n, kBlock / TC);                                                            \
      hipLaunchKernelGGL((k_update<T, WQ, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, sp, G, W); \
    }                                                                                                  \
    stat_end(kStatUpdate, (double)sizeof(T) * n * ((double)sp.nblk * WQ + 2.0 * TC),                   \
             2.0 * n * sp.nblk * WQ * TC, s);                                                          \
    break;                                                                                             \
  }
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
  const int nout = tc * tc + (r ? tc : 0);
  if (tc >= 16) {
    const int rpc = (cdiv(n, nch) + 15) / 16 * 16;
    nch = cdiv(n, rpc);
    switch (tc) {
#define C(TC)                                                                                                   \
  case TC:                                                                                                      \
    if (r)                                                                                                      \
      hipLaunchKernelGGL((k_small_gram_mfma<T, TC, true>), dim3(nch), dim3(64), 0, s, n, rpc, X, Y, r, part);   \
    else                                                                                                        \
      hipLaunchKernelGGL((k_small_gram_mfma<T, TC, false>), dim3(nch), dim3(64), 0, s, n, rpc, X, Y, r, part);  \
    break;
      C(16) C(32) C(64)
#undef C
    }
    // two-stage chunk sum; the 32 intermediate rows live past the chunk partials
    const int nsplit = 32;
    const int per = cdiv(nch, nsplit);
    double* mid = part + (size_t)nch * nout;
    hipLaunchKernelGGL(k_reduce_small_stage, dim3(cdiv(nout, kBlock), nsplit), dim3(kBlock), 0, s, nout, nch, per,
                       part, mid);
    hipLaunchKernelGGL(k_reduce_small, dim3(cdiv(nout, kBlock)), dim3(kBlock), 0, s, nout, nsplit, mid, out);
    return;
  }
  const int rpc = cdiv(n, nch);
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

void launch_factor(int mode, int tc, int tc_live, const double* in, const double* ref, double tau, double* inv,
                   double* beta, IterStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_factor, dim3(1), dim3(kBlock), 0, s, mode, tc, tc_live, in, ref, tau, inv, beta, st);
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_msdo_combine(long long len, int tc, const T* __restrict__ S, const T* __restrict__ P, const double* __restrict__ u,
               T* __restrict__ out) {
  const long long e = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  const int c = (int)(e % tc);
  out[e] = S[e] - P[e] * (T)u[c];  // beta = -u
}

template <typename T>
void launch_msdo_combine(int n, int tc, const T* S, const T* P, const double* u, T* out, hipStream_t s) {
  const long long len = (long long)n * tc;
  stat_begin(s);
  hipLaunchKernelGGL((k_msdo_combine<T>), dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, len, tc, S, P, u, out);
  stat_end(kStatSplit, 3.0 * sizeof(T) * len, 2.0 * len, s);
}
template void launch_msdo_combine<double>(int, int, const double*, const double*, const double*, double*, hipStream_t);
template void launch_msdo_combine<float>(int, int, const float*, const float*, const double*, float*, hipStream_t);

template <typename T>
void launch_times_small(int n, int tc, const T* X, const double* M, T* out, hipStream_t s) {
  switch (tc) {
#define C(TC)                                                                                         \
  case TC: {                                                                                          \
    const int nwg = cdiv(n, kBlock / TC);                                                             \
    hipLaunchKernelGGL((k_times_small<T, TC>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, X, M, out); \
    break;                                                                                            \
  }
    C(1) C(2) C(4) C(8)
#undef C
#define C(TC)                                                                                         \
  case TC: {                                                                                          \
    const int nwg = cdiv(n, SmallTile<TC>::ROWS);                                                     \
    hipLaunchKernelGGL((k_small_mfma<T, double, TC, false>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, nwg, X, \
                       nullptr, M, nullptr, out, nullptr, nullptr, nullptr, nullptr);                 \
    break;                                                                                            \
  }
    C(16) C(32) C(64)
#undef C
  }
}

constexpr int kFinalGroups = 2048;  // workgroups of the fused update (8 per CU)

template <typename T, typename TX>
int launch_final_update(int n, int tc, const T* H, const T* Y, const double* Cinv, const double* beta, T* Wq,
                        T* Zn, TX* x, T* r, double* part, hipStream_t s) {
  int nwg = 0, ntiles = 0;
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
    C(1) C(2) C(4) C(8)
#undef C
#define C(TC)                                                                                          \
  case TC:                                                                                             \
    ntiles = cdiv(n, SmallTile<TC, true>::ROWS);                                                       \
    nwg = std::min(ntiles, kFinalGroups);                                                              \
    stat_begin(s);                                                                                     \
    hipLaunchKernelGGL((k_small_mfma<T, TX, TC, true>), dim3(pad8(nwg)), dim3(kBlock), 0, s, n, nwg, ntiles, H, Y, \
                       Cinv, beta, Wq, Zn, x, r, part);                                                \
    stat_end(kStatFinal, 4.0 * sizeof(T) * n * TC + (double)n * (2 * sizeof(TX) + 2 * sizeof(T)),      \
             4.0 * n * TC * TC + 4.0 * n * TC, s);                                                     \
    break;
    C(16) C(32) C(64)
#undef C
  }
  return nwg;
}

template <typename T>
void launch_trisolve(const DevTri& M, int which, int tc, const T* X, T* Y, hipStream_t s) {
  const DevCsr& F = which == 0 ? M.L : M.U;
  const int* lp = which == 0 ? M.lvl_ptr_L : M.lvl_ptr_U;
  const int* lr = which == 0 ? M.lvl_rows_L : M.lvl_rows_U;
  // LDS-resident sweeps when one group's rows fit for at least one column (<= 128 KB)
  constexpr size_t kTriLds = 128 * 1024;
  int cw = 0;
  for (int c = 8; c >= 1; c /= 2)
    if (tc % c == 0 && (size_t)M.maxrows * c * sizeof(T) <= kTriLds) {
      cw = c;
      break;
    }
  if (M.loc && cw > 0) {
    const int* kr = which == 0 ? M.kr_L : M.kr_U;
    const int* lcol = which == 0 ? M.lcol_L : M.lcol_U;
    const size_t lds = (size_t)M.maxrows * cw * sizeof(T);
    const dim3 grid(M.ngroups, tc / cw);
    stat_begin(s);
    switch (cw) {
#define C(CW)                                                                                                \
  case CW:                                                                                                   \
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_trisolve_lds<T, CW>),                          \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                         \
    hipLaunchKernelGGL((k_trisolve_lds<T, CW>), grid, dim3(kBlock), lds, s, which, tc, kr, lcol, vals_of<T>(F), \
                       lp, lr, M.maxlev, M.loc, X, Y);                                                       \
    break;
      C(1) C(2) C(4) C(8)
#undef C
    }
    stat_end(kStatSplit, (double)F.nnz * (sizeof(T) + 4) + 4.0 * (F.n + 1) + 2.0 * sizeof(T) * F.n * tc,
             2.0 * F.nnz * tc, s);
    return;
  }
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
  template void launch_spmm<T>(const DevCsr&, int, const T*, T*, hipStream_t, int);                           \
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
