/*
 * ecg.h - C ABI of the MI355X (gfx950) flexibly enlarged Conjugate Gradient solver.
 *
 * The method is flexibly SRE-CG2 (Section 4.3, Algorithm 3 of "Flexibly Enlarged
 * Conjugate Gradient methods"; MSDO-CG, Algorithms 2, 4 and 5, is a variant): the
 * residual is split over t subdomains
 * (operator T^t, eq. (Tt)); every iteration adds a block of t search vectors that is
 * A-orthonormalised against the stored blocks (CGS2) and against itself (Pre-CholQR,
 * Section 5); x and r follow the short recurrences of Algorithm 1; once the relative
 * change of the residual norm falls below switchTol the block width is halved and the
 * next block is T^{t/2}(r) on merged subdomains (Section 4.2).
 *
 * Conventions for every entry point:
 *  - Every function returns ecg_status.  Nothing throws across the ABI.  On a status
 *    other than ECG_OK / ECG_ENOTCONV, ecg_last_error() returns a message describing
 *    the failure (thread-local, valid until the next call on the same thread).
 *  - Pointers documented as "device" must point to device memory of the current HIP
 *    device (e.g. from hipMalloc or a torch tensor on cuda:0); "host" pointers to host
 *    memory.  Arrays are dense, contiguous, in the stated element type.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  All device work is
 *    enqueued on it.  Functions return after the work they describe has completed
 *    unless stated otherwise.
 *  - Invalid arguments are rejected with ECG_EINVAL before any device work.
 *    A HIP runtime error gives ECG_EHIP with the HIP error string in ecg_last_error().
 *  - Opaque objects are owned by the library and freed by their *_destroy function.
 *
 * Block layout: an n x t block of vectors is stored row-major ("[n][t]": the t values
 * of one unknown are contiguous).  The solver uses this layout internally; it is
 * visible to callers only through ecg_debug_* entry points.
 */
#ifndef ECG_H
#define ECG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ECG_OK = 0,
  ECG_ENOTCONV = 1,      /* k_max reached before the tolerance; x and report are valid */
  ECG_EINVAL = -1,       /* invalid argument (nothing was enqueued) */
  ECG_ENOMEM = -2,       /* workspace too small or library allocation failed */
  ECG_EHIP = -3,         /* HIP runtime error */
  ECG_EBREAKDOWN = -4    /* a block lost every column (all deflated), or a t x t Cholesky
                            pivot was not positive with deflation disabled; x and report
                            hold the last completed iterate */
} ecg_status;

typedef enum {
  ECG_REDUCE_NONE = 0,            /* SRE-CG2, Algorithm 1: t never changes */
  ECG_REDUCE_SWITCHTOL_ONCE = 1,  /* Algorithm 3: halve t once, when tol1 < switch_tol */
  ECG_REDUCE_SWITCHTOL_REPEAT = 2,/* halve again at each later tol1 < switch_tol, at least
                                     min_gap iterations apart, down to t_min */
  ECG_REDUCE_SCHEDULE = 3         /* halve exactly at the iterations listed in schedule */
} ecg_reduce;

typedef enum {
  ECG_FP64 = 0,          /* every step in FP64 */
  ECG_FP32_REFINED = 1   /* SpMM, Gram products and block updates in FP32 (FP32
                            accumulation); t x t Grams, Cholesky factors, x, the true
                            residual and the outer refinement in FP64 */
} ecg_precision;

typedef enum {
  ECG_SRE_CG2 = 0,         /* next block A W_{k-1} (Algorithms 1 and 3) */
  ECG_MSDO_CG = 1,         /* next block [T(r_{k-1})] + P_{k-1} diag(beta_k),
                              beta_k = -V_{k-1}^T r_{k-1} (Algorithms 2, 4 and 5) */
  ECG_MODIFIED_MSDO = 2    /* next block [T(r_{k-1})] (modified MSDO-CG, Section 2.2) */
} ecg_variant;

/* Restarted variants (Section 3): a restart at iteration k empties the stored blocks Q and
 * takes the candidate [T(r_{k-1})] at the current width, as at k = 1 (for MSDO-CG without
 * the beta term).  The stopping test stays relative to ||r_0||. */
typedef enum {
  ECG_RESTART_NONE = 0,
  ECG_RESTART_EVERY = 1,  /* restart when k mod restart_every == 1 (k > 1) */
  ECG_RESTART_TOL = 2     /* restart when |rho_k - rho_{k-1}| / rho_c < restart_tol, tested
                             where the switch is tested, with rho_c the residual norm the
                             current cycle started from (rho_0 before the first restart);
                             at most max_restarts times (0 = no limit) */
} ecg_restart;

typedef enum {
  ECG_PRECOND_NONE = 0,
  ECG_PRECOND_SPLIT = 1  /* split preconditioner M = L L^T given as an ecg_precond
                            (Section 4.5, option 2, eq. (zsre2)) */
} ecg_precond_kind;

typedef struct ecg_operator ecg_operator;    /* device copy of a sparse matrix (CSR) */
typedef struct ecg_partition ecg_partition;  /* device copy of the subdomain map */
typedef struct ecg_precond ecg_precond;      /* split preconditioner M = L L^T */

typedef struct {
  double tol;              /* stop when ||r_k|| <= tol * ||r_0|| (recursive residual) */
  int32_t kmax;            /* loop runs while k < kmax (at most kmax-1 iterations); for
                              FP32_REFINED the budget of all inner iterations together */
  int32_t reduce;          /* ecg_reduce */
  double switch_tol;       /* switchTol of Section 4.2 */
  int32_t t_min;           /* never halve below this width (>= 1) */
  int32_t min_gap;         /* REPEAT: iterations between two halvings (>= 1) */
  const int32_t* schedule; /* host; SCHEDULE: iterations k at which to halve */
  int32_t n_schedule;
  int32_t precision;       /* ecg_precision */
  double inner_tol;        /* FP32_REFINED: relative tolerance of each inner solve */
  int32_t max_outer;       /* FP32_REFINED: maximum refinement steps (>= 1) */
  int32_t replace_every;   /* FP32_REFINED: recompute r = b - A x in FP64 every this many
                              inner iterations (0 = never).  An inner solve whose true
                              residual falls by less than 10% over four replacements (and at
                              least 100 iterations) ends and the next refinement step
                              starts; refinement stops when a step gains less than 10%. */
  int32_t trunc;           /* > 0: A-orthonormalise against the last trunc blocks only
                              (truncated SRE-CG2, Section 3); 0 = all stored blocks */
  int64_t q_budget_bytes;  /* bytes of workspace reserved for stored blocks; 0 = room for
                              kmax-1 blocks of width t (or trunc blocks).  Blocks are packed
                              by their width; when the next one does not fit, the oldest
                              are dropped (truncation to the blocks that fit). */
  double deflate_tol;      /* drop a column whose Cholesky pivot <= deflate_tol times a
                              reference: its squared norm before the A-orthonormalisation
                              against the stored blocks (Euclidean step), its own diagonal
                              entry (A step); < 0 disables deflation (then a non-positive
                              pivot is ECG_EBREAKDOWN).  A dropped column stays a zero
                              column of the block. */
  int32_t precond;         /* ecg_precond_kind */
  const ecg_precond* M;    /* used when precond == ECG_PRECOND_SPLIT */
  int32_t variant;         /* ecg_variant */
  int32_t restart;         /* ecg_restart */
  int32_t restart_every;   /* RESTART_EVERY: cycle length j (>= 1) */
  double restart_tol;      /* RESTART_TOL: restartTol */
  int32_t max_restarts;    /* RESTART_TOL: limit on the number of restarts, 0 = none */
  int32_t restart_at_switch; /* != 0: every halving also empties Q (restarted flexible
                              variant); a halving takes precedence over a restart */
  int32_t refine_keep_q;   /* FP32_REFINED, != 0: the stored blocks are kept across residual
                              replacements and refinement steps.  Each time r is recomputed
                              from x (a replacement, the start of a refinement step) the
                              iterate is re-projected, x += Q (Q^T r), so that r is again
                              orthogonal to the stored blocks, and the next refinement step
                              extends the kept blocks instead of starting from none.
                              2: the same, except that a refinement step drops the kept
                              blocks when re-projecting its residual on them leaves more than
                              half of its norm (they would be swept every iteration for
                              little gain).  0: every refinement step starts from an empty
                              Q (replacements do not re-project). */
} ecg_options;

typedef struct {
  int32_t iters;            /* completed block iterations (all inner iterations summed
                               for FP32_REFINED) */
  int32_t n_switch;         /* number of halvings */
  int32_t switch_iters[8];  /* iteration k at which each halved block was formed (FP32_REFINED:
                               numbered within the refinement step's inner solve) */
  int32_t t_final;          /* block width at the end */
  int32_t outer_iters;      /* refinement steps (1 for FP64) */
  int32_t deflated_cols;    /* columns dropped by deflation */
  int32_t trunc_used;       /* the trunc option in force (0 = all stored blocks) */
  int32_t blocks_dropped;   /* stored blocks evicted because q_budget_bytes was full */
  int64_t vectors_stored;   /* sum of the widths of all blocks created (the paper's mem) */
  double relres_recursive;  /* ||r_k|| / ||r_0|| of the recursion */
  double relres_true;       /* ||b - A x|| / ||b||, recomputed in FP64 at the end */
  double seconds;           /* wall time of the solve, host clock */
  int32_t status;           /* ecg_status of the solve */
  int32_t n_restart;        /* number of restarts (including those at a halving) */
  int32_t restart_iters[8]; /* iteration k of the first restarts (numbered like switch_iters) */
  int64_t vectors_peak;     /* largest sum of widths stored within one restart cycle (the
                               mem of the paper's restarted runs; = vectors_stored without
                               restarts) */
} ecg_report;

/* Fill *o with defaults: tol 1e-8, kmax 20000, no reduction, switch_tol 1e-5, t_min 1,
 * min_gap 1, FP64, inner_tol 1e-4, max_outer 20, replace_every 25, trunc 0,
 * q_budget_bytes 0, deflate_tol 1e-14, no preconditioner, SRE-CG2, no restarts
 * (restart_every 0, restart_tol 1e-5, max_restarts 0, restart_at_switch 0),
 * refine_keep_q 2. */
ecg_status ecg_options_default(ecg_options* o);

/* Sparse SPD matrix A (n x n) in CSR form, copied to the device.
 * rowptr: int64[n+1], colind: int32[nnz] (each row sorted ascending, entries in [0,n)),
 * vals: double[nnz].  on_device != 0: the three arrays are device pointers, else host.
 * nnz must be < 2^31.  The matrix must be symmetric; this is not checked. */
ecg_status ecg_operator_create_csr(int64_t n, int64_t nnz, const int64_t* rowptr,
                                   const int32_t* colind, const double* vals, int on_device,
                                   void* hip_stream, ecg_operator** out);
void ecg_operator_destroy(ecg_operator* A);
/* n and nnz of an operator (host out-pointers). */
ecg_status ecg_operator_info(const ecg_operator* A, int64_t* n, int64_t* nnz);

/* Subdomain map (Section 2: disjoint delta_1..delta_t).  part: int32[n] with values in
 * [0, t), every subdomain non-empty (else ECG_EINVAL).  Halving merges subdomains 2i
 * and 2i+1 (Section 4): the map after l halvings is part >> l.  1 <= t <= 64. */
ecg_status ecg_partition_create(int64_t n, int32_t t, const int32_t* part, int on_device,
                                void* hip_stream, ecg_partition** out);
void ecg_partition_destroy(ecg_partition* P);

/* Block-Jacobi IC(0) preconditioner on the subdomains of P (Section 5.3): A restricted
 * to each subdomain (couplings between subdomains dropped) is factored by incomplete
 * Cholesky with zero fill, L_i L_i^T, in the matrix's own ordering.  The factorisation
 * runs on the device.  Fails with ECG_EBREAKDOWN if a pivot is not positive. */
ecg_status ecg_precond_create_bj_ic0(const ecg_operator* A, const ecg_partition* P,
                                     void* hip_stream, ecg_precond** out);

typedef enum {
  ECG_BJ_IC0 = 0,  /* incomplete Cholesky with zero fill of every block */
  ECG_BJ_CHOL = 1  /* exact Cholesky of every block (eq. (cholprec)) */
} ecg_bj_kind;

/* Block-Jacobi preconditioner on nblocks diagonal blocks of A chosen independently of the
 * ECG partition (Section 5.3: the paper uses 64 or 128 blocks for every t, the t
 * subdomains being unions of consecutive blocks).  block: int32[n], block[i] in
 * [0, nblocks), every block non-empty (device or host per on_device).  Couplings between
 * blocks are dropped; each block keeps the matrix order of its rows.
 * ECG_BJ_CHOL stores each factor as a band: the band of a block is the largest distance,
 * in that order, between a row and a column it couples to, and must be <= 128 (else
 * ECG_EINVAL): grid blocks at most 128 cells wide along the fastest axis.  Factorisation
 * runs on the device; a non-positive pivot gives ECG_EBREAKDOWN. */
ecg_status ecg_precond_create_bj(const ecg_operator* A, int32_t nblocks, const int32_t* block,
                                 int on_device, int32_t kind, void* hip_stream,
                                 ecg_precond** out);

/* Factorised approximate inverse M^{-1} = G G^T (so L^{-1} = G^T, L^{-T} = G in
 * eq. (zsre2)).  G is lower triangular in CSR (int64 rowptr, int32 colind, double vals,
 * each row sorted with the diagonal last), device or host per on_device.  Every
 * diagonal entry must be positive (checked; ECG_EINVAL otherwise). */
ecg_status ecg_precond_create_factor(int64_t n, int64_t nnz, const int64_t* rowptr,
                                     const int32_t* colind, const double* vals, int on_device,
                                     void* hip_stream, ecg_precond** out);
void ecg_precond_destroy(ecg_precond* M);

/* Bytes of device workspace ecg_solve needs for this operator, partition and options. */
ecg_status ecg_workspace_size(const ecg_operator* A, const ecg_partition* P,
                              const ecg_options* o, size_t* bytes);

/* Solve A x = b.  b: device double[n]; x: device double[n], holds x0 on entry and the
 * solution on exit.  workspace: device, >= ecg_workspace_size bytes, 256-byte aligned;
 * its contents on entry are irrelevant.  rep: host, filled on every return that got past
 * argument checking.  rho_hist: host, nullable, length >= kmax; receives ||r_k|| for
 * k = 0..iters (FP64 solves only).  Returns ECG_OK, ECG_ENOTCONV or an error. */
ecg_status ecg_solve(const ecg_operator* A, const ecg_partition* P, const double* b, double* x,
                     const ecg_options* o, void* workspace, size_t ws_bytes, void* hip_stream,
                     ecg_report* rep, double* rho_hist);

/* ecg_solve without a workspace argument, for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid hipMalloc): the solve runs
 * in a static device array of the library, 64 MiB (67108864 bytes) per device, kept from the
 * first call on a device until the process ends.  The call allocates nothing.  Arguments
 * and results are those of ecg_solve; hip_stream must belong to the current device.  A
 * solve whose ecg_workspace_size exceeds 64 MiB returns ECG_ENOMEM before any device work
 * (lower kmax, or bound the stored blocks with q_budget_bytes or trunc).  Every call on a
 * device shares that device's array and leaves its contents behind (the solve does not
 * depend on them): calls that overlap in time on one device, from several threads or
 * streams, race and must not be made. */
ecg_status ecg_solve_noalloc(const ecg_operator* A, const ecg_partition* P, const double* b, double* x,
                             const ecg_options* o, void* hip_stream, ecg_report* rep,
                             double* rho_hist);

/* y = A x for one vector (device double[n] each); used for true residuals. */
ecg_status ecg_spmv(const ecg_operator* A, const double* x, double* y, void* hip_stream);

/* ---- per-kernel timing ----------------------------------------------------------
 * When enabled, ecg_solve brackets every kernel launch of the classes below with HIP
 * events on its own stream and accumulates, per class: launches, event-measured
 * milliseconds, and the algorithmic bytes and flops of those launches (the data the
 * method must move: each stored column read once per sweep, each block row read or
 * written once).  Classes:
 *   0 SpMM Y = A X            bytes nnz*(w+4) + 4(n+1) + 2 w n t
 *   1 CGS2 Gram partials      bytes w n (m_span + t)        (one launch per span)
 *   2 CGS2 Gram chunk sums    bytes of the partial sums read and G written
 *   3 CGS2 update W -= Q G    bytes w n (m_span + 2t)       (one launch per span)
 *   4 t x t Grams             bytes w n (2t [+1])
 *   5 t x t factor            bytes 0
 *   6 H = C R^{-1}            bytes 2 w n t
 *   7 fused final update      bytes 4 w n t + traffic of x and r
 *   8 split / preconditioner  bytes as the kernels stream them
 *   9 residuals and norms     bytes of the vectors read and written
 * w = bytes per value of the block data (8 FP64, 4 FP32).  Timing adds a little host
 * overhead per launch; leave it off for wall-clock measurements.  Process-global. */
#define ECG_NSTAT 10
typedef struct {
  int64_t count[ECG_NSTAT];
  double ms[ECG_NSTAT];
  double bytes[ECG_NSTAT];
  double flops[ECG_NSTAT];
} ecg_kernel_stats;

ecg_status ecg_stats_enable(int on);
/* Copy the accumulated statistics into *out (host); reset != 0 clears them. */
ecg_status ecg_stats_read(ecg_kernel_stats* out, int reset);

/* Print "ecg: k=... rho/rho0=... t=... m=... elapsed=..." to stderr every `every`
 * iterations of ecg_solve (0 = never, the default).  Process-global. */
ecg_status ecg_progress(int32_t every);

/* Thread-local message for the last failing call. */
const char* ecg_last_error(void);

/* ---- building blocks exposed for kernel-level tests (device pointers, FP64) ---- */

/* Y = A X for a row-major n x t block (t in 1..64). */
ecg_status ecg_debug_spmm(const ecg_operator* A, int32_t t, const double* X, double* Y,
                          void* hip_stream);
/* Y = A X with a chosen product kernel: kernel 0 = CSR, 1 = diagonal form, 2 = grid stencil
 * (diagonal offsets -c, -b, -a, 0, a, b, c or -c, -a, 0, a, c with b dividing c and c
 * dividing n), 3 = 3-D grid stencil with its planes staged in LDS, 4 = the same with the
 * planes brought into LDS by direct buffer loads (3 and 4: seven diagonals, a = 1, at least
 * 4 lanes of 16 bytes per block row, nx a multiple of 16 / (bytes per value), and n t and
 * 7 n values within 32-bit byte offsets), 5 = SELL-C-sigma (C = 64 rows per
 * slice, rows sorted by length within windows of 1024; kept for matrices without a diagonal
 * form), -1 = the one the solver uses.
 * precision 0: X and Y are double, 1: float.  Row-major n x t blocks, t a power of two in
 * 1..64.  Every kernel builds a row as a chain of fused multiply-adds in the stored (CSR)
 * or ascending-offset order, so for rows stored in ascending column order and finite X all
 * of them give bitwise equal results.  ECG_EINVAL when the operator has no such form. */
ecg_status ecg_debug_spmm_kernel(const ecg_operator* A, int32_t kernel, int32_t precision, int32_t t,
                                 const void* X, void* Y, void* hip_stream);
/* out = [T^t(v)] with the map part >> level: out[i][j] = v[i] if (part[i]>>level) == j. */
ecg_status ecg_debug_split(const ecg_partition* P, int32_t level, const double* v, double* out,
                           void* hip_stream);
/* G = Q^T Y where Q is nb blocks of width wq stored block-major ([nb][n][wq]) and Y is a
 * row-major n x t block.  G: device double[nb*wq][t]. */
ecg_status ecg_debug_gram(int64_t n, int32_t nb, int32_t wq, const double* Q, int32_t t,
                          const double* Y, double* G, void* hip_stream);
/* W -= Q G (same layouts as ecg_debug_gram; W row-major n x t, updated in place). */
ecg_status ecg_debug_update(int64_t n, int32_t nb, int32_t wq, const double* Q, int32_t t,
                            const double* G, double* W, void* hip_stream);
/* FP32 forms of the two kernels above (the FP32_REFINED path), same layouts. */
ecg_status ecg_debug_gram_f32(int64_t n, int32_t nb, int32_t wq, const float* Q, int32_t t,
                              const float* Y, float* G, void* hip_stream);
ecg_status ecg_debug_update_f32(int64_t n, int32_t nb, int32_t wq, const float* Q, int32_t t,
                                const float* G, float* W, void* hip_stream);
/* Apply the preconditioner factors to a row-major n x t block: which = 0: Y = L^{-1} X,
 * which = 1: Y = L^{-T} X. */
ecg_status ecg_debug_precond_apply(const ecg_precond* M, int32_t which, int32_t t,
                                   const double* X, double* Y, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ECG_H */
