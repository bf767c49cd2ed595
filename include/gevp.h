/*
 * gevp.h -- C ABI of the MI355X seeded solver for sequences of dense complex
 * Hermitian generalized eigenproblems.
 *
 * The problem (the paper, section 1, eq. (3) and the paragraph before it):
 * for every k-point and every outer SCF iteration, find the lowest nev
 * eigenpairs of A x = lambda B x, A Hermitian (the Hamiltonian), B Hermitian
 * positive definite (the overlap), eigenvalues in ascending order (eq. (1)).
 * Successive iterations form a chain of correlated problems, and the previous
 * iteration's eigenvectors seed the next solve (section 2, first paragraph and
 * paragraph "Eigenvectors evolution").
 *
 * Method: Cholesky reduction to standard form C = L^{-1} A L^{-H}, then a
 * Chebyshev-filtered subspace iteration started from the seed block, with
 * CholQR orthonormalisation, Rayleigh-Ritz and residual-based locking, then
 * X = L^{-H} Y.  The paper names an improved subspace iteration as the
 * intended solver for the fast iterations (section 3) but gives no details;
 * the filter is the Chebyshev form of Zhou & Saad.
 *
 * Conventions for every entry point:
 *  - Matrices are complex128 (two doubles, real then imaginary) in
 *    column-major order with a leading dimension >= the row count, in DEVICE
 *    memory of the handle's device.  Only the lower triangles of A and B are
 *    read (LAPACK uplo = 'L').  A, B and X0 are never written.
 *  - The caller owns every buffer passed in.  Device workspace: by default the
 *    handle allocates it on first use with hipMalloc, grows it as needed and
 *    frees it in gevp_destroy; after gevp_set_workspace the handle works only
 *    in the caller's buffer (e.g. a torch tensor) and allocates no device
 *    memory at all, returning GEVP_ERR_WORKSPACE when a call needs more.
 *  - Work runs on the stream set with gevp_set_stream (default: the null
 *    stream).  gevp_solve returns after its work has completed, because its
 *    status depends on convergence; gevp_backward and the gevp_k_* kernels
 *    are asynchronous.
 *  - A handle is not thread-safe: one handle per host thread and stream.
 *  - Errors are returned as a status code and never raised across the ABI.
 */
#ifndef GEVP_H
#define GEVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gevp_ctx* gevp_handle;

typedef enum {
  GEVP_OK = 0,
  GEVP_ERR_INVALID = 1,    /* a bad argument; info->lapack_info = -(argument index) */
  GEVP_ERR_NOT_HPD = 2,    /* Cholesky of B failed; info->lapack_info = n + pivot (1-based) */
  GEVP_ERR_NOCONV = 3,     /* maxit reached; outputs hold the best pairs and residuals */
  GEVP_ERR_HIP = 4,        /* a HIP runtime call failed */
  GEVP_ERR_NONFINITE = 5,  /* NaN or Inf in A, B or X0 */
  GEVP_ERR_ALLOC = 6,      /* workspace allocation failed */
  GEVP_ERR_SINGULAR = 7,   /* a shifted matrix of the contour filter had a zero or
                              non-finite pivot */
  GEVP_ERR_WORKSPACE = 8   /* the buffer given to gevp_set_workspace is too small
                              for this call (see gevp_workspace_size) */
} gevp_status;

typedef enum {
  GEVP_FP64 = 0,   /* every step in FP64 */
  GEVP_FP32 = 1,   /* filter products in FP32 MFMA, everything else FP64 */
  GEVP_BF16X3 = 2  /* filter products in split-BF16 (3 products, FP32 accumulate) */
} gevp_precision;

/* Options; a zero-initialised struct selects every default. */
typedef struct {
  int precision;            /* gevp_precision; default GEVP_FP64 */
  int nex;                  /* guard vectors; 0 = max(16, ceil(0.15 nev)) rounded to 16 */
  int deg_init;             /* filter degree of a cold first sweep; 0 = 20 */
  int deg_max;              /* per-sweep cap on a column's degree; 0 = 36 */
  int maxit;                /* outer iterations; 0 = 40 */
  int lanczos_steps;        /* spectral-bound Lanczos steps; 0 = 24 */
  unsigned long long seed;  /* random fill of non-seeded columns */
  int skip_final_residual;  /* 1: skip the original-basis residual check */
  int batch_streams;        /* gevp_solve_batched: concurrent streams; 0 = 8 */
  int seed_monitor;         /* 1: with a seed X0, report how it relates to the result
                               (gevp_info seed_*) */
  int filter;               /* gevp_filter; default GEVP_FILTER_CHEBYSHEV */
  int contour_points;       /* quadrature nodes of the contour filter; 0 = 8 */
  int lock_mode;            /* 0 (default): hard locking -- the converged prefix of wanted
                               pairs leaves the orthonormalisation and Rayleigh-Ritz of later
                               sweeps; 1: soft locking -- converged columns are only left out
                               of the filter */
  int sweep_reduction;      /* low-precision filters: the largest residual reduction one sweep
                               aims for, as a power of ten (the products' rounding floor); 0 =
                               default (4 for split-BF16, 6 for FP32) */
  int reserved[2];
} gevp_opts;

/* Filter of the subspace iteration.  The contour filter (section 3 names a
 * Sakurai-Sugiura solver as a candidate for the fast iterations) applies
 * sum_j w_j (z_j I - C)^{-1} to the block, the trapezoidal rule on a circle
 * around the wanted eigenvalues (see gevp_k_contour_filter).  It needs the
 * Ritz values of a seed to place the circle, so it is used for seeded solves
 * with k0 > nev (and n <= 65535); other solves take the Chebyshev filter.  With
 * opts.precision = GEVP_FP64 its factorisations and solves are FP64; with
 * GEVP_FP32 or GEVP_BF16X3 they are FP32 and act only on the Ritz residuals
 * (residual-correction form: (z I - C)^{-1} q = [q + (z I - C)^{-1} r] / (z - theta)
 * for a Ritz pair), so the result still reaches FP64 residuals. */
typedef enum {
  GEVP_FILTER_CHEBYSHEV = 0,
  GEVP_FILTER_CONTOUR = 1
} gevp_filter;

/* Diagnostics, filled on return when a non-NULL pointer is passed. */
typedef struct {
  int64_t lapack_info;    /* zhegv-style: 0, -i bad argument, n+i Cholesky pivot i */
  int outer_iters;        /* filter + QR + Rayleigh-Ritz sweeps */
  int nconv;              /* converged wanted pairs (nev on success) */
  int block;              /* nev + nex */
  int qr_fallbacks;       /* shifted-CholQR fallbacks taken */
  int64_t col_degrees;    /* filter GEMM column-steps summed over sweeps (8 n^2 flops each) */
  double max_resid;       /* max_i ||A x_i - lambda_i B x_i||_2 / ||A||_2 (original basis) */
  double normA, normB;    /* Lanczos estimates of ||A||_2, ||B||_2 */
  double filter_flops;    /* useful filter flops, 8 n^2 per column-degree */
  double ms[8];           /* stage times (ms), profiling bit 0: see gevp_stage */
  double filter_kernel_ms;  /* summed duration of the filter GEMM launches, profiling bit 1 */
  int64_t filter_launches;  /* number of those launches */
  /* Seed monitor (opts.seed_monitor, seeded solves; section 2, paragraph
     "Eigenvectors evolution": how far eigenvectors move between SCF steps).
     With k = min(nev, k0) and M = X0(:, :k)^H B X(:, :k) (both blocks
     B-orthonormal, so the singular values of M are the cosines of the
     principal angles between the two spans; formed in the reduced basis as
     (L^H X0)^H (L^H X)):
       seed_sin_rms   = the RMS sine of those angles, sqrt(sum_j ||r_j||_B^2 / k)
                        with r_j the B-orthogonal projection residual of seed
                        column j onto span X(:, :k) (equal to
                        sqrt(k - ||M||_F^2) in exact arithmetic, but free of
                        its cancellation, so it resolves angles down to
                        rounding level);
       seed_dev_mean, seed_dev_max: per result column j, the deviation angle
                        arccos(max_i |M(i, j)|) / (pi/2) (1 = orthogonal), mean and max;
       seed_reindexed = columns j matched to a seed column other than j;
       seed_dev_std  = standard deviation of the deviation angles.
     The matching minimises the summed deviation angles over permutations: each
     column's largest overlap when those are distinct (then optimal), else a
     linear assignment on arccos|M| solved on the device in O(k^3).
     -1 (and 0) when not computed. */
  double seed_sin_rms;
  double seed_dev_mean, seed_dev_max;
  int seed_reindexed;
  /* Contour filter (opts.filter = GEVP_FILTER_CONTOUR and used): the circle's
     diameter [contour_a, contour_b], its nodes, how many times the filter was
     applied and the block columns filtered, summed over the applications
     (converged columns are not filtered again); 0 otherwise.  Work: nq
     factorisations of 8 n^3 / 3 flops and 8 n^2 nq flops per filtered column. */
  int contour_points;
  double contour_a, contour_b;
  int contour_applications;
  int64_t contour_columns;
  double seed_dev_std;    /* see the seed monitor fields above */
  /* FP64 complex GEMM launches (profiling bit 4, every stream of the solve):
     summed duration (HIP events around each launch, split-K reduction
     included), algorithmic flops (8 m n k for a dense product, half of it
     where only one triangle of the output or of op(A) is involved) and the
     number of launches */
  double gemm_kernel_ms;
  double gemm_flops;
  int64_t gemm_launches;
  int locked;             /* columns hard-locked in the last sweep */
} gevp_info;

typedef enum {
  GEVP_STAGE_STAGE = 0,   /* input mirroring and scans */
  GEVP_STAGE_CHOL = 1,    /* Cholesky of B */
  GEVP_STAGE_REDUCE = 2,  /* C = L^{-1} A L^{-H} */
  GEVP_STAGE_BOUNDS = 3,  /* Lanczos bounds */
  GEVP_STAGE_FILTER = 4,  /* Chebyshev filter */
  GEVP_STAGE_QR = 5,      /* CholQR */
  GEVP_STAGE_RR = 6,      /* Rayleigh-Ritz incl. the small eigensolve */
  GEVP_STAGE_FINAL = 7    /* back-transform and residual */
} gevp_stage;

/* Create a handle on HIP device `device`.  The workspace is allocated lazily. */
gevp_status gevp_create(gevp_handle* h, int device);

/* Run subsequent work on `hip_stream` (a hipStream_t; NULL = null stream). */
gevp_status gevp_set_stream(gevp_handle h, void* hip_stream);

/* Profiling bits: 1 = per-stage HIP event times into gevp_info.ms (adds a
 * synchronisation per stage); 2 = HIP events around every filter product
 * (its operand conversion, product and split-K reduction kernels), summed
 * into gevp_info.filter_kernel_ms (no added synchronisation), and around the
 * scan and apply kernels of gevp_update_thresholded (gevp_update_info.scan_ms,
 * apply_ms); 4 = HIP events around every FP64 GEMM launch, summed into
 * gevp_info.gemm_kernel_ms with their flops. */
gevp_status gevp_set_profiling(gevp_handle h, int flags);

/* Free the workspace and the handle. */
void gevp_destroy(gevp_handle h);

const char* gevp_status_string(gevp_status s);

/* Block width nev + nex that gevp_solve uses for these options. */
int64_t gevp_block_size(const gevp_opts* opts, int64_t n, int64_t nev);

/* Device workspace, in bytes, that gevp_solve needs for a problem of order n
 * with nev wanted pairs and these options (any seed), including six fixed
 * split-K buffers of 128 MiB for the streams a solve may use.  Also enough for
 * gevp_backward with the same n and nev columns.  *bytes is written; the
 * handle is not touched and may be NULL. */
gevp_status gevp_workspace_size(gevp_handle h, const gevp_opts* opts, int64_t n, int64_t nev,
                                size_t* bytes);

/* The same for gevp_solve_batched over `count` problems of orders n[i] with
 * nev[i] wanted pairs: every concurrent stream gets an equal share, sized for
 * the largest problem. */
gevp_status gevp_workspace_size_batched(gevp_handle h, const gevp_opts* opts, int count,
                                        const int64_t* n, const int64_t* nev, size_t* bytes);

/* Work in caller-owned device memory from now on (the paper states the
 * problem, section 1, eq. (3); where the memory comes from is the caller's
 * choice, e.g. a torch tensor).  dev_ptr: device memory of the handle's
 * device, 256-byte aligned, `bytes` >= 6 x 128 MiB + 256 (the split-K slots
 * at its top end), owned by the caller and left valid until the handle is
 * destroyed or the workspace replaced.  The handle then calls no hipMalloc
 * or hipFree for device memory; a call that needs more than the buffer
 * returns GEVP_ERR_WORKSPACE before launching anything.  Memory the handle
 * had allocated itself is freed here.  dev_ptr = NULL returns to
 * library-managed memory.  Waits for the handle's streams.  Calls that share
 * a handle must not overlap (one handle per stream, as always). */
gevp_status gevp_set_workspace(gevp_handle h, void* dev_ptr, size_t bytes);

/*
 * Lowest eigenpairs of A x = lambda B x.
 *   n        order of A and B (n >= 1)
 *   A, lda   device complex128 n x n, Hermitian, lower triangle read
 *   B, ldb   device complex128 n x n, Hermitian positive definite, lower read
 *   X0, ldx0, k0
 *            optional seed block (device complex128 n x k0, k0 <= block), the
 *            previous SCF iteration's eigenvectors in the original basis;
 *            X0 = NULL or k0 = 0 is a cold start.  Columns beyond k0 are
 *            filled from a counter-based random generator (opts->seed); an
 *            all-zero seed column is replaced by a fixed pseudo-random one,
 *            and linearly dependent ones are handled by the orthonormalisation
 *            (shifted CholQR when needed).
 *   nev      wanted pairs, 1 <= nev <= n
 *   tol      convergence: ||A x_i - lambda_i B x_i||_2 <= tol ||A||_2 for
 *            every i < nev (tol > 0; 1e-10 is typical)
 *   kx       columns returned, nev <= kx <= block: the first nev are the
 *            wanted pairs, the rest are the guard Ritz pairs (useful as the
 *            next seed)
 *   lambda   device float64[kx], ascending
 *   X, ldx   device complex128 n x kx, B-orthonormal eigenvectors; the
 *            largest-modulus entry of each column is real and positive
 *   resid    optional device float64[kx]: ||A x_i - lambda_i B x_i||_2 (without it
 *            the final check forms the residuals of the nev wanted pairs only)
 *   info     optional host struct
 * Returns GEVP_OK, or GEVP_ERR_NOCONV with the best pairs written.
 */
gevp_status gevp_solve(gevp_handle h, const gevp_opts* opts, int64_t n,
                       const void* A, int64_t lda, const void* B, int64_t ldb,
                       const void* X0, int64_t ldx0, int64_t k0,
                       int64_t nev, double tol, int64_t kx,
                       double* lambda, void* X, int64_t ldx, double* resid,
                       gevp_info* info);

/*
 * Batched k-points: `count` independent problems of uneven size (the paper,
 * section 1: one pencil per Bloch vector k).  Arrays of length count hold
 * per-problem arguments as in gevp_solve (X0[i] may be NULL).  kx[i] = nev[i]
 * when kx is NULL.  infos may be NULL.  Returns the worst status.
 * The problems run concurrently on opts->batch_streams HIP streams owned by
 * the handle (one host thread each), largest first; every stream waits for
 * the work already queued on the handle's stream, and the call returns when
 * all problems are done.  Each stream keeps a workspace sized for the largest
 * problem it has solved.
 */
gevp_status gevp_solve_batched(gevp_handle h, const gevp_opts* opts, int count,
                               const int64_t* n, const void* const* A, const int64_t* lda,
                               const void* const* B, const int64_t* ldb,
                               const void* const* X0, const int64_t* ldx0, const int64_t* k0,
                               const int64_t* nev, double tol, const int64_t* kx,
                               double* const* lambda, void* const* X, const int64_t* ldx,
                               double* const* resid, gevp_info* infos);

/*
 * Launch configuration of gevp_solve_batched (section 1: one pencil per Bloch
 * vector k; the problems of a batch share the GPU).
 *   streams     concurrent streams; > 0 overrides opts->batch_streams (at most
 *               16 and at most count; ignored while a caller-owned workspace is
 *               set, whose shares gevp_workspace_size_batched sized for the
 *               options' rule)
 *   split_mode  split-K of the FP64 and split-BF16 products: 0 = cost model
 *               over all compute units, 1 = over one stream's share of them,
 *               2 = no split-K
 *   seconds     the measured time of one batched call (autotuner output)
 */
typedef struct {
  int streams;
  int split_mode;
  double seconds;
  int reserved[4];
} gevp_tuning;

/*
 * Autotuner of gevp_solve_batched: the same arguments, solved once untimed
 * (workspace set-up) and then once per candidate configuration — streams in
 * {4, 8, 12, 16} (those <= count, plus count itself when below 16) times the
 * three split modes — timed on the host around each complete call.  The
 * fastest configuration is kept in the handle for later gevp_solve_batched
 * calls and written to *best (may be NULL); the outputs hold the last call's
 * results.  Costs about a dozen batched solves; allocates workspace like
 * gevp_solve_batched.  Returns the status of the last call, or that of the
 * first failing one.
 */
gevp_status gevp_autotune_batched(gevp_handle h, const gevp_opts* opts, int count,
                                  const int64_t* n, const void* const* A, const int64_t* lda,
                                  const void* const* B, const int64_t* ldb,
                                  const void* const* X0, const int64_t* ldx0, const int64_t* k0,
                                  const int64_t* nev, double tol, const int64_t* kx,
                                  double* const* lambda, void* const* X, const int64_t* ldx,
                                  double* const* resid, gevp_tuning* best);

/* Set (t != NULL; streams 0..16, split_mode 0..2, else GEVP_ERR_INVALID) or
 * clear (t == NULL) the handle's batched launch configuration, e.g. one read
 * back from a tuning cache. */
gevp_status gevp_set_tuning(gevp_handle h, const gevp_tuning* t);

/* The handle's batched launch configuration (zeros when none is set). */
gevp_status gevp_get_tuning(gevp_handle h, gevp_tuning* t);

/*
 * Adjoint of L = sum_i w_i lambda_i (first-order perturbation of a
 * B-orthonormal pair: d lambda_i = x_i^H (dA - lambda_i dB) x_i):
 *   dA = X diag(w) X^H,    dB = -X diag(w .* lambda) X^H     (full n x n)
 * X: device complex128 n x nev (ldx); lambda, w: device float64[nev];
 * dA, dB: device complex128 n x n outputs, either may be NULL.
 */
gevp_status gevp_backward(gevp_handle h, int64_t n, int64_t nev, const void* X, int64_t ldx,
                          const double* lambda, const double* w,
                          void* dA, int64_t ldda, void* dB, int64_t lddb);

/*
 * gevp_backward for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and asynchronous behaviour, but the n x nev scaled copy
 * of X lives in a fixed 32 MiB device array of the library (one per device,
 * held until the process ends; its device address is taken once per device
 * by gevp_create) and no call here allocates or frees memory, creates events
 * or splits K.  n * nev * 16 bytes must not exceed 32 MiB (e.g. n = 4096,
 * nev <= 512): larger problems return GEVP_ERR_WORKSPACE with nothing
 * launched.  Every call on a device shares that device's array: calls that
 * overlap on one device (other streams, other handles or threads) race and
 * must be ordered by the caller.  The array keeps the last call's contents;
 * nothing in it needs to start at zero.
 */
gevp_status gevp_backward_noalloc(gevp_handle h, int64_t n, int64_t nev, const void* X,
                                  int64_t ldx, const double* lambda, const double* w, void* dA,
                                  int64_t ldda, void* dB, int64_t lddb);

/* ---- kernel-level entry points (the building blocks, exposed for tests) ---- */

/*
 * D = alpha op(A) op(B) + beta Cm + gamma diag-scaled E on FP64 MFMA, complex128.
 *   opA, opB: 'N' or 'C' (conjugate transpose).  op(A) is m x k, op(B) k x n.
 *   Cm may alias D; Cm / E may be NULL (term dropped).  gcol (device float64[n])
 *   scales the E term per column when non-NULL.  Asynchronous.
 */
gevp_status gevp_k_zgemm(gevp_handle h, char opA, char opB, int64_t m, int64_t n, int64_t k,
                         double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                         double beta, const void* Cm, int64_t ldc,
                         double gamma, const void* E, int64_t lde, const double* gcol,
                         void* D, int64_t ldd);

/*
 * The structured forms of gevp_k_zgemm that the solver uses internally (no E
 * term).  lower = 1: square output (m == n), only the 64 x 64 tiles that touch
 * the lower triangle are computed (entries of tiles entirely above the
 * diagonal are left as they were; the other entries of the diagonal tiles are
 * written).  upperA = 1: only the upper triangle of op(A) is used; entries
 * below its diagonal read as zero whatever the memory holds.  Asynchronous.
 */
gevp_status gevp_k_zgemm_tri(gevp_handle h, char opA, char opB, int64_t m, int64_t n, int64_t k,
                             double alpha, const void* A, int64_t lda, const void* B, int64_t ldb,
                             double beta, const void* Cm, int64_t ldc, void* D, int64_t ldd,
                             int lower, int upperA);

/*
 * One step of the low-precision residual-correction filter (the Chebyshev
 * recurrence of the mixed-precision forms), per column j < m:
 *   D(:, j) = alpha_j C G(:, j) + beta_j G(:, j) + gamma_j P(:, j) + delta_j R(:, j)
 * C: device complex128 n x n Hermitian (full storage), converted internally to
 * the precision's format (GEVP_FP32: complex64; GEVP_BF16X3: split-BF16 row
 * planes).  G, P, R, D: device complex64 n x m; D may alias P.
 * alpha..delta: device float64[m].  Asynchronous.
 */
gevp_status gevp_k_filter_gemm(gevp_handle h, int precision, int64_t n, int64_t m,
                               const void* C, int64_t ldc, const void* G, int64_t ldg,
                               const void* P, int64_t ldp, const void* R, int64_t ldr, void* D,
                               int64_t ldd, const double* alpha, const double* beta,
                               const double* gamma, const double* delta);

/* y = M x for an n x n Hermitian M stored in full (device complex128,
 * column-major, ld ldm >= n; only the 64 x 64 tiles on and below the diagonal
 * are read), x and y device vectors of n complex128 (y must not overlap M or
 * x).  The matrix-vector product of the Lanczos spectral bounds that set the
 * Chebyshev filter's interval (section 3: the filter damps the unwanted part
 * of the spectrum, whose ends the bounds estimate).  Asynchronous. */
gevp_status gevp_k_hemv(gevp_handle h, int64_t n, const void* M, int64_t ldm, const void* x, void* y);

/* In-place Cholesky of the lower triangle of the n x n Hermitian M (upper
 * triangle zeroed).  Synchronous; returns GEVP_ERR_NOT_HPD with *pivot
 * (1-based) on failure. */
gevp_status gevp_k_potrf(gevp_handle h, int64_t n, void* M, int64_t ldm, int64_t* pivot);

/* Triangular solves with the lower-triangular L (n x n):
 *   side 'L', trans 'N':  R <- L^{-1} R        (R is n x m)
 *   side 'L', trans 'C':  R <- L^{-H} R        (R is n x m)
 *   side 'R', trans 'C':  R <- R L^{-H}        (R is m x n)
 * Asynchronous. */
gevp_status gevp_k_trsm(gevp_handle h, char side, char trans, int64_t n, int64_t m,
                        const void* L, int64_t ldl, void* R, int64_t ldr);

/* Seed monitor of a k x k cross-overlap M = X0^H B X of two B-orthonormal
 * blocks (device complex128, 1 <= k <= 8192): stats (host double[5]) receives
 * sin_rms, dev_mean, dev_max, reindexed and dev_std as in gevp_info, match
 * (optional host int[k]) the seed column matched to each column.  When two
 * columns share a best match, the matching is the minimum-total-angle
 * assignment, solved on the device.  Synchronous. */
gevp_status gevp_k_seed_monitor(gevp_handle h, int64_t k, const void* M, int64_t ldm, double* stats,
                                int* match);

/* Eigen-decomposition of a small Hermitian matrix (n <= 2048) on the GPU:
 * H = Z diag(theta) Z^H, theta ascending.  H (lower read) is overwritten.
 * Synchronous. */
gevp_status gevp_k_heev(gevp_handle h, int64_t n, void* H, int64_t ldh,
                        double* theta, void* Z, int64_t ldz);

/* ------------------------------------------------------------------------
 * Contour-integral filter pieces (section 3: Sakurai-Sugiura solver named as
 * a candidate for the fast iterations; trapezoidal quadrature of the
 * resolvent on a circle, first moment).
 * ------------------------------------------------------------------------ */

/* LU factorisation without row exchanges of z I - C, z = zr + i zi:
 * LU (n x n, ld ldlu) receives the packed factors (L unit lower strictly
 * below the diagonal, U on and above).  C (device complex128 n x n) is read in
 * full.  For Hermitian C and zi != 0 every pivot is nonzero in exact
 * arithmetic (-i (z I - C) has Hermitian part zi I); for other inputs the
 * factorisation may break down.  n <= 65535.  Synchronous; returns GEVP_ERR_SINGULAR with
 * *pivot = the first zero or non-finite pivot (1-based), else *pivot = 0. */
gevp_status gevp_k_lu_shifted(gevp_handle h, int64_t n, const void* C, int64_t ldc, double zr,
                              double zi, void* LU, int64_t ldlu, int64_t* pivot);

/* Y = sum_j w_j (z_j I - C)^{-1} V for the nq-point trapezoidal rule on the
 * circle with diameter [a, b] on the real axis:
 *   z_j = gamma + rho e^{i t_j}, w_j = rho e^{i t_j} / nq,
 *   t_j = 2 pi (j + 1/2) / nq, gamma = (a + b) / 2, rho = (b - a) / 2,
 * so an eigenvector of a Hermitian C with eigenvalue lambda is scaled by
 * 1 / (1 + t^nq), t = (lambda - gamma) / rho.  C: device complex128 n x n
 * (read in full); V: n x m; Y: n x m (must not overlap V); a < b finite,
 * 1 <= nq <= 256, n and m <= 65535.  Factors every z_j I - C (workspace nq n^2 complex128).
 * Synchronous; GEVP_ERR_SINGULAR if a factorisation broke down. */
gevp_status gevp_k_contour_filter(gevp_handle h, int64_t n, const void* C, int64_t ldc,
                                  const void* V, int64_t ldv, int64_t m, double a, double b, int nq,
                                  void* Y, int64_t ldy);

/* ------------------------------------------------------------------------
 * Thresholded partial update of a Hermitian matrix between two SCF
 * iterations (section 2, paragraph "Matrix generation").  The paper measures
 * the change between adjacent Hamiltonians at one k-point by the largest
 * entry variation delta and proposes updating only the entries whose change,
 * normalised by delta, exceeds a threshold p_t; the other entries keep their
 * previous values (and need not be regenerated).
 *
 * Readings: delta is the largest modulus |A_new(i,j) - A(i,j)| over the
 * stored lower triangle (diagonal included); an entry is updated when
 * |A_new(i,j) - A(i,j)| > p_t * delta (strict), evaluated in FP64 as
 *   dr*dr + di*di > (p_t*p_t) * delta^2,  dr, di the real and imaginary
 *   differences, every operation rounded separately (no fused multiply-add).
 *
 * Mask layout (both functions): uint32 words, column-major with leading
 * dimension ldmask >= ceil(n/32): bit (i mod 32) of word mask[j*ldmask + i/32]
 * is entry (i, j).  Only bits with i >= j and i < n are ever set.
 * ------------------------------------------------------------------------ */
typedef struct {
  double delta;            /* max |A_new - A| over the lower triangle; NaN if non-finite */
  int64_t entries;         /* n (n + 1) / 2 */
  int64_t updated;         /* entries taken from A_new */
  int64_t tiles;           /* 64 x 64 tiles of the lower triangle */
  int64_t tiles_touched;   /* tiles with at least one updated entry */
  int64_t tiles_copied;    /* tiles whose every entry was above threshold */
  int nonfinite;           /* 1 when a change was NaN, Inf, or overflowed when squared */
  int reserved;
  double scan_ms, apply_ms; /* profiling flag 2 and info given: durations of the scan
                               and the apply kernel (HIP events on the handle's
                               stream); else 0 */
  int64_t rechecked;       /* entries whose 16-bit code of |dA|^2 tied with the
                              threshold's and were decided by re-reading both
                              matrices */
} gevp_update_info;

/*
 * A <- A with every lower entry whose change exceeds p_t * delta taken from
 * A_new.
 *   n          order (n >= 0; n = 0 does nothing)
 *   A, lda     device complex128 n x n, lower triangle read and updated in
 *              place; the strict upper triangle is never written.  Loads of
 *              the edge tiles may touch (and ignore) any entry of the n x n
 *              storage.
 *   A_new, ldn device complex128 n x n, the newly generated matrix (lower
 *              triangle used); must not overlap A unless it is A itself
 *   p_t        threshold as a fraction of delta, 0 <= p_t < inf
 *              (p_t = 0: every changed entry; p_t >= 1: none)
 *   mask       optional device uint32 words (layout above, ldmask words per
 *              column): receives the updated entries; every word of rows
 *              < n is written
 *   info       optional host struct.  With info the call waits for the
 *              result; without it the call is asynchronous on the handle's
 *              stream.
 * A non-finite change (or one whose square overflows) cancels the whole
 * update: A and the mask's set bits are left as if nothing were above
 * threshold, and with info the call returns GEVP_ERR_NONFINITE.
 * Pointers must be 16-byte aligned (mask: 4-byte); otherwise, and for a bad
 * size or p_t, GEVP_ERR_INVALID with nothing launched.  With n = 0 the
 * pointers are not looked at.
 */
gevp_status gevp_update_thresholded(gevp_handle h, int64_t n, void* A, int64_t lda,
                                    const void* A_new, int64_t ldn, double p_t, uint32_t* mask,
                                    int64_t ldmask, gevp_update_info* info);

/*
 * The fast-iteration update of the same paragraph: only part of the entries
 * of the next matrix were regenerated (those marked in `mask`, e.g. by a
 * previous gevp_update_thresholded); they are copied from S into A, every
 * other entry of A is left alone.  Lower-triangle bits only (i >= j); S is
 * read only where a bit is set.  Asynchronous; A and S must not overlap.
 * Errors as for gevp_update_thresholded.
 */
gevp_status gevp_update_masked(gevp_handle h, int64_t n, void* A, int64_t lda, const void* S,
                               int64_t lds, const uint32_t* mask, int64_t ldmask);

#ifdef __cplusplus
}
#endif
#endif /* GEVP_H */
