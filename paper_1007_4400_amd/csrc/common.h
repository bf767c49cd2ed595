// Internal declarations shared by the HIP sources of libgevp.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/gevp.h"

typedef double2 zd;  // complex128 stored as (re, im)

// ---------------------------------------------------------------- host side

#define GEVP_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) {                                                         \
      if (gevp_log_enabled())                                                       \
        fprintf(stderr, "[gevp] %s failed: %s (%s:%d)\n", #expr, hipGetErrorString(_e), \
                __FILE__, __LINE__);                                                \
      return GEVP_ERR_HIP;                                                          \
    }                                                                               \
  } while (0)

#define GEVP_TRY(expr)                   \
  do {                                   \
    gevp_status _s = (expr);             \
    if (_s != GEVP_OK) return _s;        \
  } while (0)

// GEVP_LOG=1: failures and per-sweep diagnostics on stderr; GEVP_LOG=2 also
// prints every timed FP64 GEMM launch (profiling bit 4) with its shape
int gevp_log_enabled();
// event pair around one filter product (profiling bit 2), see solver.hip
gevp_status fev_mark(gevp_ctx* c);
// event pair around one FP64 GEMM launch (profiling bit 4); gev_end also adds
// the launch's algorithmic flops to the context's tally
gevp_status gev_begin(gevp_ctx* c);
// shape = {form (opA * 2 + opB), m, n, k, split-K factor, work-groups}
gevp_status gev_end(gevp_ctx* c, double flops, const int64_t* shape = nullptr);
int gevp_device_cus(int device);  // compute units of a device (cached)

struct gevp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int profiling = 0;
  // bump-allocated workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_used = 0;
  // event pairs around filter GEMM launches (profiling bit 1)
  hipEvent_t* fev = nullptr;
  int fev_cap = 0;
  int fev_used = 0;
  // event pairs around FP64 GEMM launches (profiling bit 4) and their flops
  hipEvent_t* gev = nullptr;
  int gev_cap = 0;
  int gev_used = 0;
  double gev_flops = 0.0;
  std::vector<double> gev_shape;  // GEVP_LOG=2: 7 values per timed launch (shape, flops)
  // replayable launch sequences (the tridiagonalisation's one launch per
  // reflector, heev.hip): executable graphs keyed by their kernel arguments,
  // captured on a private stream, released by destroy
  struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t cap_stream = nullptr;
  // split-K partial products of launch_zgemm (grown on demand, freed by destroy)
  void* skw = nullptr;
  size_t skw_bytes = 0;
  // second stream of a seeded solve (own split-K buffer; created on demand)
  gevp_ctx* aux = nullptr;
  // false for the worker contexts of gevp_solve_batched: problems already run
  // concurrently there, so a solve keeps all its work on its own stream
  bool inner_streams = true;
  // panel stream of the Cholesky factorisation and its two events (on demand)
  gevp_ctx* panel = nullptr;
  hipEvent_t pev[2] = {nullptr, nullptr};
  // per-stream sub-contexts of gevp_solve_batched (own stream and workspace)
  std::vector<gevp_ctx*> workers;
  // streams of the contour filter's independent quadrature nodes (on demand)
  std::vector<gevp_ctx*> qctx;
  bool owns_stream = false;
  // Caller-owned device memory (gevp_set_workspace): ws and skw point into it
  // and are never allocated or freed by the library.  On the handle, ext_base
  // / ext_bytes describe the whole region; sub-contexts only borrow slices.
  bool ext = false;
  char* ext_base = nullptr;
  size_t ext_bytes = 0;
  // set for the duration of a call that must not allocate: launch_zgemm then
  // never splits K (which needs the split-K buffer)
  bool no_split = false;
  // split-K cost models count the compute units divided by this (a batched
  // worker shares the GPU with the other streams)
  int cu_div = 1;
  // launch configuration of gevp_solve_batched chosen by gevp_autotune_batched
  // or gevp_set_tuning (0 streams: the options' rule)
  int tune_streams = 0;
  int tune_split = 0;
  double tune_seconds = 0.0;
};

// Split-K partial products of launch_zgemm: one fixed-size buffer per stream
// context (2048 partial 64 x 64 complex128 tiles).
constexpr size_t SKW_BYTES = (size_t)2048 * 64 * 64 * 16;
// Slots of a caller-owned workspace reserved for split-K buffers, at its top
// end: the handle's stream, the second stream of a seeded solve, the panel
// stream of the Cholesky factorisation and three quadrature-node streams.
constexpr int EXT_SLOTS = 6;
enum { SLOT_MAIN = 0, SLOT_AUX = 1, SLOT_PANEL = 2, SLOT_QUAD0 = 3 };
// Lend slot `slot` of parent's caller-owned workspace to the sub-context
// child (no-op when parent manages its own memory).
void ext_assign(gevp_ctx* parent, gevp_ctx* child, int slot);

// Workspace carving.  reserve() (re)allocates when `bytes` exceeds the current
// size; take() hands out 256-byte aligned pieces until reset().
gevp_status ws_reserve(gevp_ctx* c, size_t bytes);
void* ws_take(gevp_ctx* c, size_t bytes);
inline size_t ws_round(size_t b) { return (b + 255) & ~size_t(255); }

// ---- kernel launchers (host functions, asynchronous on c->stream)

// D = alpha op(A) op(B) + beta Cm + gamma diag(gcol) E   (FP64 MFMA, complex128)
// When `coef` (device double[3]) is non-null it supplies alpha, beta, gamma.
// lower = 1 computes only the 64 x 64 tiles that touch the lower triangle
// (Hermitian updates whose upper triangle is never read).  upperA = 1 uses only
// the upper triangle of op(A) (e.g. L^H): each output row block skips the K
// range below its first row and entries below op(A)'s diagonal read as zero.  Products with few
// output tiles and a long K run split-K through c->skw (see zgemm.hip).
// A2 (op(A) = 'N' only): op(A) is [A; A2] stacked, rows 0..m1-1 from A and
// rows m1..m-1 from A2 (same lda): two products that share op(B) in one
// launch, so their tiles fill the rounds together.
gevp_status launch_zgemm(gevp_ctx* c, int opA, int opB, int64_t m, int64_t n, int64_t k,
                         double alpha, const zd* A, int64_t lda, const zd* B, int64_t ldb,
                         double beta, const zd* Cm, int64_t ldc, double gamma, const zd* E,
                         int64_t lde, const double* gcol, zd* D, int64_t ldd,
                         const double* coef = nullptr, int lower = 0, int upperA = 0,
                         int64_t m1 = 0, const zd* A2 = nullptr);

// Blocked Cholesky of the lower triangle; Dinv (n x 64 column-major, ld =
// ldi) receives the inverses of the 64 x 64 diagonal blocks; *info_dev
// (device int) receives the first failing pivot (1-based) or stays 0.  If
// given, `midpoint` is recorded on c->stream once half the block columns
// are queued (from there on the factorisation leaves most compute units idle).
// If R is given (n x m, ld ldr), it is overwritten by L^{-1} R, the forward
// substitution carried along panel by panel: each block row of R is solved
// with its panel's diagonal block as soon as that panel is factored and
// updated with the panel below it, work that overlaps the factorisation of
// the next panel.
gevp_status chol_lower(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* Dinv, int64_t ldi,
                       int* info_dev, hipEvent_t midpoint = nullptr, zd* R = nullptr,
                       int64_t ldr = 0, int64_t m = 0);
// R <- L^{-1} R (R n x m) ;  R <- L^{-H} R ;  R <- R L^{-H} (R m x n)
// lhu = 1: the strictly upper triangle of L holds L^H (see launch_mirror_lower),
// and the off-diagonal products read those blocks as stored instead of
// conjugate-transposing the blocks below the diagonal
gevp_status trsm_left_lower_n(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                              const zd* Dinv, int64_t ldi, zd* R, int64_t ldr);
gevp_status trsm_left_lower_c(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                              const zd* Dinv, int64_t ldi, zd* R, int64_t ldr, int lhu = 0);
gevp_status trsm_right_lower_c(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                               const zd* Dinv, int64_t ldi, zd* R, int64_t ldr);
// Lower triangle only of R <- R L^{-H} for square n x n R: rows below each
// column block's start are all that is computed (the Hermitian C = W L^{-H}).
gevp_status trsm_right_lower_c_lowerpart(gevp_ctx* c, int64_t n, const zd* L, int64_t ldl,
                                         const zd* Dinv, int64_t ldi, zd* R, int64_t ldr, int lhu = 0);
// Inverses of the 64 x 64 diagonal blocks of an already factored L.
gevp_status diag_block_inverses(gevp_ctx* c, int64_t n, const zd* L, int64_t ldl, zd* Dinv,
                                int64_t ldi);

// Contour-integral filter (contour.hip).  lu_nopiv: M = L U in place without
// row exchanges (L unit lower, packed), DinvL / DinvU (n x 64, ld ldi) receive
// the inverses of the 64 x 64 diagonal blocks of L and U, *info_dev the first
// failing pivot.  contour_factor forms and factors z_j I - C for the nq nodes
// of the circle with diameter [a, b] into `work` (contour_work_bytes(n, mmax,
// nq)), *pivot = first failing pivot or 0 (waits for the result);
// contour_apply then forms Y = sum_j w_j (z_j I - C)^{-1} V for m <= mmax
// columns (Y must not overlap V).
gevp_status lu_nopiv(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* DinvL, zd* DinvU,
                     int64_t ldi, int* info_dev);
gevp_status trsm_left_upper_n(gevp_ctx* c, int64_t n, int64_t m, const zd* U, int64_t ldu,
                              const zd* DinvU, int64_t ldi, zd* R, int64_t ldr);
size_t contour_work_bytes(int64_t n, int64_t mmax, int nq);
gevp_status contour_factor(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, double a, double b,
                           int nq, void* work, int64_t mmax, int* pivot);
gevp_status contour_apply(gevp_ctx* c, int64_t n, int64_t m, const zd* V, int64_t ldv, zd* Y,
                          int64_t ldy, double a, double b, int nq, void* work, int64_t mmax);
// FP32 form (residual correction): contour_factor32 factors the nq shifted
// matrices in complex64 into `work` (contour32_work_bytes); contour_residual
// forms R(:, j) = W(:, perm[j]) - theta[perm[j]] Qp(:, j) and thp[j] =
// theta[perm[j]] for j in [s0, nb) (Qp: the degree-sorted Ritz vectors);
// contour_apply32 then forms Y = f(theta) Q + sum_j w_j (z_j I - C)^{-1} R
// diag(1 / (z_j - theta)) for m columns, the solves in FP32.
size_t contour32_work_bytes(int64_t n, int64_t mmax, int nq);
gevp_status contour_factor32(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, double a, double b,
                             int nq, void* work, int64_t mmax, int* pivot);
gevp_status contour_residual(gevp_ctx* c, int64_t n, int64_t nb, int64_t s0, const int* perm,
                             const zd* W, int64_t ldw, const double* theta, const zd* Qp, int64_t ldq,
                             zd* R, int64_t ldr, double* thp);
gevp_status contour_apply32(gevp_ctx* c, int64_t n, int64_t m, const zd* Q, int64_t ldq, const zd* R,
                            int64_t ldr, const double* theta, zd* Y, int64_t ldy, double a, double b,
                            int nq, void* work, int64_t mmax);

// Small Hermitian eigensolver (n <= 2048): H (full storage, overwritten),
// theta ascending, Z (n x n) unitary.  work >= heev_work_bytes(n).
size_t heev_work_bytes(int64_t n);
// Eigen-decomposition of the real symmetric tridiagonal T (diagonal d[n],
// off-diagonal e[n-1]): theta ascending by Sturm-count multisection, the
// orthonormal eigenvectors by inverse iteration, Zt[i * n + j] = component i
// of eigenvector j.  work >= tridiag_eig_work_bytes(n).  Asynchronous.
size_t tridiag_eig_work_bytes(int64_t n);
gevp_status tridiag_eig(gevp_ctx* c, int64_t n, const double* d, const double* e, double* theta,
                        double* Zt, void* work);
gevp_status heev_small(gevp_ctx* c, int64_t n, zd* H, int64_t ldh, double* theta, zd* Z,
                       int64_t ldz, void* work);

// elementwise / reduction kernels (vec_kernels.hip)
gevp_status launch_mirror_lower(gevp_ctx* c, int64_t n, const zd* S, int64_t lds, zd* D,
                                int64_t ldd, int* flag_nonfinite);
gevp_status launch_copy2d(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                          zd* D, int64_t ldd);
gevp_status launch_check_finite(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S,
                                int64_t lds, int* flag);
gevp_status launch_randn(gevp_ctx* c, int64_t rows, int64_t cols, zd* V, int64_t ldv,
                         int64_t col_offset, unsigned long long seed);
gevp_status launch_colnorm_scale(gevp_ctx* c, int64_t rows, int64_t cols, zd* V, int64_t ldv);
gevp_status launch_resid_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* W, int64_t ldw,
                              const zd* V, int64_t ldv, const double* theta, double* out);
gevp_status launch_colnorms(gevp_ctx* c, int64_t rows, int64_t cols, const zd* V, int64_t ldv,
                            double* out);
// seed monitor of a k x k cross-overlap M (stat: 3k doubles; out: 6
// doubles).  seed_monitor_stats also solves the angle-minimising matching on
// the device when best matches collide, then copies the results and waits:
// res = sin_rms, dev_mean, dev_max, reindexed, dev_std under that matching,
// match[j] = matched seed column (may be null).  Beyond k = 4096 the
// matching's work arrays need a device scratch of 48 (k + 1) bytes.
// rnorm (device, k, optional): norms of the projection residuals of the seed
// columns onto the result's span; sin_rms then comes from them instead of
// from k - ||M||_F^2.
gevp_status launch_seed_monitor(gevp_ctx* c, int64_t k, const zd* M, int64_t ldm, double* stat,
                                double* out, const double* rnorm = nullptr);
gevp_status seed_monitor_stats(gevp_ctx* c, int64_t k, const zd* M, int64_t ldm, double* stat,
                               double* out, double res[5], int* match,
                               const double* rnorm = nullptr, void* scratch = nullptr,
                               size_t scratch_bytes = 0);
gevp_status launch_gather_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                               const int* perm, zd* D, int64_t ldd);
gevp_status launch_phase_normalize(gevp_ctx* c, int64_t rows, int64_t cols, zd* X, int64_t ldx);
// y = M x for a Hermitian M stored in full (only the tiles on and below the
// diagonal are read); work >= hemv_work_bytes(n) (partial vectors)
size_t hemv_work_bytes(int64_t n);
gevp_status launch_hemv(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, const zd* x, zd* y,
                        void* work);
gevp_status launch_add_diag(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, const double* shift);
gevp_status launch_scale_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                              const double* w, zd* D, int64_t ldd);
gevp_status launch_copy_real(gevp_ctx* c, int64_t n, const double* s, double* d);
// locking helpers (nb <= 2048): theta/resid[j] <- theta/resid[perm[j]] for j < nl;
// stable merge of the ascending runs [0, nl) and [nl, nb) of theta (resid
// follows), order[p] = the index that lands at position p
gevp_status launch_permute_prefix(gevp_ctx* c, double* theta, double* resid, const int* perm,
                                  int64_t nl);
gevp_status launch_merge_runs(gevp_ctx* c, double* theta, double* resid, int64_t nb, int64_t nl,
                              int* order);
// out[0] = max |M - I| over the lower triangle of M (n >= 1); part: scratch
// of MAX_OFFIDENT_PARTS doubles
constexpr int MAX_OFFIDENT_PARTS = 128;
gevp_status launch_max_offident(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, double* out,
                                double* part);

// Lanczos bounds: runs `steps` steps on the Hermitian M (full storage) and
// writes into out[0..5]: theta_min, theta_max, beta_last, upper bound
// (theta_max + beta_last), spectrum-fraction estimate (see lanczos.hip),
// max(|theta_min|, |theta_max|).  frac = wanted fraction for out[4].
gevp_status lanczos_bounds(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, int steps,
                           unsigned long long seed, double frac, double* out, void* work);
size_t lanczos_work_bytes(int64_t n, int steps);

// Controller (single work-group): decides convergence, the next filter
// interval, per-column degrees, the degree-sorted column permutation and the
// filter coefficients.  See solver.hip for the status layout.
struct CtlParams {
  int nb, nev, deg_max, deg_init;
  int mode;         // 0: from Ritz data, 1: cold start, 2: Ritz data, residual-correction filter
  double u_target;  // mode 2: smallest per-sweep residual reduction worth aiming for
  double margin;    // degrees aim at tol / margin (convergence is still tested at tol)
  // mode 2: when every wanted column can reach tol / margin with a reduction
  // of at most 1 / u_reach, the sweep aims there at once, with degrees up to
  // deg_reach (a sweep more than the rounding floor u_target usually allows)
  double u_reach;
  int deg_reach;
};
gevp_status launch_control(gevp_ctx* c, const CtlParams& p, const double* theta,
                           const double* resid, const double* bounds, const double* norms,
                           double tol_rel, int* status_i, double* status_d, int* perm,
                           double* coefs, double* rho0 = nullptr, double* coef2 = nullptr);

// mixed-precision filter pieces (cgemm32.hip)
gevp_status launch_cgemm32_filter(gevp_ctx* c, int64_t m, int64_t n, int64_t k, const void* A,
                                  int64_t lda, const void* G, int64_t ldg, const void* P,
                                  int64_t ldp, const void* R, int64_t ldr, void* D, int64_t ldd,
                                  const double* al, const double* be, const double* ga,
                                  const double* de);
gevp_status launch_to_c32(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                          void* D, int64_t ldd);
gevp_status launch_resid_start32(gevp_ctx* c, int64_t rows, int64_t cols, const zd* W,
                                 const zd* Q, int64_t ld, const double* theta, const int* perm,
                                 const double* rho0, double sc, void* R, void* G1, void* G0,
                                 int64_t ldl);
size_t bf16_planes_bytes(int64_t n);
gevp_status launch_split_rows_bf16(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, void* planes);
gevp_status launch_cgemm_bf16x3_filter(gevp_ctx* c, int64_t m, int64_t n, int64_t k,
                                       const void* planes, const void* G, int64_t ldg,
                                       const void* P, int64_t ldp, const void* R, int64_t ldr,
                                       void* D, int64_t ldd, const double* al, const double* be,
                                       const double* ga, const double* de, void* work);
// workspace of launch_cgemm_bf16x3_filter for a k x k C and up to `cols` columns
size_t bf16_filter_work_bytes(int64_t k, int64_t cols);
gevp_status launch_add_correction32(gevp_ctx* c, int64_t rows, int64_t cols, const zd* Q,
                                    int64_t ldq, const int* perm, const void* G, int64_t ldg,
                                    zd* Y, int64_t ldy);
