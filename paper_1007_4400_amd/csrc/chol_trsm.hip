// Cholesky factorisation and triangular solves, FP64 complex, recursive.
//
// Every level of the recursion splits the triangle in two halves (rounded to
// the 64-wide block), so the off-diagonal work is one large GEMM on the FP64
// matrix cores per level; only the 64 x 64 diagonal blocks are factored by a
// single work-group in LDS, which also writes the block's inverse.  The
// triangular solves then apply those inverses with GEMMs (base case, in place:
// a 64-wide block fits one output tile of the GEMM, so every tile reads its
// whole K range before it writes) and recurse exactly like the factorisation.
#include <climits>

#include "common.h"

namespace {
constexpr int NB = 64;

// Register-resident 64 x 64 block algorithms.  Thread t owns row i = t % 64
// and the 16 columns c = kq + 4m (kq = t / 64, m = 0..15), so the four waves
// split the columns and a wave reads a broadcast buffer at a uniform index.

__device__ __forceinline__ zd zmul(zd a, zd b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// X = inv(L) for the lower-triangular n x n L held in S[col][row], by
// right-looking forward substitution on L X = I: row k of X is finished at
// step k and broadcast through a double-buffered row buffer (one barrier per
// step).  X is written to Dinv (zeros above the diagonal).
__device__ void reg_inverse_to(zd (*S)[NB], zd (*xrow)[NB], int n, zd* Dinv, int64_t ldi) {
  const int tid = threadIdx.x, i = tid & 63, kq = tid >> 6;
  zd b[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) b[m] = make_double2((kq + 4 * m == i) ? 1.0 : 0.0, 0.0);
  for (int k = 0; k < n; ++k) {
    zd* xr = xrow[k & 1];
    if (i == k) {
      const zd lkk = S[k][k];
      const double dd = lkk.x * lkk.x + lkk.y * lkk.y;
      const zd r = make_double2(lkk.x / dd, -lkk.y / dd);  // 1 / l_kk
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        b[m] = zmul(b[m], r);
        xr[kq + 4 * m] = b[m];
      }
    }
    __syncthreads();
    // rows i > k subtract l_ik * x_k; every load is unconditional (valid
    // addresses) and a 0/1 factor masks the update, so no branch splits the
    // batch of LDS reads
    const double fk = (i > k && i < n) ? 1.0 : 0.0;
    zd lik = S[k][i];
    lik.x *= fk;
    lik.y *= fk;
    zd xv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) xv[m] = xr[kq + 4 * m];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const zd t = zmul(lik, xv[m]);
      b[m].x -= t.x;
      b[m].y -= t.y;
    }
  }
  if (i < n) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int c = kq + 4 * m;
      if (c < n) Dinv[i + (int64_t)c * ldi] = (c <= i) ? b[m] : make_double2(0.0, 0.0);
    }
  }
}

// Factor the n x n (n <= 64) diagonal block at M (lower triangle read), write
// L back (upper part of the block zeroed) and inv(L) to Dinv.  Right-looking
// in registers: column j (current values) is broadcast through a
// double-buffered column buffer, one barrier per column; the 1/l_jj scaling is
// folded into the updates and applied at the end.  A non-positive or
// non-finite pivot is recorded in *info (atomic min of the 1-based global
// index) and replaced by 1 so the kernel always finishes.
__global__ __launch_bounds__(256) void k_potrf_block(zd* M, int64_t ldm, int n, zd* Dinv,
                                                     int64_t ldi, int* info, int goff) {
  __shared__ zd S[NB][NB];  // S[col][row]: the factor, for the inverse
  __shared__ zd cb[2][NB];
  __shared__ double piv[NB];
  const int tid = threadIdx.x, i = tid & 63, kq = tid >> 6;
  zd a[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = kq + 4 * m;
    a[m] = (i < n && c < n && i >= c) ? M[i + (int64_t)c * ldm] : make_double2(0.0, 0.0);
  }
  for (int j = 0; j < n; ++j) {
    if (kq == (j & 3)) {
      // a[j / 4] without a dynamic register index (keeps a[] out of scratch)
      zd v = a[0];
#pragma unroll
      for (int m = 1; m < 16; ++m)
        if (m == (j >> 2)) v = a[m];
      cb[j & 1][i] = v;
    }
    __syncthreads();
    double d = cb[j & 1][j].x;
    const bool badp = !(d > 0.0) || !isfinite(d);
    if (badp) d = 1.0;
    if (tid == 0) {
      piv[j] = d;
      if (badp) atomicMin(info, goff + j + 1);
    }
    const double id = 1.0 / d;  // 1 / l_jj^2
    // a_ic -= a_ij conj(a_cj) / l_jj^2 for j < c <= i; unconditional loads,
    // a 0/1 factor masks the update (no branch between the LDS reads)
    const zd ci = cb[j & 1][i];
    const double fi = (i > j && i < n) ? id : 0.0;
    const zd cs = make_double2(ci.x * fi, ci.y * fi);
    zd ck[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) ck[m] = cb[j & 1][kq + 4 * m];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int c = kq + 4 * m;
      const double f = (c > j && c <= i) ? 1.0 : 0.0;
      const double sr = cs.x * ck[m].x + cs.y * ck[m].y, si = cs.y * ck[m].x - cs.x * ck[m].y;
      a[m].x -= f * sr;
      a[m].y -= f * si;
    }
  }
  __syncthreads();
  // scale and write L; keep it in S for the inverse
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = kq + 4 * m;
    zd v = make_double2(0.0, 0.0);
    if (i < n && c < n && i >= c) {
      const double lc = sqrt(piv[c]);
      v = (i == c) ? make_double2(lc, 0.0) : make_double2(a[m].x / lc, a[m].y / lc);
    }
    S[c][i] = v;
    if (i < n && c < n) M[i + (int64_t)c * ldm] = v;
  }
  __syncthreads();
  reg_inverse_to(S, cb, n, Dinv, ldi);
}

// inverse of the n x n (n <= 64) lower-triangular block at L into Dinv
__global__ __launch_bounds__(256) void k_trtri_block(const zd* L, int64_t ldl, int64_t ntot, zd* Dinv,
                                                     int64_t ldi) {
  __shared__ zd S[NB][NB];
  __shared__ zd xr[2][NB];
  const int tid = threadIdx.x;
  const int64_t off = (int64_t)blockIdx.x * NB;
  const int n = (int)((ntot - off) < NB ? (ntot - off) : NB);
  const zd* Lb = L + off + off * ldl;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e & (NB - 1), j = e >> 6;
    S[j][i] = (i < n && j < n && i >= j) ? Lb[i + (int64_t)j * ldl] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  reg_inverse_to(S, xr, n, Dinv + off, ldi);
}

__global__ void k_zero_upper(zd* M, int64_t ldm, int64_t n) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < j && i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    M[i + j * ldm] = make_double2(0.0, 0.0);
}

inline int64_t split64(int64_t n) { return ((n / 2 + NB - 1) / NB) * NB; }

gevp_status chol_rec(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* Dinv, int64_t ldi,
                     int* info, int64_t goff) {
  if (n <= NB) {
    hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), 0, c->stream, M, ldm, (int)n, Dinv,
                       ldi, info, (int)goff);
    GEVP_HIP_TRY(hipGetLastError());
    return GEVP_OK;
  }
  const int64_t h = split64(n);
  GEVP_TRY(chol_rec(c, h, M, ldm, Dinv, ldi, info, goff));
  zd* M21 = M + h;
  GEVP_TRY(trsm_right_lower_c(c, h, n - h, M, ldm, Dinv, ldi, M21, ldm));
  zd* M22 = M + h + h * ldm;
  GEVP_TRY(launch_zgemm(c, 0, 1, n - h, n - h, h, -1.0, M21, ldm, M21, ldm, 1.0, M22, ldm, 0.0,
                        nullptr, 0, nullptr, M22, ldm, nullptr, 1));
  return chol_rec(c, n - h, M22, ldm, Dinv + h, ldi, info, goff + h);
}
}  // namespace

gevp_status chol_lower(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* Dinv, int64_t ldi,
                       int* info_dev) {
  GEVP_TRY(chol_rec(c, n, M, ldm, Dinv, ldi, info_dev, 0));
  if (n > 1) {
    dim3 g((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), (unsigned)n);
    hipLaunchKernelGGL(k_zero_upper, g, dim3(256), 0, c->stream, M, ldm, n);
    GEVP_HIP_TRY(hipGetLastError());
  }
  return GEVP_OK;
}

gevp_status diag_block_inverses(gevp_ctx* c, int64_t n, const zd* L, int64_t ldl, zd* Dinv,
                                int64_t ldi) {
  if (n <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_trtri_block, dim3((unsigned)((n + NB - 1) / NB)), dim3(256), 0, c->stream, L,
                     ldl, n, Dinv, ldi);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

// R (n x m) <- L^{-1} R
gevp_status trsm_left_lower_n(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                              const zd* Dinv, int64_t ldi, zd* R, int64_t ldr) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB)
    return launch_zgemm(c, 0, 0, n, m, n, 1.0, Dinv, ldi, R, ldr, 0.0, nullptr, 0, 0.0, nullptr,
                        0, nullptr, R, ldr);
  const int64_t h = split64(n);
  GEVP_TRY(trsm_left_lower_n(c, h, m, L, ldl, Dinv, ldi, R, ldr));
  GEVP_TRY(launch_zgemm(c, 0, 0, n - h, m, h, -1.0, L + h, ldl, R, ldr, 1.0, R + h, ldr, 0.0,
                        nullptr, 0, nullptr, R + h, ldr));
  return trsm_left_lower_n(c, n - h, m, L + h + h * ldl, ldl, Dinv + h, ldi, R + h, ldr);
}

// R (n x m) <- L^{-H} R
gevp_status trsm_left_lower_c(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                              const zd* Dinv, int64_t ldi, zd* R, int64_t ldr) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB)
    return launch_zgemm(c, 1, 0, n, m, n, 1.0, Dinv, ldi, R, ldr, 0.0, nullptr, 0, 0.0, nullptr,
                        0, nullptr, R, ldr);
  const int64_t h = split64(n);
  GEVP_TRY(trsm_left_lower_c(c, n - h, m, L + h + h * ldl, ldl, Dinv + h, ldi, R + h, ldr));
  // R1 -= L21^H R2   (L21 is (n-h) x h)
  GEVP_TRY(launch_zgemm(c, 1, 0, h, m, n - h, -1.0, L + h, ldl, R + h, ldr, 1.0, R, ldr, 0.0,
                        nullptr, 0, nullptr, R, ldr));
  return trsm_left_lower_c(c, h, m, L, ldl, Dinv, ldi, R, ldr);
}

// R (m x n) <- R L^{-H}
gevp_status trsm_right_lower_c(gevp_ctx* c, int64_t n, int64_t m, const zd* L, int64_t ldl,
                               const zd* Dinv, int64_t ldi, zd* R, int64_t ldr) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB)
    return launch_zgemm(c, 0, 1, m, n, n, 1.0, R, ldr, Dinv, ldi, 0.0, nullptr, 0, 0.0, nullptr,
                        0, nullptr, R, ldr);
  const int64_t h = split64(n);
  GEVP_TRY(trsm_right_lower_c(c, h, m, L, ldl, Dinv, ldi, R, ldr));
  // R2 -= R1 L21^H   (R1 = R[:, :h], L21 is (n-h) x h)
  GEVP_TRY(launch_zgemm(c, 0, 1, m, n - h, h, -1.0, R, ldr, L + h, ldl, 1.0, R + h * ldr, ldr,
                        0.0, nullptr, 0, nullptr, R + h * ldr, ldr));
  return trsm_right_lower_c(c, n - h, m, L + h + h * ldl, ldl, Dinv + h, ldi, R + h * ldr, ldr);
}

namespace {
// rows [c0, n) of columns [c0, c0 + nn) of R <- R L^{-H}
gevp_status trsm_rlc_lower_rec(gevp_ctx* c, int64_t n, int64_t c0, int64_t nn, const zd* L,
                               int64_t ldl, const zd* Dinv, int64_t ldi, zd* R, int64_t ldr) {
  const zd* Lb = L + c0 + c0 * ldl;
  zd* Rb = R + c0 + c0 * ldr;
  const int64_t rows = n - c0;
  if (nn <= NB)
    return launch_zgemm(c, 0, 1, rows, nn, nn, 1.0, Rb, ldr, Dinv + c0, ldi, 0.0, nullptr, 0, 0.0,
                        nullptr, 0, nullptr, Rb, ldr);
  const int64_t h = split64(nn);
  GEVP_TRY(trsm_rlc_lower_rec(c, n, c0, h, L, ldl, Dinv, ldi, R, ldr));
  // R[c0+h:, c0+h : c0+nn] -= R[c0+h:, c0 : c0+h] L21^H,  L21 = L[c0+h : c0+nn, c0 : c0+h]
  GEVP_TRY(launch_zgemm(c, 0, 1, n - c0 - h, nn - h, h, -1.0, Rb + h, ldr, Lb + h, ldl, 1.0,
                        Rb + h + h * ldr, ldr, 0.0, nullptr, 0, nullptr, Rb + h + h * ldr, ldr));
  return trsm_rlc_lower_rec(c, n, c0 + h, nn - h, L, ldl, Dinv, ldi, R, ldr);
}
}  // namespace

gevp_status trsm_right_lower_c_lowerpart(gevp_ctx* c, int64_t n, const zd* L, int64_t ldl,
                                         const zd* Dinv, int64_t ldi, zd* R, int64_t ldr) {
  if (n <= 0) return GEVP_OK;
  return trsm_rlc_lower_rec(c, n, 0, n, L, ldl, Dinv, ldi, R, ldr);
}
