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

// Inverse of the lower-triangular n x n (n <= 64) factor held in S[col][row]
// (strict upper part free), by column-parallel forward substitution: a group
// of four lanes owns column c of X = inv(L) and walks rows i = c..n-1,
// x_i = -(sum_{c<=k<i} L(i,k) x_k) / L(i,i); lane q sums the k with
// (k - c) % 4 == q and keeps exactly those x_k (strict part stored
// transposed in S's upper triangle, S[i][c] = X(i,c); diagonal in dg), so
// no lane reads another lane's LDS writes.  Result written to Dinv.
__device__ void lds_inverse_to(zd (*S)[NB], zd* dg, int n, zd* Dinv, int64_t ldi) {
  const int tid = threadIdx.x;
  const int c = tid >> 2, q = tid & 3;
  if (c < n) {
    for (int i = c; i < n; ++i) {
      zd xi;
      if (i == c) {
        const zd d = S[c][c];
        const double dd = d.x * d.x + d.y * d.y;
        xi = make_double2(d.x / dd, -d.y / dd);
      } else {
        double sr = 0.0, si = 0.0;
        for (int k = c + q; k < i; k += 4) {
          const zd l = S[k][i];
          const zd x = (k == c) ? dg[c] : S[k][c];
          sr += l.x * x.x - l.y * x.y;
          si += l.x * x.y + l.y * x.x;
        }
        sr += __shfl_xor(sr, 1, 64);
        si += __shfl_xor(si, 1, 64);
        sr += __shfl_xor(sr, 2, 64);
        si += __shfl_xor(si, 2, 64);
        const zd d = S[i][i];
        const double dd = d.x * d.x + d.y * d.y;
        // xi = -(s) / d
        xi = make_double2(-(sr * d.x + si * d.y) / dd, -(si * d.x - sr * d.y) / dd);
      }
      if (((i - c) & 3) == q) {
        if (i == c) dg[c] = xi; else S[i][c] = xi;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += 256) {
    const int i = e % n, j = e / n;
    zd v = make_double2(0.0, 0.0);
    if (i == j) v = dg[i];
    else if (i > j) v = S[i][j];
    Dinv[i + (int64_t)j * ldi] = v;
  }
}

// Factor the n x n (n <= 64) diagonal block at M (lower triangle read) and
// write L (upper part of the block zeroed) back, then write inv(L) to Dinv.
// Right-looking, one barrier per column: the update of step j reads the
// unscaled column j (scaling by 1/l_jj is folded into the update and applied
// to the stored column at the end).  A non-positive or non-finite pivot is
// recorded in *info (atomic min of the 1-based global index) and replaced by
// 1 so the kernel always finishes.
__global__ __launch_bounds__(256) void k_potrf_block(zd* M, int64_t ldm, int n, zd* Dinv,
                                                     int64_t ldi, int* info, int goff) {
  __shared__ zd S[NB][NB];  // S[col][row]
  __shared__ zd dg[NB];
  __shared__ double piv[NB];
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e & (NB - 1), j = e >> 6;
    zd v = make_double2(0.0, 0.0);
    if (i < n && j < n && i >= j) v = M[i + (int64_t)j * ldm];
    S[j][i] = v;
  }
  __syncthreads();
  const int i = tid & 63, kq = tid >> 6;
  for (int j = 0; j < n; ++j) {
    double d = S[j][j].x;
    const bool badp = !(d > 0.0) || !isfinite(d);
    if (badp) d = 1.0;
    if (badp && tid == 0) atomicMin(info, goff + j + 1);
    const double id = 1.0 / d;  // 1 / l_jj^2
    if (tid == 0) piv[j] = d;
    if (i > j && i < n) {
      const zd ci = S[j][i];
      for (int k = j + 1 + kq; k <= i; k += 4) {
        const zd ck = S[j][k];
        zd s = S[k][i];  // s -= ci conj(ck) / l_jj^2
        s.x -= (ci.x * ck.x + ci.y * ck.y) * id;
        s.y -= (ci.y * ck.x - ci.x * ck.y) * id;
        S[k][i] = s;
      }
    }
    __syncthreads();
  }
  // scale the columns: l_jj = sqrt(d_j), l_ij = s_ij / l_jj
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e & (NB - 1), j = e >> 6;
    if (j < n && r >= j && r < n) {
      const double lj = sqrt(piv[j]);
      if (r == j) S[j][j] = make_double2(lj, 0.0);
      else S[j][r] = make_double2(S[j][r].x / lj, S[j][r].y / lj);
    }
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += 256) {
    const int r = e % n, j = e / n;
    M[r + (int64_t)j * ldm] = (r >= j) ? S[j][r] : make_double2(0.0, 0.0);
  }
  // the strict upper triangle of S is zero; it now receives inv(L)
  __syncthreads();
  lds_inverse_to(S, dg, n, Dinv, ldi);
}

// inverse of the n x n (n <= 64) lower-triangular block at L into Dinv
__global__ __launch_bounds__(256) void k_trtri_block(const zd* L, int64_t ldl, int64_t ntot, zd* Dinv,
                                                     int64_t ldi) {
  __shared__ zd S[NB][NB];
  __shared__ zd dg[NB];
  const int tid = threadIdx.x;
  const int64_t off = (int64_t)blockIdx.x * NB;
  const int n = (int)((ntot - off) < NB ? (ntot - off) : NB);
  const zd* Lb = L + off + off * ldl;
  for (int e = tid; e < NB * NB; e += 256) {
    const int i = e & (NB - 1), j = e >> 6;
    S[j][i] = (i < n && j < n && i >= j) ? Lb[i + (int64_t)j * ldl] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  lds_inverse_to(S, dg, n, Dinv + off, ldi);
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
                        nullptr, 0, nullptr, M22, ldm));
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
