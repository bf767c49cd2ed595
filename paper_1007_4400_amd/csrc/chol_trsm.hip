// Cholesky factorisation and triangular solves, FP64 complex.
//
// The factorisation is right-looking in panels of 384 columns with one panel
// of lookahead on a second stream (see chol_lower); each 64 x 64 diagonal
// block is factored and inverted by one work-group in LDS.  The triangular solves
// recurse: every level splits the triangle in two halves (rounded to the
// 64-wide block), so the off-diagonal work is one large GEMM on the FP64
// matrix cores per level, and the base case applies a diagonal block's
// inverse with a GEMM (in place: a 64-wide block fits one output tile of the
// GEMM, so every tile reads its whole K range before it writes).
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
// L back (upper part of the block zeroed) and inv(L) to Dinv.
//
// Blocked right-looking in LDS with 16-wide panels.  Per panel: one wave
// factors the 16 x 16 diagonal block and inverts it (lanes own a row and
// four columns; a wave's LDS accesses are ordered, so no barrier is needed
// inside), then all threads form the panel below as A21 inv(L11)^H and
// update the trailing lower triangle.  inv(L) is then assembled block row by
// block row from the diagonal inverses: X_IJ = -X_II sum_{K=J}^{I-1} L_IK X_KJ.
// Entries past n are the identity, so a ragged block needs no special case.
// A non-positive or non-finite pivot is recorded in *info (atomic min of the
// 1-based global index) and replaced by 1 so the kernel always finishes.
constexpr int PB = 16;       // panel width
constexpr int SLD = NB + 1;  // LDS column stride in complex entries (odd: rows spread over banks)
// L and inv(L) share one array: L in the lower triangle (column-major,
// S[c * SLD + r], r >= c), the strict lower triangle of inv(L) transposed into
// the upper one (X(i, j), i > j, at S[i * SLD + j]), inv(L)'s diagonal in a
// separate vector.  66.5 KB of LDS instead of 133 KB, so the factor fits on a
// compute unit next to one work-group of the trailing-update GEMM (which holds
// 66.5 KB) instead of waiting for a unit with both of its GEMM work-groups
// gone.
constexpr size_t POTRF_LDS = sizeof(zd) * (NB * SLD + NB);

__device__ __forceinline__ zd zmulc(zd a, zd b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

__global__ __launch_bounds__(256) void k_potrf_block(zd* M, int64_t ldm, int n, zd* Dinv,
                                                     int64_t ldi, int* info, int goff) {
  extern __shared__ double potrf_lds[];
  zd* S = reinterpret_cast<zd*>(potrf_lds);  // L, S[c * SLD + r], r >= c
  zd* Xd = S + NB * SLD;                     // diagonal of inv(L)
  // entry (i, j), i >= j, of inv(L)
  auto X = [&](int i, int j) -> zd& { return (i == j) ? Xd[i] : S[i * SLD + j]; };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  {
    // all sixteen loads in flight before the first LDS store
    zd v[NB * NB / 256];
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int e = tid + 256 * q, r = e & (NB - 1), c = e >> 6;
      v[q] = make_double2((r == c && (r >= n || c >= n)) ? 1.0 : 0.0, 0.0);
      if (r < n && c < n && r >= c) v[q] = M[r + (int64_t)c * ldm];
    }
#pragma unroll
    for (int q = 0; q < NB * NB / 256; ++q) {
      const int e = tid + 256 * q, r = e & (NB - 1), c = e >> 6;
      S[c * SLD + r] = v[q];  // zeros above the diagonal: inv(L)'s entries go there later
    }
  }
  __syncthreads();
  for (int p0 = 0; p0 < NB; p0 += PB) {
    if (wave == 0) {
      // lane: row r of the diagonal block, columns cg + 4m (m = 0..3)
      const int r = lane & 15, cg = lane >> 4;
      for (int j = 0; j < PB; ++j) {
        const int gj = p0 + j;
        zd* colj = S + gj * SLD + p0;
        double d = colj[j].x;
        const bool bad = !(d > 0.0) || !isfinite(d);
        if (bad) d = 1.0;
        if (lane == 0 && bad && gj < n) atomicMin(info, goff + gj + 1);
        const double ljj = sqrt(d), il = 1.0 / ljj;
        if (cg == (j & 3)) {
          if (r == j) {
            colj[r] = make_double2(ljj, 0.0);
          } else if (r > j) {
            const zd v = colj[r];
            colj[r] = make_double2(v.x * il, v.y * il);
          }
        }
        __builtin_amdgcn_wave_barrier();
        const zd lr = colj[r];  // L(r, j)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int c = cg + 4 * m;
          if (c > j && c <= r) {
            const zd t = zmulc(lr, colj[c]);
            zd* a = S + (p0 + c) * SLD + p0 + r;
            const zd v = *a;
            *a = make_double2(v.x - t.x, v.y - t.y);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      // inverse of the diagonal block: right-looking forward substitution on
      // L11 X = I for the lane's four columns
      zd x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = make_double2((cg + 4 * m == r) ? 1.0 : 0.0, 0.0);
      for (int k = 0; k < PB; ++k) {
        zd* colk = S + (p0 + k) * SLD + p0;
        if (r == k) {
          const double il = 1.0 / colk[k].x;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            x[m] = make_double2(x[m].x * il, x[m].y * il);
            if (cg + 4 * m <= k) X(p0 + k, p0 + cg + 4 * m) = x[m];  // row k, lower part
          }
        }
        __builtin_amdgcn_wave_barrier();
        if (r > k) {
          const zd lrk = colk[r];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const zd xk = (cg + 4 * m <= k) ? X(p0 + k, p0 + cg + 4 * m) : make_double2(0.0, 0.0);
            const zd t = make_double2(lrk.x * xk.x - lrk.y * xk.y, lrk.x * xk.y + lrk.y * xk.x);
            x[m] = make_double2(x[m].x - t.x, x[m].y - t.y);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    const int R = NB - p0 - PB;  // rows below the panel
    if (R > 0) {
      // L21 = A21 inv(L11)^H: entry (row, c) = sum_{k <= c} A21(row, k) conj(X11(c, k))
      zd v[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int e = tid + 256 * q;
        v[q] = make_double2(0.0, 0.0);
        if (e < R * PB) {
          const int row = p0 + PB + e % R, c = e / R;
          for (int k = 0; k <= c; ++k) {
            const zd t = zmulc(S[(p0 + k) * SLD + row], X(p0 + c, p0 + k));
            v[q].x += t.x;
            v[q].y += t.y;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int e = tid + 256 * q;
        if (e < R * PB) S[(p0 + e / R) * SLD + p0 + PB + e % R] = v[q];
      }
      __syncthreads();
      // trailing lower triangle: A22 -= L21 L21^H
      for (int e = tid; e < R * R; e += 256) {
        const int rr = p0 + PB + e % R, cc = p0 + PB + e / R;
        if (rr < cc) continue;
        zd acc = S[cc * SLD + rr];
#pragma unroll 4
        for (int k = 0; k < PB; ++k) {
          const zd t = zmulc(S[(p0 + k) * SLD + rr], S[(p0 + k) * SLD + cc]);
          acc.x -= t.x;
          acc.y -= t.y;
        }
        S[cc * SLD + rr] = acc;
      }
      __syncthreads();
    }
  }
  // off-diagonal blocks of inv(L), block row I = 1..3
  for (int I = 1; I < NB / PB; ++I) {
    // T_IJ = sum_{K=J}^{I-1} L_IK X_KJ, into X's block (I, J)
    zd v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = tid + 256 * q;
      v[q] = make_double2(0.0, 0.0);
      if (e < I * PB * PB) {
        const int J = e >> 8, r = e & 15, c = (e >> 4) & 15;
        const int row = I * PB + r, col = J * PB + c;
        for (int k = J * PB + c; k < I * PB; ++k) {  // X(k, col) = 0 for k < col
          const zd l = S[k * SLD + row], xk = X(k, col);
          v[q].x += l.x * xk.x - l.y * xk.y;
          v[q].y += l.x * xk.y + l.y * xk.x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = tid + 256 * q;
      if (e < I * PB * PB) {
        const int J = e >> 8, r = e & 15, c = (e >> 4) & 15;
        X(I * PB + r, J * PB + c) = v[q];
      }
    }
    __syncthreads();
    // X_IJ = -X_II T_IJ (X_II lower triangular)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = tid + 256 * q;
      v[q] = make_double2(0.0, 0.0);
      if (e < I * PB * PB) {
        const int J = e >> 8, r = e & 15, c = (e >> 4) & 15;
        const int row = I * PB + r, col = J * PB + c;
        for (int k = 0; k <= r; ++k) {
          const zd xi = X(row, I * PB + k), t = X(I * PB + k, col);
          v[q].x -= xi.x * t.x - xi.y * t.y;
          v[q].y -= xi.x * t.y + xi.y * t.x;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int e = tid + 256 * q;
      if (e < I * PB * PB) {
        const int J = e >> 8, r = e & 15, c = (e >> 4) & 15;
        X(I * PB + r, J * PB + c) = v[q];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < NB * NB; e += 256) {
    const int r = e & (NB - 1), c = e >> 6;
    if (r < n && c < n) {
      M[r + (int64_t)c * ldm] = (r >= c) ? S[c * SLD + r] : make_double2(0.0, 0.0);
      Dinv[r + (int64_t)c * ldi] = (r >= c) ? X(r, c) : make_double2(0.0, 0.0);
    }
  }
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

}  // namespace

namespace {
gevp_status panel_ctx(gevp_ctx* c, gevp_ctx** out) {
  if (!c->panel) {
    gevp_ctx* w = new gevp_ctx();
    w->device = c->device;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return GEVP_ERR_HIP;
    }
    w->owns_stream = true;
    c->panel = w;
    ext_assign(c, w, SLOT_PANEL);
  }
  for (hipEvent_t& e : c->pev)
    if (!e) GEVP_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  *out = c->panel;
  return GEVP_OK;
}

gevp_status potrf_leaf(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* Dinv, int64_t ldi, int* info,
                       int64_t goff) {
  static const bool attr = [] {
    (void)hipFuncSetAttribute((const void*)k_potrf_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)POTRF_LDS);
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(256), POTRF_LDS, c->stream, M, ldm, (int)n, Dinv,
                     ldi, info, (int)goff);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
}  // namespace

namespace {
// out (k x m) = in^H, in (m x k): 32 x 32 tiles through LDS, both sides coalesced
__global__ __launch_bounds__(256) void k_copy_ct(const zd* in, int64_t ldin, zd* out, int64_t ldout,
                                                 int64_t m, int64_t k) {
  __shared__ zd t[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;  // tile of `in`: rows bi, columns bj
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + tx, j = bj * 32 + r;
    if (i < m && j < k) t[r][tx] = in[i + j * ldin];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {  // out(j, i) = conj(in(i, j)): j = bj*32 + tx, i = bi*32 + r
    const int64_t j = bj * 32 + tx, i = bi * 32 + r;
    if (i < m && j < k) {
      const zd v = t[tx][r];
      out[j + i * ldout] = make_double2(v.x, -v.y);
    }
  }
}

gevp_status copy_ct(gevp_ctx* c, int64_t m, int64_t k, const zd* in, int64_t ldin, zd* out,
                    int64_t ldout) {
  if (m <= 0 || k <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_copy_ct, dim3((unsigned)((m + 31) / 32), (unsigned)((k + 31) / 32)),
                     dim3(256), 0, c->stream, in, ldin, out, ldout, m, k);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
}  // namespace

// Right-looking blocked Cholesky in 384-wide panels with one panel of
// lookahead.  A panel is factored on the panel stream, 64 columns at a time:
// the diagonal block in LDS (k_potrf_block, which also writes its inverse to
// Dinv), the rows below by an in-place product with that inverse,
// L21 = A21 L11^{-H}, and the panel's remaining columns by a rank-64 update.
// The panel's conjugate transpose is then copied into the upper block row
// (space the factor does not use until it is zeroed at the end), so the
// rank-384 trailing updates multiply both operands as stored.  The main
// stream applies the panel first to the next panel's columns, after which
// the panel stream may factor that panel, then to the rest of the lower
// triangle, which overlaps the factorisation.
gevp_status chol_lower(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* Dinv, int64_t ldi,
                       int* info_dev, hipEvent_t midpoint, zd* R, int64_t ldr, int64_t m) {
  constexpr int64_t PW = 6 * NB;  // measured at n = 8192: 30 ms; 128: 31, 256: 32, 512: 33
  if (n <= 0) {
    if (midpoint) GEVP_HIP_TRY(hipEventRecord(midpoint, c->stream));
    return GEVP_OK;
  }
  const bool rhs = R != nullptr && m > 0;
  if (n <= NB) {
    GEVP_TRY(potrf_leaf(c, n, M, ldm, Dinv, ldi, info_dev, 0));
    if (rhs) GEVP_TRY(trsm_left_lower_n(c, n, m, M, ldm, Dinv, ldi, R, ldr));
    if (midpoint) GEVP_HIP_TRY(hipEventRecord(midpoint, c->stream));
  } else {
    const int64_t half = ((n + NB - 1) / NB / 2) * NB;  // first row of the second half
    bool mid_done = false;
    gevp_ctx* pc = c;  // without inner streams the panels run in order on c's stream
    if (c->inner_streams) {
      GEVP_TRY(panel_ctx(c, &pc));
      pc->profiling = c->profiling & 4;
    }
    const bool two = pc != c;
    hipEvent_t evp = c->pev[0], evn = c->pev[1];
    // the panel stream starts after the work already queued on the main stream
    if (two) {
      GEVP_HIP_TRY(hipEventRecord(evn, c->stream));
      GEVP_HIP_TRY(hipStreamWaitEvent(pc->stream, evn, 0));
    }
    for (int64_t p0 = 0; p0 < n; p0 += PW) {
      const int64_t pw = std::min<int64_t>(PW, n - p0), pend = p0 + pw;
      // factor the panel (columns p0 .. pend-1, all rows below p0)
      for (int64_t r0 = p0; r0 < pend; r0 += NB) {
        const int64_t kb = std::min<int64_t>(NB, pend - r0), below = n - r0 - kb;
        zd* Mkk = M + r0 + r0 * ldm;
        GEVP_TRY(potrf_leaf(pc, kb, Mkk, ldm, Dinv + r0, ldi, info_dev, r0));
        if (below <= 0) continue;
        zd* L21 = Mkk + kb;
        GEVP_TRY(launch_zgemm(pc, 0, 1, below, kb, kb, 1.0, L21, ldm, Dinv + r0, ldi, 0.0, nullptr,
                              0, 0.0, nullptr, 0, nullptr, L21, ldm));
        const int64_t w = pend - r0 - kb;  // panel columns right of this block
        if (w > 0) {
          zd* A2 = M + (r0 + kb) + (r0 + kb) * ldm;
          GEVP_TRY(launch_zgemm(pc, 0, 1, below, w, kb, -1.0, L21, ldm, L21, ldm, 1.0, A2, ldm, 0.0,
                                nullptr, 0, nullptr, A2, ldm));
        }
      }
      const int64_t rest = n - pend;
      const zd* Lp = M + pend + p0 * ldm;  // rest x pw, below the panel's diagonal block
      zd* LpH = M + p0 + pend * ldm;       // pw x rest, the upper block row
      if (rest > 0) GEVP_TRY(copy_ct(pc, rest, pw, Lp, ldm, LpH, ldm));
      if (two) {
        GEVP_HIP_TRY(hipEventRecord(evp, pc->stream));
        GEVP_HIP_TRY(hipStreamWaitEvent(c->stream, evp, 0));
      }
      if (rest > 0) {
        const int64_t pw1 = std::min<int64_t>(PW, rest);
        zd* A2 = M + pend + pend * ldm;
        // next panel's columns: A2(:, :pw1) -= Lp LpH(:, :pw1)
        GEVP_TRY(launch_zgemm(c, 0, 0, rest, pw1, pw, -1.0, Lp, ldm, LpH, ldm, 1.0, A2, ldm, 0.0,
                              nullptr, 0, nullptr, A2, ldm));
        if (two) {
          GEVP_HIP_TRY(hipEventRecord(evn, c->stream));
          GEVP_HIP_TRY(hipStreamWaitEvent(pc->stream, evn, 0));
        }
        const int64_t rest2 = rest - pw1;
        if (rest2 > 0) {  // the rest of the trailing lower triangle
          zd* A3 = A2 + pw1 + pw1 * ldm;
          GEVP_TRY(launch_zgemm(c, 0, 0, rest2, rest2, pw, -1.0, Lp + pw1, ldm, LpH + pw1 * ldm,
                                ldm, 1.0, A3, ldm, 0.0, nullptr, 0, nullptr, A3, ldm, nullptr, 1));
        }
      }
      if (rhs) {
        // block row of the forward substitution: R_p <- L_pp^{-1} R_p (every
        // earlier panel's update of these rows is queued before it on this
        // stream), then the rows below: R_rest -= L_rest,p R_p
        GEVP_TRY(trsm_left_lower_n(c, pw, m, M + p0 + p0 * ldm, ldm, Dinv + p0, ldi, R + p0, ldr));
        if (rest > 0)
          GEVP_TRY(launch_zgemm(c, 0, 0, rest, m, pw, -1.0, Lp, ldm, R + p0, ldr, 1.0, R + pend, ldr,
                                0.0, nullptr, 0, nullptr, R + pend, ldr));
      }
      if (midpoint && !mid_done && pend >= half) {
        GEVP_HIP_TRY(hipEventRecord(midpoint, c->stream));
        mid_done = true;
      }
    }
  }
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
                              const zd* Dinv, int64_t ldi, zd* R, int64_t ldr, int lhu) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB)
    return launch_zgemm(c, 1, 0, n, m, n, 1.0, Dinv, ldi, R, ldr, 0.0, nullptr, 0, 0.0, nullptr,
                        0, nullptr, R, ldr);
  const int64_t h = split64(n);
  GEVP_TRY(trsm_left_lower_c(c, n - h, m, L + h + h * ldl, ldl, Dinv + h, ldi, R + h, ldr, lhu));
  // R1 -= L21^H R2   (L21 is (n-h) x h; with lhu its conjugate transpose is the
  // block above the diagonal, read as stored)
  if (lhu)
    GEVP_TRY(launch_zgemm(c, 0, 0, h, m, n - h, -1.0, L + h * ldl, ldl, R + h, ldr, 1.0, R, ldr,
                          0.0, nullptr, 0, nullptr, R, ldr));
  else
    GEVP_TRY(launch_zgemm(c, 1, 0, h, m, n - h, -1.0, L + h, ldl, R + h, ldr, 1.0, R, ldr, 0.0,
                          nullptr, 0, nullptr, R, ldr));
  return trsm_left_lower_c(c, h, m, L, ldl, Dinv, ldi, R, ldr, lhu);
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
                               int64_t ldl, const zd* Dinv, int64_t ldi, zd* R, int64_t ldr,
                               int lhu) {
  const zd* Lb = L + c0 + c0 * ldl;
  zd* Rb = R + c0 + c0 * ldr;
  const int64_t rows = n - c0;
  if (nn <= NB)
    return launch_zgemm(c, 0, 1, rows, nn, nn, 1.0, Rb, ldr, Dinv + c0, ldi, 0.0, nullptr, 0, 0.0,
                        nullptr, 0, nullptr, Rb, ldr);
  const int64_t h = split64(nn);
  GEVP_TRY(trsm_rlc_lower_rec(c, n, c0, h, L, ldl, Dinv, ldi, R, ldr, lhu));
  // R[c0+h:, c0+h : c0+nn] -= R[c0+h:, c0 : c0+h] L21^H,  L21 = L[c0+h : c0+nn, c0 : c0+h]
  // (with lhu, L21^H = L[c0 : c0+h, c0+h : c0+nn] as stored)
  if (lhu)
    GEVP_TRY(launch_zgemm(c, 0, 0, n - c0 - h, nn - h, h, -1.0, Rb + h, ldr, Lb + h * ldl, ldl,
                          1.0, Rb + h + h * ldr, ldr, 0.0, nullptr, 0, nullptr, Rb + h + h * ldr,
                          ldr));
  else
    GEVP_TRY(launch_zgemm(c, 0, 1, n - c0 - h, nn - h, h, -1.0, Rb + h, ldr, Lb + h, ldl, 1.0,
                          Rb + h + h * ldr, ldr, 0.0, nullptr, 0, nullptr, Rb + h + h * ldr, ldr));
  return trsm_rlc_lower_rec(c, n, c0 + h, nn - h, L, ldl, Dinv, ldi, R, ldr, lhu);
}
}  // namespace

gevp_status trsm_right_lower_c_lowerpart(gevp_ctx* c, int64_t n, const zd* L, int64_t ldl,
                                         const zd* Dinv, int64_t ldi, zd* R, int64_t ldr, int lhu) {
  if (n <= 0) return GEVP_OK;
  return trsm_rlc_lower_rec(c, n, 0, n, L, ldl, Dinv, ldi, R, ldr, lhu);
}
