// Contour-integral filter (Sakurai-Sugiura), FP64 complex.
//
// The paper names a Sakurai-Sugiura eigensolver as a candidate for the fast
// iterations (section 3) without details; this is the published method's
// first moment with Rayleigh-Ritz extraction: for the reduced C = L^{-1} A L^{-H}
// and a circle through a < b on the real axis, the spectral projector onto
// the eigenvalues inside is approximated by the trapezoidal rule
//     Y = sum_j w_j (z_j I - C)^{-1} V,
//     z_j = gamma + rho e^{i t_j},  w_j = rho e^{i t_j} / nq,  t_j = 2 pi (j + 1/2) / nq,
// which acts on an eigenvector with eigenvalue lambda as 1 / (1 + t^nq),
// t = (lambda - gamma) / rho.
//
// Each shifted matrix M_j = z_j I - C is factored once, M_j = L_j U_j, without
// row exchanges: -i M_j has Hermitian part Im(z_j) I, positive definite, so
// every leading block is nonsingular and the growth stays bounded.  The
// factorisation is right-looking by 256-wide panels: inside a panel one
// work-group factors each 64 x 64 diagonal block in registers and writes the
// inverses of its two triangles, the block's column and row pieces are
// products with those inverses, and the trailing matrix gets one FP64
// matrix-core GEMM per panel (K = 256).  The nq factorisations are
// independent and run on four streams (the caller's and three more), so one
// factorisation's latency-bound diagonal blocks overlap another's GEMMs.
// Applying the filter is two triangular solves per node (the existing
// recursive lower solve with the unit-lower block inverses, and an upper solve
// written here), accumulated with the complex weights into one partial sum per
// stream.
#include <cmath>
#include <vector>

#include "common.h"

namespace {
constexpr int NB = 64;
constexpr int QSTREAMS = 4;
constexpr int64_t GRID_Y_MAX = 65535;  // column kernels put the column index in grid.y
constexpr int CGS = 16;       // column groups of the block LU (one per wave)
constexpr int EPT = NB / CGS; // entries per thread

typedef float2 zf;

// complex element types of the factorisation: FP64 (zd) and FP32 (zf)
template <class T> struct Cx;
template <> struct Cx<zd> {
  typedef double R;
  static __device__ __forceinline__ zd mk(double re, double im) { return make_double2(re, im); }
};
template <> struct Cx<zf> {
  typedef float R;
  static __device__ __forceinline__ zf mk(float re, float im) { return make_float2(re, im); }
};

template <class T>
__device__ __forceinline__ T zmul(T a, T b) {
  return Cx<T>::mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class T>
__device__ __forceinline__ T zsub(T a, T b) {
  return Cx<T>::mk(a.x - b.x, a.y - b.y);
}

// One 64 x 64 diagonal block (kb <= 64 rows and columns in use, the rest
// padded with the identity): M = L U in place without row exchanges (L unit
// lower, stored strictly below the diagonal), then inv(L) into DinvL and
// inv(U) into DinvU (64 x 64 each, leading dimension ldi).  1024 threads:
// thread t holds row i = t % 64 at columns c = t / 64 + 16 m (m = 0..3) in
// registers, four waves per SIMD, so the latency of one wave's dependent FP64
// chain is hidden by the others (a quarter of the threads measured 4x slower:
// latency-bound with one wave per SIMD).  Step
// k reads the pivot row and column k from double-buffered LDS (one barrier
// per step); the next step's row and column are published from inside the
// unrolled update loop under a per-element test, so every register index is a
// constant.  *info receives goff + the first failing pivot (1-based).
template <class T>
__global__ __launch_bounds__(1024) void k_getrf_block(T* M, int64_t ldm, int kb, T* DinvL, T* DinvU,
                                                     int64_t ldi, int* info, int goff) {
  typedef typename Cx<T>::R R;
  __shared__ T rowb[2][NB], colb[2][NB], rpiv[2];
  __shared__ T rowl[2][NB], coll[2][NB], rowu[2][NB], colu[2][NB];
  __shared__ T dinv[NB];
  // the column group is uniform over a wave: column tests become scalar branches
  const int tid = threadIdx.x, i = tid & 63, cg = __builtin_amdgcn_readfirstlane(tid >> 6);
  T a[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int j = cg + CGS * m;
    a[m] = (i < kb && j < kb) ? M[i + (int64_t)j * ldm] : Cx<T>::mk(i == j ? R(1) : R(0), R(0));
    if (i == 0) rowb[0][j] = a[m];
    if (j == 0) colb[0][i] = a[m];
    if (i == 0 && j == 0) {
      const R d = a[m].x * a[m].x + a[m].y * a[m].y;
      rpiv[0] = Cx<T>::mk(a[m].x / d, -a[m].y / d);
      if (!(d > R(0)) || !isfinite(d)) atomicMin(info, goff + 1);
    }
  }
  // factorisation; the reciprocal of the next pivot is published with its row
  for (int k = 0; k < NB; ++k) {
    const int b = k & 1, nb = b ^ 1;
    __syncthreads();
    if (i > k) {
      const T l = zmul(colb[b][i], rpiv[b]);
      // all LDS reads first, then a branch-free update (a zero multiplier for
      // columns j <= k), so the reads are not serialised behind branches
      T r[EPT];
#pragma unroll
      for (int m = 0; m < EPT; ++m) r[m] = rowb[b][cg + CGS * m];
      const T zero = Cx<T>::mk(R(0), R(0));
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int j = cg + CGS * m;
        const T lm = (j > k) ? l : zero;
        const T u = zsub(a[m], zmul(lm, r[m]));
        a[m] = (j == k) ? l : u;
      }
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int j = cg + CGS * m;
        if (j == k + 1) {
          colb[nb][i] = a[m];
          if (i == k + 1) {
            const R d = a[m].x * a[m].x + a[m].y * a[m].y;
            rpiv[nb] = Cx<T>::mk(a[m].x / d, -a[m].y / d);
            if (!(d > R(0)) || !isfinite(d)) atomicMin(info, goff + k + 2);
          }
        }
      }
      if (i == k + 1) {
#pragma unroll
        for (int m = 0; m < EPT; ++m) rowb[nb][cg + CGS * m] = a[m];
      }
    }
  }
  // store the factors; diagonal inverses of U for the backward sweep; the
  // first step's operands of the inverse sweeps
  T bl[EPT], bu[EPT];
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int j = cg + CGS * m;
    if (i < kb && j < kb) M[i + (int64_t)j * ldm] = a[m];
    if (j == i) {
      const R d = a[m].x * a[m].x + a[m].y * a[m].y;
      dinv[i] = Cx<T>::mk(a[m].x / d, -a[m].y / d);
    }
    const R e = (j == i) ? R(1) : R(0);
    bl[m] = Cx<T>::mk(e, R(0));
    bu[m] = Cx<T>::mk(e, R(0));
    if (i == 0) rowl[0][j] = bl[m];  // row 0 of inv(L)
    if (j == 0) coll[0][i] = a[m];   // l_i0
    if (j == NB - 1) colu[0][i] = a[m];  // u_i,63
  }
  __syncthreads();
  if (i == NB - 1) {  // row 63 of inv(U)
    const T di = dinv[NB - 1];
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      bu[m] = zmul(bu[m], di);
      rowu[0][cg + CGS * m] = bu[m];
    }
  }
  // inverses: forward sweep for L (unit lower, step k) and backward sweep for
  // U (row ku = 63 - k) together; bl, bu hold rows of the right-hand sides I
  for (int k = 0; k < NB; ++k) {
    const int b = k & 1, nb = b ^ 1, ku = NB - 1 - k;
    __syncthreads();
    {
      // branch-free: rows outside the update range use a zero multiplier
      const T zero = Cx<T>::mk(R(0), R(0));
      const T l = (i > k) ? coll[b][i] : zero;
      const T u = (i < ku) ? colu[b][i] : zero;
      T rl[EPT], ru[EPT];
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        rl[m] = rowl[b][cg + CGS * m];
        ru[m] = rowu[b][cg + CGS * m];
      }
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        bl[m] = zsub(bl[m], zmul(l, rl[m]));
        bu[m] = zsub(bu[m], zmul(u, ru[m]));
      }
    }
    // next step's operands: row k+1 of inv(L) is final now; row ku-1 of
    // inv(U) is final once divided by its pivot
    if (k + 1 < NB) {
      const T di = dinv[ku - 1];
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int j = cg + CGS * m;
        if (i == k + 1) rowl[nb][j] = bl[m];
        if (i == ku - 1) {
          bu[m] = zmul(bu[m], di);
          rowu[nb][j] = bu[m];
        }
        if (j == k + 1) coll[nb][i] = a[m];
        if (j == ku - 1) colu[nb][i] = a[m];
      }
    }
  }
#pragma unroll
  for (int m = 0; m < EPT; ++m) {
    const int j = cg + CGS * m;
    if (i < kb) {
      DinvL[i + (int64_t)j * ldi] = bl[m];
      DinvU[i + (int64_t)j * ldi] = bu[m];
    }
  }
}

// M = z I - C (n x n, both full storage)
__global__ __launch_bounds__(256) void k_shift_neg(int64_t n, const zd* __restrict__ C, int64_t ldc,
                                                   double zr, double zi, zd* __restrict__ M,
                                                   int64_t ldm) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const zd c = C[i + j * ldc];
    M[i + j * ldm] = (i == j) ? make_double2(zr - c.x, zi - c.y) : make_double2(-c.x, -c.y);
  }
}

// Y = w T (first) or Y += w T, complex scalar w, rows x cols
__global__ __launch_bounds__(256) void k_zaxpy_cols(int64_t rows, double wr, double wi,
                                                    const zd* __restrict__ T, int64_t ldt,
                                                    zd* __restrict__ Y, int64_t ldy, int first) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const zd t = T[i + j * ldt];
    const zd v = make_double2(wr * t.x - wi * t.y, wr * t.y + wi * t.x);
    if (first) {
      Y[i + j * ldy] = v;
    } else {
      const zd y = Y[i + j * ldy];
      Y[i + j * ldy] = make_double2(y.x + v.x, y.y + v.y);
    }
  }
}

// Y = S1 + S2 + ... (up to QSTREAMS partial sums, column-major rows x cols)
__global__ __launch_bounds__(256) void k_sum_parts(int64_t rows, int parts, const zd* __restrict__ S,
                                                   int64_t lds, int64_t pstride, zd* __restrict__ Y,
                                                   int64_t ldy) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    zd s = S[i + j * lds];
    for (int p = 1; p < parts; ++p) {
      const zd t = S[p * pstride + i + j * lds];
      s.x += t.x;
      s.y += t.y;
    }
    Y[i + j * ldy] = s;
  }
}

// ---- residual-correction form in FP32.  For a Ritz pair (theta, q) with
// residual r = C q - theta q, (z I - C)^{-1} q = [q + (z I - C)^{-1} r] / (z - theta),
// so sum_j w_j (z_j I - C)^{-1} q = f(theta) q + sum_j w_j (z_j I - C)^{-1} r / (z_j - theta)
// with f(theta) = sum_j w_j / (z_j - theta).  Only the second term goes through
// the FP32 factorisations; its rounding error is relative to |r|, which
// shrinks as the pairs converge.

// M = z I - C in complex64 (C complex128, full storage)
__global__ __launch_bounds__(256) void k_shift_neg32(int64_t n, const zd* __restrict__ C, int64_t ldc,
                                                     double zr, double zi, zf* __restrict__ M,
                                                     int64_t ldm) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const zd c = C[i + j * ldc];
    M[i + j * ldm] = (i == j) ? make_float2((float)(zr - c.x), (float)(zi - c.y))
                              : make_float2((float)-c.x, (float)-c.y);
  }
}

// T(:, j) = R(:, j) / (z - theta_j), rounded to complex64
__global__ __launch_bounds__(256) void k_scale_to32(int64_t rows, const zd* __restrict__ R, int64_t ldr,
                                                    const double* __restrict__ theta, double zr,
                                                    double zi, zf* __restrict__ T, int64_t ldt) {
  const int64_t j = blockIdx.y;
  const double a = zr - theta[j], b = zi;
  const double d = a * a + b * b;
  const double sr = a / d, si = -b / d;  // 1 / (z - theta_j)
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const zd r = R[i + j * ldr];
    T[i + j * ldt] = make_float2((float)(r.x * sr - r.y * si), (float)(r.x * si + r.y * sr));
  }
}

// Acc = w T (first) or Acc += w T; T complex64, Acc complex128
__global__ __launch_bounds__(256) void k_zaxpy32(int64_t rows, double wr, double wi,
                                                 const zf* __restrict__ T, int64_t ldt,
                                                 zd* __restrict__ Acc, int64_t lda, int first) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const zf t = T[i + j * ldt];
    const zd v = make_double2(wr * t.x - wi * t.y, wr * t.y + wi * t.x);
    if (first) {
      Acc[i + j * lda] = v;
    } else {
      const zd y = Acc[i + j * lda];
      Acc[i + j * lda] = make_double2(y.x + v.x, y.y + v.y);
    }
  }
}

// Y(:, j) = f(theta_j) Q(:, j) + sum of the per-stream partial sums,
// f(theta) = sum_q w_q / (z_q - theta) (zw: nq nodes, then nq weights)
__global__ __launch_bounds__(256) void k_contour_combine(int64_t rows, int parts,
                                                         const zd* __restrict__ Q, int64_t ldq,
                                                         const double* __restrict__ theta,
                                                         const zd* __restrict__ zw, int nq,
                                                         const zd* __restrict__ S, int64_t lds,
                                                         int64_t pstride, zd* __restrict__ Y,
                                                         int64_t ldy) {
  const int64_t j = blockIdx.y;
  double fr = 0.0, fi = 0.0;
  for (int q = 0; q < nq; ++q) {
    const zd z = zw[q], w = zw[nq + q];
    const double a = z.x - theta[j], b = z.y, d = a * a + b * b;
    fr += (w.x * a + w.y * b) / d;
    fi += (w.y * a - w.x * b) / d;
  }
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const zd qv = Q[i + j * ldq];
    zd s = make_double2(fr * qv.x - fi * qv.y, fr * qv.y + fi * qv.x);
    for (int p = 0; p < parts; ++p) {
      const zd t = S[p * pstride + i + j * lds];
      s.x += t.x;
      s.y += t.y;
    }
    Y[i + j * ldy] = s;
  }
}

// R(:, j) = W(:, perm[j]) - theta[perm[j]] Qp(:, j) for j in [s0, m); thp[j] = theta[perm[j]]
__global__ __launch_bounds__(256) void k_contour_residual(int64_t rows, int64_t s0, const int* __restrict__ perm,
                                                          const zd* __restrict__ W, int64_t ldw,
                                                          const double* __restrict__ theta,
                                                          const zd* __restrict__ Qp, int64_t ldq,
                                                          zd* __restrict__ R, int64_t ldr,
                                                          double* __restrict__ thp) {
  const int64_t j = s0 + blockIdx.y;
  const int pj = perm[j];
  const double th = theta[pj];
  if (blockIdx.x == 0 && threadIdx.x == 0) thp[j] = th;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256) {
    const zd w = W[i + (int64_t)pj * ldw], q = Qp[i + j * ldq];
    R[i + j * ldr] = make_double2(w.x - th * q.x, w.y - th * q.y);
  }
}

// coefficient columns of the FP32 products: ones, minus ones, zeros (n each)
__global__ void k_fill_coefs(int64_t n, double* co) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    co[i] = 1.0;
    co[n + i] = -1.0;
    co[2 * n + i] = 0.0;
  }
}

inline dim3 grid_cols(int64_t rows, int64_t cols) {
  int64_t gx = (rows + 255) / 256;
  if (gx > 16) gx = 16;
  return dim3((unsigned)gx, (unsigned)cols);
}

inline int64_t split64(int64_t n) { return ((n / 2 + NB - 1) / NB) * NB; }

// quadrature stream i of the handle (created once, non-blocking, default priority)
gevp_status quad_ctx(gevp_ctx* c, int i, gevp_ctx** out) {
  while ((int)c->qctx.size() <= i) {
    gevp_ctx* w = new gevp_ctx();
    w->device = c->device;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return GEVP_ERR_HIP;
    }
    w->owns_stream = true;
    w->inner_streams = false;
    c->qctx.push_back(w);
    ext_assign(c, w, SLOT_QUAD0 + (int)c->qctx.size() - 1);
  }
  *out = c->qctx[i];
  return GEVP_OK;
}

// The nodes run on c's own stream and up to QSTREAMS - 1 further streams
// (c's stream is idle meanwhile; with four hardware queues per process, more
// streams would share queues and serialise).  The further streams start after
// the work queued on c's stream; every exit waits for them (they write
// workspace the next call reuses).
struct QuadStreams {
  gevp_ctx* c;
  int count = 0;
  gevp_ctx* s[QSTREAMS] = {};
  hipEvent_t fork = nullptr, join[QSTREAMS] = {};
  explicit QuadStreams(gevp_ctx* ctx) : c(ctx) {}
  gevp_status open(int want) {
    s[0] = c;
    count = (!c->inner_streams || want <= 1) ? 1 : (want < QSTREAMS ? want : QSTREAMS);
    if (count == 1) return GEVP_OK;
    GEVP_HIP_TRY(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    GEVP_HIP_TRY(hipEventRecord(fork, c->stream));
    for (int q = 1; q < count; ++q) {
      GEVP_TRY(quad_ctx(c, q - 1, &s[q]));
      GEVP_HIP_TRY(hipEventCreateWithFlags(&join[q], hipEventDisableTiming));
      GEVP_HIP_TRY(hipStreamWaitEvent(s[q]->stream, fork, 0));
    }
    return GEVP_OK;
  }
  gevp_status close() {
    for (int q = 1; q < count; ++q) {
      GEVP_HIP_TRY(hipEventRecord(join[q], s[q]->stream));
      GEVP_HIP_TRY(hipStreamWaitEvent(c->stream, join[q], 0));
    }
    return GEVP_OK;
  }
  ~QuadStreams() {
    for (int q = 1; q < count; ++q)
      if (s[q]) (void)hipStreamSynchronize(s[q]->stream);
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
  }
};

struct ContourLayout {
  zd* LU;
  zd* DinvL;
  zd* DinvU;
  zd* T;    // per stream: n x m solve buffer
  zd* Acc;  // per stream: n x m partial sum
  int* info;
  size_t lu_stride, dinv_stride, blk_stride;
};

ContourLayout carve(void* work, int64_t n, int64_t m, int nq) {
  ContourLayout L;
  char* p = (char*)work;
  L.lu_stride = (size_t)n * n;
  L.dinv_stride = (size_t)n * NB;
  L.blk_stride = (size_t)n * m;
  L.LU = (zd*)p;
  p += ws_round(sizeof(zd) * L.lu_stride * nq);
  L.DinvL = (zd*)p;
  p += ws_round(sizeof(zd) * L.dinv_stride * nq);
  L.DinvU = (zd*)p;
  p += ws_round(sizeof(zd) * L.dinv_stride * nq);
  L.T = (zd*)p;
  p += ws_round(sizeof(zd) * L.blk_stride * QSTREAMS);
  L.Acc = (zd*)p;
  p += ws_round(sizeof(zd) * L.blk_stride * QSTREAMS);
  L.info = (int*)p;
  return L;
}

void node(double a, double b, int nq, int j, zd* z, zd* w) {
  const double gamma = 0.5 * (a + b), rho = 0.5 * (b - a);
  const double t = 6.283185307179586476925 * (j + 0.5) / nq;
  const double ct = std::cos(t), st = std::sin(t);
  *z = make_double2(gamma + rho * ct, rho * st);
  *w = make_double2(rho * ct / nq, rho * st / nq);
}

}  // namespace

// ---------------------------------------------------------------------------

gevp_status lu_nopiv(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, zd* DinvL, zd* DinvU,
                     int64_t ldi, int* info_dev) {
  // Panels of PW columns; inside a panel a right-looking LU by 64-wide blocks
  // restricted to the panel's columns; then the panel's row block
  // U12 = L11^{-1} A12 by the recursive lower solve, and one trailing update
  // with K = PW (a K = 64 update per block would re-read and re-write the
  // trailing matrix four times as often: HBM-bound at about 30 TFLOP/s).
  constexpr int64_t PW = 256;
  for (int64_t r0 = 0; r0 < n; r0 += PW) {
    const int64_t kb = std::min<int64_t>(PW, n - r0);
    const int64_t pend = r0 + kb;  // first column after the panel
    for (int64_t s0 = r0; s0 < pend; s0 += NB) {
      const int64_t sb = std::min<int64_t>(NB, pend - s0);
      const int64_t below = n - s0 - sb, pc = pend - s0 - sb;
      zd* Mss = M + s0 + s0 * ldm;
      hipLaunchKernelGGL(k_getrf_block<zd>, dim3(1), dim3(1024), 0, c->stream, Mss, ldm, (int)sb,
                         DinvL + s0, DinvU + s0, ldi, info_dev, (int)s0);
      GEVP_HIP_TRY(hipGetLastError());
      zd* A21 = Mss + sb;
      zd* A12 = Mss + sb * ldm;
      // L21 = A21 U11^{-1} and U12 = L11^{-1} A12 in place (one 64-wide
      // output tile side: every tile reads its whole K range before it writes)
      if (below > 0)
        GEVP_TRY(launch_zgemm(c, 0, 0, below, sb, sb, 1.0, A21, ldm, DinvU + s0, ldi, 0.0, nullptr,
                              0, 0.0, nullptr, 0, nullptr, A21, ldm));
      if (pc > 0) {
        GEVP_TRY(launch_zgemm(c, 0, 0, sb, pc, sb, 1.0, DinvL + s0, ldi, A12, ldm, 0.0, nullptr, 0,
                              0.0, nullptr, 0, nullptr, A12, ldm));
        if (below > 0)
          GEVP_TRY(launch_zgemm(c, 0, 0, below, pc, sb, -1.0, A21, ldm, A12, ldm, 1.0, Mss + sb + sb * ldm,
                                ldm, 0.0, nullptr, 0, nullptr, Mss + sb + sb * ldm, ldm));
      }
    }
    const int64_t rest = n - pend;
    if (rest > 0) {
      zd* Mrr = M + r0 + r0 * ldm;
      zd* A12 = Mrr + kb * ldm;
      GEVP_TRY(trsm_left_lower_n(c, kb, rest, Mrr, ldm, DinvL + r0, ldi, A12, ldm));
      GEVP_TRY(launch_zgemm(c, 0, 0, rest, rest, kb, -1.0, Mrr + kb, ldm, A12, ldm, 1.0,
                            Mrr + kb + kb * ldm, ldm, 0.0, nullptr, 0, nullptr, Mrr + kb + kb * ldm,
                            ldm));
    }
  }
  return GEVP_OK;
}

// R (n x m) <- U^{-1} R, U upper triangular (the upper part of a packed LU)
gevp_status trsm_left_upper_n(gevp_ctx* c, int64_t n, int64_t m, const zd* U, int64_t ldu,
                              const zd* DinvU, int64_t ldi, zd* R, int64_t ldr) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB)
    return launch_zgemm(c, 0, 0, n, m, n, 1.0, DinvU, ldi, R, ldr, 0.0, nullptr, 0, 0.0, nullptr,
                        0, nullptr, R, ldr);
  const int64_t h = split64(n);
  GEVP_TRY(trsm_left_upper_n(c, n - h, m, U + h + h * ldu, ldu, DinvU + h, ldi, R + h, ldr));
  // R1 -= U12 R2   (U12 = U[:h, h:])
  GEVP_TRY(launch_zgemm(c, 0, 0, h, m, n - h, -1.0, U + h * ldu, ldu, R + h, ldr, 1.0, R, ldr, 0.0,
                        nullptr, 0, nullptr, R, ldr));
  return trsm_left_upper_n(c, h, m, U, ldu, DinvU, ldi, R, ldr);
}

// ---- FP32 factorisation and solves (products on the FP32 matrix cores by the
// general form of the complex64 filter kernel: D = alpha A G + gamma P with
// per-column coefficient vectors taken from co = [ones | minus ones | zeros])

namespace {
struct Co32 {
  const double *one, *mone, *zero;
};

// D = alpha A G (+ P when acc): m x n, inner dimension k
gevp_status gemm32(gevp_ctx* c, int64_t m, int64_t n, int64_t k, const zf* A, int64_t lda,
                   const zf* G, int64_t ldg, zf* D, int64_t ldd, bool minus, bool acc, const Co32& co) {
  return launch_cgemm32_filter(c, m, n, k, A, lda, G, ldg, D, ldd, D, ldd, D, ldd,
                               minus ? co.mone : co.one, co.zero, acc ? co.one : co.zero, co.zero);
}

gevp_status trsm32_lower(gevp_ctx* c, int64_t n, int64_t m, const zf* L, int64_t ldl,
                         const zf* Dinv, int64_t ldi, zf* R, int64_t ldr, const Co32& co) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB) return gemm32(c, n, m, n, Dinv, ldi, R, ldr, R, ldr, false, false, co);
  const int64_t h = split64(n);
  GEVP_TRY(trsm32_lower(c, h, m, L, ldl, Dinv, ldi, R, ldr, co));
  GEVP_TRY(gemm32(c, n - h, m, h, L + h, ldl, R, ldr, R + h, ldr, true, true, co));
  return trsm32_lower(c, n - h, m, L + h + h * ldl, ldl, Dinv + h, ldi, R + h, ldr, co);
}

gevp_status trsm32_upper(gevp_ctx* c, int64_t n, int64_t m, const zf* U, int64_t ldu,
                         const zf* Dinv, int64_t ldi, zf* R, int64_t ldr, const Co32& co) {
  if (n <= 0 || m <= 0) return GEVP_OK;
  if (n <= NB) return gemm32(c, n, m, n, Dinv, ldi, R, ldr, R, ldr, false, false, co);
  const int64_t h = split64(n);
  GEVP_TRY(trsm32_upper(c, n - h, m, U + h + h * ldu, ldu, Dinv + h, ldi, R + h, ldr, co));
  GEVP_TRY(gemm32(c, h, m, n - h, U + h * ldu, ldu, R + h, ldr, R, ldr, true, true, co));
  return trsm32_upper(c, h, m, U, ldu, Dinv, ldi, R, ldr, co);
}

// the FP32 counterpart of lu_nopiv (same panels and block kernel)
gevp_status lu_nopiv32(gevp_ctx* c, int64_t n, zf* M, int64_t ldm, zf* DinvL, zf* DinvU, int64_t ldi,
                       int* info_dev, const Co32& co) {
  constexpr int64_t PW = 256;
  for (int64_t r0 = 0; r0 < n; r0 += PW) {
    const int64_t kb = std::min<int64_t>(PW, n - r0);
    const int64_t pend = r0 + kb;
    for (int64_t s0 = r0; s0 < pend; s0 += NB) {
      const int64_t sb = std::min<int64_t>(NB, pend - s0);
      const int64_t below = n - s0 - sb, pc = pend - s0 - sb;
      zf* Mss = M + s0 + s0 * ldm;
      hipLaunchKernelGGL(k_getrf_block<zf>, dim3(1), dim3(1024), 0, c->stream, Mss, ldm, (int)sb,
                         DinvL + s0, DinvU + s0, ldi, info_dev, (int)s0);
      GEVP_HIP_TRY(hipGetLastError());
      zf* A21 = Mss + sb;
      zf* A12 = Mss + sb * ldm;
      if (below > 0)
        GEVP_TRY(gemm32(c, below, sb, sb, A21, ldm, DinvU + s0, ldi, A21, ldm, false, false, co));
      if (pc > 0) {
        GEVP_TRY(gemm32(c, sb, pc, sb, DinvL + s0, ldi, A12, ldm, A12, ldm, false, false, co));
        if (below > 0)
          GEVP_TRY(gemm32(c, below, pc, sb, A21, ldm, A12, ldm, Mss + sb + sb * ldm, ldm, true, true,
                          co));
      }
    }
    const int64_t rest = n - pend;
    if (rest > 0) {
      zf* Mrr = M + r0 + r0 * ldm;
      zf* A12 = Mrr + kb * ldm;
      GEVP_TRY(trsm32_lower(c, kb, rest, Mrr, ldm, DinvL + r0, ldi, A12, ldm, co));
      GEVP_TRY(gemm32(c, rest, rest, kb, Mrr + kb, ldm, A12, ldm, Mrr + kb + kb * ldm, ldm, true, true,
                      co));
    }
  }
  return GEVP_OK;
}

struct Contour32Layout {
  zf* LU;
  zf* DinvL;
  zf* DinvU;
  zf* T;    // per stream: n x m complex64 solve buffer
  zd* Acc;  // per stream: n x m complex128 partial sum
  double* co;
  zd* zw;
  int* info;
  size_t lu_stride, dinv_stride, blk_stride;
};

Contour32Layout carve32(void* work, int64_t n, int64_t m, int nq) {
  Contour32Layout L;
  char* p = (char*)work;
  L.lu_stride = (size_t)n * n;
  L.dinv_stride = (size_t)n * NB;
  L.blk_stride = (size_t)n * m;
  L.LU = (zf*)p;
  p += ws_round(sizeof(zf) * L.lu_stride * nq);
  L.DinvL = (zf*)p;
  p += ws_round(sizeof(zf) * L.dinv_stride * nq);
  L.DinvU = (zf*)p;
  p += ws_round(sizeof(zf) * L.dinv_stride * nq);
  L.T = (zf*)p;
  p += ws_round(sizeof(zf) * L.blk_stride * QSTREAMS);
  L.Acc = (zd*)p;
  p += ws_round(sizeof(zd) * L.blk_stride * QSTREAMS);
  L.co = (double*)p;
  p += ws_round(sizeof(double) * 3 * n);
  L.zw = (zd*)p;
  p += ws_round(sizeof(zd) * 2 * nq);
  L.info = (int*)p;
  return L;
}
}  // namespace

size_t contour32_work_bytes(int64_t n, int64_t m, int nq) {
  return ws_round(sizeof(zf) * (size_t)n * n * nq) + 2 * ws_round(sizeof(zf) * (size_t)n * NB * nq) +
         ws_round(sizeof(zf) * (size_t)n * m * QSTREAMS) +
         ws_round(sizeof(zd) * (size_t)n * m * QSTREAMS) + ws_round(sizeof(double) * 3 * n) +
         ws_round(sizeof(zd) * 2 * nq) + ws_round(sizeof(int) * 4) + 256;
}

gevp_status contour_factor32(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, double a, double b,
                             int nq, void* work, int64_t mmax, int* pivot) {
  Contour32Layout L = carve32(work, n, mmax, nq);
  const Co32 co{L.co, L.co + n, L.co + 2 * n};
  hipLaunchKernelGGL(k_fill_coefs, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 64)), dim3(256), 0,
                     c->stream, n, L.co);
  GEVP_HIP_TRY(hipGetLastError());
  const int big = 0x7fffffff;
  GEVP_HIP_TRY(hipMemcpyAsync(L.info, &big, sizeof(int), hipMemcpyHostToDevice, c->stream));
  QuadStreams qs(c);
  GEVP_TRY(qs.open(nq));
  for (int j = 0; j < nq; ++j) {
    gevp_ctx* s = qs.s[j % qs.count];
    zd z, w;
    node(a, b, nq, j, &z, &w);
    zf* M = L.LU + L.lu_stride * j;
    hipLaunchKernelGGL(k_shift_neg32, dim3((unsigned)((n + 255) / 256 < 16 ? (n + 255) / 256 : 16),
                                           (unsigned)n),
                       dim3(256), 0, s->stream, n, C, ldc, z.x, z.y, M, n);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_TRY(lu_nopiv32(s, n, M, n, L.DinvL + L.dinv_stride * j, L.DinvU + L.dinv_stride * j, n,
                        L.info, co));
  }
  GEVP_TRY(qs.close());
  int f = big;
  GEVP_HIP_TRY(hipMemcpyAsync(&f, L.info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
  *pivot = (f == big) ? 0 : f;
  return GEVP_OK;
}

gevp_status contour_apply32(gevp_ctx* c, int64_t n, int64_t m, const zd* Q, int64_t ldq, const zd* R,
                            int64_t ldr, const double* theta, zd* Y, int64_t ldy, double a, double b,
                            int nq, void* work, int64_t mmax) {
  if (m <= 0) return GEVP_OK;
  Contour32Layout L = carve32(work, n, mmax, nq);
  const Co32 co{L.co, L.co + n, L.co + 2 * n};
  std::vector<zd> zw(2 * nq);
  for (int j = 0; j < nq; ++j) node(a, b, nq, j, &zw[j], &zw[nq + j]);
  GEVP_HIP_TRY(hipMemcpyAsync(L.zw, zw.data(), sizeof(zd) * 2 * nq, hipMemcpyHostToDevice, c->stream));
  QuadStreams qs(c);
  GEVP_TRY(qs.open(nq));
  std::vector<int> firsts(qs.count, 1);
  for (int j = 0; j < nq; ++j) {
    const int q = j % qs.count;
    gevp_ctx* s = qs.s[q];
    const zd z = zw[j], w = zw[nq + j];
    zf* T = L.T + L.blk_stride * q;
    zd* Acc = L.Acc + L.blk_stride * q;
    const zf* LU = L.LU + L.lu_stride * j;
    hipLaunchKernelGGL(k_scale_to32, grid_cols(n, m), dim3(256), 0, s->stream, n, R, ldr, theta, z.x, z.y,
                       T, n);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_TRY(trsm32_lower(s, n, m, LU, n, L.DinvL + L.dinv_stride * j, n, T, n, co));
    GEVP_TRY(trsm32_upper(s, n, m, LU, n, L.DinvU + L.dinv_stride * j, n, T, n, co));
    hipLaunchKernelGGL(k_zaxpy32, grid_cols(n, m), dim3(256), 0, s->stream, n, w.x, w.y, T, n, Acc, n,
                       firsts[q]);
    GEVP_HIP_TRY(hipGetLastError());
    firsts[q] = 0;
  }
  GEVP_TRY(qs.close());
  hipLaunchKernelGGL(k_contour_combine, grid_cols(n, m), dim3(256), 0, c->stream, n, qs.count, Q, ldq,
                     theta, L.zw, nq, L.Acc, n, (int64_t)L.blk_stride, Y, ldy);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status contour_residual(gevp_ctx* c, int64_t n, int64_t nb, int64_t s0, const int* perm,
                             const zd* W, int64_t ldw, const double* theta, const zd* Qp, int64_t ldq,
                             zd* R, int64_t ldr, double* thp) {
  if (s0 >= nb) return GEVP_OK;
  hipLaunchKernelGGL(k_contour_residual, grid_cols(n, nb - s0), dim3(256), 0, c->stream, n, s0, perm, W,
                     ldw, theta, Qp, ldq, R, ldr, thp);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

size_t contour_work_bytes(int64_t n, int64_t m, int nq) {
  return ws_round(sizeof(zd) * (size_t)n * n * nq) + 2 * ws_round(sizeof(zd) * (size_t)n * NB * nq) +
         2 * ws_round(sizeof(zd) * (size_t)n * m * QSTREAMS) + ws_round(sizeof(int) * 4) + 256;
}

gevp_status contour_factor(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, double a, double b,
                           int nq, void* work, int64_t mmax, int* pivot) {
  ContourLayout L = carve(work, n, mmax, nq);
  const int big = 0x7fffffff;
  GEVP_HIP_TRY(hipMemcpyAsync(L.info, &big, sizeof(int), hipMemcpyHostToDevice, c->stream));
  QuadStreams qs(c);
  GEVP_TRY(qs.open(nq));
  for (int j = 0; j < nq; ++j) {
    gevp_ctx* s = qs.s[j % qs.count];
    zd z, w;
    node(a, b, nq, j, &z, &w);
    zd* M = L.LU + L.lu_stride * j;
    hipLaunchKernelGGL(k_shift_neg, dim3((unsigned)((n + 255) / 256 < 16 ? (n + 255) / 256 : 16),
                                         (unsigned)n),
                       dim3(256), 0, s->stream, n, C, ldc, z.x, z.y, M, n);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_TRY(lu_nopiv(s, n, M, n, L.DinvL + L.dinv_stride * j, L.DinvU + L.dinv_stride * j, n,
                      L.info));
  }
  GEVP_TRY(qs.close());
  int f = big;
  GEVP_HIP_TRY(hipMemcpyAsync(&f, L.info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
  *pivot = (f == big) ? 0 : f;
  return GEVP_OK;
}

gevp_status contour_apply(gevp_ctx* c, int64_t n, int64_t m, const zd* V, int64_t ldv, zd* Y,
                          int64_t ldy, double a, double b, int nq, void* work, int64_t mmax) {
  if (m <= 0) return GEVP_OK;
  ContourLayout L = carve(work, n, mmax, nq);
  QuadStreams qs(c);
  GEVP_TRY(qs.open(nq));
  std::vector<int> firsts(qs.count, 1);
  for (int j = 0; j < nq; ++j) {
    const int q = j % qs.count;
    gevp_ctx* s = qs.s[q];
    zd z, w;
    node(a, b, nq, j, &z, &w);
    zd* T = L.T + L.blk_stride * q;
    zd* Acc = L.Acc + L.blk_stride * q;
    const zd* LU = L.LU + L.lu_stride * j;
    GEVP_TRY(launch_copy2d(s, n, m, V, ldv, T, n));
    GEVP_TRY(trsm_left_lower_n(s, n, m, LU, n, L.DinvL + L.dinv_stride * j, n, T, n));
    GEVP_TRY(trsm_left_upper_n(s, n, m, LU, n, L.DinvU + L.dinv_stride * j, n, T, n));
    hipLaunchKernelGGL(k_zaxpy_cols, grid_cols(n, m), dim3(256), 0, s->stream, n, w.x, w.y, T, n,
                       Acc, n, firsts[q]);
    GEVP_HIP_TRY(hipGetLastError());
    firsts[q] = 0;
  }
  GEVP_TRY(qs.close());
  hipLaunchKernelGGL(k_sum_parts, grid_cols(n, m), dim3(256), 0, c->stream, n, qs.count, L.Acc, n,
                     (int64_t)L.blk_stride, Y, ldy);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

extern "C" {

gevp_status gevp_k_lu_shifted(gevp_handle h, int64_t n, const void* C, int64_t ldc, double zr,
                              double zi, void* LU, int64_t ldlu, int64_t* pivot) {
  if (!h || n < 1 || n > GRID_Y_MAX || !C || ldc < n || !LU || ldlu < n || !std::isfinite(zr) ||
      !std::isfinite(zi))
    return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_TRY(ws_reserve(h, 2 * ws_round(sizeof(zd) * n * NB) + ws_round(sizeof(int) * 4) + 256));
  zd* DL = (zd*)ws_take(h, sizeof(zd) * n * NB);
  zd* DU = (zd*)ws_take(h, sizeof(zd) * n * NB);
  int* info = (int*)ws_take(h, sizeof(int) * 4);
  const int big = 0x7fffffff;
  GEVP_HIP_TRY(hipMemcpyAsync(info, &big, sizeof(int), hipMemcpyHostToDevice, h->stream));
  hipLaunchKernelGGL(k_shift_neg, dim3((unsigned)((n + 255) / 256 < 16 ? (n + 255) / 256 : 16),
                                       (unsigned)n),
                     dim3(256), 0, h->stream, n, (const zd*)C, ldc, zr, zi, (zd*)LU, ldlu);
  GEVP_HIP_TRY(hipGetLastError());
  GEVP_TRY(lu_nopiv(h, n, (zd*)LU, ldlu, DL, DU, n, info));
  int f = big;
  GEVP_HIP_TRY(hipMemcpyAsync(&f, info, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  if (pivot) *pivot = (f == big) ? 0 : f;
  return (f == big) ? GEVP_OK : GEVP_ERR_SINGULAR;
}

gevp_status gevp_k_contour_filter(gevp_handle h, int64_t n, const void* C, int64_t ldc,
                                  const void* V, int64_t ldv, int64_t m, double a, double b, int nq,
                                  void* Y, int64_t ldy) {
  if (!h || n < 1 || n > GRID_Y_MAX || !C || ldc < n || !V || ldv < n || m < 0 ||
      m > GRID_Y_MAX || !Y || ldy < n)
    return GEVP_ERR_INVALID;
  if (!(a < b) || !std::isfinite(a) || !std::isfinite(b) || nq < 1 || nq > 256)
    return GEVP_ERR_INVALID;
  if (m == 0) return GEVP_OK;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  GEVP_TRY(ws_reserve(h, contour_work_bytes(n, m, nq) + 256));
  void* work = ws_take(h, contour_work_bytes(n, m, nq));
  int piv = 0;
  GEVP_TRY(contour_factor(h, n, (const zd*)C, ldc, a, b, nq, work, m, &piv));
  if (piv) return GEVP_ERR_SINGULAR;
  GEVP_TRY(contour_apply(h, n, m, (const zd*)V, ldv, (zd*)Y, ldy, a, b, nq, work, m));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  return GEVP_OK;
}

}  // extern "C"
