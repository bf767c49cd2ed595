// Complex128 GEMM on the FP64 matrix cores of gfx950 (v_mfma_f64_16x16x4f64).
//
//   D = alpha op(A) op(B) + beta Cm + gamma diag(gcol) E
//
// op() is identity or conjugate transpose.  The complex product is formed
// from four real products per 16 x 16 block:
//   Re += Ar Br - Ai Bi,   Im += Ar Bi + Ai Br
// on interleaved (re, im) operands, so no planar copy of the inputs exists.
//
// Tiling: a 256-thread work-group owns a 64 x 64 complex output tile; each of
// its four waves owns 32 x 32 (2 x 2 MFMA blocks, 8 accumulators).  K is
// walked in slices of 16 complex values staged through LDS (double buffered,
// with the next slice's global loads in flight during the current slice's
// MFMAs).  Rows of the LDS slices are padded by one element so that the
// transposing stores of the 'C' / column-major operands are conflict-free.
//
// XCD-aware order: the hardware deals work-groups to the 8 XCDs round-robin,
// so consecutive block ids are remapped to consecutive tiles of ONE XCD, with
// the column tiles of a row panel adjacent; a row panel of A (the Hamiltonian
// in the filter) is then reused out of that XCD's L2.
//
// The Chebyshev filter uses the epilogue with Cm = the B operand and E = the
// previous iterate, coefficients read from device memory (`coef`).
#include "common.h"

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64, BN = 64, KT = 16, NTHR = 256;
constexpr int PADA = BM + 1, PADB = BN + 1;
// The in-place base cases of the triangular solves rely on a 64-wide block
// fitting in one output tile.
static_assert(BM >= 64 && BN >= 64, "trsm base cases need 64-wide tiles");

struct ZgemmParams {
  int M, N, K;
  int opA, opB;
  const zd* A;
  int64_t lda;
  const zd* B;
  int64_t ldb;
  const zd* Cm;
  int64_t ldc;
  const zd* E;
  int64_t lde;
  const double* gcol;
  zd* D;
  int64_t ldd;
  double alpha, beta, gamma;
  const double* coef;
  int tiles_n;
  int total;
  int remap;
};

__device__ __forceinline__ zd zconj(zd a) { return make_double2(a.x, -a.y); }

// FILTER only names the kernel differently for the Chebyshev filter launches
// (coefficients from device memory), so profiles separate them.
template <int FILTER>
__global__ __launch_bounds__(NTHR, 2) void k_zgemm(ZgemmParams p) {
  __shared__ zd As[2][KT][PADA];
  __shared__ zd Bs[2][KT][PADB];

  const int tid = threadIdx.x;
  int L = blockIdx.x;
  if (p.remap) {
    const int per = p.total >> 3;
    L = (L & 7) * per + (L >> 3);
  }
  const int tm = L / p.tiles_n, tn = L - tm * p.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;

  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;

  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0, 0, 0, 0};
      accI[i][j] = d4{0, 0, 0, 0};
    }

  zd ra[4], rb[4];
  const zd zero = make_double2(0.0, 0.0);

  auto load = [&](int k0) {
    if (p.opA == 0) {  // A col-major M x K: thread -> (m = tid%64, k = tid/64 + 4i)
      const int m = tid & 63, gm = row0 + m;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + (tid >> 6) + 4 * i;
        ra[i] = (gm < p.M && gk < p.K) ? p.A[gm + (int64_t)gk * p.lda] : zero;
      }
    } else {  // A stored K x M: op(A)(m,k) = conj(A[k + m lda]); k fastest
      const int k = tid & 15, gk = k0 + k;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = row0 + (tid >> 4) + 16 * i;
        ra[i] = (gm < p.M && gk < p.K) ? zconj(p.A[gk + (int64_t)gm * p.lda]) : zero;
      }
    }
    if (p.opB == 0) {  // B col-major K x N: k fastest
      const int k = tid & 15, gk = k0 + k;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gn = col0 + (tid >> 4) + 16 * i;
        rb[i] = (gn < p.N && gk < p.K) ? p.B[gk + (int64_t)gn * p.ldb] : zero;
      }
    } else {  // B stored N x K: op(B)(k,n) = conj(B[n + k ldb]); n fastest
      const int n = tid & 63, gn = col0 + n;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gk = k0 + (tid >> 6) + 4 * i;
        rb[i] = (gn < p.N && gk < p.K) ? zconj(p.B[gn + (int64_t)gk * p.ldb]) : zero;
      }
    }
  };
  auto store = [&](int buf) {
    if (p.opA == 0) {
      const int m = tid & 63;
#pragma unroll
      for (int i = 0; i < 4; ++i) As[buf][(tid >> 6) + 4 * i][m] = ra[i];
    } else {
      const int k = tid & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) As[buf][k][(tid >> 4) + 16 * i] = ra[i];
    }
    if (p.opB == 0) {
      const int k = tid & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[buf][k][(tid >> 4) + 16 * i] = rb[i];
    } else {
      const int n = tid & 63;
#pragma unroll
      for (int i = 0; i < 4; ++i) Bs[buf][(tid >> 6) + 4 * i][n] = rb[i];
    }
  };

  const int nk = (p.K + KT - 1) / KT;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) load((t + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int kk = ks * 4 + lg;
      zd a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][kk][wr * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kk][wc * 32 + j * 16 + l16];
      // four independent accumulator sweeps keep the MFMA pipe busy
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, accR[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, accI[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[i].y, b[j].y, accR[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].x, accI[i][j], 0, 0, 0);
    }
    if (t + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

  double alpha = p.alpha, beta = p.beta, gamma = p.gamma;
  if (p.coef) {
    alpha = p.coef[0];
    beta = p.coef[1];
    gamma = p.coef[2];
  }
  const bool useC = (p.Cm != nullptr) && (beta != 0.0);
  const bool useE = (p.E != nullptr) && (gamma != 0.0);
  // D layout of v_mfma_f64_16x16x4: lane l, register r -> row l/16 + 4r, col l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wc * 32 + j * 16 + l16;
      if (col >= p.N) continue;
      const double g = useE ? gamma * (p.gcol ? p.gcol[col] : 1.0) : 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + i * 16 + lg + 4 * r;
        if (row >= p.M) continue;
        double vr = alpha * accR[i][j][r], vi = alpha * accI[i][j][r];
        if (useC) {
          const zd cv = p.Cm[row + (int64_t)col * p.ldc];
          vr += beta * cv.x;
          vi += beta * cv.y;
        }
        if (useE) {
          const zd ev = p.E[row + (int64_t)col * p.lde];
          vr += g * ev.x;
          vi += g * ev.y;
        }
        p.D[row + (int64_t)col * p.ldd] = make_double2(vr, vi);
      }
    }
}
}  // namespace

gevp_status launch_zgemm(gevp_ctx* c, int opA, int opB, int64_t m, int64_t n, int64_t k,
                         double alpha, const zd* A, int64_t lda, const zd* B, int64_t ldb,
                         double beta, const zd* Cm, int64_t ldc, double gamma, const zd* E,
                         int64_t lde, const double* gcol, zd* D, int64_t ldd,
                         const double* coef) {
  if (m <= 0 || n <= 0) return GEVP_OK;
  if (m > INT32_MAX || n > INT32_MAX || k > INT32_MAX) return GEVP_ERR_INVALID;
  ZgemmParams p;
  p.M = (int)m;
  p.N = (int)n;
  p.K = (int)(k < 0 ? 0 : k);
  p.opA = opA;
  p.opB = opB;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.Cm = Cm;
  p.ldc = ldc;
  p.E = E;
  p.lde = lde;
  p.gcol = gcol;
  p.D = D;
  p.ldd = ldd;
  p.alpha = alpha;
  p.beta = beta;
  p.gamma = gamma;
  p.coef = coef;
  p.tiles_n = (int)((n + BN - 1) / BN);
  const int64_t tiles_m = (m + BM - 1) / BM;
  const int64_t total = tiles_m * p.tiles_n;
  if (total > INT32_MAX) return GEVP_ERR_INVALID;
  p.total = (int)total;
  p.remap = (total % 8 == 0 && total >= 64) ? 1 : 0;
  if (coef)
    hipLaunchKernelGGL(k_zgemm<1>, dim3((unsigned)total), dim3(NTHR), 0, c->stream, p);
  else
    hipLaunchKernelGGL(k_zgemm<0>, dim3((unsigned)total), dim3(NTHR), 0, c->stream, p);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
