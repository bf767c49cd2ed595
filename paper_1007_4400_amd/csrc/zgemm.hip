// Complex128 GEMM on the FP64 matrix cores of gfx950 (v_mfma_f64_16x16x4f64).
//
//   D = alpha op(A) op(B) + beta Cm + gamma diag(gcol) E
//
// op() is identity or conjugate transpose.  The complex product is formed
// from three real products per 16 x 16 block (Gauss's three-multiplication
// form, as in the 3M complex GEMMs):
//   P1 += Ar Br,   P2 += Ai Bi,   P3 += (Ar + Ai)(Br + Bi)
//   Re = P1 - P2,  Im = P3 - P1 - P2
// on interleaved (re, im) operands (the two sums are formed in registers from
// the LDS slices), so no planar copy of the inputs exists.  Three MFMAs per
// block and K step instead of four; the error of Im is bounded by the unit
// roundoff times (|Ar| + |Ai|)(|Br| + |Bi|) instead of times |A||B|, a factor
// of at most 2 in the normwise bounds.
//
// Tiling: a 256-thread work-group owns a 64 x 64 complex output tile; each of
// its four waves owns 32 x 32 (2 x 2 MFMA blocks, 12 accumulators).  K is
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
//
// Split-K: a product with few output tiles and a long K (a Gram matrix
// Y^H Y of a tall block, say) splits K over several work-groups chosen by a
// cost model (rounds of two work-groups per compute unit times slices per
// part, plus the reduction); each writes its raw partial tile to the
// handle's buffer and a second kernel sums the parts in a fixed order and
// applies the epilogue, so results do not depend on scheduling.  upperA = 1
// declares op(A) upper triangular (L^H, or the upper triangle of a matrix
// whose lower triangle holds something else): a row block starts its K walk
// at its own first row, and the entries below the diagonal of op(A) read as
// zero, so only the upper triangle is ever used.  A split whose K range lies
// entirely below a row block's diagonal contributes a zero partial tile.
#include <atomic>

#include <algorithm>

#include "common.h"

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64, BN = 64, KT = 16, NTHR = 256;
constexpr int PADA = BM + 1, PADB = BN + 1;
constexpr int64_t SPLIT_TILES_MAX = 2048;  // partial tiles the split-K buffer holds (128 MiB)
constexpr int SKINNY_K_MAX = 1024;         // longest K for the skinny-tile kernels
static_assert(SKW_BYTES == (size_t)SPLIT_TILES_MAX * 64 * 64 * 16, "split-K buffer size");
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
  int tiles;  // output tiles; blocks = tiles * splits
  int total;
  int remap;
  int lower;  // 1: only tiles that touch the lower triangle (row >= col) are computed
  int upperA;       // op(A) upper triangular: slices below the tile's first row are zero
  int splits, nks;  // K split in `splits` parts of nks slices
  zd* part;         // splits > 1: raw partial tiles [split][tile][col][row]
  const zd* A2;     // op(A) = 'N' only: rows >= M1 of op(A) are rows - M1 of A2 (same lda)
  int M1;
};

__device__ __forceinline__ zd zconj(zd a) { return make_double2(a.x, -a.y); }

// Output tile of linear index `tile`: row-major over all tiles, or, for a
// lower-triangle launch (p.lower: square output, only tiles on or below the
// diagonal exist), row-major over the lower triangle of tiles: row tm holds
// tm + 1 tiles and starts at tm (tm + 1) / 2.
__device__ __forceinline__ void tile_coords(const ZgemmParams& p, int tile, int& tm, int& tn) {
  if (p.lower) {
    int r = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((int64_t)r * (r + 1) / 2 > tile) --r;  // correct the rounding of the root
    while ((int64_t)(r + 1) * (r + 2) / 2 <= tile) ++r;
    tm = r;
    tn = tile - (int)((int64_t)r * (r + 1) / 2);
  } else {
    tm = tile / p.tiles_n;
    tn = tile - tm * p.tiles_n;
  }
}

// One output tile; the operand forms are compile-time constants, so each
// kernel below carries only its own load and LDS-store pattern.
template <int OPA, int OPB>
__device__ __forceinline__ void zgemm_tile(const ZgemmParams& p) {
  __shared__ zd As[2][KT][PADA];
  __shared__ zd Bs[2][KT][PADB];

  const int tid = threadIdx.x;
  int L = blockIdx.x;
  if (p.remap) {
    const int per = p.total >> 3;
    L = (L & 7) * per + (L >> 3);
  }
  const int kc = L / p.tiles, tile = L - kc * p.tiles;
  int tm, tn;
  tile_coords(p, tile, tm, tn);
  const int row0 = tm * BM, col0 = tn * BN;

  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;

  d4 acc1[2][2], acc2[2][2], acc3[2][2];  // P1, P2, P3 of the three-product form
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc1[i][j] = d4{0, 0, 0, 0};
      acc2[i][j] = d4{0, 0, 0, 0};
      acc3[i][j] = d4{0, 0, 0, 0};
    }

  zd ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;  // next slice, in registers
  constexpr int opA = OPA, opB = OPB;

  // A col-major M x K: thread -> (m = tid%64, k = tid/64 + 4i); A stored K x M
  // ('C'): op(A)(m,k) = conj(A[k + m lda]), k fastest.  B col-major K x N: k
  // fastest; B stored N x K ('C'): op(B)(k,n) = conj(B[n + k ldb]), n fastest.
#define LDA_(i, dst)                                                                  \
  do {                                                                                \
    if (opA == 0) {                                                                   \
      const int gm_ = row0 + (tid & 63), gk_ = k0 + (tid >> 6) + 4 * (i);             \
      const bool lo_ = gm_ >= p.M1;                                                   \
      const zd* ab_ = lo_ ? p.A2 : p.A;                                               \
      const int gr_ = lo_ ? gm_ - p.M1 : gm_;                                         \
      dst = (gm_ < p.M && gk_ < p.K && !(p.upperA && gk_ < gm_)) ? ab_[gr_ + (int64_t)gk_ * p.lda]: make_double2(0.0, 0.0); \
    } else {                                                                          \
      const int gk_ = k0 + (tid & 15), gm_ = row0 + (tid >> 4) + 16 * (i);            \
      dst = (gm_ < p.M && gk_ < p.K && !(p.upperA && gk_ < gm_)) ? zconj(p.A[gk_ + (int64_t)gm_ * p.lda]) : make_double2(0.0, 0.0); \
    }                                                                                 \
  } while (0)
#define LDB_(i, dst)                                                                  \
  do {                                                                                \
    if (opB == 0) {                                                                   \
      const int gk_ = k0 + (tid & 15), gn_ = col0 + (tid >> 4) + 16 * (i);            \
      dst = (gn_ < p.N && gk_ < p.K) ? p.B[gk_ + (int64_t)gn_ * p.ldb]: make_double2(0.0, 0.0);      \
    } else {                                                                          \
      const int gn_ = col0 + (tid & 63), gk_ = k0 + (tid >> 6) + 4 * (i);             \
      dst = (gn_ < p.N && gk_ < p.K) ? zconj(p.B[gn_ + (int64_t)gk_ * p.ldb]) : make_double2(0.0, 0.0); \
    }                                                                                 \
  } while (0)
#define LOAD_(kk0)          \
  do {                      \
    const int k0 = (kk0);   \
    LDA_(0, ra0);           \
    LDA_(1, ra1);           \
    LDA_(2, ra2);           \
    LDA_(3, ra3);           \
    LDB_(0, rb0);           \
    LDB_(1, rb1);           \
    LDB_(2, rb2);           \
    LDB_(3, rb3);           \
  } while (0)
#define STA_(i, v)                                                   \
  do {                                                               \
    if (opA == 0) As[buf_][(tid >> 6) + 4 * (i)][tid & 63] = v;      \
    else As[buf_][tid & 15][(tid >> 4) + 16 * (i)] = v;              \
  } while (0)
#define STB_(i, v)                                                   \
  do {                                                               \
    if (opB == 0) Bs[buf_][tid & 15][(tid >> 4) + 16 * (i)] = v;     \
    else Bs[buf_][(tid >> 6) + 4 * (i)][tid & 63] = v;               \
  } while (0)
#define STORE_(b)           \
  do {                      \
    const int buf_ = (b);   \
    STA_(0, ra0);           \
    STA_(1, ra1);           \
    STA_(2, ra2);           \
    STA_(3, ra3);           \
    STB_(0, rb0);           \
    STB_(1, rb1);           \
    STB_(2, rb2);           \
    STB_(3, rb3);           \
  } while (0)

  const int nk = (p.K + KT - 1) / KT;
  int t0 = kc * p.nks;
  const int t1 = (t0 + p.nks < nk) ? t0 + p.nks : nk;
  if (p.upperA && row0 / KT > t0) t0 = row0 / KT;
  if (t0 < t1) {
    LOAD_(t0 * KT);
    STORE_(0);
  }
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    const int cur = (t - t0) & 1;
    if (t + 1 < t1) LOAD_((t + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int kk = ks * 4 + lg;
      zd a[2], b[2];
      double sa[2], sb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = As[cur][kk][wr * 32 + i * 16 + l16];
        sa[i] = a[i].x + a[i].y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        b[j] = Bs[cur][kk][wc * 32 + j * 16 + l16];
        sb[j] = b[j].x + b[j].y;
      }
      // three independent accumulator sweeps keep the MFMA pipe busy
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc1[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc2[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[i], sb[j], acc3[i][j], 0, 0, 0);
    }
    if (t + 1 < t1) STORE_(cur ^ 1);
    __syncthreads();
  }
#undef LDA_
#undef LDB_
#undef LOAD_
#undef STA_
#undef STB_
#undef STORE_

  // the complex result of the three products
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = acc1[i][j] - acc2[i][j];
      accI[i][j] = acc3[i][j] - acc1[i][j] - acc2[i][j];
    }
  // D layout of v_mfma_f64_16x16x4: lane l, register r -> row l/16 + 4r, col l%16
  if (p.splits > 1) {  // raw partial tile, [col][row] within the tile
    zd* pt = p.part + ((int64_t)kc * p.tiles + tile) * (BM * BN);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          pt[(wc * 32 + j * 16 + l16) * BM + wr * 32 + i * 16 + lg + 4 * r] =
              make_double2(accR[i][j][r], accI[i][j][r]);
    return;
  }
  double alpha = p.alpha, beta = p.beta, gamma = p.gamma;
  if (p.coef) {
    alpha = p.coef[0];
    beta = p.coef[1];
    gamma = p.coef[2];
  }
  const bool useC = (p.Cm != nullptr) && (beta != 0.0);
  const bool useE = (p.E != nullptr) && (gamma != 0.0);
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

// Both operands as stored.  FILTER only names the kernel differently for the
// Chebyshev filter launches (coefficients from device memory), so profiles
// separate them.
template <int FILTER>
__global__ __launch_bounds__(NTHR, 2) void k_zgemm(ZgemmParams p) { zgemm_tile<0, 0>(p); }
// op(B) = B^H, op(A) = A^H, both conjugate-transposed
__global__ __launch_bounds__(NTHR, 2) void k_zgemm_nc(ZgemmParams p) { zgemm_tile<0, 1>(p); }
__global__ __launch_bounds__(NTHR, 2) void k_zgemm_cn(ZgemmParams p) { zgemm_tile<1, 0>(p); }
__global__ __launch_bounds__(NTHR, 2) void k_zgemm_cc(ZgemmParams p) { zgemm_tile<1, 1>(p); }

// Skinny tiles for products with at most 64 rows (TALL: 64 x 16 output
// tiles) or at most 64 columns (16 x 64 tiles) and a short K: the base cases
// and 64-wide updates of the triangular solves and the panel products of the
// Cholesky factorisation.  With 64 x 64 tiles such a product has one tile per
// 64 columns (or rows), so 15 work-groups for a 64 x 948 result, and each of
// their waves runs a chain of 12 MFMAs per 4 K; here each of the four waves
// owns one 16 x 16 block (3 MFMAs per 4 K), so the work-groups are four times
// as many and their chains four times shorter.  A tile still spans every row
// (TALL) or every column (wide) of the result, so a base case that writes its
// right operand in place (TALL) or its left operand in place (wide) reads its
// whole K range before it writes, as with the 64 x 64 tiles.
template <int OPA, int OPB, int TALL>
__global__ __launch_bounds__(NTHR) void k_zgemm_sk(ZgemmParams p) {
  constexpr int SM = TALL ? 64 : 16, SN = TALL ? 16 : 64;
  __shared__ zd As[2][KT][SM + 1];
  __shared__ zd Bs[2][KT][SN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_n = (p.N + SN - 1) / SN;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int row0 = tm * SM, col0 = tn * SN;
  const int l16 = lane & 15, lg = lane >> 4;
  const int bm = TALL ? wave : 0, bn = TALL ? 0 : wave;  // this wave's 16 x 16 block
  d4 acc1 = d4{0, 0, 0, 0}, acc2 = d4{0, 0, 0, 0}, acc3 = d4{0, 0, 0, 0};  // three-product form
  constexpr int LA = SM * KT / NTHR, LB = SN * KT / NTHR;  // loads per thread and slice
  zd ra[LA], rb[LB];
  // thread -> (m, k) of op(A) and (k, n) of op(B), the stored layout's fast
  // index on consecutive threads
  auto a_mk = [&](int i, int& m, int& k) {
    if (OPA == 0) { m = tid % SM; k = tid / SM + (NTHR / SM) * i; }
    else { k = tid & 15; m = (tid >> 4) + 16 * i; }
  };
  auto b_kn = [&](int i, int& k, int& n) {
    if (OPB == 0) { k = tid & 15; n = (tid >> 4) + 16 * i; }
    else { n = tid % SN; k = tid / SN + (NTHR / SN) * i; }
  };
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      int m, k;
      a_mk(i, m, k);
      const int gm = row0 + m, gk = k0 + k;
      ra[i] = (gm < p.M && gk < p.K)
                  ? (OPA == 0 ? p.A[gm + (int64_t)gk * p.lda] : zconj(p.A[gk + (int64_t)gm * p.lda]))
                  : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      int k, n;
      b_kn(i, k, n);
      const int gn = col0 + n, gk = k0 + k;
      rb[i] = (gn < p.N && gk < p.K)
                  ? (OPB == 0 ? p.B[gk + (int64_t)gn * p.ldb] : zconj(p.B[gn + (int64_t)gk * p.ldb]))
                  : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int b) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      int m, k;
      a_mk(i, m, k);
      As[b][k][m] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      int k, n;
      b_kn(i, k, n);
      Bs[b][k][n] = rb[i];
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
      const zd a = As[cur][kk][bm * 16 + l16], b = Bs[cur][kk][bn * 16 + l16];
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x + a.y, b.x + b.y, acc3, 0, 0, 0);
    }
    if (t + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
  const d4 accR = acc1 - acc2, accI = acc3 - acc1 - acc2;
  const int col = col0 + bn * 16 + l16;
  if (col >= p.N) return;
  const bool useC = (p.Cm != nullptr) && (p.beta != 0.0);
  const bool useE = (p.E != nullptr) && (p.gamma != 0.0);
  const double g = useE ? p.gamma * (p.gcol ? p.gcol[col] : 1.0) : 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + bm * 16 + lg + 4 * r;
    if (row >= p.M) continue;
    double vr = p.alpha * accR[r], vi = p.alpha * accI[r];
    if (useC) {
      const zd cv = p.Cm[row + (int64_t)col * p.ldc];
      vr += p.beta * cv.x;
      vi += p.beta * cv.y;
    }
    if (useE) {
      const zd ev = p.E[row + (int64_t)col * p.lde];
      vr += g * ev.x;
      vi += g * ev.y;
    }
    p.D[row + (int64_t)col * p.ldd] = make_double2(vr, vi);
  }
}

// Split-K: sum of the partial tiles in split order, then the epilogue; one
// thread per output element, consecutive threads on consecutive rows.
__global__ __launch_bounds__(256) void k_zgemm_splitk_reduce(ZgemmParams p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)BM * BN;
  if (e >= (int64_t)p.tiles * per) return;
  const int tile = (int)(e / per);
  const int w = (int)(e - (int64_t)tile * per);
  const int cl = w / BM, rl = w - cl * BM;
  int tm, tn;
  tile_coords(p, tile, tm, tn);
  const int row = tm * BM + rl, col = tn * BN + cl;
  if (row >= p.M || col >= p.N) return;
  double ar = 0.0, ai = 0.0;
  for (int kc = 0; kc < p.splits; ++kc) {
    const zd v = p.part[((int64_t)kc * p.tiles + tile) * per + w];
    ar += v.x;
    ai += v.y;
  }
  double alpha = p.alpha, beta = p.beta, gamma = p.gamma;
  if (p.coef) {
    alpha = p.coef[0];
    beta = p.coef[1];
    gamma = p.coef[2];
  }
  double vr = alpha * ar, vi = alpha * ai;
  if (p.Cm != nullptr && beta != 0.0) {
    const zd cv = p.Cm[row + (int64_t)col * p.ldc];
    vr += beta * cv.x;
    vi += beta * cv.y;
  }
  if (p.E != nullptr && gamma != 0.0) {
    const double g = gamma * (p.gcol ? p.gcol[col] : 1.0);
    const zd ev = p.E[row + (int64_t)col * p.lde];
    vr += g * ev.x;
    vi += g * ev.y;
  }
  p.D[row + (int64_t)col * p.ldd] = make_double2(vr, vi);
}

// K splits for T tiles of nk slices when `slots` work-groups run at once:
// minimise rounds(T s) * ceil(nk / s) plus the reduction (about 1/100 of a
// slice per partial tile), keeping at least 8 slices per part
int zgemm_splits(int64_t T, int nk, int64_t slots, int64_t max_parts) {
  int best = 1;
  double best_cost = (double)((T + slots - 1) / slots) * nk;
  for (int s = 2; s <= 16; ++s) {
    const int nks = (nk + s - 1) / s;
    if (nks < 8) break;
    const int se = (nk + nks - 1) / nks;
    if (T * se > max_parts) break;
    const double cost = (double)((T * se + slots - 1) / slots) * nks + 0.01 * (double)(T * se) + 2.0;
    if (cost < 0.95 * best_cost) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}
}  // namespace

gevp_status launch_zgemm(gevp_ctx* c, int opA, int opB, int64_t m, int64_t n, int64_t k,
                         double alpha, const zd* A, int64_t lda, const zd* B, int64_t ldb,
                         double beta, const zd* Cm, int64_t ldc, double gamma, const zd* E,
                         int64_t lde, const double* gcol, zd* D, int64_t ldd,
                         const double* coef, int lower, int upperA, int64_t m1, const zd* A2) {
  if (m <= 0 || n <= 0) return GEVP_OK;
  // a stacked left operand [A; A2]: plain 'N' form only
  if (A2 && (opA != 0 || lower || upperA || coef || m1 <= 0 || m1 >= m)) return GEVP_ERR_INVALID;
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
  p.A2 = A2;
  p.M1 = A2 ? (int)m1 : (int)m;
  p.tiles_n = (int)((n + BN - 1) / BN);
  const int64_t tiles_m = (m + BM - 1) / BM;
  // a lower-triangle launch enumerates only the tiles on or below the
  // diagonal (square outputs; BM == BN), so the grid carries no empty
  // work-groups and the XCD ranges below get equal shares of the work
  static_assert(BM == BN, "lower-triangle tile enumeration");
  if (lower && m != n) return GEVP_ERR_INVALID;
  const int64_t total = lower ? tiles_m * (tiles_m + 1) / 2 : tiles_m * p.tiles_n;
  if (total > INT32_MAX) return GEVP_ERR_INVALID;
  p.tiles = (int)total;
  p.lower = lower;
  // skinny tiles: at most 64 rows (TALL) or columns (wide), fewer 64 x 64
  // tiles than compute units, a short K.  A result written over its right
  // operand needs tiles that span all rows (TALL), over its left operand
  // tiles that span all columns (wide).
  int skinny = 0;
  if (!lower && !upperA && !coef && !A2 && p.K <= SKINNY_K_MAX &&
      total < (int64_t)gevp_device_cus(c->device)) {
    if (m <= BM && (const zd*)D != A) skinny = 1;
    else if (n <= BN && (const zd*)D != B) skinny = 2;
  }
  const int nk = (p.K + KT - 1) / KT;
  p.upperA = upperA;
  int s = (c->no_split || skinny)
              ? 1
              : zgemm_splits(total, nk,
                             std::max<int64_t>(1, 2 * (int64_t)gevp_device_cus(c->device) / std::max(1, c->cu_div)),
                             SPLIT_TILES_MAX);
  p.nks = nk > 0 ? (nk + s - 1) / s : 1;
  p.splits = nk > 0 ? (nk + p.nks - 1) / p.nks : 1;
  p.part = nullptr;
  if (p.splits > 1) {
    const size_t need = (size_t)p.splits * total * BM * BN * sizeof(zd);
    if (need > c->skw_bytes) {
      if (c->ext) return GEVP_ERR_WORKSPACE;  // caller-owned memory is never reallocated
      if (c->skw) {
        GEVP_HIP_TRY(hipStreamSynchronize(c->stream));  // earlier launches may still read it
        GEVP_HIP_TRY(hipFree(c->skw));
        c->skw = nullptr;
        c->skw_bytes = 0;
      }
      const size_t cap = (size_t)SPLIT_TILES_MAX * BM * BN * sizeof(zd);
      if (hipMalloc(&c->skw, cap) != hipSuccess) {
        c->skw = nullptr;
        return GEVP_ERR_ALLOC;
      }
      c->skw_bytes = cap;
    }
    p.part = (zd*)c->skw;
  }
  const int64_t blocks = total * p.splits;
  p.total = (int)blocks;
  // XCD-aware order: the hardware deals work-groups to the eight XCDs in
  // turn; the remap gives each XCD a contiguous range of tiles (rows of
  // output tiles share their A panel in that XCD's L2).  A product with a
  // triangular op(A) has tiles of unequal work (row block i runs K from its
  // first row), so it keeps the dealt order: every XCD then gets every
  // eighth tile, heavy rows first.
  p.remap = (!upperA && blocks % 8 == 0 && blocks >= 64) ? 1 : 0;
  const dim3 grid((unsigned)blocks), thr(NTHR);
  // FP64 GEMM timing (profiling bit 4): not the FP64 filter (coef), which is
  // timed as a filter product by the caller
  const bool timed = (coef == nullptr) && (c->profiling & 4);
  if (skinny) {
    const int64_t sm = skinny == 1 ? 64 : 16, sn = skinny == 1 ? 16 : 64;
    const int64_t sk_tiles = ((m + sm - 1) / sm) * ((n + sn - 1) / sn);
    if (timed) GEVP_TRY(gev_begin(c));
    const dim3 sg((unsigned)sk_tiles), st(NTHR);
    if (skinny == 1) {
      if (opA == 0 && opB == 0) hipLaunchKernelGGL((k_zgemm_sk<0, 0, 1>), sg, st, 0, c->stream, p);
      else if (opA == 0) hipLaunchKernelGGL((k_zgemm_sk<0, 1, 1>), sg, st, 0, c->stream, p);
      else if (opB == 0) hipLaunchKernelGGL((k_zgemm_sk<1, 0, 1>), sg, st, 0, c->stream, p);
      else hipLaunchKernelGGL((k_zgemm_sk<1, 1, 1>), sg, st, 0, c->stream, p);
    } else {
      if (opA == 0 && opB == 0) hipLaunchKernelGGL((k_zgemm_sk<0, 0, 0>), sg, st, 0, c->stream, p);
      else if (opA == 0) hipLaunchKernelGGL((k_zgemm_sk<0, 1, 0>), sg, st, 0, c->stream, p);
      else if (opB == 0) hipLaunchKernelGGL((k_zgemm_sk<1, 0, 0>), sg, st, 0, c->stream, p);
      else hipLaunchKernelGGL((k_zgemm_sk<1, 1, 0>), sg, st, 0, c->stream, p);
    }
    GEVP_HIP_TRY(hipGetLastError());
    if (timed) {
      const int64_t shape[6] = {opA * 2 + opB, m, n, p.K, 1, sk_tiles};
      GEVP_TRY(gev_end(c, 8.0 * (double)m * (double)n * (double)p.K, shape));
    }
    return GEVP_OK;
  }
  if (timed) GEVP_TRY(gev_begin(c));
  if (opA == 0 && opB == 0) {
    if (coef)
      hipLaunchKernelGGL(k_zgemm<1>, grid, thr, 0, c->stream, p);
    else
      hipLaunchKernelGGL(k_zgemm<0>, grid, thr, 0, c->stream, p);
  } else if (opA == 0) {
    hipLaunchKernelGGL(k_zgemm_nc, grid, thr, 0, c->stream, p);
  } else if (opB == 0) {
    hipLaunchKernelGGL(k_zgemm_cn, grid, thr, 0, c->stream, p);
  } else {
    hipLaunchKernelGGL(k_zgemm_cc, grid, thr, 0, c->stream, p);
  }
  GEVP_HIP_TRY(hipGetLastError());
  if (p.splits > 1) {
    const int64_t elems = total * BM * BN;
    hipLaunchKernelGGL(k_zgemm_splitk_reduce, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                       c->stream, p);
    GEVP_HIP_TRY(hipGetLastError());
  }
  if (timed) {
    // algorithmic flops: 8 per complex multiply-add of the product as
    // defined (only the lower triangle of a square output when `lower`,
    // only the upper-triangular part of op(A) when `upperA`)
    const double md = (double)m, nd = (double)n, kd = (double)p.K;
    double fl = 8.0 * md * nd * kd;
    if (lower && m == n) fl = 8.0 * kd * nd * (nd + 1.0) * 0.5;
    if (upperA) {
      const double rows = std::min(md, kd);  // row i of op(A) starts at column i
      fl = 8.0 * nd * (rows * kd - rows * (rows - 1.0) * 0.5);
    }
    const int64_t shape[6] = {opA * 2 + opB, m, n, p.K, p.splits, blocks};
    GEVP_TRY(gev_end(c, fl, shape));
  }
  return GEVP_OK;
}

int gevp_device_cus(int dev) {
  static std::atomic<int> cache[64];
  if (dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load();
  if (v > 0) return v;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
    cu = 256;
  cache[dev].store(cu);
  return cu;
}
