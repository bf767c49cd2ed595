// Split-BF16 complex filter GEMM on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation):
//
//   D(:, j) = alpha_j C G(:, j) + beta_j G(:, j) + gamma_j P(:, j) + delta_j R(:, j)
//
// Every real operand x is split as x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (both round-to-nearest-even), and a real product is
// formed from three BF16 products hi*hi + hi*lo + lo*hi; the dropped lo*lo
// term and the split itself leave a relative error near 2^-16 per product,
// which the residual-correction recurrence tolerates (its rounding errors are
// relative to the correction, not to the iterate).  A complex multiply-add is
// four real products, so twelve MFMAs per 16 x 16 x 32 block.
//
// A is the reduced matrix C, stored once per solve as four BF16 planes
// (re hi, re lo, im hi, im lo) of its ROWS: C is Hermitian, so row i is the
// conjugate of stored column i and the conversion reads columns
// contiguously; in the planes 8 consecutive k of one row (one MFMA fragment)
// are 16 contiguous bytes.  B is the FP32 complex iterate, split into planes
// while it is staged into LDS.
//
// Tiling: 512 threads (8 waves, 2 x 4) own a 128 x 128 complex output tile,
// each wave 64 x 32 (4 x 2 MFMA blocks); K advances 32 per slice through a
// double-buffered LDS stage (row stride padded by 16 bytes so a fragment
// read by 16 lanes touches 64 distinct banks), with the next slice's global
// loads in flight during the current slice's MFMAs.
#include "common.h"

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float2 zf;

namespace {
constexpr int BM = 128, BN = 128, KT = 32, NTHR = 512;
constexpr int ROWB = 4 * KT * 2 + 16;  // bytes per staged row/column: 4 planes x 32 k x 2 B + pad

struct BfParams {
  int M, N, K;        // K = order of C; Kp (padded to 32) = KG * 8
  int KG;             // k-groups of 8 per plane row
  const uint4* A;     // planes: [(row * KG + g) * 4 + plane] 16-byte chunks
  const zf* B;
  int64_t ldb;
  const zf* P;
  int64_t ldp;
  const zf* R;
  int64_t ldr;
  zf* D;
  int64_t ldd;
  const double* alpha;
  const double* beta;
  const double* gamma;
  const double* delta;
  int tiles_n, total, remap;
};

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// hi/lo split of 8 floats into two 16-byte chunks
__device__ __forceinline__ void split8(const float* x, uint4& hi, uint4& lo) {
  unsigned h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const unsigned short hh = bf16_rne(x[e]);
    h[e] = hh;
    l[e] = bf16_rne(x[e] - bf16_f(hh));
  }
  hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
  lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
}

__device__ __forceinline__ unsigned pack_split(float a, float b, unsigned& lo) {
  const unsigned short ha = bf16_rne(a), hb = bf16_rne(b);
  const unsigned short la = bf16_rne(a - bf16_f(ha)), lb = bf16_rne(b - bf16_f(hb));
  lo = (unsigned)la | ((unsigned)lb << 16);
  return (unsigned)ha | ((unsigned)hb << 16);
}
__device__ __forceinline__ void split8v(float x0, float x1, float x2, float x3, float x4, float x5,
                                        float x6, float x7, uint4& hi, uint4& lo) {
  unsigned l0, l1, l2, l3;
  const unsigned h0 = pack_split(x0, x1, l0), h1 = pack_split(x2, x3, l1);
  const unsigned h2 = pack_split(x4, x5, l2), h3 = pack_split(x6, x7, l3);
  hi = make_uint4(h0, h1, h2, h3);
  lo = make_uint4(l0, l1, l2, l3);
}

__device__ __forceinline__ bf8 as_bf8(uint4 v) { return __builtin_bit_cast(bf8, v); }
__device__ __forceinline__ uint4 negbf(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

__global__ __launch_bounds__(NTHR, 1) void k_cgemm_bf16x3_filter(BfParams p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  // stage b: A rows at lds + b * BM * ROWB, B columns after both A stages
  auto As = [&](int b) { return lds + b * (BM * ROWB); };
  auto Bs = [&](int b) { return lds + 2 * BM * ROWB + b * (BN * ROWB); };

  const int tid = threadIdx.x;
  int L = blockIdx.x;
  if (p.remap) {
    const int per = p.total >> 3;
    L = (L & 7) * per + (L >> 3);
  }
  const int tm = L / p.tiles_n, tn = L - tm * p.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // 2 x 4 waves; wave tile 64 x 32
  const int l16 = lane & 15, lg = lane >> 4;

  f4 accR[4][2], accI[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }

  // staging assignment: thread -> (row/col = tid / 4, k-group q = tid % 4);
  // held in plain vector registers (no arrays, so nothing lands in scratch)
  const int sr = tid >> 2, sq = tid & 3;
  uint4 pa0, pa1, pa2, pa3;  // planes of one k-group of row sr
  float4 gb0, gb1, gb2, gb3;  // 8 complex of column sr, k-group sq (re, im interleaved)
  const uint4 z4 = make_uint4(0, 0, 0, 0);
  const float4 zf4 = make_float4(0.f, 0.f, 0.f, 0.f);

#define GLOAD(t)                                                                 \
  do {                                                                           \
    const int g_ = (t) * 4 + sq;                                                 \
    const int gm_ = row0 + sr;                                                   \
    if (gm_ < p.M && g_ < p.KG) {                                                \
      const uint4* src_ = p.A + ((int64_t)gm_ * p.KG + g_) * 4;                  \
      pa0 = src_[0];                                                             \
      pa1 = src_[1];                                                             \
      pa2 = src_[2];                                                             \
      pa3 = src_[3];                                                             \
    } else {                                                                     \
      pa0 = pa1 = pa2 = pa3 = z4;                                                \
    }                                                                            \
    const int gn_ = col0 + sr;                                                   \
    const int k0_ = g_ * 8;                                                      \
    if (gn_ < p.N && k0_ + 8 <= p.K) {                                           \
      const float4* col_ = (const float4*)(p.B + (int64_t)gn_ * p.ldb + k0_);   \
      gb0 = col_[0];                                                             \
      gb1 = col_[1];                                                             \
      gb2 = col_[2];                                                             \
      gb3 = col_[3];                                                             \
    } else if (gn_ < p.N) {                                                      \
      const zf* col_ = p.B + (int64_t)gn_ * p.ldb;                               \
      const zf v0 = (k0_ + 0 < p.K) ? col_[k0_ + 0] : make_float2(0.f, 0.f);     \
      const zf v1 = (k0_ + 1 < p.K) ? col_[k0_ + 1] : make_float2(0.f, 0.f);     \
      const zf v2 = (k0_ + 2 < p.K) ? col_[k0_ + 2] : make_float2(0.f, 0.f);     \
      const zf v3 = (k0_ + 3 < p.K) ? col_[k0_ + 3] : make_float2(0.f, 0.f);     \
      const zf v4 = (k0_ + 4 < p.K) ? col_[k0_ + 4] : make_float2(0.f, 0.f);     \
      const zf v5 = (k0_ + 5 < p.K) ? col_[k0_ + 5] : make_float2(0.f, 0.f);     \
      const zf v6 = (k0_ + 6 < p.K) ? col_[k0_ + 6] : make_float2(0.f, 0.f);     \
      const zf v7 = (k0_ + 7 < p.K) ? col_[k0_ + 7] : make_float2(0.f, 0.f);     \
      gb0 = make_float4(v0.x, v0.y, v1.x, v1.y);                                 \
      gb1 = make_float4(v2.x, v2.y, v3.x, v3.y);                                 \
      gb2 = make_float4(v4.x, v4.y, v5.x, v5.y);                                 \
      gb3 = make_float4(v6.x, v6.y, v7.x, v7.y);                                 \
    } else {                                                                     \
      gb0 = gb1 = gb2 = gb3 = zf4;                                               \
    }                                                                            \
  } while (0)

#define SSTORE(buf)                                                              \
  do {                                                                           \
    uint4* ra_ = (uint4*)(As(buf) + sr * ROWB);                                  \
    ra_[0 * 4 + sq] = pa0;                                                       \
    ra_[1 * 4 + sq] = pa1;                                                       \
    ra_[2 * 4 + sq] = pa2;                                                       \
    ra_[3 * 4 + sq] = pa3;                                                       \
    uint4 rh_, rl_, ih_, il_;                                                    \
    split8v(gb0.x, gb0.z, gb1.x, gb1.z, gb2.x, gb2.z, gb3.x, gb3.z, rh_, rl_);   \
    split8v(gb0.y, gb0.w, gb1.y, gb1.w, gb2.y, gb2.w, gb3.y, gb3.w, ih_, il_);   \
    uint4* rb_ = (uint4*)(Bs(buf) + sr * ROWB);                                  \
    rb_[0 * 4 + sq] = rh_;                                                       \
    rb_[1 * 4 + sq] = rl_;                                                       \
    rb_[2 * 4 + sq] = ih_;                                                       \
    rb_[3 * 4 + sq] = il_;                                                       \
  } while (0)

  const int nk = (p.KG + 3) / 4;
  if (nk > 0) {
    GLOAD(0);
    SSTORE(0);
  }
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) GLOAD(t + 1);
    // fragments: lane -> (row/col l16 of the block, k-group lg)
    uint4 bf[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint4* src = (const uint4*)(Bs(cur) + (wc * 32 + j * 16 + l16) * ROWB);
#pragma unroll
      for (int q = 0; q < 4; ++q) bf[j][q] = src[q * 4 + lg];
    }
    uint4 nbh[2], nbl[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      nbh[j] = negbf(bf[j][2]);
      nbl[j] = negbf(bf[j][3]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4* src = (const uint4*)(As(cur) + (wr * 64 + i * 16 + l16) * ROWB);
      const bf8 arh = as_bf8(src[0 * 4 + lg]), arl = as_bf8(src[1 * 4 + lg]);
      const bf8 aih = as_bf8(src[2 * 4 + lg]), ail = as_bf8(src[3 * 4 + lg]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bf8 brh = as_bf8(bf[j][0]), brl = as_bf8(bf[j][1]);
        const bf8 bih = as_bf8(bf[j][2]), bil = as_bf8(bf[j][3]);
        const bf8 nih = as_bf8(nbh[j]), nil = as_bf8(nbl[j]);
        f4 r = accR[i][j], m = accI[i][j];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brh, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bih, m, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, brl, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arh, bil, m, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, brh, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(arl, bih, m, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, nih, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brh, m, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, nil, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aih, brl, m, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, nih, r, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ail, brh, m, 0, 0, 0);
        accR[i][j] = r;
        accI[i][j] = m;
      }
    }
    if (t + 1 < nk) SSTORE(cur ^ 1);
    __syncthreads();
  }
#undef GLOAD
#undef SSTORE
  // D layout of v_mfma_f32_16x16x32_bf16: lane l, register r -> row 4 (l/16) + r, col l%16
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = col0 + wc * 32 + j * 16 + l16;
    if (col >= p.N) continue;
    const float al = (float)p.alpha[col], be = (float)p.beta[col];
    const float ga = (float)p.gamma[col], de = (float)p.delta[col];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 64 + i * 16 + 4 * lg + r;
        if (row >= p.M) continue;
        const zf g = p.B[row + (int64_t)col * p.ldb];
        float vr = al * accR[i][j][r] + be * g.x, vi = al * accI[i][j][r] + be * g.y;
        if (ga != 0.f) {
          const zf q = p.P[row + (int64_t)col * p.ldp];
          vr += ga * q.x;
          vi += ga * q.y;
        }
        if (de != 0.f) {
          const zf q = p.R[row + (int64_t)col * p.ldr];
          vr += de * q.x;
          vi += de * q.y;
        }
        p.D[row + (int64_t)col * p.ldd] = make_float2(vr, vi);
      }
  }
}

// Planes of the rows of the Hermitian C: row i, k-group g holds
// C(i, 8g .. 8g+7) = conj(C_st(8g .. 8g+7, i)), split into re hi/lo, im hi/lo.
__global__ void k_split_rows_bf16(int64_t n, int KG, const zd* C, int64_t ldc, uint4* planes) {
  const int64_t i = blockIdx.y;
  const zd* col = C + i * ldc;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < KG; g += gridDim.x * blockDim.x) {
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = (int64_t)g * 8 + e;
      const zd v = (k < n) ? col[k] : make_double2(0.0, 0.0);
      re[e] = (float)v.x;
      im[e] = (float)(-v.y);
    }
    uint4 rh, rl, ih, il;
    split8(re, rh, rl);
    split8(im, ih, il);
    uint4* o = planes + (i * KG + g) * 4;
    o[0] = rh;
    o[1] = rl;
    o[2] = ih;
    o[3] = il;
  }
}
}  // namespace

size_t bf16_planes_bytes(int64_t n) {
  const int64_t KG = ((n + 31) / 32) * 4;
  return (size_t)n * KG * 64;
}

gevp_status launch_split_rows_bf16(gevp_ctx* c, int64_t n, const zd* C, int64_t ldc, void* planes) {
  if (n <= 0) return GEVP_OK;
  const int KG = (int)(((n + 31) / 32) * 4);
  const unsigned gxs = (unsigned)((KG + 255) / 256);
  hipLaunchKernelGGL(k_split_rows_bf16, dim3(gxs, (unsigned)n), dim3(256), 0, c->stream, n, KG, C, ldc,
                     (uint4*)planes);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_cgemm_bf16x3_filter(gevp_ctx* c, int64_t m, int64_t n, int64_t k,
                                       const void* planes, const void* G, int64_t ldg,
                                       const void* P, int64_t ldp, const void* R, int64_t ldr,
                                       void* D, int64_t ldd, const double* al, const double* be,
                                       const double* ga, const double* de) {
  if (m <= 0 || n <= 0) return GEVP_OK;
  BfParams p;
  p.M = (int)m;
  p.N = (int)n;
  p.K = (int)k;
  p.KG = (int)(((k + 31) / 32) * 4);
  p.A = (const uint4*)planes;
  p.B = (const zf*)G;
  p.ldb = ldg;
  p.P = (const zf*)P;
  p.ldp = ldp;
  p.R = (const zf*)R;
  p.ldr = ldr;
  p.D = (zf*)D;
  p.ldd = ldd;
  p.alpha = al;
  p.beta = be;
  p.gamma = ga;
  p.delta = de;
  p.tiles_n = (int)((n + BN - 1) / BN);
  const int64_t total = ((m + BM - 1) / BM) * p.tiles_n;
  p.total = (int)total;
  p.remap = (total % 8 == 0 && total >= 64) ? 1 : 0;
  const size_t shm = (size_t)2 * (BM + BN) * ROWB;
  // 136 KB of LDS per work-group (gfx950 has 160 KB per CU); set once,
  // thread-safely (batched solves launch from several host threads)
  static const bool attr_set = [&]() {
    (void)hipFuncSetAttribute((const void*)k_cgemm_bf16x3_filter,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    return true;
  }();
  (void)attr_set;
  hipLaunchKernelGGL(k_cgemm_bf16x3_filter, dim3((unsigned)total), dim3(NTHR), shm, c->stream, p);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
