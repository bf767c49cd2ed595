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
// are 16 contiguous bytes.  B, the FP32 complex iterate, is split into the
// same plane layout (per column) by a pass before the product, so the main
// loop moves both operands as plain 16-byte chunks and does no conversion.
//
// Tiling: 512 threads (8 waves, 2 x 4) own a 128 x 128 complex output tile,
// each wave 64 x 32 (4 x 2 MFMA blocks); K advances 32 per slice.  The
// operands go from global memory into LDS by direct transfers (no staging
// registers, no LDS stores); a staged row is 256 bytes with its 16-byte
// chunks XOR-swizzled by the row index so that fragment reads meet no bank
// conflicts.  The rows of C, streamed from HBM, are staged three slices
// deep and the iterate's columns two (3 x 32 KB + 2 x 32 KB = the 160 KB of
// LDS); each stage is its own LDS array and the loop is unrolled by six so
// that every stage index is a constant: the compiler can then tell a stage
// being read from the stages whose transfers are in flight, and the only
// waits on the transfers are the kernel's own (a __syncthreads() would also
// drain the transfers two slices ahead).  Measured at n = 8192 and 948
// columns: 1.23 ms per launch against 1.27 ms with two stages of both
// operands, 1.43 ms when the loop staged through registers and LDS stores,
// 1.65 ms with 64 x 64 wave tiles (one wave per SIMD), 1.34 ms with
// 256 x 64 tiles, and no change from raising the wave priority around the
// MFMAs.
//
// One work-group per compute unit runs at a time (160 KB of LDS), so a grid
// of T tiles takes ceil(T / CUs) rounds.  When that rounds badly (T = 384 on
// 256 CUs costs two full rounds for 1.5 rounds of work) the K range is split
// in s parts: each work-group writes its FP32 partial tile to a workspace
// and a second kernel sums the s partials in a fixed order and applies the
// epilogue, so the result does not depend on scheduling.
#include "common.h"

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float2 zf;

namespace {
constexpr int BM = 128, BN = 128;  // output tile; K advances 32 (one MFMA K) per slice

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
  const uint4* Bp;    // B planes: [(col * KG + g) * 4 + plane]
  zf* part;           // split-K partial tiles (splits > 1)
  int tiles_n, tiles, total, remap;
  int nks;            // K slices per split
  int splits;
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

__device__ __forceinline__ bf8 as_bf8(uint4 v) { return __builtin_bit_cast(bf8, v); }
__device__ __forceinline__ uint4 negbf(uint4 v) {
  return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

// The operands move straight from global memory into LDS
// (global_load_lds_dwordx4: lane i of a wave instruction writes 16 bytes at
// the wave's LDS base + 16 i): no staging registers, no LDS store
// instructions.  A staged row is 256 bytes without padding; its sixteen
// 16-byte chunks are XOR-swizzled (physical chunk = logical chunk ^
// SWZ(row)) so that fragment reads meet no bank conflicts.  Per
// K slice the work-group issues 64 wave instructions (4 rows each: 32 for the
// rows of C, 32 for the iterate's columns), 8 per wave: the rows of C two
// slices ahead of the MFMAs, the iterate's columns one.  Rows past the matrix
// load row 0 instead (valid memory; their outputs are never stored).
constexpr int DROW = 256;  // bytes per staged row
// chunk swizzle of a staged row: the two 2-bit halves of row % 16 swapped.
// Measured on this kernel's fragment reads (16 rows x 4 k-groups of 16 B per
// wave instruction): no bank-conflict cycles, against 4 per read with
// (row % 16) itself and 12 per read with (row / 2) % 16.
#define SWZ(row) ((((row) & 3) << 2) | (((row) >> 2) & 3))
// stages: three of the rows of C, two of the iterate's columns, 32 KB each
constexpr size_t A_STAGE = (size_t)BM * DROW, B_STAGE = (size_t)BN * DROW;
static_assert(3 * A_STAGE + 2 * B_STAGE == 160 * 1024, "the LDS of one compute unit");

template <int V>
struct ic {
  static constexpr int value = V;
};

__global__ __launch_bounds__(512, 1) void k_cgemm_bf16x3_filter(BfParams p) {
  // one array per stage, so that alias analysis separates a stage being read
  // from the stages whose transfers are still in flight
  __shared__ __attribute__((aligned(16))) unsigned char sA0[A_STAGE], sA1[A_STAGE], sA2[A_STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char sB0[B_STAGE], sB1[B_STAGE];
  constexpr int WNB = 2, WC = 4;
  auto As = [&](auto S) -> unsigned char* {
    if constexpr (decltype(S)::value == 0) return sA0;
    else if constexpr (decltype(S)::value == 1) return sA1;
    else return sA2;
  };
  auto Bs = [&](auto S) -> unsigned char* {
    if constexpr (decltype(S)::value == 0) return sB0;
    else return sB1;
  };

  const int tid = threadIdx.x;
  int L = blockIdx.x;
  if (p.remap) {
    const int per = p.total >> 3;
    L = (L & 7) * per + (L >> 3);
  }
  const int kc = L / p.tiles, tile = L - kc * p.tiles;
  const int tm = tile / p.tiles_n, tn = tile - tm * p.tiles_n;
  const int row0 = tm * BM, col0 = tn * BN;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int l16 = lane & 15, lg = lane >> 4;

  f4 accR[4][WNB], accI[4][WNB];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      accR[i][j] = f4{0, 0, 0, 0};
      accI[i][j] = f4{0, 0, 0, 0};
    }

  // this lane's part of the wave's 8 transfers per slice: transfer k moves
  // row 4 (wi & 31) + lane / 16 (wi = wave + 8 k; below 32: rows of C, else
  // iterate columns), physical chunk lane % 16, which carries logical chunk
  // (lane % 16) ^ (row & 15).  Its global address is a per-lane base plus
  // 256 bytes per slice.
  const unsigned char* gsrc[8];
  int ldst[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int wi = wave + 8 * k;
    const int blk = wi & 31;
    const int row = 4 * blk + (lane >> 4);
    const int lc = (lane & 15) ^ SWZ(row);
    const int gofs = (lc >> 2) * 64 + (lc & 3) * 16;  // bytes within the slice's 256
    if (wi < 32) {
      const int gm = (row0 + row < p.M) ? row0 + row : 0;
      gsrc[k] = (const unsigned char*)(p.A + (int64_t)gm * p.KG * 4) + gofs;
      ldst[k] = blk * 4 * DROW;
    } else {
      const int gn = (col0 + row < p.N) ? col0 + row : 0;
      gsrc[k] = (const unsigned char*)(p.Bp + (int64_t)gn * p.KG * 4) + gofs;
      ldst[k] = blk * 4 * DROW;
    }
  }
  // wave instructions k = 0..3 move rows of C (wi < 32), k = 4..7 iterate columns
  auto issueA = [&](int t, auto buf) {
    unsigned char* stage = As(buf);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      __builtin_amdgcn_global_load_lds((const void*)(gsrc[k] + (int64_t)t * 256),
                                       (__attribute__((address_space(3))) void*)(stage + ldst[k]),
                                       16, 0, 0);
  };
  auto issueB = [&](int t, auto buf) {
    unsigned char* stage = Bs(buf);
#pragma unroll
    for (int k = 4; k < 8; ++k)
      __builtin_amdgcn_global_load_lds((const void*)(gsrc[k] + (int64_t)t * 256),
                                       (__attribute__((address_space(3))) void*)(stage + ldst[k]),
                                       16, 0, 0);
  };
  auto frag = [&](const unsigned char* base, int row, int q) {
    return *(const uint4*)(base + row * DROW + (((lg * 4 + q) ^ SWZ(row)) << 4));
  };
  // one K slice: every fragment of stage `cur` is read into registers first,
  // then the next slice's transfers are issued, then the MFMAs run, so the
  // transfers overlap the MFMAs (an LDS read after a transfer is issued
  // would wait for it)
  uint4 bf[WNB][4], af[4][4];
  auto read_frags = [&](auto ca, auto cb) {
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      const int col = wc * 16 * WNB + j * 16 + l16;
#pragma unroll
      for (int q = 0; q < 4; ++q) bf[j][q] = frag(Bs(cb), col, q);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wr * 64 + i * 16 + l16;
#pragma unroll
      for (int q = 0; q < 4; ++q) af[i][q] = frag(As(ca), row, q);
    }
  };
  auto mfmas = [&]() {
    uint4 nbh[WNB], nbl[WNB];
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      nbh[j] = negbf(bf[j][2]);
      nbl[j] = negbf(bf[j][3]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bf8 arh = as_bf8(af[i][0]), arl = as_bf8(af[i][1]);
      const bf8 aih = as_bf8(af[i][2]), ail = as_bf8(af[i][3]);
#pragma unroll
      for (int j = 0; j < WNB; ++j) {
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
  };

  const int nk = (p.KG + 3) / 4;
  const int t0 = kc * p.nks;
  const int t1 = (t0 + p.nks < nk) ? t0 + p.nks : nk;
  const int nloc = t1 - t0;
  // issue order: A(0), B(0), A(1), then per slice u: B(u+1), A(u+2); at the
  // end of slice u everything but this wave's last A transfers (slice u+2,
  // four instructions) must have landed.  Slice u uses A stage u mod 3 and B
  // stage u mod 2; the loop is unrolled by 6 so both are constants.
  if (nloc > 0) {
    issueA(t0, ic<0>{});
    issueB(t0, ic<0>{});
  }
  if (nloc > 1) {
    issueA(t0 + 1, ic<1>{});
    asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  __builtin_amdgcn_s_barrier();
  auto body = [&](auto SA, auto SB, int u) {
    constexpr int sa = decltype(SA)::value, sb = decltype(SB)::value;
    read_frags(SA, SB);
    if (u + 1 < nloc) issueB(t0 + u + 1, ic<1 - sb>{});
    if (u + 2 < nloc) issueA(t0 + u + 2, ic<(sa + 2) % 3>{});
    __builtin_amdgcn_sched_barrier(0);
    mfmas();
    __builtin_amdgcn_sched_barrier(0);
    if (u + 2 < nloc)
      asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // a bare barrier: __syncthreads() would also drain the slice-(u+2) transfers
    __builtin_amdgcn_s_barrier();
  };
  int u = 0;
  for (; u + 6 <= nloc; u += 6) {
    body(ic<0>{}, ic<0>{}, u);
    body(ic<1>{}, ic<1>{}, u + 1);
    body(ic<2>{}, ic<0>{}, u + 2);
    body(ic<0>{}, ic<1>{}, u + 3);
    body(ic<1>{}, ic<0>{}, u + 4);
    body(ic<2>{}, ic<1>{}, u + 5);
  }
  for (; u < nloc; ++u) {
    switch (u % 6) {
      case 0: body(ic<0>{}, ic<0>{}, u); break;
      case 1: body(ic<1>{}, ic<1>{}, u); break;
      case 2: body(ic<2>{}, ic<0>{}, u); break;
      case 3: body(ic<0>{}, ic<1>{}, u); break;
      case 4: body(ic<1>{}, ic<0>{}, u); break;
      default: body(ic<2>{}, ic<1>{}, u); break;
    }
  }
  // D layout of v_mfma_f32_16x16x32_bf16: lane l, register r -> row 4 (l/16) + r, col l%16
  if (p.splits > 1) {
    zf* pt = p.part + ((int64_t)kc * p.tiles + tile) * (BM * BN);
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      const int cl = wc * 16 * WNB + j * 16 + l16;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          pt[cl * BM + wr * 64 + i * 16 + 4 * lg + r] = make_float2(accR[i][j][r], accI[i][j][r]);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < WNB; ++j) {
    const int col = col0 + wc * 16 * WNB + j * 16 + l16;
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

// Sum of the split-K partial tiles in split order, then the epilogue; one
// thread per output element, consecutive threads on consecutive rows.
__global__ __launch_bounds__(256) void k_bf16_splitk_reduce(BfParams p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)BM * BN;
  if (e >= (int64_t)p.tiles * per) return;
  const int tile = (int)(e / per);
  const int w = (int)(e - (int64_t)tile * per);
  const int cl = w / BM, rl = w - cl * BM;
  const int tm = tile / p.tiles_n, tn = tile - tm * p.tiles_n;
  const int row = tm * BM + rl, col = tn * BN + cl;
  if (row >= p.M || col >= p.N) return;
  float ar = 0.f, ai = 0.f;
  for (int kc = 0; kc < p.splits; ++kc) {
    const zf v = p.part[((int64_t)kc * p.tiles + tile) * per + w];
    ar += v.x;
    ai += v.y;
  }
  const float al = (float)p.alpha[col], be = (float)p.beta[col];
  const float ga = (float)p.gamma[col], de = (float)p.delta[col];
  const zf g = p.B[row + (int64_t)col * p.ldb];
  float vr = al * ar + be * g.x, vi = al * ai + be * g.y;
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

// Planes of the columns of the FP32 complex iterate G (k rows): column c,
// k-group g holds G(8g .. 8g+7, c) split into re hi/lo, im hi/lo (rows past
// k are zero).
__global__ __launch_bounds__(256) void k_split_cols_bf16(int k, int KG, int cols, const zf* G,
                                                         int64_t ldg, uint4* planes) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)cols * KG) return;
  const int c = (int)(e / KG), g = (int)(e - (int64_t)c * KG);
  const zf* col = G + (int64_t)c * ldg;
  const int k0 = g * 8;
  float re[8], im[8];
  if (k0 + 8 <= k) {
    const float4* v = (const float4*)(col + k0);
    const float4 v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
    re[0] = v0.x; im[0] = v0.y; re[1] = v0.z; im[1] = v0.w;
    re[2] = v1.x; im[2] = v1.y; re[3] = v1.z; im[3] = v1.w;
    re[4] = v2.x; im[4] = v2.y; re[5] = v2.z; im[5] = v2.w;
    re[6] = v3.x; im[6] = v3.y; re[7] = v3.z; im[7] = v3.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const zf v = (k0 + q < k) ? col[k0 + q] : make_float2(0.f, 0.f);
      re[q] = v.x;
      im[q] = v.y;
    }
  }
  uint4 rh, rl, ih, il;
  split8(re, rh, rl);
  split8(im, ih, il);
  uint4* o = planes + e * 4;
  o[0] = rh;
  o[1] = rl;
  o[2] = ih;
  o[3] = il;
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

namespace {
constexpr int PART_TILES_MAX = 1024;  // partial tiles the workspace holds

// K splits for T tiles of nk slices on `cus` compute units: minimise
// rounds(T s) * ceil(nk / s) plus the reduction's traffic (about 1/40 of a
// slice per partial tile), keeping at least 8 slices per part
int choose_splits(int64_t T, int nk, int cus) {
  int best = 1;
  double best_cost = (double)((T + cus - 1) / cus) * nk;
  for (int s = 2; s <= 8; ++s) {
    const int nks = (nk + s - 1) / s;
    if (nks < 8) break;
    const int se = (nk + nks - 1) / nks;
    if (T * se > PART_TILES_MAX) break;
    const double cost = (double)((T * se + cus - 1) / cus) * nks + 0.025 * (double)(T * se) + 2.0;
    if (cost < 0.95 * best_cost) {
      best = s;
      best_cost = cost;
    }
  }
  return best;
}
}  // namespace

size_t bf16_filter_work_bytes(int64_t k, int64_t cols) {
  const int64_t KG = ((k + 31) / 32) * 4;
  return ws_round((size_t)cols * KG * 64) + ws_round((size_t)PART_TILES_MAX * BM * BN * sizeof(zf));
}

gevp_status launch_cgemm_bf16x3_filter(gevp_ctx* c, int64_t m, int64_t n, int64_t k,
                                       const void* planes, const void* G, int64_t ldg,
                                       const void* P, int64_t ldp, const void* R, int64_t ldr,
                                       void* D, int64_t ldd, const double* al, const double* be,
                                       const double* ga, const double* de, void* work) {
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
  char* wb = (char*)work;
  uint4* bp = (uint4*)wb;
  p.Bp = bp;
  p.part = (zf*)(wb + ws_round((size_t)n * p.KG * 64));
  // the event pair (profiling bit 2) brackets the whole product: the split of
  // the iterate into planes, the product and the split-K reduction
  GEVP_TRY(fev_mark(c));
  // B planes
  {
    const int64_t items = n * (int64_t)p.KG;
    hipLaunchKernelGGL(k_split_cols_bf16, dim3((unsigned)((items + 255) / 256)), dim3(256), 0,
                       c->stream, (int)k, p.KG, (int)n, (const zf*)G, ldg, bp);
    GEVP_HIP_TRY(hipGetLastError());
  }
  p.tiles_n = (int)((n + BN - 1) / BN);
  const int64_t tiles = ((m + BM - 1) / BM) * p.tiles_n;
  const int nk = (p.KG + 3) / 4;
  const int s = c->no_split ? 1 : choose_splits(tiles, nk, std::max(1, gevp_device_cus(c->device) / std::max(1, c->cu_div)));
  p.nks = (nk + s - 1) / s;
  p.splits = (nk + p.nks - 1) / p.nks;
  p.tiles = (int)tiles;
  const int64_t total = tiles * p.splits;
  p.total = (int)total;
  p.remap = (total % 8 == 0 && total >= 64) ? 1 : 0;
  // the stages are static LDS arrays (the 160 KB of a compute unit): no
  // dynamic LDS
  hipLaunchKernelGGL(k_cgemm_bf16x3_filter, dim3((unsigned)total), dim3(512), 0, c->stream, p);
  GEVP_HIP_TRY(hipGetLastError());
  if (p.splits > 1) {
    const int64_t elems = tiles * BM * BN;
    hipLaunchKernelGGL(k_bf16_splitk_reduce, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0,
                       c->stream, p);
    GEVP_HIP_TRY(hipGetLastError());
  }
  GEVP_TRY(fev_mark(c));
  return GEVP_OK;
}
