// Thresholded partial update of a Hermitian matrix between two SCF iterations
// (section 2, paragraph "Matrix generation").
//
// delta = max |A_new(i,j) - A(i,j)| over the stored lower triangle; every lower
// entry whose change exceeds p_t * delta takes A_new's value and the others
// keep A's.  The test is |dA|^2 > (p_t * p_t) * delta^2 with each operation
// rounded on its own (no fused multiply-add anywhere on the decision path), so
// the mask is a fixed FP64 computation, reproducible bit for bit.
//
// Everything streams the lower triangle in 64 x 64 tiles: one work-group of
// four waves per tile, one wave instruction per column segment (64 complex
// entries = 1 KiB contiguous), 16 columns per wave with all loads issued before
// the first use.  The passes are HBM-bound:
//   scan   reads A and A_new (32 bytes per entry), keeps per-tile max and
//          min of |dA|^2 plus a non-finite flag, and writes a 16-bit code per
//          entry: the top 16 bits of the IEEE pattern of |dA|^2, monotone in
//          the value (non-negative doubles order like their bit patterns);
//   delta  (one work-group) reduces the tile maxima to the threshold;
//   apply  skips tiles whose max is at or below the threshold (no matrix
//          traffic), copies tiles whose min is above it without re-reading A,
//          and decides the rest from the codes: a code above the threshold's
//          code means above threshold, below means not, and only entries whose
//          code ties are re-read (both matrices) and compared exactly, so the
//          decisions are those of the plain comparison bit for bit while a
//          mixed tile reads 2 bytes per entry plus A_new where it is taken;
//          the mask words are wave ballots (bit r = row r of the column
//          segment);
//   count  (one work-group) sums the per-tile counts and gathers the result.
// Addresses past the matrix edge (ragged last tile) and above the diagonal of a
// diagonal tile are clamped into the n x n storage and their values discarded,
// so the loads need no branches; only lower-triangle entries are ever written.
// The scan's loads are non-temporal (each byte is read once per pass); the
// apply keeps ordinary loads, which measured faster for the scan that follows.
#include <cfloat>
#include <cstring>

#include "common.h"

namespace {

constexpr int UT = 64;        // tile edge
constexpr int UCOLS = 16;     // columns per wave (4 waves x 16 = 64)
constexpr int UTHREADS = 256;

// |b - a|^2 with every operation rounded separately.
__device__ __forceinline__ double sqdiff(zd a, zd b) {
#pragma clang fp contract(off)
  const double dr = b.x - a.x;
  const double di = b.y - a.y;
  const double r2 = dr * dr;
  const double i2 = di * di;
  return r2 + i2;
}

__device__ __forceinline__ zd load_nt(const zd* p) {
  zd v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}

// linear lower-triangle tile index t -> (bi, bj), bi >= bj, t = bi(bi+1)/2 + bj
__device__ __forceinline__ void tile_of(int64_t t, int64_t& bi, int64_t& bj) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > t) --r;
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  bi = r;
  bj = t - r * (r + 1) / 2;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ unsigned code_of(double s) {
  return (unsigned)((unsigned long long)__double_as_longlong(s) >> 48);
}

__global__ __launch_bounds__(UTHREADS) void k_upd_scan(int64_t n, const zd* __restrict__ A,
                                                       int64_t lda, const zd* __restrict__ An,
                                                       int64_t ldn, double* __restrict__ tmax,
                                                       double* __restrict__ tmin,
                                                       int* __restrict__ tbad,
                                                       uint16_t* __restrict__ code) {
  uint16_t* tc = code + (size_t)blockIdx.x * UT * UT;
  __shared__ double smx[4], smn[4];
  __shared__ int sbad[4];
  int64_t bi, bj;
  tile_of(blockIdx.x, bi, bj);
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = bi * UT + l;
  const int64_t ic = i < n ? i : n - 1;
  zd a[UCOLS], b[UCOLS];
#pragma unroll
  for (int c = 0; c < UCOLS; ++c) {
    int64_t j = bj * UT + w + 4 * c;
    j = j < n ? j : n - 1;
    a[c] = load_nt(A + ic + j * lda);
    b[c] = load_nt(An + ic + j * ldn);
  }
  double mx = 0.0, mn = DBL_MAX;
  bool bad = false;
#pragma unroll
  for (int c = 0; c < UCOLS; ++c) {
    const int64_t j = bj * UT + w + 4 * c;
    unsigned cd = 0;
    if (i < n && j <= i) {
      const double s = sqdiff(a[c], b[c]);
      if (!(s <= DBL_MAX)) {
        bad = true;  // NaN or overflow
      } else {
        mx = fmax(mx, s);
        mn = fmin(mn, s);
        cd = code_of(s);
      }
    }
    tc[(w + 4 * c) * UT + l] = (uint16_t)cd;
  }
  mx = wave_max(mx);
  mn = wave_min(mn);
  const bool wbad = __ballot(bad) != 0;
  if (l == 0) {
    smx[w] = mx;
    smn[w] = mn;
    sbad[w] = wbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tmax[blockIdx.x] = fmax(fmax(smx[0], smx[1]), fmax(smx[2], smx[3]));
    tmin[blockIdx.x] = fmin(fmin(smn[0], smn[1]), fmin(smn[2], smn[3]));
    tbad[blockIdx.x] = sbad[0] | sbad[1] | sbad[2] | sbad[3];
  }
}

// scal[0] = max |dA|^2, scal[1] = threshold (p_t*p_t) * scal[0],
// scal[2] = delta = sqrt(scal[0]); flag[0] = non-finite change seen
__global__ __launch_bounds__(1024) void k_upd_delta(int64_t tiles, const double* __restrict__ tmax,
                                                    const int* __restrict__ tbad, double p_t,
                                                    double* __restrict__ scal, int* __restrict__ flag) {
  __shared__ double sm[16];
  __shared__ int sb[16];
  double mx = 0.0;
  int bad = 0;
  for (int64_t t = threadIdx.x; t < tiles; t += 1024) {
    mx = fmax(mx, tmax[t]);
    bad |= tbad[t];
  }
  mx = wave_max(mx);
  const bool wbad = __ballot(bad != 0) != 0;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (l == 0) {
    sm[w] = mx;
    sb[w] = wbad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    int b = 0;
    for (int k = 0; k < 16; ++k) {
      m = fmax(m, sm[k]);
      b |= sb[k];
    }
    const double pp = p_t * p_t;
    scal[0] = m;
    scal[1] = pp * m;
    scal[2] = sqrt(m);
    flag[0] = b;
  }
}

// Writes mask words of one column segment from a wave ballot.
__device__ __forceinline__ void put_mask(uint32_t* mask, int64_t ldmask, int64_t n, int64_t bi,
                                         int64_t j, uint64_t bits, int l) {
  if (l == 0) mask[j * ldmask + 2 * bi] = (uint32_t)bits;
  if (l == 32 && bi * UT + 32 < n) mask[j * ldmask + 2 * bi + 1] = (uint32_t)(bits >> 32);
}

// kind[t]: 0 nothing updated, 1 entry-by-entry, 2 copied whole.  A tile below
// the diagonal also clears the mask words of its mirror tile above the
// diagonal (bits that are never set), so every word of rows < n is written.
__global__ __launch_bounds__(UTHREADS) void k_upd_apply(
    int64_t n, zd* __restrict__ A, int64_t lda, const zd* __restrict__ An, int64_t ldn,
    const double* __restrict__ tmax, const double* __restrict__ tmin, const double* __restrict__ scal,
    const int* __restrict__ flag, uint32_t* __restrict__ mask, int64_t ldmask, int* __restrict__ tcnt,
    int* __restrict__ tkind, const uint16_t* __restrict__ code, int* __restrict__ tamb) {
  __shared__ int scnt[4], samb[4];
  int64_t bi, bj;
  tile_of(blockIdx.x, bi, bj);
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = bi * UT + l;
  const double thr = scal[1];
  const bool none = flag[0] != 0 || !(tmax[blockIdx.x] > thr);
  const bool all = !none && tmin[blockIdx.x] > thr;
  if (mask && bi > bj && threadIdx.x < 2 * UT) {
    const int64_t jm = bi * UT + (threadIdx.x >> 1);
    if (jm < n) mask[jm * ldmask + 2 * bj + (threadIdx.x & 1)] = 0u;
  }
  int cnt = 0, amb = 0;
  if (none) {
    if (mask) {
#pragma unroll 4
      for (int c = 0; c < UCOLS; ++c) {
        const int64_t j = bj * UT + w + 4 * c;
        if (j < n) put_mask(mask, ldmask, n, bi, j, 0ull, l);
      }
    }
  } else if (all) {
    const int64_t ic = i < n ? i : n - 1;
    zd b[UCOLS];
#pragma unroll
    for (int c = 0; c < UCOLS; ++c) {
      int64_t j = bj * UT + w + 4 * c;
      j = j < n ? j : n - 1;
      b[c] = An[ic + j * ldn];
    }
#pragma unroll
    for (int c = 0; c < UCOLS; ++c) {
      const int64_t j = bj * UT + w + 4 * c;
      const bool ok = i < n && j <= i;
      if (ok) A[i + j * lda] = b[c];
      const uint64_t bits = __ballot(ok);
      cnt += __popcll(bits);
      if (mask && j < n) put_mask(mask, ldmask, n, bi, j, bits, l);
    }
  } else {
    // decide from the codes; loads only where needed (A_new when the code is
    // at or above the threshold's, A as well on a tie); lanes that need no
    // entry read the tile's first one, a single shared address
    const uint16_t* tc = code + (size_t)blockIdx.x * UT * UT;
    const unsigned ct = code_of(thr);
    const int64_t ic = i < n ? i : n - 1;
    const int64_t safe_a = bi * UT + bj * UT * lda, safe_n = bi * UT + bj * UT * ldn;
    unsigned cd[UCOLS];
#pragma unroll
    for (int c = 0; c < UCOLS; ++c) cd[c] = tc[(w + 4 * c) * UT + l];
    zd a[UCOLS], b[UCOLS];
#pragma unroll
    for (int c = 0; c < UCOLS; ++c) {
      int64_t j = bj * UT + w + 4 * c;
      const bool valid = i < n && j <= i;
      j = j < n ? j : n - 1;
      b[c] = An[(valid && cd[c] >= ct) ? ic + j * ldn : safe_n];
      a[c] = A[(valid && cd[c] == ct) ? ic + j * lda : safe_a];
    }
#pragma unroll
    for (int c = 0; c < UCOLS; ++c) {
      const int64_t j = bj * UT + w + 4 * c;
      const bool valid = i < n && j <= i;
      const bool tie = valid && cd[c] == ct;
      const bool ok = valid && (cd[c] > ct || (tie && sqdiff(a[c], b[c]) > thr));
      amb += tie ? 1 : 0;
      if (ok) A[i + j * lda] = b[c];
      const uint64_t bits = __ballot(ok);
      cnt += __popcll(bits);
      if (mask && j < n) put_mask(mask, ldmask, n, bi, j, bits, l);
    }
  }
  amb = (int)wave_sum_int(amb);
  if (l == 0) {
    scnt[w] = cnt;
    samb[w] = amb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    tcnt[blockIdx.x] = scnt[0] + scnt[1] + scnt[2] + scnt[3];
    tkind[blockIdx.x] = none ? 0 : (all ? 2 : 1);
    tamb[blockIdx.x] = samb[0] + samb[1] + samb[2] + samb[3];
  }
}

// out[0] = entries updated, out[1] = tiles with any update, out[2] = tiles
// copied whole, out[3] = the non-finite flag, out[4] = delta's bits, out[5] =
// entries decided by an exact re-check: the whole result in one block for a
// single copy to the host
__global__ __launch_bounds__(1024) void k_upd_count(int64_t tiles, const int* __restrict__ tcnt,
                                                    const int* __restrict__ tkind,
                                                    const int* __restrict__ tamb,
                                                    const double* __restrict__ scal,
                                                    const int* __restrict__ flag,
                                                    long long* __restrict__ out) {
  __shared__ long long s0[16], s1[16], s2[16], s3[16];
  long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  for (int64_t t = threadIdx.x; t < tiles; t += 1024) {
    c0 += tcnt[t];
    c1 += tcnt[t] > 0;
    c2 += tkind[t] == 2;
    c3 += tamb[t];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c0 += __shfl_xor(c0, o, 64);
    c1 += __shfl_xor(c1, o, 64);
    c2 += __shfl_xor(c2, o, 64);
    c3 += __shfl_xor(c3, o, 64);
  }
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (l == 0) {
    s0[w] = c0;
    s1[w] = c1;
    s2[w] = c2;
    s3[w] = c3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long a = 0, b = 0, c = 0, d = 0;
    for (int k = 0; k < 16; ++k) {
      a += s0[k];
      b += s1[k];
      c += s2[k];
      d += s3[k];
    }
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = flag[0];
    out[4] = __double_as_longlong(scal[2]);
    out[5] = d;
  }
}

// Masked update: lower entries whose mask bit is set take S's value.
__global__ __launch_bounds__(UTHREADS) void k_upd_masked(int64_t n, zd* __restrict__ A, int64_t lda,
                                                         const zd* __restrict__ S, int64_t lds,
                                                         const uint32_t* __restrict__ mask,
                                                         int64_t ldmask) {
  int64_t bi, bj;
  tile_of(blockIdx.x, bi, bj);
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t i = bi * UT + l;
  const int64_t word = 2 * bi + (l >> 5);
  const bool row_ok = i < n;
  uint32_t mw[UCOLS];
#pragma unroll
  for (int c = 0; c < UCOLS; ++c) {
    const int64_t j = bj * UT + w + 4 * c;
    mw[c] = (row_ok && j < n) ? mask[j * ldmask + word] : 0u;
  }
#pragma unroll
  for (int c = 0; c < UCOLS; ++c) {
    const int64_t j = bj * UT + w + 4 * c;
    if (row_ok && j <= i && ((mw[c] >> (l & 31)) & 1u)) A[i + j * lda] = S[i + j * lds];
  }
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

gevp_status gevp_update_thresholded(gevp_handle h, int64_t n, void* A_, int64_t lda,
                                    const void* An_, int64_t ldn, double p_t, uint32_t* mask,
                                    int64_t ldmask, gevp_update_info* info) {
  if (!h || n < 0 || !(p_t >= 0.0) || !(p_t <= DBL_MAX)) return GEVP_ERR_INVALID;
  const int64_t nt = (n + UT - 1) / UT;
  const int64_t tiles = nt * (nt + 1) / 2;
  if (info) {
    *info = gevp_update_info{};
    info->entries = n * (n + 1) / 2;
    info->tiles = tiles;
  }
  if (n == 0) return GEVP_OK;
  if (!A_ || !An_ || lda < n || ldn < n || !aligned16(A_) || !aligned16(An_))
    return GEVP_ERR_INVALID;
  const int64_t words = (n + 31) / 32;
  if (mask && (ldmask < words || ((uintptr_t)mask & 3))) return GEVP_ERR_INVALID;
  if (tiles > INT32_MAX || n > INT32_MAX) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  const size_t need = 2 * ws_round(sizeof(double) * tiles) + 4 * ws_round(sizeof(int) * tiles) +
                      ws_round(sizeof(uint16_t) * UT * UT * (size_t)tiles) +
                      ws_round(sizeof(double) * 4) + ws_round(sizeof(int) * 4) +
                      ws_round(sizeof(long long) * 8) + 256;
  GEVP_TRY(ws_reserve(h, need));
  double* tmax = (double*)ws_take(h, sizeof(double) * tiles);
  double* tmin = (double*)ws_take(h, sizeof(double) * tiles);
  int* tbad = (int*)ws_take(h, sizeof(int) * tiles);
  int* tcnt = (int*)ws_take(h, sizeof(int) * tiles);
  int* tkind = (int*)ws_take(h, sizeof(int) * tiles);
  int* tamb = (int*)ws_take(h, sizeof(int) * tiles);
  uint16_t* code = (uint16_t*)ws_take(h, sizeof(uint16_t) * UT * UT * (size_t)tiles);
  double* scal = (double*)ws_take(h, sizeof(double) * 4);
  int* flag = (int*)ws_take(h, sizeof(int) * 4);
  long long* out = (long long*)ws_take(h, sizeof(long long) * 8);
  zd* A = (zd*)A_;
  const zd* An = (const zd*)An_;
  // profiling flag 2: event pairs around the scan and the apply launch
  const bool timed = (h->profiling & 2) && info;
  if (timed) {
    h->fev_used = 0;
    GEVP_TRY(fev_mark(h));
  }
  hipLaunchKernelGGL(k_upd_scan, dim3((unsigned)tiles), dim3(UTHREADS), 0, h->stream, n, A, lda,
                     An, ldn, tmax, tmin, tbad, code);
  GEVP_HIP_TRY(hipGetLastError());
  if (timed) GEVP_TRY(fev_mark(h));
  hipLaunchKernelGGL(k_upd_delta, dim3(1), dim3(1024), 0, h->stream, tiles, tmax, tbad, p_t, scal,
                     flag);
  if (timed) GEVP_TRY(fev_mark(h));
  hipLaunchKernelGGL(k_upd_apply, dim3((unsigned)tiles), dim3(UTHREADS), 0, h->stream, n, A, lda,
                     An, ldn, tmax, tmin, scal, flag, mask, ldmask, tcnt, tkind, code, tamb);
  GEVP_HIP_TRY(hipGetLastError());
  if (timed) GEVP_TRY(fev_mark(h));
  if (!info) return GEVP_OK;
  hipLaunchKernelGGL(k_upd_count, dim3(1), dim3(1024), 0, h->stream, tiles, tcnt, tkind, tamb, scal,
                     flag, out);
  GEVP_HIP_TRY(hipGetLastError());
  long long ho[6];
  GEVP_HIP_TRY(hipMemcpyAsync(ho, out, sizeof(ho), hipMemcpyDeviceToHost, h->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(h->stream));
  if (timed) {
    float ms0 = 0.f, ms1 = 0.f;
    GEVP_HIP_TRY(hipEventElapsedTime(&ms0, h->fev[0], h->fev[1]));
    GEVP_HIP_TRY(hipEventElapsedTime(&ms1, h->fev[2], h->fev[3]));
    info->scan_ms = ms0;
    info->apply_ms = ms1;
    h->fev_used = 0;
  }
  double delta;
  memcpy(&delta, &ho[4], sizeof(delta));
  info->nonfinite = (int)ho[3];
  info->delta = ho[3] ? __builtin_nan("") : delta;
  info->updated = ho[0];
  info->tiles_touched = ho[1];
  info->tiles_copied = ho[2];
  info->rechecked = ho[5];
  return ho[3] ? GEVP_ERR_NONFINITE : GEVP_OK;
}

gevp_status gevp_update_masked(gevp_handle h, int64_t n, void* A_, int64_t lda, const void* S_,
                               int64_t lds, const uint32_t* mask, int64_t ldmask) {
  if (!h || n < 0) return GEVP_ERR_INVALID;
  if (n == 0) return GEVP_OK;
  if (!A_ || !S_ || !mask || lda < n || lds < n) return GEVP_ERR_INVALID;
  if (!aligned16(A_) || !aligned16(S_) || ((uintptr_t)mask & 3)) return GEVP_ERR_INVALID;
  if (ldmask < (n + 31) / 32) return GEVP_ERR_INVALID;
  const int64_t nt = (n + UT - 1) / UT;
  const int64_t tiles = nt * (nt + 1) / 2;
  if (tiles > INT32_MAX) return GEVP_ERR_INVALID;
  GEVP_HIP_TRY(hipSetDevice(h->device));
  hipLaunchKernelGGL(k_upd_masked, dim3((unsigned)tiles), dim3(UTHREADS), 0, h->stream, n, (zd*)A_,
                     lda, (const zd*)S_, lds, mask, ldmask);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

}  // extern "C"
