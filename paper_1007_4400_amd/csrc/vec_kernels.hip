// Bandwidth-bound helper kernels: input mirroring and scans, transposes,
// column norms and residual norms (wave64 reductions), column gathers,
// counter-based random fill, phase normalisation, Hermitian matrix-vector
// products for the Lanczos bounds; and the seed monitor's statistics with
// its angle-minimising matching (one work-group).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum for 256 threads; every thread gets the result
__device__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return s;
}

__device__ __forceinline__ bool finite2(zd v) { return isfinite(v.x) && isfinite(v.y); }

// Full Hermitian copy from the lower triangle, 32 x 32 tiles through LDS so
// the conjugate-transposed half is written coalesced.  Only tiles on or below
// the diagonal are launched.  In place (S == D) the strict lower triangle is
// not written at all, and a diagonal entry only when its imaginary part has
// to be cleared, so other streams may read the lower triangle meanwhile.
__global__ __launch_bounds__(256) void k_mirror_lower(const zd* S, int64_t lds, zd* D, int64_t ldd,
                                                      int64_t n, int* flag) {
  __shared__ zd t[32][33];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const bool inplace = (S == D && lds == ldd);
  bool bad = false;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + tx, j = bj * 32 + r;  // element (i, j), column j
    zd v = make_double2(0.0, 0.0);
    if (i < n && j < n && i >= j) {
      v = S[i + j * lds];
      if (i == j) {
        if (inplace && v.y != 0.0) D[i + j * ldd] = make_double2(v.x, 0.0);
        v.y = 0.0;
      }
      bad |= !finite2(v);
    }
    t[r][tx] = v;  // t[col][row]
  }
  __syncthreads();
  if (!inplace) {
    for (int r = ty; r < 32; r += 8) {
      const int64_t i = bi * 32 + tx, j = bj * 32 + r;
      if (i < n && j < n && i >= j) D[i + j * ldd] = t[r][tx];
    }
  }
  // conjugate transpose: D(j, i) = conj(S(i, j)) for i > j
  for (int r = ty; r < 32; r += 8) {
    const int64_t row = bj * 32 + tx, col = bi * 32 + r;  // D(row, col), row < col
    if (row < n && col < n && row < col) {
      const zd v = t[tx][r];
      D[row + col * ldd] = make_double2(v.x, -v.y);
    }
  }
  if (bad && flag) atomicOr(flag, 1);
}

__global__ void k_copy2d(int64_t rows, int64_t cols, const zd* S, int64_t lds, zd* D, int64_t ldd) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    D[i + j * ldd] = S[i + j * lds];
}

__global__ void k_check_finite(int64_t rows, const zd* S, int64_t lds, int* flag) {
  const int64_t j = blockIdx.y;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !finite2(S[i + j * lds]);
  if (bad) atomicOr(flag, 1);
}

// splitmix64 finaliser: counter-based, so every (seed, column, row) maps to a
// fixed value regardless of the launch shape
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_randn(int64_t rows, zd* V, int64_t ldv, int64_t col_offset, uint64_t seed) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = mix64(seed ^ mix64((uint64_t)(j + col_offset) * 0x100000001B3ull)) ^ (uint64_t)i;
    const uint64_t r1 = mix64(key), r2 = mix64(key ^ 0xD1B54A32D192ED03ull);
    const double u1 = ((r1 >> 11) + 1) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (r2 >> 11) * (1.0 / 9007199254740992.0);
    const double rad = sqrt(-log(u1));  // E|z|^2 = 1
    double s, co;
    sincos(6.283185307179586 * u2, &s, &co);
    V[i + j * ldv] = make_double2(rad * co, rad * s);
  }
}

// one work-group per column: v <- v / ||v|| (an all-zero column becomes a unit
// pseudo-random one)
__global__ __launch_bounds__(256) void k_colnorm_scale(int64_t rows, zd* V, int64_t ldv) {
  __shared__ double sh[4];
  zd* v = V + blockIdx.x * ldv;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) s += v[i].x * v[i].x + v[i].y * v[i].y;
  s = block_sum256(s, sh);
  if (s == 0.0) {
    // an all-zero column can never be orthonormalised (the shifted Cholesky
    // keeps it zero): replace it by a fixed pseudo-random direction, as a
    // missing seed vector is replaced in subspace iteration
    const uint64_t key = mix64(0x5EEDC01Dull ^ mix64((uint64_t)blockIdx.x * 0x100000001B3ull));
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
      const uint64_t r1 = mix64(key ^ (uint64_t)i), r2 = mix64(key ^ (uint64_t)i ^ 0xD1B54A32D192ED03ull);
      const zd z = make_double2((r1 >> 11) * (1.0 / 9007199254740992.0) - 0.5,
                                (r2 >> 11) * (1.0 / 9007199254740992.0) - 0.5);
      v[i] = z;
      s += z.x * z.x + z.y * z.y;
    }
    s = block_sum256(s, sh);
  }
  if (s > 0.0) {
    const double inv = 1.0 / sqrt(s);
    for (int64_t i = threadIdx.x; i < rows; i += 256) v[i] = make_double2(v[i].x * inv, v[i].y * inv);
  }
}

__global__ __launch_bounds__(256) void k_colnorms(int64_t rows, const zd* V, int64_t ldv, double* out) {
  __shared__ double sh[4];
  const zd* v = V + blockIdx.x * ldv;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) s += v[i].x * v[i].x + v[i].y * v[i].y;
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

// r_j = || W_j - theta_j V_j ||_2
__global__ __launch_bounds__(256) void k_resid_cols(int64_t rows, const zd* W, int64_t ldw,
                                                    const zd* V, int64_t ldv, const double* theta,
                                                    double* out) {
  __shared__ double sh[4];
  const int64_t j = blockIdx.x;
  const zd* w = W + j * ldw;
  const zd* v = V + j * ldv;
  const double th = theta[j];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double rx = w[i].x - th * v[i].x, ry = w[i].y - th * v[i].y;
    s += rx * rx + ry * ry;
  }
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

// Seed monitor, per column j of the k x k cross-overlap M: sum_i |M(i,j)|^2,
// max_i |M(i,j)| and its row (lowest row on ties).
__global__ __launch_bounds__(256) void k_seed_cols(int k, const zd* M, int64_t ldm, double* stat) {
  __shared__ double ss[256], sm[256];
  __shared__ int si[256];
  const int j = blockIdx.x, t = threadIdx.x;
  const zd* col = M + (int64_t)j * ldm;
  double s2 = 0.0, mx = -1.0;
  int arg = 0;
  for (int i = t; i < k; i += 256) {
    const double a = col[i].x * col[i].x + col[i].y * col[i].y;
    s2 += a;
    if (a > mx) {
      mx = a;
      arg = i;
    }
  }
  ss[t] = s2;
  sm[t] = mx;
  si[t] = arg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      ss[t] += ss[t + w];
      if (sm[t + w] > sm[t] || (sm[t + w] == sm[t] && si[t + w] < si[t])) {
        sm[t] = sm[t + w];
        si[t] = si[t + w];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    stat[3 * j] = ss[0];
    stat[3 * j + 1] = sqrt(fmax(sm[0], 0.0));
    stat[3 * j + 2] = (double)si[0];
  }
}

constexpr int SEED_K_MAX = 8192;  // columns of the seed monitor

// Seed monitor totals.  out[0] sin_rms: sqrt(sum_j rnorm[j]^2 / k) when the
// norms of the projection residuals R = X0 - P X0 (P the orthogonal projector
// onto the result's span) are given, else sqrt(max(0, k - ||M||_F^2) / k)
// from M alone (which loses its digits to cancellation below about 1e-8);
// out[1] mean and out[2] max of the per-column deviation angles
// acos(min(1, max_i |M(i,j)|)) / (pi/2) (best match per column), out[3]
// columns whose best match is not their own index, out[4] standard deviation
// of the angles, out[5] = 1 when two columns share a best match (the
// per-column matches are then no permutation and k_seed_assign solves the
// assignment).  k <= SEED_K_MAX.
__global__ __launch_bounds__(256) void k_seed_finish(int k, const double* stat, const double* rnorm,
                                                     double* out) {
  __shared__ double sf[256], sd[256], sx[256], sr[256], sq[256];
  __shared__ int hits[SEED_K_MAX];
  __shared__ int clash;
  const int t = threadIdx.x;
  for (int i = t; i < k; i += 256) hits[i] = 0;
  if (t == 0) clash = 0;
  __syncthreads();
  double f = 0.0, d = 0.0, x = 0.0, r = 0.0, q = 0.0;
  for (int j = t; j < k; j += 256) {
    f += rnorm ? rnorm[j] * rnorm[j] : stat[3 * j];
    const double dev = acos(fmin(1.0, stat[3 * j + 1])) * 0.63661977236758134;  // / (pi/2)
    d += dev;
    q += dev * dev;
    x = fmax(x, dev);
    const int best = (int)stat[3 * j + 2];
    r += (best != j) ? 1.0 : 0.0;
    if (atomicAdd(&hits[best], 1) > 0) clash = 1;
  }
  sf[t] = f;
  sd[t] = d;
  sx[t] = x;
  sr[t] = r;
  sq[t] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sf[t] += sf[t + w];
      sd[t] += sd[t + w];
      sx[t] = fmax(sx[t], sx[t + w]);
      sr[t] += sr[t + w];
      sq[t] += sq[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double mean = sd[0] / (double)k;
    out[0] = rnorm ? sqrt(sf[0] / (double)k) : sqrt(fmax(0.0, (double)k - sf[0]) / (double)k);
    out[1] = mean;
    out[2] = sx[0];
    out[3] = sr[0];
    out[4] = sqrt(fmax(0.0, sq[0] / (double)k - mean * mean));
    out[5] = clash ? 1.0 : 0.0;
  }
}

// When two result columns share a best-matching seed column (out[5] set by
// k_seed_finish), the re-indexing is the angle-minimising assignment: a
// minimum-cost perfect matching on the deviation angles acos|M(i, j)| (row:
// result column j, column: seed column i), solved by shortest augmenting
// paths with row and column potentials (Kuhn-Munkres, O(k^3)) in one
// work-group: rows are added one at a time, and every step of a path scans
// the columns in parallel and takes the smallest reduced cost (ties to the
// lowest column).  The matching replaces the best matches in stat[3 j + 2],
// and the deviation statistics out[1..4] are recomputed from it.  Without a
// clash the kernel returns at once.  The six work arrays (k + 1 entries each)
// sit in LDS up to ASG_LDS_K columns and in a device buffer beyond.
constexpr int ASG_T = 1024;
constexpr int ASG_LDS_K = 4096;
constexpr size_t asg_bytes(int64_t k) { return (size_t)(k + 1) * (3 * sizeof(double) + 3 * sizeof(int)); }
template <bool GLB>
__global__ __launch_bounds__(ASG_T) void k_seed_assign(int k, const zd* M, int64_t ldm, double* stat,
                                                       double* out, double* gbuf) {
  if (out[5] == 0.0) return;  // uniform: every best match is distinct
  extern __shared__ double asg_lds[];
  double* asg = GLB ? gbuf : asg_lds;
  double* u = asg;                       // k + 1 row potentials (1-based rows)
  double* v = u + (k + 1);               // k + 1 column potentials
  double* minv = v + (k + 1);            // k + 1
  int* row_of = (int*)(minv + (k + 1));  // k + 1; column 0 is the sentinel
  int* way = row_of + (k + 1);           // k + 1
  int* used = way + (k + 1);             // k + 1
  __shared__ double rv[ASG_T / 64];
  __shared__ int rc[ASG_T / 64];
  __shared__ int c0s;
  __shared__ double deltas;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  constexpr int NONE = 0x7fffffff;
  // (value, column) order of the path step: a real column before none, then
  // the smaller value, then the smaller column
  auto better = [](double a, int ca, double b, int cb) {
    return ca != NONE && (cb == NONE || a < b || (a == b && ca < cb));
  };
  auto cost = [&](int r, int c) {  // 1-based row r (result column), column c (seed column)
    const zd m = M[(int64_t)(r - 1) * ldm + (c - 1)];
    return acos(fmin(1.0, sqrt(m.x * m.x + m.y * m.y)));
  };
  for (int c = t; c <= k; c += ASG_T) {
    u[c] = 0.0;
    v[c] = 0.0;
    row_of[c] = 0;
    way[c] = 0;
  }
  __syncthreads();
  for (int r = 1; r <= k; ++r) {
    for (int c = t; c <= k; c += ASG_T) {
      minv[c] = 1e300;
      used[c] = 0;
    }
    if (t == 0) {
      row_of[0] = r;
      c0s = 0;
    }
    __syncthreads();
    for (;;) {
      const int c0 = c0s;
      if (t == 0) used[c0] = 1;
      __syncthreads();
      const int r0 = row_of[c0];
      // reduced costs of row r0, and the smallest over the unused columns
      double best = 1e300;
      int bc = NONE;
      for (int c = 1 + t; c <= k; c += ASG_T) {
        if (used[c]) continue;
        const double cur = cost(r0, c) - u[r0] - v[c];
        if (cur < minv[c]) {
          minv[c] = cur;
          way[c] = c0;
        }
        // c increases along this thread's columns; any unused column is a
        // valid pick, so a non-finite cost cannot leave the path without one
        if (bc == NONE || minv[c] < best) {
          best = minv[c];
          bc = c;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oc = __shfl_xor(bc, o, 64);
        if (better(ob, oc, best, bc)) {
          best = ob;
          bc = oc;
        }
      }
      if (lane == 0) {
        rv[wave] = best;
        rc[wave] = bc;
      }
      __syncthreads();
      if (t == 0) {
        double b = rv[0];
        int cc = rc[0];
        for (int w = 1; w < ASG_T / 64; ++w)
          if (better(rv[w], rc[w], b, cc)) {
            b = rv[w];
            cc = rc[w];
          }
        deltas = b;
        c0s = cc;
      }
      __syncthreads();
      const double delta = deltas;
      for (int c = t; c <= k; c += ASG_T) {
        if (used[c]) {
          u[row_of[c]] += delta;
          v[c] -= delta;
        } else {
          minv[c] -= delta;
        }
      }
      __syncthreads();
      const bool free_col = row_of[c0s] == 0;  // uniform: c0s and row_of[] are shared
      __syncthreads();                         // read by all before the path is flipped
      if (free_col) break;
    }
    if (t == 0) {  // flip the augmenting path
      int c0 = c0s;
      do {
        const int c1 = way[c0];
        row_of[c0] = row_of[c1];
        c0 = c1;
      } while (c0 != 0);
    }
    __syncthreads();
  }
  // the matching (seed column of result column j) and its statistics
  __shared__ double sd[ASG_T / 64], sq[ASG_T / 64], sx[ASG_T / 64], sr[ASG_T / 64];
  double d = 0.0, q = 0.0, x = 0.0, re = 0.0;
  for (int c = 1 + t; c <= k; c += ASG_T) {
    const int j = row_of[c] - 1, i = c - 1;  // result column j takes seed column i
    stat[3 * j + 2] = (double)i;
    const double dv = cost(j + 1, c) * 0.63661977236758134;  // / (pi/2)
    d += dv;
    q += dv * dv;
    x = fmax(x, dv);
    re += (i != j) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    d += __shfl_xor(d, o, 64);
    q += __shfl_xor(q, o, 64);
    x = fmax(x, __shfl_xor(x, o, 64));
    re += __shfl_xor(re, o, 64);
  }
  if (lane == 0) {
    sd[wave] = d;
    sq[wave] = q;
    sx[wave] = x;
    sr[wave] = re;
  }
  __syncthreads();
  if (t == 0) {
    double D = 0.0, Q = 0.0, X = 0.0, R = 0.0;
    for (int w = 0; w < ASG_T / 64; ++w) {
      D += sd[w];
      Q += sq[w];
      X = fmax(X, sx[w]);
      R += sr[w];
    }
    const double mean = D / (double)k;
    out[1] = mean;
    out[2] = X;
    out[3] = R;
    out[4] = sqrt(fmax(0.0, Q / (double)k - mean * mean));
  }
}

// Locked columns after a filter sweep: entries j < nl of theta and resid
// become those of column perm[j] (in place, through LDS; nb <= 2048).
__global__ __launch_bounds__(256) void k_permute_prefix(double* theta, double* resid, const int* perm,
                                                        int nl) {
  __shared__ double st[2048], sr[2048];
  for (int j = threadIdx.x; j < nl; j += 256) {
    st[j] = theta[perm[j]];
    sr[j] = resid[perm[j]];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nl; j += 256) {
    theta[j] = st[j];
    resid[j] = sr[j];
  }
}

// Stable merge of the two ascending runs theta[0, nl) and theta[nl, nb):
// position of entry j in the merged order (runs of equal values keep the
// first run first); theta and resid are rewritten in merged order and
// order[p] = j is the column that lands at position p.  One work-group,
// nb <= 2048.
__global__ __launch_bounds__(256) void k_merge_runs(double* theta, double* resid, int nb, int nl,
                                                    int* order) {
  __shared__ double st[2048], sr[2048];
  for (int j = threadIdx.x; j < nb; j += 256) {
    st[j] = theta[j];
    sr[j] = resid[j];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nb; j += 256) {
    const double v = st[j];
    int lo, hi, base;
    if (j < nl) {  // entries of the second run strictly below v
      lo = nl;
      hi = nb;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st[mid] < v) lo = mid + 1; else hi = mid;
      }
      base = j + (lo - nl);
    } else {  // entries of the first run at or below v
      lo = 0;
      hi = nl;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st[mid] <= v) lo = mid + 1; else hi = mid;
      }
      base = (j - nl) + lo;
    }
    order[base] = j;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < nb; p += 256) {
    const int j = order[p];
    theta[p] = st[j];
    resid[p] = sr[j];
  }
}

__global__ void k_gather_cols(int64_t rows, const zd* S, int64_t lds, const int* perm, zd* D,
                              int64_t ldd) {
  const int64_t j = blockIdx.y;
  const zd* s = S + (int64_t)perm[j] * lds;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x)
    D[i + j * ldd] = s[i];
}

__global__ void k_scale_cols(int64_t rows, const zd* S, int64_t lds, const double* w, zd* D,
                             int64_t ldd) {
  const int64_t j = blockIdx.y;
  const double a = w[j];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const zd v = S[i + j * lds];
    D[i + j * ldd] = make_double2(a * v.x, a * v.y);
  }
}

// Largest-modulus entry of each column made real and positive (lowest index
// among entries within 1e-12 relative of the maximum).
__global__ __launch_bounds__(256) void k_phase_normalize(int64_t rows, zd* X, int64_t ldx) {
  __shared__ double shm[256];
  __shared__ int shi[256];
  zd* x = X + blockIdx.x * ldx;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) m = fmax(m, hypot(x[i].x, x[i].y));
  shm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + s]);
    __syncthreads();
  }
  const double amax = shm[0];
  __syncthreads();
  int best = INT32_MAX;
  for (int64_t i = threadIdx.x; i < rows; i += 256)
    if (hypot(x[i].x, x[i].y) >= amax * (1.0 - 1e-12)) {
      best = (int)i;
      break;
    }
  shi[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) shi[threadIdx.x] = min(shi[threadIdx.x], shi[threadIdx.x + s]);
    __syncthreads();
  }
  const int piv = shi[0];
  if (amax == 0.0 || piv == INT32_MAX) return;
  const zd p = x[piv];
  const double a = hypot(p.x, p.y);
  const double cr = p.x / a, ci = -p.y / a;  // conj(p)/|p|
  __syncthreads();
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const zd v = x[i];
    x[i] = make_double2(v.x * cr - v.y * ci, v.x * ci + v.y * cr);
  }
}

// y = M x for a Hermitian M stored in full, reading only the 64 x 64 tiles on
// and below the diagonal: the tile (I, J), I > J, gives y_I += T x_J and
// y_J += T^H x_I, a diagonal tile y_I += T x_I.  One work-group per tile
// (lane = row, each wave 16 columns, loads first) writes its two partial
// 64-vectors; k_hemv_reduce sums, for every block I, the partials of the
// tiles in block row I and block column I.  Half the bytes of a column-by-
// column product.
constexpr int HV = 64;  // tile order
__device__ __forceinline__ int64_t hv_pair(int64_t I, int64_t J) { return I * (I + 1) / 2 + J; }

__global__ __launch_bounds__(256) void k_hemv_tiles(int64_t n, const zd* M, int64_t ldm, const zd* x,
                                                    zd* P1, zd* P2) {
  __shared__ zd xs[2][HV];
  __shared__ zd ys[4][HV];
  const int64_t p = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > p) --I;  // correct the rounding of the root
  while ((I + 1) * (I + 2) / 2 <= p) ++I;
  const int64_t J = p - I * (I + 1) / 2;
  const int64_t r0 = I * HV, c0 = J * HV;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // every global load of the tile in flight before the first is used: the
  // matrix entries (indices clamped into the matrix, out-of-range entries
  // zeroed after the load) and the two slices of x
  const int64_t row = r0 + lane, rowc = min(row, n - 1);
  zd a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t col = c0 + wave * 16 + q;
    a[q] = M[rowc + min(col, n - 1) * ldm];
  }
  const zd xj = x[min(c0 + lane, n - 1)], xi = x[min(r0 + lane, n - 1)];
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (row >= n || c0 + wave * 16 + q >= n) a[q] = make_double2(0.0, 0.0);
  if (tid < HV) {
    xs[0][tid] = (c0 + tid < n) ? xj : make_double2(0.0, 0.0);  // x_J
    xs[1][tid] = (r0 + tid < n) ? xi : make_double2(0.0, 0.0);  // x_I
  }
  __syncthreads();
  // y_I partial: the lane's row over the wave's 16 columns
  double yr = 0.0, yi = 0.0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const zd v = xs[0][wave * 16 + q];
    yr += a[q].x * v.x - a[q].y * v.y;
    yi += a[q].x * v.y + a[q].y * v.x;
  }
  ys[wave][lane] = make_double2(yr, yi);
  if (I != J) {
    // y_J partial for the wave's 16 columns: sum over the 64 rows of
    // conj(T(r, c)) x_I(r), a reduce-scatter over the lanes (after the four
    // halving steps lane l holds column (l >> 2) summed over 16 lanes)
    const zd xi = xs[1][lane];
    double vr[16], vi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      vr[q] = a[q].x * xi.x + a[q].y * xi.y;
      vi[q] = a[q].x * xi.y - a[q].y * xi.x;
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int o = 32 >> st, m = 16 >> st, h = m >> 1;
      const bool up = (lane & o) != 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q < h) {
          const double sr = up ? vr[q] : vr[q + h], si = up ? vi[q] : vi[q + h];
          const double kr = up ? vr[q + h] : vr[q], ki = up ? vi[q + h] : vi[q];
          vr[q] = kr + __shfl_xor(sr, o, 64);
          vi[q] = ki + __shfl_xor(si, o, 64);
        }
      }
    }
    double tr = vr[0], ti = vi[0];
    tr += __shfl_xor(tr, 2, 64);
    ti += __shfl_xor(ti, 2, 64);
    tr += __shfl_xor(tr, 1, 64);
    ti += __shfl_xor(ti, 1, 64);
    if ((lane & 3) == 0) P2[p * HV + wave * 16 + (lane >> 2)] = make_double2(tr, ti);
  }
  __syncthreads();
  if (tid < HV) {
    zd t = ys[0][tid];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      t.x += ys[w][tid].x;
      t.y += ys[w][tid].y;
    }
    P1[p * HV + tid] = t;
  }
}

// y_I = sum over the partials of block row I (tiles (I, J), J <= I) and of
// block column I (tiles (K, I), K > I): nbk terms per row, split over four
// thread groups, each with eight loads in flight.
__global__ __launch_bounds__(256) void k_hemv_reduce(int64_t n, int64_t nbk, const zd* P1, const zd* P2,
                                                     zd* y) {
  __shared__ zd part[4][HV];
  const int64_t I = blockIdx.x;
  const int r = threadIdx.x & (HV - 1), g = threadIdx.x >> 6;
  double sr = 0.0, si = 0.0;
  for (int64_t k0 = g; k0 < nbk; k0 += 4 * 8) {
    zd v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t k = min(k0 + 4 * u, nbk - 1);  // clamped: every load valid
      v[u] = (k <= I) ? P1[hv_pair(I, k) * HV + r] : P2[hv_pair(k, I) * HV + r];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + 4 * u < nbk) {
        sr += v[u].x;
        si += v[u].y;
      }
  }
  part[g][r] = make_double2(sr, si);
  __syncthreads();
  if (g == 0 && I * HV + r < n) {
    const zd a = part[0][r], b = part[1][r], c = part[2][r], d = part[3][r];
    y[I * HV + r] = make_double2(a.x + b.x + c.x + d.x, a.y + b.y + c.y + d.y);
  }
}

__global__ void k_add_diag(int64_t n, zd* M, int64_t ldm, const double* shift) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) M[i + i * ldm].x += shift[0];
}

__global__ void k_copy_real(int64_t n, const double* s, double* d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// out[0] = max_ij |M(i,j) - delta_ij| (one work-group)
// max |M - I| over all entries; a non-finite entry gives +inf (fmax alone
// would drop a NaN), so a block with NaN never passes a tolerance test
// max |M - I| over the lower triangle of a Hermitian M (the upper triangle is
// not read): one partial maximum per work-group, columns dealt round-robin
__global__ __launch_bounds__(256) void k_max_offident(int64_t n, const zd* M, int64_t ldm, double* part) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
    for (int64_t i = j + threadIdx.x; i < n; i += 256) {
      zd v = M[i + j * ldm];
      if (i == j) v.x -= 1.0;
      const double h = hypot(v.x, v.y);
      mx = (h != h) ? INFINITY : fmax(mx, h);
    }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_max_parts(int cnt, const double* part, double* out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < cnt; i += 256) mx = fmax(mx, part[i]);  // partials are never NaN
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

inline unsigned gx(int64_t rows) {
  int64_t b = (rows + 255) / 256;
  return (unsigned)(b < 64 ? (b < 1 ? 1 : b) : 64);
}
}  // namespace

gevp_status launch_mirror_lower(gevp_ctx* c, int64_t n, const zd* S, int64_t lds, zd* D,
                                int64_t ldd, int* flag) {
  if (n <= 0) return GEVP_OK;
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_mirror_lower, dim3(t, t), dim3(256), 0, c->stream, S, lds, D, ldd, n, flag);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_copy2d(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                          zd* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_copy2d, dim3(gx(rows), (unsigned)cols), dim3(256), 0, c->stream, rows, cols,
                     S, lds, D, ldd);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_check_finite(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                                int* flag) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_check_finite, dim3(gx(rows), (unsigned)cols), dim3(256), 0, c->stream, rows,
                     S, lds, flag);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_randn(gevp_ctx* c, int64_t rows, int64_t cols, zd* V, int64_t ldv,
                         int64_t col_offset, unsigned long long seed) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_randn, dim3(gx(rows), (unsigned)cols), dim3(256), 0, c->stream, rows, V, ldv,
                     col_offset, (uint64_t)seed);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_colnorm_scale(gevp_ctx* c, int64_t rows, int64_t cols, zd* V, int64_t ldv) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_colnorm_scale, dim3((unsigned)cols), dim3(256), 0, c->stream, rows, V, ldv);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_colnorms(gevp_ctx* c, int64_t rows, int64_t cols, const zd* V, int64_t ldv,
                            double* out) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_colnorms, dim3((unsigned)cols), dim3(256), 0, c->stream, rows, V, ldv, out);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_resid_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* W, int64_t ldw,
                              const zd* V, int64_t ldv, const double* theta, double* out) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_resid_cols, dim3((unsigned)cols), dim3(256), 0, c->stream, rows, W, ldw, V,
                     ldv, theta, out);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_seed_monitor(gevp_ctx* c, int64_t k, const zd* M, int64_t ldm, double* stat,
                                double* out, const double* rnorm) {
  if (k <= 0) return GEVP_OK;
  if (k > SEED_K_MAX) return GEVP_ERR_INVALID;
  hipLaunchKernelGGL(k_seed_cols, dim3((unsigned)k), dim3(256), 0, c->stream, (int)k, M, ldm, stat);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_seed_finish, dim3(1), dim3(256), 0, c->stream, (int)k, stat, rnorm, out);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status seed_monitor_stats(gevp_ctx* c, int64_t k, const zd* M, int64_t ldm, double* stat,
                               double* out, double res[5], int* match, const double* rnorm,
                               void* scratch, size_t scratch_bytes) {
  GEVP_TRY(launch_seed_monitor(c, k, M, ldm, stat, out, rnorm));
  if (k <= ASG_LDS_K) {
    static const bool attr = [] {
      (void)hipFuncSetAttribute((const void*)k_seed_assign<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)asg_bytes(ASG_LDS_K));
      return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(k_seed_assign<false>, dim3(1), dim3(ASG_T), asg_bytes(k), c->stream, (int)k, M,
                       ldm, stat, out, nullptr);
  } else {
    if (!scratch || scratch_bytes < asg_bytes(k)) return GEVP_ERR_INVALID;
    hipLaunchKernelGGL(k_seed_assign<true>, dim3(1), dim3(ASG_T), 0, c->stream, (int)k, M, ldm, stat,
                       out, (double*)scratch);
  }
  GEVP_HIP_TRY(hipGetLastError());
  double h[6];
  std::vector<double> st(3 * k);
  GEVP_HIP_TRY(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  GEVP_HIP_TRY(hipMemcpyAsync(st.data(), stat, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, c->stream));
  GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 5; ++i) res[i] = h[i];
  if (match)
    for (int64_t j = 0; j < k; ++j) match[j] = (int)st[3 * j + 2];
  return GEVP_OK;
}

gevp_status launch_gather_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                               const int* perm, zd* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_gather_cols, dim3(gx(rows), (unsigned)cols), dim3(256), 0, c->stream, rows,
                     S, lds, perm, D, ldd);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_scale_cols(gevp_ctx* c, int64_t rows, int64_t cols, const zd* S, int64_t lds,
                              const double* w, zd* D, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_scale_cols, dim3(gx(rows), (unsigned)cols), dim3(256), 0, c->stream, rows, S,
                     lds, w, D, ldd);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_phase_normalize(gevp_ctx* c, int64_t rows, int64_t cols, zd* X, int64_t ldx) {
  if (rows <= 0 || cols <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_phase_normalize, dim3((unsigned)cols), dim3(256), 0, c->stream, rows, X, ldx);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

size_t hemv_work_bytes(int64_t n) {
  const int64_t nbk = (n + HV - 1) / HV;
  return 2 * ws_round(sizeof(zd) * HV * (size_t)(nbk * (nbk + 1) / 2));
}

gevp_status launch_hemv(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, const zd* x, zd* y,
                        void* work) {
  if (n <= 0) return GEVP_OK;
  const int64_t nbk = (n + HV - 1) / HV, pairs = nbk * (nbk + 1) / 2;
  zd* P1 = (zd*)work;
  zd* P2 = (zd*)((char*)work + ws_round(sizeof(zd) * HV * (size_t)pairs));
  hipLaunchKernelGGL(k_hemv_tiles, dim3((unsigned)pairs), dim3(256), 0, c->stream, n, M, ldm, x, P1, P2);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_hemv_reduce, dim3((unsigned)nbk), dim3(256), 0, c->stream, n, nbk, P1, P2, y);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_add_diag(gevp_ctx* c, int64_t n, zd* M, int64_t ldm, const double* shift) {
  if (n <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_add_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, M,
                     ldm, shift);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_permute_prefix(gevp_ctx* c, double* theta, double* resid, const int* perm,
                                  int64_t nl) {
  if (nl <= 0) return GEVP_OK;
  if (nl > 2048) return GEVP_ERR_INVALID;
  hipLaunchKernelGGL(k_permute_prefix, dim3(1), dim3(256), 0, c->stream, theta, resid, perm, (int)nl);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_merge_runs(gevp_ctx* c, double* theta, double* resid, int64_t nb, int64_t nl,
                              int* order) {
  if (nb <= 0) return GEVP_OK;
  if (nb > 2048) return GEVP_ERR_INVALID;
  hipLaunchKernelGGL(k_merge_runs, dim3(1), dim3(256), 0, c->stream, theta, resid, (int)nb, (int)nl,
                     order);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_copy_real(gevp_ctx* c, int64_t n, const double* s, double* d) {
  if (n <= 0) return GEVP_OK;
  hipLaunchKernelGGL(k_copy_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, s,
                     d);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_max_offident(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, double* out,
                                double* part) {
  if (n <= 0) return GEVP_ERR_INVALID;
  const int g = (int)std::min<int64_t>(n, MAX_OFFIDENT_PARTS);
  hipLaunchKernelGGL(k_max_offident, dim3(g), dim3(256), 0, c->stream, n, M, ldm, part);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(256), 0, c->stream, g, part, out);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
