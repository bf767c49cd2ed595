// Small dense Hermitian eigensolver for the Rayleigh-Ritz step (n up to a few
// thousand), all on the GPU in FP64:
//
//  1. Householder tridiagonalisation H = U T U^H, one fused kernel per
//     reflector.  Kernel s finishes the rank-2 update of reflector s-1 on the
//     columns it owns, forms reflector s from column s (which every
//     work-group reconstructs redundantly from the old column and the
//     previous reflector, so no extra grid-wide barrier is needed), and
//     accumulates p = tau H v for reflector s on its columns.  Hermitian
//     symmetry turns each row dot product into a contiguous column dot.
//  2. Eigenvalues of the real tridiagonal T by multisection on Sturm counts,
//     one wave per eigenvalue (64 points per round).
//  3. Eigenvectors of T by inverse iteration (tridiagonal LU with partial
//     pivoting), one thread per eigenvalue, recurrences in registers; members
//     of numerically degenerate clusters are then made orthonormal by
//     modified Gram-Schmidt.
//  4. Z = U Z_T with U = I - V T V^H for all reflectors at once: T^{-1} is
//     diag(1/tau) plus the strict upper triangle of V^H V, so Z <- Z - V (T
//     (V^H Z)) is a Gram product, a triangular solve and two products on the
//     FP64 matrix cores.
#include <cfloat>

#include "common.h"

namespace {
constexpr int HT = 256;  // threads per work-group

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ double bsum(double v, double* sh) {
  v = wsum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  const double s = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return s;
}
__device__ __forceinline__ zd cmul(zd a, zd b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ zd cconj(zd a) { return make_double2(a.x, -a.y); }

struct TrdArgs {
  int n;
  zd* H;
  int64_t ldh;
  zd* V;  // reflectors, column s holds v_s (v_s[s+1] = 1)
  int64_t ldv;
  zd* tau;
  double* d;
  double* e;
  zd* pb;       // 2 x n : p of the previous / current reflector
  zd* pp;       // 2 x G : per-work-group partial sums v^H p
  int G;
};

// Reflector s (0 <= s <= n-2); s == n-1 finishes the last diagonal entry.
// One pass over global memory per step: every thread first loads its share
// of column s, v_{s-1} and p_{s-1} (rows s .. n-1, at most QMAX per thread)
// together with one partial sum, everything else is formed in registers and
// LDS: w_{s-1} = p - K v (K from the partials), the updated column s, the
// reflector, and the staged vectors v_s, w_{s-1}, v_{s-1} that the column
// updates read.
// LDS: sm = [v_s | w_{s-1} | v_{s-1}], each n complex; sh: 8 doubles.
constexpr int QMAX = 8;  // rows per thread: n <= QMAX * HT

__device__ __forceinline__ zd bsum2(zd v, double* sh) {
  v.x = wsum(v.x);
  v.y = wsum(v.y);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    sh[2 * w] = v.x;
    sh[2 * w + 1] = v.y;
  }
  __syncthreads();
  const zd r = make_double2(sh[0] + sh[2] + sh[4] + sh[6], sh[1] + sh[3] + sh[5] + sh[7]);
  __syncthreads();
  return r;
}

__device__ void hetrd_body(const TrdArgs& a, int s, zd* sm, double* sh, zd* bc) {
  const int n = a.n, tid = threadIdx.x, wg = blockIdx.x;
  const int prev = s - 1;
  zd* vs = sm;            // v_s
  zd* sw = sm + n;        // w_{s-1}
  zd* sv = sm + 2 * n;    // v_{s-1}
  const zd* vp = (prev >= 0) ? a.V + (int64_t)prev * a.ldv : nullptr;
  const zd* pprev = (prev >= 0) ? a.pb + (int64_t)(prev & 1) * n : nullptr;
  const zd* cs = a.H + (int64_t)s * a.ldh;
  // ---- the one round of global loads
  zd hc[QMAX], vv[QMAX], pv[QMAX];
  zd ppart = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int i = s + tid + q * HT;
    hc[q] = (i < n) ? cs[i] : make_double2(0.0, 0.0);
    vv[q] = (prev >= 0 && i < n) ? vp[i] : make_double2(0.0, 0.0);
    pv[q] = (prev >= 0 && i < n) ? pprev[i] : make_double2(0.0, 0.0);
  }
  if (prev >= 0 && tid < a.G) ppart = a.pp[(int64_t)(prev & 1) * a.G + tid];
  const zd taup = (prev >= 0) ? a.tau[prev] : make_double2(0.0, 0.0);
  // ---- K = 1/2 conj(tau) sum(partials); w = p - K v
  zd K = make_double2(0.0, 0.0);
  if (prev >= 0) {
    const zd ps = bsum2(ppart, sh);
    const zd k2 = cmul(cconj(taup), ps);
    K = make_double2(0.5 * k2.x, 0.5 * k2.y);
  }
  zd ww[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const zd kv = cmul(K, vv[q]);
    ww[q] = make_double2(pv[q].x - kv.x, pv[q].y - kv.y);
  }
  // v_s and w_s of the previous reflector (row s, owned by thread 0, q = 0)
  if (tid == 0) {
    bc[0] = vv[0];
    bc[1] = ww[0];
  }
  __syncthreads();
  const zd vps = bc[0], wps = bc[1];
  // updated column s: H(i,s) - v_i conj(w_s) - w_i conj(v_s)
  double sig = 0.0;
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int i = s + tid + q * HT;
    const zd t1 = cmul(vv[q], cconj(wps)), t2 = cmul(ww[q], cconj(vps));
    hc[q].x -= t1.x + t2.x;
    hc[q].y -= t1.y + t2.y;
    if (i >= s + 2 && i < n) sig += hc[q].x * hc[q].x + hc[q].y * hc[q].y;
    if (i == s + 1) bc[2] = hc[q];
    if (i == s) bc[3] = hc[q];
  }
  sig = bsum(sig, sh);  // its barriers also publish bc[2], bc[3]
  if (s == n - 1) {  // finish: last diagonal entry only
    if (wg == 0 && tid == 0) a.d[s] = bc[3].x;
    return;
  }
  const zd alpha = bc[2];
  zd tau = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
  double beta;
  if (sig == 0.0 && alpha.y == 0.0) {
    beta = alpha.x;
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig);
    beta = (alpha.x >= 0.0) ? -nrm : nrm;
    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    const zd den = make_double2(alpha.x - beta, alpha.y);  // scal = 1 / den
    const double dd = den.x * den.x + den.y * den.y;
    scal = make_double2(den.x / dd, -den.y / dd);
  }
  // stage v_s, w_{s-1}, v_{s-1} in LDS
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int i = s + tid + q * HT;
    if (i < n) {
      vs[i] = (i == s + 1) ? make_double2(1.0, 0.0) : (i > s + 1 ? cmul(hc[q], scal) : make_double2(0.0, 0.0));
      sw[i] = ww[q];
      sv[i] = vv[q];
    }
  }
  __syncthreads();
  if (wg == 0) {
    zd* vcol = a.V + (int64_t)s * a.ldv;
    for (int i = tid; i < n; i += HT) vcol[i] = (i > s) ? vs[i] : make_double2(0.0, 0.0);
    if (tid == 0) {
      a.tau[s] = tau;
      a.e[s] = beta;
      a.d[s] = bc[3].x;
    }
  }
  // own columns j >= s+1, j % G == wg: finish the previous update on rows
  // >= s+1 and accumulate p_s[j] = tau sum_i conj(H(i,j)) v_i (Hermitian
  // symmetry turns the row product into a contiguous column product)
  const int lane = tid & 63, wave = tid >> 6;
  zd part = make_double2(0.0, 0.0);
  zd* pcur = a.pb + (int64_t)(s & 1) * n;
  const int j0 = s + 1 + ((wg - (s + 1)) % a.G + a.G) % a.G;
  for (int j = j0 + wave * a.G; j < n; j += 4 * a.G) {
    zd* col = a.H + (int64_t)j * a.ldh;
    const zd vj = sv[j], wj = sw[j];
    double ar = 0.0, ai = 0.0;
    for (int i = s + 1 + lane; i < n; i += 64) {
      zd h = col[i];
      if (prev >= 0) {
        const zd v = sv[i], w = sw[i];
        const zd t1 = cmul(v, cconj(wj)), t2 = cmul(w, cconj(vj));
        h.x -= t1.x + t2.x;
        h.y -= t1.y + t2.y;
        col[i] = h;
      }
      const zd v = vs[i];  // conj(h) * v
      ar += h.x * v.x + h.y * v.y;
      ai += h.x * v.y - h.y * v.x;
    }
    ar = wsum(ar);
    ai = wsum(ai);
    const zd pj = cmul(tau, make_double2(ar, ai));
    if (lane == 0) {
      pcur[j] = pj;
      const zd t = cmul(cconj(vs[j]), pj);
      part.x += t.x;
      part.y += t.y;
    }
  }
  // work-group partial of v_s^H p_s
  const zd pt = bsum2(lane == 0 ? part : make_double2(0.0, 0.0), sh);
  if (tid == 0) a.pp[(int64_t)(s & 1) * a.G + wg] = pt;
}

__global__ __launch_bounds__(HT) void k_hetrd_step(TrdArgs a, int s) {
  extern __shared__ double sm[];
  __shared__ double sh[8];
  __shared__ zd bc[4];
  hetrd_body(a, s, reinterpret_cast<zd*>(sm), sh, bc);
}

// Sturm count: number of eigenvalues of T smaller than x.
__device__ int sturm(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// One wave per eigenvalue k: every round the 64 lanes evaluate Sturm counts
// at 64 interior points of [lo, hi] and the bracket shrinks to the
// sub-interval where the count passes k (65x per round).
__global__ __launch_bounds__(HT) void k_tri_bisect(const double* d, const double* e, int n,
                                                   double* theta) {
  extern __shared__ double sm[];
  double* sd = sm;
  double* se2 = sm + n;
  __shared__ double red[3];
  for (int i = threadIdx.x; i < n; i += HT) {
    sd[i] = d[i];
    se2[i] = (i < n - 1) ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double gl = DBL_MAX, gu = -DBL_MAX, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? sqrt(se2[i - 1]) : 0.0) + (i < n - 1 ? sqrt(se2[i]) : 0.0);
      gl = fmin(gl, sd[i] - r);
      gu = fmax(gu, sd[i] + r);
      if (i < n - 1) emax = fmax(emax, se2[i]);
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    red[0] = gl - 2.0 * DBL_EPSILON * tnorm * n - 1e-300;
    red[1] = gu + 2.0 * DBL_EPSILON * tnorm * n + 1e-300;
    red[2] = DBL_MIN * fmax(1.0, emax);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (HT / 64) + (threadIdx.x >> 6);
  if (k >= n) return;
  double lo = red[0], hi = red[1];
  const double pivmin = red[2];
  for (int round = 0; round < 40; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
    const double w = (hi - lo) / 65.0;
    const double x = lo + w * (lane + 1);
    const int cnt = sturm(sd, se2, n, x, pivmin);
    const unsigned long long m = __ballot(cnt > k);
    const double xs = x;
    if (m == 0ull) {
      lo = __shfl(xs, 63, 64);
    } else {
      const int q = __ffsll((long long)m) - 1;
      const double nh = __shfl(xs, q, 64);
      const double nl = (q > 0) ? __shfl(xs, q - 1 < 0 ? 0 : q - 1, 64) : lo;
      hi = nh;
      lo = nl;
    }
  }
  if (lane == 0) theta[k] = 0.5 * (lo + hi);
}

__device__ __forceinline__ uint64_t hmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Inverse iteration, thread j <-> eigenvalue j.  Scratch arrays are laid out
// [i * n + j] so that a wave's accesses are contiguous.  Output Zt[i*n + j].
// LU of T - lam I with partial pivoting: row k of U holds (U, Vv, Ww) on
// columns (k, k+1, k+2); Lm the multiplier and Sw the row swap of step k.
__global__ __launch_bounds__(64) void k_tri_invit(const double* dg, const double* eg, int n,
                                                  const double* theta, double* U, double* Vv,
                                                  double* Ww, double* Lm, double* Sw, double* Zt,
                                                  const double* tnorm_dev) {
  const double tnorm = *tnorm_dev;
  extern __shared__ double sm[];
  double* d = sm;
  double* e = sm + n;
  for (int i = threadIdx.x; i < n; i += 64) {
    d[i] = dg[i];
    e[i] = (i < n - 1) ? eg[i] : 0.0;
  }
  __syncthreads();
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= n) return;
  const double lam = theta[j];
  const double tiny = DBL_EPSILON * fmax(tnorm, DBL_MIN);
  // thread j's entry k of an n x n work array; consecutive threads are
  // consecutive addresses.  Every pass below keeps its recurrence in
  // registers; the loads it needs do not depend on the recurrence and are
  // issued IB steps at a time, so a pass costs n / IB memory latencies.
  auto at = [&](double* A, int k) -> double& { return A[(int64_t)k * n + j]; };
  constexpr int IB = 32;
  // LU with partial pivoting of T - lam I; working row k: (al, be) on columns (k, k+1)
  double al = d[0] - lam, be = (n > 1) ? e[0] : 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double ck = e[k], an = d[k + 1] - lam, bn = (k + 1 < n - 1) ? e[k + 1] : 0.0;
    if (fabs(al) >= fabs(ck)) {  // pivot on the working row
      const double piv = (al == 0.0) ? tiny : al;
      const double l = ck / piv;
      at(U, k) = piv;
      at(Vv, k) = be;
      at(Ww, k) = 0.0;
      at(Lm, k) = l;
      at(Sw, k) = 0.0;
      al = an - l * be;
      be = bn;
    } else {  // pivot on the next original row (ck, an, bn)
      const double l = al / ck;
      at(U, k) = ck;
      at(Vv, k) = an;
      at(Ww, k) = bn;
      at(Lm, k) = l;
      at(Sw, k) = 1.0;
      const double nal = be - l * an;
      be = -l * bn;
      al = nal;
    }
  }
  at(U, n - 1) = (al == 0.0) ? tiny : al;
  for (int i = 0; i < n; ++i) {
    const uint64_t r = hmix(((uint64_t)j << 32) ^ (uint64_t)i ^ 0x5DEECE66Dull);
    at(Zt, i) = ((double)(r >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
  }
  // Two sweeps of inverse iteration.  The growth of the first sweep is removed
  // by a power-of-two factor folded into the second sweep's loads (exact, no
  // extra pass); the second sweep's backward pass also accumulates the sum of
  // squares, so one final pass normalises.
  double sc = 1.0, ssq = 0.0, mx = 0.0;
  for (int it = 0; it < 2; ++it) {
    // forward: apply the row swaps and multipliers; c is the current y_k
    double c = at(Zt, 0) * sc;
    for (int k0 = 0; k0 < n - 1; k0 += IB) {
      double lv[IB], sv[IB], av[IB];
#pragma unroll
      for (int q = 0; q < IB; ++q) {
        const int k = k0 + q;
        if (k < n - 1) {
          lv[q] = at(Lm, k);
          sv[q] = at(Sw, k);
          av[q] = at(Zt, k + 1);
        }
      }
#pragma unroll
      for (int q = 0; q < IB; ++q) {
        const int k = k0 + q;
        if (k < n - 1) {
          const double a = av[q] * sc;
          if (sv[q] != 0.0) {  // rows k, k+1 swapped
            at(Zt, k) = a;
            c = c - lv[q] * a;
          } else {
            at(Zt, k) = c;
            c = a - lv[q] * c;
          }
        }
      }
    }
    at(Zt, n - 1) = c;
    // backward: U x = y with U upper triangular, bandwidth 3
    double x1 = 0.0, x2 = 0.0;
    mx = 0.0;
    ssq = 0.0;
    for (int k0 = n - 1; k0 >= 0; k0 -= IB) {
      double yv[IB], vv[IB], wv[IB], uv[IB];
#pragma unroll
      for (int q = 0; q < IB; ++q) {
        const int k = k0 - q;
        if (k >= 0) {
          yv[q] = at(Zt, k);
          vv[q] = at(Vv, k);
          wv[q] = at(Ww, k);
          uv[q] = at(U, k);
        }
      }
#pragma unroll
      for (int q = 0; q < IB; ++q) {
        const int k = k0 - q;
        if (k >= 0) {
          double y = yv[q];
          if (k + 1 < n) y -= vv[q] * x1;
          if (k + 2 < n) y -= wv[q] * x2;
          const double x = y / uv[q];
          at(Zt, k) = x;
          x2 = x1;
          x1 = x;
          mx = fmax(mx, fabs(x));
          ssq += x * x;
        }
      }
    }
    int ex = 0;
    (void)frexp(mx, &ex);
    sc = (mx > 0.0 && isfinite(mx)) ? ldexp(1.0, -ex) : 1.0;
  }
  // normalise: from the sum of squares when it is finite, else after scaling
  // by the power of two (a second pass, only for extreme growth)
  double inv;
  if (ssq > 0.0 && isfinite(ssq)) {
    inv = 1.0 / sqrt(ssq);
  } else {
    double nrm = 0.0;
    for (int k0 = 0; k0 < n; k0 += IB) {
      double zv[IB];
#pragma unroll
      for (int q = 0; q < IB; ++q)
        if (k0 + q < n) zv[q] = at(Zt, k0 + q);
#pragma unroll
      for (int q = 0; q < IB; ++q)
        if (k0 + q < n) nrm += (zv[q] * sc) * (zv[q] * sc);
    }
    inv = (nrm > 0.0 && isfinite(nrm)) ? sc / sqrt(nrm) : 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += IB) {
    double zv[IB];
#pragma unroll
    for (int q = 0; q < IB; ++q)
      if (k0 + q < n) zv[q] = at(Zt, k0 + q);
#pragma unroll
    for (int q = 0; q < IB; ++q)
      if (k0 + q < n) at(Zt, k0 + q) = zv[q] * inv;
  }
}

// Modified Gram-Schmidt inside clusters of (numerically) equal eigenvalues:
// work-group b handles the cluster that starts at index b (if any).
__global__ __launch_bounds__(HT) void k_tri_cluster_mgs(const double* theta, int n, double* Zt,
                                                        const double* tnorm_dev) {
  const double ctol = 1e3 * DBL_EPSILON * fmax(*tnorm_dev, 1e-300);
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (b >= n) return;
  const bool start = (b == 0 || theta[b] - theta[b - 1] > ctol);
  if (!start || b + 1 >= n || theta[b + 1] - theta[b] > ctol) return;
  int end = b + 1;
  while (end + 1 < n && theta[end + 1] - theta[end] <= ctol) ++end;
  for (int pass = 0; pass < 2; ++pass)
    for (int m = b; m <= end; ++m) {
      for (int q = b; q < m; ++q) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += HT) s += Zt[(int64_t)i * n + q] * Zt[(int64_t)i * n + m];
        s = bsum(s, sh);
        for (int i = threadIdx.x; i < n; i += HT) Zt[(int64_t)i * n + m] -= s * Zt[(int64_t)i * n + q];
        __syncthreads();
      }
      double s = 0.0;
      for (int i = threadIdx.x; i < n; i += HT) {
        const double v = Zt[(int64_t)i * n + m];
        s += v * v;
      }
      s = bsum(s, sh);
      const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
      for (int i = threadIdx.x; i < n; i += HT) Zt[(int64_t)i * n + m] *= inv;
      __syncthreads();
    }
}

// Zc(i, j) = Zt[i*n + j] as complex, 32 x 32 tiles through LDS
__global__ __launch_bounds__(256) void k_zt_to_complex(const double* Zt, int n, zd* Z, int64_t ldz) {
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    t[r][tx] = (i < n && j < n) ? Zt[(int64_t)i * n + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = j0 + r, i = i0 + tx;
    if (i < n && j < n) Z[i + (int64_t)j * ldz] = make_double2(t[tx][r], 0.0);
  }
}

__global__ void k_tri_norm(const double* d, const double* e, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double m = 0.0;
  for (int i = 0; i < n; ++i)
    m = fmax(m, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0));
  out[0] = m;
}
}  // namespace

// work-groups of the tridiagonalisation: one column per wave as far as the
// order allows, and at most HT, since the next step's block reduction reads
// one work-group partial per thread (measured at n = 948: 12.4 ms per
// eigensolve with 256 groups, 13.2 with 192, 17.6 with 64)
inline int trd_groups(int64_t n) { return (int)(n - 1 < HT ? (n > 1 ? n - 1 : 1) : HT); }

size_t tridiag_eig_work_bytes(int64_t n) {
  return 5 * ws_round(sizeof(double) * n * n) + ws_round(sizeof(double) * 8);  // U, Vv, Ww, Lm, Sw; norm
}

gevp_status tridiag_eig(gevp_ctx* c, int64_t n64, const double* d, const double* e, double* theta,
                        double* Zt, void* work) {
  if (n64 <= 0) return GEVP_OK;
  const int n = (int)n64;
  char* w = (char*)work;
  auto take = [&](size_t bytes) {
    void* p = w;
    w += ws_round(bytes);
    return p;
  };
  double* U = (double*)take(sizeof(double) * n * n);
  double* Vv = (double*)take(sizeof(double) * n * n);
  double* Ww = (double*)take(sizeof(double) * n * n);
  double* Lm = (double*)take(sizeof(double) * n * n);
  double* Sw = (double*)take(sizeof(double) * n * n);
  double* tn = (double*)take(sizeof(double) * 8);
  hipLaunchKernelGGL(k_tri_norm, dim3(1), dim3(64), 0, c->stream, d, e, n, tn);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_tri_bisect, dim3((n + 3) / 4), dim3(HT), sizeof(double) * 2 * n, c->stream,
                     d, e, n, theta);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_tri_invit, dim3((n + 63) / 64), dim3(64), sizeof(double) * 2 * n, c->stream,
                     d, e, n, theta, U, Vv, Ww, Lm, Sw, Zt, tn);
  GEVP_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_tri_cluster_mgs, dim3(n), dim3(HT), 0, c->stream, theta, n, Zt, tn);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

// Back-transformation Z <- Q Z, Q = G_0 G_1 ... G_{k-1} = I - V T V^H with the
// k = n - 1 reflectors G_i = I - tau_i v_i v_i^H as the columns of V.  For the
// forward accumulation (T_ii = tau_i, T(0:i-1, i) = -tau_i T(0:i-1, 0:i-1)
// V(:, 0:i-1)^H v_i) the inverse of T is diag(1/tau) + striu(V^H V) (the UT
// transform), so with L = T^{-H} = diag(conj(1/tau)) + stril(V^H V):
//   S = V^H Z,   S <- L^{-H} S (= T S),   Z <- Z - V S,
// a Gram product, a triangular solve and two products on the FP64 matrix
// cores.  A reflector with tau = 0 is the identity: its column of V is
// cleared and its diagonal entry of L set to 1, which leaves it out.
__global__ __launch_bounds__(256) void k_ut_clear(int n, int k, zd* V, int64_t ldv, const zd* tau) {
  const int i = blockIdx.x;
  if (i >= k) return;
  const zd t = tau[i];
  if (t.x != 0.0 || t.y != 0.0) return;
  for (int r = threadIdx.x; r < n; r += 256) V[r + (int64_t)i * ldv] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_ut_diag(int k, zd* L, int64_t ldl, const zd* tau) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= k) return;
  const zd t = tau[i];
  const double dd = t.x * t.x + t.y * t.y;
  // conj(1 / t) = t / |t|^2
  L[i + (int64_t)i * ldl] = (dd == 0.0) ? make_double2(1.0, 0.0) : make_double2(t.x / dd, t.y / dd);
}

size_t heev_work_bytes(int64_t n) {
  const int G = trd_groups(n);
  size_t b = 0;
  b += ws_round(sizeof(zd) * n * n);          // V (reflectors)
  b += ws_round(sizeof(zd) * n);              // tau
  b += 2 * ws_round(sizeof(double) * n);      // d, e
  b += ws_round(sizeof(zd) * 2 * n);          // pb
  b += ws_round(sizeof(zd) * 2 * G);          // pp
  b += ws_round(sizeof(double) * n * n);      // Zt
  b += tridiag_eig_work_bytes(n);
  b += 2 * ws_round(sizeof(zd) * n * n);     // L = T^{-H}, S
  b += ws_round(sizeof(zd) * n * 64);         // inverses of L's diagonal blocks
  return b;
}

// One launch per reflector: the kernel boundary is the grid-wide barrier (a
// cooperative single launch with explicit barriers measured slower, because
// each barrier must write back and invalidate the XCD caches).  Issued one by
// one, the launches cost the host about 4.4 us each at n = 948, more than the
// later, shorter steps take on the GPU; so the sequence is captured once per
// argument set into a graph and replayed (the first call also pays the
// capture).  Any failure of the graph calls falls back to direct launches.
namespace {
constexpr size_t MAX_GRAPHS = 8;

gevp_status hetrd_direct(gevp_ctx* c, hipStream_t st, const TrdArgs& a, int G, size_t sh3) {
  for (int s = 0; s <= a.n - 1; ++s) {
    hipLaunchKernelGGL(k_hetrd_step, dim3(G), dim3(HT), sh3, st, a, s);
    GEVP_HIP_TRY(hipGetLastError());
  }
  return GEVP_OK;
}

gevp_status hetrd_launches(gevp_ctx* c, const TrdArgs& a, int G, size_t sh3) {
  const std::vector<int64_t> key = {a.n, G, (int64_t)(uintptr_t)a.H, a.ldh, (int64_t)(uintptr_t)a.V,
                                    a.ldv, (int64_t)(uintptr_t)a.tau, (int64_t)(uintptr_t)a.d,
                                    (int64_t)(uintptr_t)a.e, (int64_t)(uintptr_t)a.pb,
                                    (int64_t)(uintptr_t)a.pp, (int64_t)sh3};
  for (gevp_ctx::GraphEntry& g : c->graphs)
    if (g.key == key) {
      if (hipGraphLaunch(g.exec, c->stream) == hipSuccess) return GEVP_OK;
      (void)hipGetLastError();
      return hetrd_direct(c, c->stream, a, G, sh3);
    }
  if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->cap_stream = nullptr;
    (void)hipGetLastError();
    return hetrd_direct(c, c->stream, a, G, sh3);
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    const gevp_status st = hetrd_direct(c, c->cap_stream, a, G, sh3);
    ok = (hipStreamEndCapture(c->cap_stream, &graph) == hipSuccess) && st == GEVP_OK && graph;
  }
  if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  if (!ok) {
    (void)hipGetLastError();
    if (gevp_log_enabled()) fprintf(stderr, "[gevp] tridiagonalisation graph unavailable: direct launches\n");
    return hetrd_direct(c, c->stream, a, G, sh3);
  }
  if (c->graphs.size() >= MAX_GRAPHS) {  // the oldest may still run on the stream
    GEVP_HIP_TRY(hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({key, exec});
  GEVP_HIP_TRY(hipGraphLaunch(exec, c->stream));
  return GEVP_OK;
}
}  // namespace

gevp_status heev_small(gevp_ctx* c, int64_t n64, zd* H, int64_t ldh, double* theta, zd* Z,
                       int64_t ldz, void* work) {
  if (n64 <= 0) return GEVP_OK;
  // the reflector step keeps at most QMAX rows per thread and three n-vectors in LDS
  if (n64 > (int64_t)QMAX * HT) return GEVP_ERR_INVALID;
  const int n = (int)n64;
  const int G = trd_groups(n);
  char* w = (char*)work;
  auto take = [&](size_t bytes) {
    void* p = w;
    w += ws_round(bytes);
    return p;
  };
  TrdArgs a;
  a.n = n;
  a.H = H;
  a.ldh = ldh;
  a.V = (zd*)take(sizeof(zd) * n * n);
  a.ldv = n;
  a.tau = (zd*)take(sizeof(zd) * n);
  a.d = (double*)take(sizeof(double) * n);
  a.e = (double*)take(sizeof(double) * n);
  a.pb = (zd*)take(sizeof(zd) * 2 * n);
  a.pp = (zd*)take(sizeof(zd) * 2 * G);
  a.G = G;
  double* Zt = (double*)take(sizeof(double) * n * n);
  void* tw = take(tridiag_eig_work_bytes(n));
  zd* Lut = (zd*)take(sizeof(zd) * n * n);
  zd* Sut = (zd*)take(sizeof(zd) * n * n);
  zd* Dut = (zd*)take(sizeof(zd) * n * 64);

  const size_t shv = sizeof(zd) * (size_t)n;
  const size_t sh3 = 3 * shv;  // v_s, w_{s-1}, v_{s-1}
  static const bool attr = [&]() {
    (void)hipFuncSetAttribute((const void*)k_hetrd_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(3 * sizeof(zd) * 2048));
    return true;
  }();
  (void)attr;
  if (n == 1) {
    hipLaunchKernelGGL(k_hetrd_step, dim3(1), dim3(HT), sh3, c->stream, a, 0);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_HIP_TRY(hipMemsetAsync(a.tau, 0, sizeof(zd), c->stream));
  } else {
    GEVP_HIP_TRY(hipMemsetAsync(a.tau, 0, sizeof(zd) * n, c->stream));
    GEVP_TRY(hetrd_launches(c, a, G, sh3));
  }
  GEVP_TRY(tridiag_eig(c, n, a.d, a.e, theta, Zt, tw));
  const unsigned tb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_zt_to_complex, dim3(tb, tb), dim3(256), 0, c->stream, Zt, n, Z, ldz);
  GEVP_HIP_TRY(hipGetLastError());
  if (n > 1) {
    const int k = n - 1;
    hipLaunchKernelGGL(k_ut_clear, dim3((unsigned)k), dim3(256), 0, c->stream, n, k, a.V, a.ldv, a.tau);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_TRY(launch_zgemm(c, 1, 0, k, k, n, 1.0, a.V, a.ldv, a.V, a.ldv, 0.0, nullptr, 0, 0.0, nullptr,
                          0, nullptr, Lut, k, nullptr, 1));  // lower triangle of V^H V
    hipLaunchKernelGGL(k_ut_diag, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, c->stream, k, Lut, k,
                       a.tau);
    GEVP_HIP_TRY(hipGetLastError());
    GEVP_TRY(diag_block_inverses(c, k, Lut, k, Dut, k));
    GEVP_TRY(launch_zgemm(c, 1, 0, k, n, n, 1.0, a.V, a.ldv, Z, ldz, 0.0, nullptr, 0, 0.0, nullptr, 0,
                          nullptr, Sut, k));
    GEVP_TRY(trsm_left_lower_c(c, k, n, Lut, k, Dut, k, Sut, k, 0));
    GEVP_TRY(launch_zgemm(c, 0, 0, n, n, k, -1.0, a.V, a.ldv, Sut, k, 1.0, Z, ldz, 0.0, nullptr, 0,
                          nullptr, Z, ldz));
  }
  return GEVP_OK;
}
