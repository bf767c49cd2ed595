// Spectral bounds by a few Lanczos steps, and the controller that turns
// Ritz values and residuals into the next Chebyshev filter.
//
// Lanczos: v_{j+1} beta_j = M v_j - alpha_j v_j - beta_{j-1} v_{j-1}.  The
// Ritz values of the k x k tridiagonal bracket the spectrum from inside; the
// largest plus the last beta is a safe upper bound for the filter interval
// (the damped end), and the squared first components of the Ritz vectors
// estimate the spectral density, which places the lower end of the damped
// interval for a cold start.
//
// Controller: Chebyshev filter of degree m on the damped interval [a, b]
// (centre c, half-width e), normalised at the lowest estimate mu, applied
// with the scaled three-term recurrence
//   Y1 = (s1/e)(C - cI) Y0,
//   Y_{j+1} = (2 s_{j+1}/e)(C - cI) Y_j - s_j s_{j+1} Y_{j-1},
//   s1 = e/(mu - c),  s_{j+1} = 1/(2/s1 - s_j),
// whose coefficients are written as (alpha, beta, gamma) triples for the GEMM
// epilogue D = alpha C Y + beta Y + gamma Y_prev.  A column whose Ritz value
// theta lies left of the interval gains a factor rho = |t| + sqrt(t^2 - 1),
// t = (theta - c)/e, per degree relative to the damped part, so it needs
// about m = log(r / tol) / log(rho) more degrees to converge (the degree
// chosen aims at tol / margin, one degree more, so that columns the
// first-order model misjudges still converge in this sweep); converged wanted
// columns get degree 0 (they stay in the basis), guard columns the largest
// degree of the unconverged wanted ones.  Degrees are even so every column's
// last iterate lands in the same buffer; columns are sorted by degree so the
// columns still active at step j form a contiguous suffix.
#include <cfloat>

#include "common.h"

namespace {

__global__ __launch_bounds__(1024) void k_lanczos_init(int64_t n, zd* v) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += v[i].x * v[i].x + v[i].y * v[i].y;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += sh[w];
  const double inv = 1.0 / sqrt(t);
  for (int64_t i = threadIdx.x; i < n; i += 1024) v[i] = make_double2(v[i].x * inv, v[i].y * inv);
}

__device__ double bsum1024(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// w = M v_j (given); alpha_j = Re(v_j^H w); w -= alpha_j v_j + beta_{j-1} v_{j-1};
// beta_j = ||w||; v_{j+1} = w / beta_j.  Up to LV * 1024 entries are held in
// registers (all loads of a chunk in flight at once); longer vectors go
// through in chunks, re-reading them per pass.
constexpr int LV = 8;
__global__ __launch_bounds__(1024) void k_lanczos_vec(int64_t n, const zd* vprev, const zd* vcur,
                                                      const zd* w, zd* vnext, double* alpha,
                                                      double* beta, int j) {
  __shared__ double sh[16];
  const int64_t t = threadIdx.x, chunk = 1024 * LV;
  const bool one = n <= chunk;  // uniform
  zd vv[LV], ww[LV], pv[LV];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int64_t i = i0 + t + 1024 * u;
      const bool in = i < n;
      vv[u] = in ? vcur[i] : make_double2(0.0, 0.0);
      ww[u] = in ? w[i] : make_double2(0.0, 0.0);
      pv[u] = (in && j > 0) ? vprev[i] : make_double2(0.0, 0.0);
    }
  };
  double s = 0.0;
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    load(i0);
#pragma unroll
    for (int u = 0; u < LV; ++u) s += vv[u].x * ww[u].x + vv[u].y * ww[u].y;
  }
  const double a = bsum1024(s, sh);
  const double bp = (j > 0) ? beta[j - 1] : 0.0;
  zd rr[LV];
  double q = 0.0;
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    if (!one) load(i0);
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      rr[u] = make_double2(ww[u].x - a * vv[u].x - bp * pv[u].x, ww[u].y - a * vv[u].y - bp * pv[u].y);
      q += rr[u].x * rr[u].x + rr[u].y * rr[u].y;
      const int64_t i = i0 + t + 1024 * u;
      if (!one && i < n) vnext[i] = rr[u];
    }
  }
  const double b = sqrt(bsum1024(q, sh));
  const double inv = (b > 0.0) ? 1.0 / b : 0.0;
  if (one) {
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int64_t i = t + 1024 * u;
      if (i < n) vnext[i] = make_double2(rr[u].x * inv, rr[u].y * inv);
    }
  } else {
    for (int64_t i = t; i < n; i += 1024) vnext[i] = make_double2(vnext[i].x * inv, vnext[i].y * inv);
  }
  if (t == 0) {
    alpha[j] = a;
    beta[j] = b;
  }
}

// Summary of the k Ritz values theta (ascending) of the Lanczos tridiagonal
// and the first components Zt[0 * k + j] of its eigenvectors (from
// tridiag_eig: Sturm-count multisection and inverse iteration).  The squared
// first components are the weights the start vector gives each Ritz value,
// a coarse estimate of the spectral density.  Single thread; k <= 64.
__global__ void k_lanczos_summary(const double* theta, const double* Zt, const double* beta, int k,
                                  double frac, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double blast = beta[k - 1];
  const double tlo = theta[0], thi = theta[k - 1];
  out[0] = tlo;
  out[1] = thi;
  out[2] = blast;
  out[3] = thi + fabs(blast);
  // the point where the cumulative weight reaches frac, interpolated inside
  // the Ritz interval that crosses it
  double cum = 0.0, est = thi;
  for (int j = 0; j < k; ++j) {
    const double z = Zt[j];
    const double wgt = z * z;
    if (cum + wgt >= frac) {
      const double left = (j > 0) ? theta[j - 1] : tlo;
      const double t = (wgt > 0.0) ? (frac - cum) / wgt : 1.0;
      est = left + t * (theta[j] - left);
      break;
    }
    cum += wgt;
  }
  out[4] = est;
  out[5] = fmax(fabs(tlo), fabs(thi));
}

// status_i: [0] nconv  [1] maxdeg  [2] done  [3] unused  [4 + j - 1] s_j (j = 1..maxdeg)
// status_d: [0] a  [1] b  [2] c  [3] e  [4] tol_abs  [5] sum of column degrees  [6] mu
__global__ __launch_bounds__(256) void k_control(CtlParams p, const double* theta,
                                                 const double* resid, const double* bounds,
                                                 const double* norms, double tol_rel, int* si,
                                                 double* sd, int* perm, double* coefs,
                                                 double* rho0, double* coef2) {
  extern __shared__ int deg[];  // nb
  __shared__ int cnt[256];
  __shared__ int sh_nconv, sh_maxdeg;
  const int tid = threadIdx.x, nb = p.nb, nev = p.nev;
  const double normA = norms[0], normB = norms[1];
  const double tol_abs = tol_rel * normA / sqrt(fmax(normB, DBL_MIN));
  double a, mu;
  const double b = bounds[3];
  if (p.mode == 1) {
    a = bounds[4];
    mu = bounds[0];
  } else {  // modes 0 and 2: from the Ritz values
    a = theta[nb - 1];
    mu = fmin(theta[0], bounds[0]);
  }
  // a damped interval narrower than a few thousand rounding units of its
  // ends (e.g. every eigenvalue equal) would divide rounding noise by its
  // half-width: widen it to a thousandth of the scale instead
  if (!(b - a > 1e3 * DBL_EPSILON * fmax(fmax(fabs(a), fabs(b)), DBL_MIN)))
    a = b - 1e-3 * fmax(fabs(b), 1.0);
  if (!(mu < a)) mu = a - 0.5 * (b - a);
  const double e = 0.5 * (b - a), c = 0.5 * (b + a);
  if (tid == 0) {
    int nc = 0;
    if (p.mode != 1)
      while (nc < nev && resid[nc] <= tol_abs) ++nc;
    sh_nconv = nc;
  }
  // largest reduction a wanted column needs (mode 2): within 1 / u_reach, one
  // sweep aims for the tolerance directly instead of stopping at u_target
  __shared__ double red_sh[256];
  double rmax = 0.0;
  if (p.mode == 2)
    for (int i = tid; i < nev && i < nb; i += 256)
      if (resid[i] > tol_abs) rmax = fmax(rmax, resid[i] * p.margin / tol_abs);
  red_sh[tid] = rmax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red_sh[tid] = fmax(red_sh[tid], red_sh[tid + s]);
    __syncthreads();
  }
  const bool reach = p.mode == 2 && p.u_reach > 0.0 && red_sh[0] * p.u_reach <= 1.0;
  const double u_cap = reach ? p.u_reach : p.u_target;
  const int dmax = reach ? max(p.deg_max, p.deg_reach) : p.deg_max;
  const bool done = (p.mode != 1) && sh_nconv >= nev;
  // per-column degrees
  for (int i = tid; i < nb; i += 256) {
    int m;
    if (p.mode == 1) {
      m = p.deg_init;
    } else if (i < nev) {
      if (resid[i] <= tol_abs) {
        m = 0;
      } else {
        const double t = (theta[i] - c) / e;
        if (t >= -1.0) {
          m = dmax;
        } else {
          const double rho = fabs(t) + sqrt(t * t - 1.0);
          // reduction wanted this sweep; a low-precision filter (mode 2) cannot
          // beat its rounding floor, so it aims no further than u_target
          double red = resid[i] * p.margin / tol_abs;
          if (p.mode == 2 && red * u_cap > 1.0) red = 1.0 / u_cap;
          const double need = log(red) / log(rho);
          m = (int)ceil(need) + 1;
          if (m < 2) m = 2;
          if (m > dmax) m = dmax;
        }
      }
    } else {
      m = -1;  // guard: filled below
    }
    m = (m > 0) ? (m + (m & 1)) : m;
    deg[i] = m;
  }
  __syncthreads();
  if (tid == 0) {
    int mx = 0;
    for (int i = 0; i < nb && i < nev; ++i) mx = max(mx, deg[i]);
    if (p.mode == 1) mx = deg[0];
    if (mx == 0 && !done) mx = 2;
    if (mx > dmax + (dmax & 1)) mx = dmax + (dmax & 1);
    sh_maxdeg = done ? 0 : mx;
  }
  __syncthreads();
  for (int i = tid; i < nb; i += 256)
    if (deg[i] < 0) deg[i] = sh_maxdeg;
  __syncthreads();
  // stable counting sort by degree (degrees <= 255)
  for (int i = tid; i < 256; i += 256) cnt[i] = 0;
  __syncthreads();
  if (tid == 0) {
    long long sum = 0;
    for (int i = 0; i < nb; ++i) {
      cnt[deg[i]]++;
      sum += deg[i];
    }
    int acc = 0;
    for (int v = 0; v < 256; ++v) {
      const int cv = cnt[v];
      cnt[v] = acc;
      acc += cv;
    }
    // s_j = number of columns with degree < j
    for (int j = 1; j <= sh_maxdeg; ++j) si[4 + j - 1] = cnt[j];
    for (int i = 0; i < nb; ++i) perm[cnt[deg[i]]++] = i;
    si[0] = sh_nconv;
    si[1] = sh_maxdeg;
    si[2] = done ? 1 : 0;
    si[3] = 0;
    sd[0] = a;
    sd[1] = b;
    sd[2] = c;
    sd[3] = e;
    sd[4] = tol_abs;
    sd[5] = (double)sum;
    sd[6] = mu;
    double rmax = 0.0, rmin = 1e300;
    for (int i = 0; i < nev && i < nb; ++i) {
      rmax = fmax(rmax, resid[i]);
      rmin = fmin(rmin, resid[i]);
    }
    sd[7] = rmax;
    sd[8] = rmin;
    // filter coefficients, step j at coefs[3 (j - 1)]
    const double s1 = e / (mu - c);
    double sg = s1;
    for (int j = 1; j <= sh_maxdeg; ++j) {
      double al, be, ga;
      if (j == 1) {
        al = s1 / e;
        be = -s1 * c / e;
        ga = 0.0;
      } else {
        const double sn = 1.0 / (2.0 / s1 - sg);
        al = 2.0 * sn / e;
        be = -2.0 * sn * c / e;
        ga = -sg * sn;
        sg = sn;
      }
      coefs[3 * (j - 1) + 0] = al;
      coefs[3 * (j - 1) + 1] = be;
      coefs[3 * (j - 1) + 2] = ga;
    }
  }
  if (p.mode != 2) return;
  __syncthreads();
  // Residual-correction filter, per column in degree-sorted order: with
  // theta' = (theta - c)/e and T_j the Chebyshev polynomials,
  // g_{j+1} = a_j (C' g_j + r') - b_j g_{j-1},  a_j = 2 T_j/T_{j+1},
  // b_j = T_{j-1}/T_{j+1}, g_1 = r'/theta'; with rho_j = T_j/T_{j+1}:
  // rho_0 = 1/theta', rho_j = 1/(2 theta' - rho_{j-1}).  Step s (computing
  // g_{s+1}) stores alpha = a_s/e, beta = -a_s c/e, gamma = -b_s, delta = a_s.
  const int md = sh_maxdeg;
  for (int j = tid; j < nb; j += 256) {
    const int col = perm[j];
    double tp = (theta[col] - c) / e;
    if (tp > -1.0) tp = -1.0;
    double rprev = 1.0 / tp;
    rho0[j] = rprev;
    for (int st = 1; st < md; ++st) {
      const double r = 1.0 / (2.0 * tp - rprev);
      const double a = 2.0 * r, bb = rprev * r;
      double* row = coef2 + (size_t)(st - 1) * 4 * nb;
      row[j] = a / e;
      row[nb + j] = -a * c / e;
      row[2 * nb + j] = -bb;
      row[3 * nb + j] = a;
      rprev = r;
    }
  }
}
}  // namespace

size_t lanczos_work_bytes(int64_t n, int steps) {
  if (steps > 64) steps = 64;
  return ws_round(sizeof(zd) * n * 4) + 2 * ws_round(sizeof(double) * (steps + 1)) +
         ws_round(sizeof(double) * 64) + ws_round(sizeof(double) * 64 * 64) +
         tridiag_eig_work_bytes(64) + hemv_work_bytes(n);
}

gevp_status lanczos_bounds(gevp_ctx* c, int64_t n, const zd* M, int64_t ldm, int steps,
                           unsigned long long seed, double frac, double* out, void* work) {
  if (steps > 64) steps = 64;
  if (steps > n) steps = (int)n;
  if (steps < 1) steps = 1;
  char* w = (char*)work;
  zd* V = (zd*)w;
  w += ws_round(sizeof(zd) * n * 4);
  double* alpha = (double*)w;
  w += ws_round(sizeof(double) * (steps + 1));
  double* beta = (double*)w;
  w += ws_round(sizeof(double) * (steps + 1));
  double* rv = (double*)w;  // Ritz values
  w += ws_round(sizeof(double) * 64);
  double* Zt = (double*)w;  // eigenvectors of the tridiagonal, row-major
  w += ws_round(sizeof(double) * 64 * 64);
  void* tw = w;
  w += tridiag_eig_work_bytes(64);
  void* hw = w;  // partial vectors of the matrix-vector products
  zd* buf[3] = {V, V + n, V + 2 * n};
  zd* wv = V + 3 * n;
  GEVP_TRY(launch_randn(c, n, 1, buf[0], n, 0, seed));
  hipLaunchKernelGGL(k_lanczos_init, dim3(1), dim3(1024), 0, c->stream, n, buf[0]);
  GEVP_HIP_TRY(hipGetLastError());
  for (int j = 0; j < steps; ++j) {
    zd* vc = buf[j % 3];
    zd* vp = buf[(j + 2) % 3];
    zd* vn = buf[(j + 1) % 3];
    GEVP_TRY(launch_hemv(c, n, M, ldm, vc, wv, hw));
    hipLaunchKernelGGL(k_lanczos_vec, dim3(1), dim3(1024), 0, c->stream, n, vp, vc, wv, vn, alpha,
                       beta, j);
    GEVP_HIP_TRY(hipGetLastError());
  }
  GEVP_TRY(tridiag_eig(c, steps, alpha, beta, rv, Zt, tw));
  hipLaunchKernelGGL(k_lanczos_summary, dim3(1), dim3(64), 0, c->stream, rv, Zt, beta, steps, frac,
                     out);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}

gevp_status launch_control(gevp_ctx* c, const CtlParams& p, const double* theta,
                           const double* resid, const double* bounds, const double* norms,
                           double tol_rel, int* status_i, double* status_d, int* perm,
                           double* coefs, double* rho0, double* coef2) {
  if (p.mode == 2 && (!rho0 || !coef2)) return GEVP_ERR_INVALID;
  hipLaunchKernelGGL(k_control, dim3(1), dim3(256), sizeof(int) * p.nb, c->stream, p, theta, resid,
                     bounds, norms, tol_rel, status_i, status_d, perm, coefs, rho0, coef2);
  GEVP_HIP_TRY(hipGetLastError());
  return GEVP_OK;
}
