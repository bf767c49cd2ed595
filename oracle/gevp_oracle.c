/*
 * gevp_oracle.c -- plain, slow, FP64 CPU reference for the generalized
 * Hermitian eigenproblem A x = lambda B x (B Hermitian positive definite).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header or constant with the GPU
 * path.
 *
 * What it computes (the paper, section 1, eq. (3) and the paragraph before
 * it): for every k-point the Hamiltonian A and overlap B are dense Hermitian
 * matrices and the wanted states are the solutions of sum_G' [A - lambda B] c
 * = 0 with the lowest eigenvalues first (the ordering eps_1 <= eps_2 <= ... of
 * eq. (1)).  The paper solves these "full data" problems with the LAPACK QR
 * algorithm (section 2, paragraph "Eigenvectors evolution"); this file is that
 * textbook dense route written out from Golub & Van Loan, Matrix
 * Computations, ch. 4 (Cholesky), ch. 5 (Householder), ch. 8 (symmetric QR):
 *
 *   1. B = L L^H                      (unblocked Cholesky, no pivoting)
 *   2. C = L^{-1} A L^{-H}            (two forward substitutions)
 *   3. C = U T U^H                    (Householder tridiagonalisation, T real)
 *   4. T = Z diag(theta) Z^T          (implicit Wilkinson-shift QR, Givens)
 *   5. sort ascending, keep the lowest nev
 *   6. X = L^{-H} U Z(:, 1:nev)       (back substitution)
 *
 * plus independent checks used to pin it: inertia counts by an LDL^H
 * factorisation of A - sigma B (Sylvester's law, no QR involved), bisection
 * on those counts, inverse iteration, residual and B-orthonormality norms,
 * and the eigenvalue gradient dA = X diag(w) X^H, dB = -X diag(w lambda) X^H.
 *
 * Conventions: every matrix is column-major complex128 with a leading
 * dimension; only the lower triangles of A and B are read.  Return codes:
 * 0 ok, -i bad argument i, n+j Cholesky of B failed at (1-based) pivot j,
 * 1 the tridiagonal QR did not converge in 30 n sweeps.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ---- full Hermitian copy from the lower triangle (uplo = 'L' reading) ---- */
static void herm_from_lower(int n, const zc* A, int lda, zc* F) {
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      if (i > j)
        F[IDX(i, j, n)] = A[IDX(i, j, lda)];
      else if (i == j)
        F[IDX(i, j, n)] = creal(A[IDX(i, i, lda)]);
      else
        F[IDX(i, j, n)] = conj(A[IDX(j, i, lda)]);
    }
}

/* ---- step 1: Cholesky B = L L^H, in place on a full n x n copy.
 * Column j: l_jj = sqrt(b_jj - sum_k |l_jk|^2), l_ij = (b_ij - sum_k l_ik
 * conj(l_jk)) / l_jj.  Returns 0 or j+1 for a non-positive pivot. */
int oref_potrf(int n, zc* L, int ld) {
  for (int j = 0; j < n; ++j) {
    double s = creal(L[IDX(j, j, ld)]);
    for (int k = 0; k < j; ++k) {
      zc l = L[IDX(j, k, ld)];
      s -= creal(l) * creal(l) + cimag(l) * cimag(l);
    }
    if (!(s > 0.0) || !isfinite(s)) return j + 1;
    double ljj = sqrt(s);
    L[IDX(j, j, ld)] = ljj;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      zc t = L[IDX(i, j, ld)];
      for (int k = 0; k < j; ++k) t -= L[IDX(i, k, ld)] * conj(L[IDX(j, k, ld)]);
      L[IDX(i, j, ld)] = t / ljj;
    }
    for (int i = 0; i < j; ++i) L[IDX(i, j, ld)] = 0.0;
  }
  return 0;
}

/* forward substitution L y = b for each of m right-hand sides (columns of Y) */
static void fwd_subst(int n, const zc* L, int ldl, int m, zc* Y, int ldy) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < m; ++c) {
    zc* y = Y + (size_t)c * ldy;
    for (int i = 0; i < n; ++i) {
      zc t = y[i];
      for (int k = 0; k < i; ++k) t -= L[IDX(i, k, ldl)] * y[k];
      y[i] = t / L[IDX(i, i, ldl)];
    }
  }
}

/* back substitution L^H x = y for each of m right-hand sides */
static void back_subst_h(int n, const zc* L, int ldl, int m, zc* Y, int ldy) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < m; ++c) {
    zc* y = Y + (size_t)c * ldy;
    for (int i = n - 1; i >= 0; --i) {
      zc t = y[i];
      /* (L^H)_{ik} = conj(L_{ki}) for k > i */
      for (int k = i + 1; k < n; ++k) t -= conj(L[IDX(k, i, ldl)]) * y[k];
      y[i] = t / conj(L[IDX(i, i, ldl)]);
    }
  }
}

/* ---- step 2: C = L^{-1} A L^{-H} from full Hermitian A; C overwrites W.
 * W = L^{-1} A; V = L^{-1} W^H; C = V^H; then C = (C + C^H)/2. */
static void reduce_to_standard(int n, const zc* L, zc* W /* in: A full, out: C */) {
  zc* T = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  fwd_subst(n, L, n, n, W, n);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) T[IDX(i, j, n)] = conj(W[IDX(j, i, n)]);
  fwd_subst(n, L, n, n, T, n);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) W[IDX(i, j, n)] = conj(T[IDX(j, i, n)]);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) {
      zc h = 0.5 * (W[IDX(i, j, n)] + conj(W[IDX(j, i, n)]));
      if (i == j) h = creal(h);
      W[IDX(i, j, n)] = h;
      W[IDX(j, i, n)] = conj(h);
    }
  free(T);
}

/* ---- step 3: Householder tridiagonalisation of Hermitian C (full storage).
 * For column k the reflector G_k = I - tau v v^H (v_0 = 1) maps
 * x = C(k+1:n, k) to beta e_1 with beta real: beta = -sign(Re x_0) ||x||,
 * tau = (beta - x_0)/beta, v = x / (x_0 - beta).  The two-sided update
 * G^H C G is C - v w^H - w v^H with p = tau C v, w = p - (1/2) conj(tau)
 * (v^H p) v.  On exit d, e hold T (real) and V, tau the reflectors
 * (column k of V stores v for reflector k, starting at row k+1). */
static void hetrd(int n, zc* C, double* d, double* e, zc* V, zc* tau) {
  zc* p = (zc*)malloc(sizeof(zc) * n);
  for (int k = 0; k < n - 1; ++k) {
    int m = n - k - 1; /* length of x */
    zc* x = C + IDX(k + 1, k, n);
    double sig = 0.0;
    for (int i = 1; i < m; ++i) sig += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    zc alpha = x[0];
    zc t = 0.0;
    double beta;
    zc* v = V + IDX(0, k, n);
    memset(v, 0, sizeof(zc) * n);
    if (sig == 0.0 && cimag(alpha) == 0.0) {
      /* already in the wanted form: no reflection */
      beta = creal(alpha);
      t = 0.0;
    } else {
      double nrm = sqrt(creal(alpha) * creal(alpha) + cimag(alpha) * cimag(alpha) + sig);
      beta = (creal(alpha) >= 0.0) ? -nrm : nrm;
      t = (beta - alpha) / beta;
      zc scal = 1.0 / (alpha - beta);
      v[k + 1] = 1.0;
      for (int i = 1; i < m; ++i) v[k + 1 + i] = x[i] * scal;
    }
    tau[k] = t;
    e[k] = beta;
    if (t != 0.0) {
      zc* vv = v + k + 1;
      zc* CC = C + IDX(k + 1, k + 1, n);
      /* p = tau * C22 * v */
#pragma omp parallel for schedule(static)
      for (int i = 0; i < m; ++i) {
        zc s = 0.0;
        for (int j = 0; j < m; ++j) s += CC[IDX(i, j, n)] * vv[j];
        p[i] = t * s;
      }
      zc vhp = 0.0;
      for (int i = 0; i < m; ++i) vhp += conj(vv[i]) * p[i];
      zc K = 0.5 * conj(t) * vhp;
      for (int i = 0; i < m; ++i) p[i] -= K * vv[i]; /* p is now w */
#pragma omp parallel for schedule(static)
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i)
          CC[IDX(i, j, n)] -= vv[i] * conj(p[j]) + p[i] * conj(vv[j]);
    }
    /* column k of the reduced matrix is (beta, 0, ..., 0) below the diagonal */
    x[0] = beta;
    for (int i = 1; i < m; ++i) x[i] = 0.0;
  }
  for (int k = 0; k < n; ++k) d[k] = creal(C[IDX(k, k, n)]);
  free(p);
}

/* ---- step 4: implicit symmetric QR with Wilkinson shift (G&VL 8.3).
 * d[0..n-1], e[0..n-2] (e[i] couples i and i+1).  Z is n x n real, stored
 * row-major (Z[i*n + k]); each Givens similarity T <- G T G^T in the plane
 * (k, k+1) with G = [c s; -s c] is accumulated as Z <- Z G^T.
 * Returns 0 on success, 1 when 30 n steps were not enough. */
static int tridiag_qr(int n, double* d, double* e, double* Z) {
  const double eps = 2.220446049250313e-16;
  long iters = 0, maxit = 30L * n;
  int m = n - 1;
  /* absolute floor eps ||T||_1 so that blocks whose diagonal is near zero
   * still deflate (a backward-stable criterion) */
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i)
    tnorm = fmax(tnorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0));
  const double floor_abs = eps * tnorm;
  double* cs = (double*)malloc(sizeof(double) * 2 * (n > 1 ? n : 1));
  while (m > 0) {
    if (fabs(e[m - 1]) <= eps * (fabs(d[m - 1]) + fabs(d[m])) || fabs(e[m - 1]) <= floor_abs) {
      e[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && fabs(e[l - 1]) > eps * (fabs(d[l - 1]) + fabs(d[l])) && fabs(e[l - 1]) > floor_abs) --l;
    if (l > 0) e[l - 1] = 0.0;
    if (++iters > maxit) { free(cs); return 1; }
    /* Wilkinson shift from the trailing 2x2 block [a b; b c] */
    double a = d[m - 1], b = e[m - 1], c = d[m];
    double del = 0.5 * (a - c);
    double den = del + copysign(hypot(del, b), del);
    double mu = (den != 0.0) ? c - b * b / den : c - fabs(b);
    double x = d[l] - mu, z = e[l];
    int nrot = 0;
    for (int k = l; k < m; ++k) {
      double r = hypot(x, z);
      double cc, ss;
      if (r == 0.0) { cc = 1.0; ss = 0.0; } else { cc = x / r; ss = z / r; }
      if (k > l) e[k - 1] = r;
      double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = cc * cc * dk + 2.0 * cc * ss * ek + ss * ss * dk1;
      d[k + 1] = ss * ss * dk - 2.0 * cc * ss * ek + cc * cc * dk1;
      e[k] = cc * ss * (dk1 - dk) + (cc * cc - ss * ss) * ek;
      if (k < m - 1) {
        x = e[k];
        z = ss * e[k + 1];
        e[k + 1] = cc * e[k + 1];
      }
      cs[2 * nrot] = cc;
      cs[2 * nrot + 1] = ss;
      ++nrot;
    }
    /* apply the sweep's rotations to every row of Z (rows are independent) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double* zr = Z + (size_t)i * n;
      for (int q = 0; q < nrot; ++q) {
        int k = l + q;
        double cc = cs[2 * q], ss = cs[2 * q + 1];
        double z0 = zr[k], z1 = zr[k + 1];
        zr[k] = cc * z0 + ss * z1;
        zr[k + 1] = -ss * z0 + cc * z1;
      }
    }
  }
  free(cs);
  return 0;
}

/* stable ascending order of theta (insertion sort on an index array is
 * O(n^2) but trivially correct; n is at most a few thousand here) */
static void stable_argsort(int n, const double* th, int* idx) {
  for (int i = 0; i < n; ++i) idx[i] = i;
  /* merge sort for O(n log n) with stability */
  int* tmp = (int*)malloc(sizeof(int) * n);
  for (int w = 1; w < n; w *= 2) {
    for (int lo = 0; lo < n; lo += 2 * w) {
      int mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
      int a = lo, b = mid, o = lo;
      while (a < mid && b < hi) tmp[o++] = (th[idx[b]] < th[idx[a]]) ? idx[b++] : idx[a++];
      while (a < mid) tmp[o++] = idx[a++];
      while (b < hi) tmp[o++] = idx[b++];
    }
    memcpy(idx, tmp, sizeof(int) * n);
  }
  free(tmp);
}

/* make the largest-modulus entry of each column real and positive; among
 * entries within 1e-12 (relative) of the maximum the lowest index wins */
void oref_phase_normalize(int n, int m, zc* X, int ldx) {
  for (int c = 0; c < m; ++c) {
    zc* x = X + (size_t)c * ldx;
    double amax = 0.0;
    for (int i = 0; i < n; ++i) amax = fmax(amax, cabs(x[i]));
    if (amax == 0.0) continue;
    int piv = 0;
    for (int i = 0; i < n; ++i)
      if (cabs(x[i]) >= amax * (1.0 - 1e-12)) { piv = i; break; }
    zc ph = conj(x[piv]) / cabs(x[piv]);
    for (int i = 0; i < n; ++i) x[i] *= ph;
  }
}

/* ---- the whole direct solve: lowest nev eigenpairs of (A, B) ---- */
int oref_solve(int n, const zc* A, int lda, const zc* B, int ldb, int nev,
               double* lam, zc* X, int ldx) {
  if (n < 1) return -1;
  if (lda < n) return -3;
  if (ldb < n) return -5;
  if (nev < 1 || nev > n) return -6;
  if (ldx < n) return -9;
  size_t nn = (size_t)n * n;
  zc* L = (zc*)malloc(sizeof(zc) * nn);
  zc* C = (zc*)malloc(sizeof(zc) * nn);
  herm_from_lower(n, B, ldb, L);
  int info = oref_potrf(n, L, n);
  if (info) { free(L); free(C); return n + info; }
  herm_from_lower(n, A, lda, C);
  reduce_to_standard(n, L, C);
  double* d = (double*)malloc(sizeof(double) * n);
  double* e = (double*)malloc(sizeof(double) * (n > 1 ? n : 1));
  zc* V = (zc*)malloc(sizeof(zc) * nn);
  zc* tau = (zc*)malloc(sizeof(zc) * (n > 1 ? n : 1));
  hetrd(n, C, d, e, V, tau);
  double* Z = (double*)calloc(nn, sizeof(double));
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  int qr = tridiag_qr(n, d, e, Z);
  int* idx = (int*)malloc(sizeof(int) * n);
  stable_argsort(n, d, idx);
  /* Y(:, c) = U z_{idx[c]} with U = G_0 G_1 ... G_{n-2}: apply from the last
   * reflector to the first, G_k y = y - tau_k v_k (v_k^H y). */
#pragma omp parallel for schedule(dynamic, 2)
  for (int c = 0; c < nev; ++c) {
    zc* y = X + (size_t)c * ldx;
    for (int i = 0; i < n; ++i) y[i] = Z[(size_t)i * n + idx[c]];
    for (int k = n - 2; k >= 0; --k) {
      if (tau[k] == 0.0) continue;
      const zc* v = V + IDX(0, k, n);
      zc s = 0.0;
      for (int i = k + 1; i < n; ++i) s += conj(v[i]) * y[i];
      s *= tau[k];
      for (int i = k + 1; i < n; ++i) y[i] -= s * v[i];
    }
    lam[c] = d[idx[c]];
  }
  back_subst_h(n, L, n, nev, X, ldx);
  oref_phase_normalize(n, nev, X, ldx);
  free(L); free(C); free(d); free(e); free(V); free(tau); free(Z); free(idx);
  return qr ? 1 : 0;
}

/* ---- per-pair residual ||A x_i - lambda_i B x_i||_2 (A, B read as lower) and
 * max |X^H B X - I|.  Only columns listed in cols (or all when cols==NULL). */
void oref_residuals(int n, const zc* A, int lda, const zc* B, int ldb, int m,
                    const double* lam, const zc* X, int ldx, double* res, double* orth) {
  zc* Af = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  zc* Bf = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  herm_from_lower(n, A, lda, Af);
  herm_from_lower(n, B, ldb, Bf);
  zc* BX = (zc*)malloc(sizeof(zc) * (size_t)n * m);
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < m; ++c) {
    const zc* x = X + (size_t)c * ldx;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      zc ax = 0.0, bx = 0.0;
      for (int j = 0; j < n; ++j) {
        ax += Af[IDX(i, j, n)] * x[j];
        bx += Bf[IDX(i, j, n)] * x[j];
      }
      BX[(size_t)c * n + i] = bx;
      zc r = ax - lam[c] * bx;
      s += creal(r) * creal(r) + cimag(r) * cimag(r);
    }
    res[c] = sqrt(s);
  }
  double om = 0.0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      zc s = 0.0;
      for (int i = 0; i < n; ++i) s += conj(X[(size_t)a * ldx + i]) * BX[(size_t)b * n + i];
      if (a == b) s -= 1.0;
      om = fmax(om, cabs(s));
    }
  *orth = om;
  free(Af); free(Bf); free(BX);
}

/* residual of selected single pairs, O(n^2) each: for sampling large runs */
void oref_pair_residual(int n, const zc* A, int lda, const zc* B, int ldb,
                        double lam, const zc* x, double* res, double* xbx) {
  double s = 0.0;
  zc q = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int i = 0; i < n; ++i) {
    zc ax = 0.0, bx = 0.0;
    for (int j = 0; j < n; ++j) {
      zc a = (i >= j) ? A[IDX(i, j, lda)] : conj(A[IDX(j, i, lda)]);
      zc b = (i >= j) ? B[IDX(i, j, ldb)] : conj(B[IDX(j, i, ldb)]);
      if (i == j) { a = creal(a); b = creal(b); }
      ax += a * x[j];
      bx += b * x[j];
    }
    zc r = ax - lam * bx;
    s += creal(r) * creal(r) + cimag(r) * cimag(r);
  }
  for (int i = 0; i < n; ++i) {
    zc bx = 0.0;
    for (int j = 0; j < n; ++j) {
      zc b = (i >= j) ? B[IDX(i, j, ldb)] : conj(B[IDX(j, i, ldb)]);
      if (i == j) b = creal(b);
      bx += b * x[j];
    }
    q += conj(x[i]) * bx;
  }
  *res = sqrt(s);
  *xbx = creal(q);
}

/* ---- Sylvester inertia: number of eigenvalues of (A, B) below sigma.
 * A - sigma B = L (C - sigma I) L^H is congruent to C - sigma I, so the count
 * of negative pivots of an LDL^H factorisation (no pivoting) of A - sigma B
 * is the count of eigenvalues < sigma.  Returns -1 on an exactly zero pivot. */
long oref_inertia(int n, const zc* A, int lda, const zc* B, int ldb, double sigma) {
  zc* M = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  double* D = (double*)malloc(sizeof(double) * n);
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) M[IDX(i, j, n)] = A[IDX(i, j, lda)] - sigma * B[IDX(i, j, ldb)];
  long neg = 0;
  for (int j = 0; j < n; ++j) {
    double dj = creal(M[IDX(j, j, n)]);
    for (int k = 0; k < j; ++k) {
      zc l = M[IDX(j, k, n)];
      dj -= (creal(l) * creal(l) + cimag(l) * cimag(l)) * D[k];
    }
    if (dj == 0.0 || !isfinite(dj)) { free(M); free(D); return -1; }
    D[j] = dj;
    if (dj < 0.0) ++neg;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < n; ++i) {
      zc t = M[IDX(i, j, n)];
      for (int k = 0; k < j; ++k) t -= M[IDX(i, k, n)] * conj(M[IDX(j, k, n)]) * D[k];
      M[IDX(i, j, n)] = t / dj;
    }
  }
  free(M); free(D);
  return neg;
}

/* ---- bisection for the k-th smallest eigenvalue (0-based) on inertia counts,
 * within [lo, hi] which must bracket the spectrum; stops at an absolute width
 * of tol.  Independent of the QR route. */
double oref_bisect(int n, const zc* A, int lda, const zc* B, int ldb, int k,
                   double lo, double hi, double tol) {
  while (hi - lo > tol) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    long c = oref_inertia(n, A, lda, B, ldb, mid);
    if (c < 0) { mid = nextafter(mid, hi); c = oref_inertia(n, A, lda, B, ldb, mid); }
    if (c > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

/* dense complex solve M x = r by Gaussian elimination with partial pivoting
 * (M overwritten) -- used by inverse iteration only */
static int zgesv_small(int n, zc* M, zc* r) {
  for (int j = 0; j < n; ++j) {
    int p = j;
    for (int i = j + 1; i < n; ++i) if (cabs(M[IDX(i, j, n)]) > cabs(M[IDX(p, j, n)])) p = i;
    if (M[IDX(p, j, n)] == 0.0) M[IDX(p, j, n)] = 1e-300;
    if (p != j) {
      for (int c = 0; c < n; ++c) { zc t = M[IDX(j, c, n)]; M[IDX(j, c, n)] = M[IDX(p, c, n)]; M[IDX(p, c, n)] = t; }
      zc t = r[j]; r[j] = r[p]; r[p] = t;
    }
    for (int i = j + 1; i < n; ++i) {
      zc f = M[IDX(i, j, n)] / M[IDX(j, j, n)];
      for (int c = j; c < n; ++c) M[IDX(i, c, n)] -= f * M[IDX(j, c, n)];
      r[i] -= f * r[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    zc t = r[i];
    for (int c = i + 1; c < n; ++c) t -= M[IDX(i, c, n)] * r[c];
    r[i] = t / M[IDX(i, i, n)];
  }
  return 0;
}

/* ---- inverse iteration for the eigenvector of (A, B) at a given eigenvalue
 * estimate mu: x <- (A - mu B)^{-1} B x, B-normalised; `iters` passes.
 * x holds the start vector on entry. */
void oref_inverse_iteration(int n, const zc* A, int lda, const zc* B, int ldb, double mu,
                            int iters, zc* x) {
  zc* Af = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  zc* Bf = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  zc* M = (zc*)malloc(sizeof(zc) * (size_t)n * n);
  zc* r = (zc*)malloc(sizeof(zc) * n);
  herm_from_lower(n, A, lda, Af);
  herm_from_lower(n, B, ldb, Bf);
  for (int it = 0; it < iters; ++it) {
    for (size_t q = 0; q < (size_t)n * n; ++q) M[q] = Af[q] - mu * Bf[q];
    for (int i = 0; i < n; ++i) {
      zc s = 0.0;
      for (int j = 0; j < n; ++j) s += Bf[IDX(i, j, n)] * x[j];
      r[i] = s;
    }
    zgesv_small(n, M, r);
    zc q = 0.0;
    for (int i = 0; i < n; ++i) {
      zc s = 0.0;
      for (int j = 0; j < n; ++j) s += Bf[IDX(i, j, n)] * r[j];
      q += conj(r[i]) * s;
    }
    double nrm = sqrt(creal(q));
    for (int i = 0; i < n; ++i) x[i] = r[i] / nrm;
  }
  free(Af); free(Bf); free(M); free(r);
}

/* ---- eigenvalue gradient for L = sum_i w_i lambda_i (first-order
 * perturbation, d lambda_i = x_i^H (dA - lambda_i dB) x_i with x_i^H B x_i = 1):
 *   G_A = X diag(w) X^H,   G_B = -X diag(w .* lambda) X^H   (full n x n) */
void oref_grad(int n, int m, const zc* X, int ldx, const double* lam, const double* w,
               zc* GA, int ldga, zc* GB, int ldgb) {
#pragma omp parallel for schedule(static)
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      zc sa = 0.0, sb = 0.0;
      for (int c = 0; c < m; ++c) {
        zc t = X[(size_t)c * ldx + i] * conj(X[(size_t)c * ldx + j]);
        sa += w[c] * t;
        sb += w[c] * lam[c] * t;
      }
      if (GA) GA[IDX(i, j, ldga)] = sa;
      if (GB) GB[IDX(i, j, ldgb)] = -sb;
    }
}
