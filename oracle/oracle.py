"""ctypes front-end of the FP64 CPU oracle in ``gevp_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product package never imports it.

Every function takes and returns numpy arrays in the mathematical sense
(``A[i, j]`` is row i, column j); conversion to the column-major storage the C
code reads happens here.  Only the lower triangles of A and B are read, the
LAPACK ``uplo='L'`` convention.

Functions and the parts of the paper they follow:

* ``solve``            -- lowest ``nev`` eigenpairs of A x = lambda B x with
                          B Hermitian positive definite (section 1, eq. (3);
                          the "full data" direct iteration of section 2).
* ``residuals``        -- ||A x_i - lambda_i B x_i||_2 and max |X^H B X - I|.
* ``pair_residual``    -- the same for one pair, O(n^2): for sampled checks.
* ``norm2_lower``      -- a lower bound of ||A||_2 by power iteration (for
                          residual checks that must not borrow the solver's
                          own norm estimate).
* ``inertia``          -- number of eigenvalues below sigma (Sylvester).
* ``bisect``           -- k-th eigenvalue by bisection on inertia counts.
* ``inverse_iteration``-- eigenvector at a given eigenvalue estimate.
* ``grad``             -- gradient of sum_i w_i lambda_i with respect to A, B.
* ``seed_monitor``, ``seed_monitor_from_overlap``
                       -- how far a block of eigenvectors moved between two SCF
                          steps: principal angles and per-vector deviation
                          angles after an angle-minimising re-indexing
                          (section 2, paragraph "Eigenvectors evolution");
                          plain numpy/scipy, FP64.
* ``threshold_update`` -- partial update of a Hermitian matrix between two
                          SCF steps: only entries whose change exceeds a
                          fraction p_t of the largest change are taken over
                          (section 2, paragraph "Matrix generation"); plain
                          numpy, FP64.
* ``masked_update``    -- the same update driven by a given entry mask.
* ``contour_points``, ``contour_filter``, ``lu_nopivot``, ``contour_solve``
                       -- the contour-integral (Sakurai-Sugiura) filter the paper
                          names as a candidate solver for the fast iterations
                          (section 3, second paragraph): a trapezoidal quadrature
                          of the resolvent on a circle, applied to a block, inside
                          a Rayleigh-Ritz iteration; plain numpy, FP64.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # type: ignore

            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.oref_solve.argtypes = [I, P, I, P, I, I, P, P, I]
        lib.oref_solve.restype = I
        lib.oref_residuals.argtypes = [I, P, I, P, I, I, P, P, I, P, P]
        lib.oref_residuals.restype = None
        lib.oref_pair_residual.argtypes = [I, P, I, P, I, D, P, P, P]
        lib.oref_pair_residual.restype = None
        lib.oref_inertia.argtypes = [I, P, I, P, I, D]
        lib.oref_inertia.restype = ctypes.c_long
        lib.oref_bisect.argtypes = [I, P, I, P, I, I, D, D, D]
        lib.oref_bisect.restype = D
        lib.oref_inverse_iteration.argtypes = [I, P, I, P, I, D, I, P]
        lib.oref_inverse_iteration.restype = None
        lib.oref_grad.argtypes = [I, I, P, I, P, P, P, I, P, I]
        lib.oref_grad.restype = None
        lib.oref_potrf.argtypes = [I, P, I]
        lib.oref_potrf.restype = I
        _lib = lib
    return _lib


def _colmajor(M):
    return np.asfortranarray(np.asarray(M, dtype=np.complex128))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, n):
        self.code = code
        if code > n:
            msg = f"B is not positive definite (Cholesky pivot {code - n})"
        elif code == 1:
            msg = "tridiagonal QR did not converge"
        else:
            msg = f"invalid argument {-code}"
        super().__init__(msg)


def solve(A, B, nev):
    """Lowest ``nev`` eigenpairs (lam ascending, X B-orthonormal, phase
    normalised so the largest-modulus entry of each column is real > 0)."""
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    n = A.shape[0]
    lam = np.empty(nev, dtype=np.float64)
    X = np.empty((n, nev), dtype=np.complex128, order="F")
    rc = lib.oref_solve(n, _ptr(A), n, _ptr(B), n, nev, _ptr(lam), _ptr(X), n)
    if rc != 0:
        raise OracleError(rc, n)
    return lam, np.array(X)


def solve_status(A, B, nev):
    """Like ``solve`` but returns the raw status code instead of raising."""
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    n = A.shape[0]
    lam = np.empty(max(nev, 1), dtype=np.float64)
    X = np.empty((n, max(nev, 1)), dtype=np.complex128, order="F")
    return lib.oref_solve(n, _ptr(A), n, _ptr(B), n, nev, _ptr(lam), _ptr(X), n)


def residuals(A, B, lam, X):
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    X = _colmajor(X)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    n, m = X.shape
    res = np.empty(m, dtype=np.float64)
    orth = np.zeros(1, dtype=np.float64)
    lib.oref_residuals(n, _ptr(A), n, _ptr(B), n, m, _ptr(lam), _ptr(X), n, _ptr(res), _ptr(orth))
    return res, float(orth[0])


def pair_residual(A, B, lam_i, x):
    """(||A x - lam B x||_2, x^H B x) for one pair; A, B may be column-major
    device-sized host arrays (only the lower triangles are read)."""
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    n = A.shape[0]
    r = np.zeros(1)
    q = np.zeros(1)
    lib.oref_pair_residual(n, _ptr(A), n, _ptr(B), n, float(lam_i), _ptr(x), _ptr(r), _ptr(q))
    return float(r[0]), float(q[0])


def norm2_lower(A, iters=40, seed=0):
    """Lower bound of the spectral norm of the Hermitian matrix whose lower
    triangle is A's (the diagonal's real part is used).  Power iteration:
    for any v != 0, ||A v|| / ||v|| <= ||A||_2, and the largest quotient seen
    over ``iters`` steps is returned; it converges to ||A||_2 at the rate
    (|lambda_2| / |lambda_1|)^(2k) for a dominant eigenvalue of multiplicity
    one.  Memory: one lower-triangular copy of A."""
    A = np.asarray(A, dtype=np.complex128)
    n = A.shape[0]
    Lo = np.tril(A, -1)
    dg = np.real(np.diagonal(A)).copy()
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    best = 0.0
    for _ in range(int(iters)):
        # (L + D + L^H) v with L the strict lower triangle
        w = Lo @ v + dg * v + np.conj(Lo.T @ np.conj(v))
        nw = float(np.linalg.norm(w))
        best = max(best, nw)
        if nw == 0.0:
            break
        v = w / nw
    return best


def inertia(A, B, sigma):
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    n = A.shape[0]
    return int(lib.oref_inertia(n, _ptr(A), n, _ptr(B), n, float(sigma)))


def bisect(A, B, k, lo, hi, tol=1e-14):
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    n = A.shape[0]
    return float(lib.oref_bisect(n, _ptr(A), n, _ptr(B), n, int(k), float(lo), float(hi), float(tol)))


def inverse_iteration(A, B, mu, x0, iters=3):
    lib = _load()
    A = _colmajor(A)
    B = _colmajor(B)
    x = np.array(x0, dtype=np.complex128)
    n = A.shape[0]
    lib.oref_inverse_iteration(n, _ptr(A), n, _ptr(B), n, float(mu), int(iters), _ptr(x))
    return x


def grad(X, lam, w):
    """G_A = X diag(w) X^H and G_B = -X diag(w * lam) X^H."""
    lib = _load()
    X = _colmajor(X)
    n, m = X.shape
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    GA = np.empty((n, n), dtype=np.complex128, order="F")
    GB = np.empty((n, n), dtype=np.complex128, order="F")
    lib.oref_grad(n, m, _ptr(X), n, _ptr(lam), _ptr(w), _ptr(GA), n, _ptr(GB), n)
    return np.array(GA), np.array(GB)


def cholesky(B):
    """Lower Cholesky factor of B (lower triangle read); raises if not HPD."""
    lib = _load()
    n = B.shape[0]
    L = np.array(np.tril(B), dtype=np.complex128, order="F")
    rc = lib.oref_potrf(n, _ptr(L), n)
    if rc:
        raise OracleError(n + rc, n)
    return np.array(L)


def seed_monitor_from_overlap(M):
    """Seed monitor statistics of a k x k cross-overlap M = X0^H B X of two
    B-orthonormal blocks (section 2, paragraph "Eigenvectors evolution":
    deviation angles between corresponding eigenvectors of adjacent
    iterations, the eigenvectors re-indexed by an angle-minimising match).

    The singular values of M are the cosines of the principal angles between
    the two spans, so sum sin^2 = k - ||M||_F^2.  The match pi (result column j
    <- seed column pi(j)) minimises the summed deviation angles
    sum_j arccos(min(1, |M[pi(j), j]|)) over permutations (a linear assignment,
    solved by scipy).  Returns (sin_rms, dev_mean, dev_max, reindexed, dev_std,
    dev, pi) with dev[j] = arccos(min(1, |M[pi(j), j]|)) / (pi/2), reindexed =
    #{j: pi(j) != j} and dev_std the population standard deviation."""
    from scipy.optimize import linear_sum_assignment

    M = np.asarray(M, dtype=np.complex128)
    k = M.shape[0]
    absM = np.abs(M)
    sin_rms = float(np.sqrt(max(0.0, k - float(np.sum(absM ** 2))) / k))
    cost = np.arccos(np.minimum(1.0, absM)).T  # cost[j, i]: result column j <- seed column i
    rows, pi = linear_sum_assignment(cost)
    assert np.array_equal(rows, np.arange(k))
    dev = np.array([np.arccos(min(1.0, absM[pi[j], j])) / (np.pi / 2) for j in range(k)])
    reindexed = int(np.sum(pi != np.arange(k)))
    return sin_rms, float(dev.mean()), float(dev.max()), reindexed, float(dev.std()), dev, pi


def seed_monitor(X0, X, B, k):
    """seed_monitor_from_overlap of M = X0[:, :k]^H B X[:, :k]; returns
    (sin_rms, dev_mean, dev_max, reindexed, dev) for the first k columns.

    Here sin_rms comes from the projection residual instead of k - ||M||_F^2,
    which cancels to rounding noise once the angles fall below about 1e-8:
    with X B-orthonormal, R = X0 - X (X^H B X0) = X0 - X M^H is the part of
    X0 B-orthogonal to span(X), and sum of sin^2 of the principal angles is
    trace(R^H B R) (both blocks B-orthonormal with k columns)."""
    X0 = np.asarray(X0, dtype=np.complex128)[:, :k]
    X = np.asarray(X, dtype=np.complex128)[:, :k]
    B = np.asarray(B, dtype=np.complex128)
    M = X0.conj().T @ (B @ X)
    r = seed_monitor_from_overlap(M)
    R = X0 - X @ M.conj().T
    s2 = float(np.real(np.sum(R.conj() * (B @ R))))
    sin_rms = float(np.sqrt(max(0.0, s2) / k))
    return sin_rms, r[1], r[2], r[3], r[5]


def threshold_update(A_cur, A_new, p_t):
    """Thresholded partial update (section 2, paragraph "Matrix generation").

    The paper measures the change between the Hamiltonians of two adjacent
    SCF iterations by the largest entry variation delta = max |A_new - A_cur|
    and normalises the difference by it; entries whose normalised change
    exceeds the threshold p_t (a fraction of delta) are the ones that need
    recomputing, all others keep their previous value.

    Readings: entries are complex, so "largest variation" is the largest
    modulus; only the stored lower triangle (diagonal included) takes part,
    which for a Hermitian change gives the same delta and a mask that mirrors
    onto the upper triangle; "above threshold" is strict.  The comparison
    |dA_ij| > p_t * delta is taken in squared form,
        s_ij = dr*dr + di*di  >  (p_t*p_t) * max s,
    every operation rounded on its own (numpy does not fuse), so the decision
    is a fixed FP64 computation.  Non-finite changes never pass the test.

    Returns (A_out, mask, delta, updated): A_out equals A_cur except on the
    masked entries, which hold A_new's values (the upper triangle is A_cur's);
    mask is a boolean n x n array, True only on updated lower entries;
    delta = sqrt(max s); updated = mask.sum()."""
    A_cur = np.asarray(A_cur, dtype=np.complex128)
    A_new = np.asarray(A_new, dtype=np.complex128)
    n = A_cur.shape[0]
    lower = np.tril(np.ones((n, n), dtype=bool))
    dr = A_new.real - A_cur.real
    di = A_new.imag - A_cur.imag
    with np.errstate(invalid="ignore", over="ignore"):
        s = dr * dr + di * di
    s = np.where(lower, s, 0.0)
    finite = np.isfinite(s)
    if not finite.all():
        # a non-finite change disables the whole update
        return A_cur.copy(), np.zeros((n, n), dtype=bool), float("nan"), 0
    smax = float(s.max()) if n else 0.0
    thr = (p_t * p_t) * smax
    mask = lower & (s > thr)
    A_out = np.where(mask, A_new, A_cur)
    return A_out, mask, float(np.sqrt(smax)), int(mask.sum())


def masked_update(A_cur, A_src, mask):
    """Apply a precomputed entry mask: masked lower-triangle entries take
    A_src's value, everything else keeps A_cur's (the fast iterations of
    section 2, paragraph "Matrix generation", where only part of the entries
    have been regenerated)."""
    A_cur = np.asarray(A_cur, dtype=np.complex128)
    n = A_cur.shape[0]
    m = np.asarray(mask, dtype=bool) & np.tril(np.ones((n, n), dtype=bool))
    return np.where(m, np.asarray(A_src, dtype=np.complex128), A_cur)


# ---------------------------------------------------------------------------
# contour-integral (Sakurai-Sugiura) filter
#
# The paper names a Sakurai-Sugiura eigensolver as a candidate for the fast,
# seeded iterations (section 3) without details.  Written here from the
# published method (Sakurai & Sugiura 2003; with Rayleigh-Ritz extraction,
# Sakurai & Tadano 2007), first moment only: the spectral projector onto the
# eigenvalues inside a closed curve G,
#     P = (1 / 2 pi i) * contour integral over G of (z I - C)^{-1} dz,
# for the reduced matrix C = L^{-1} A L^{-H}, discretised by the trapezoidal
# rule on a circle, and applied to a block V (the previous eigenvectors).


def contour_points(a, b, nq):
    """Nodes and weights of the nq-point trapezoidal rule on the circle whose
    diameter is [a, b] on the real axis: z_j = gamma + rho e^{i t_j},
    w_j = rho e^{i t_j} / nq, t_j = 2 pi (j + 1/2) / nq (no node on the real
    axis), gamma = (a + b) / 2, rho = (b - a) / 2.  With dz = i rho e^{it} dt the
    rule approximates (1 / 2 pi i) * integral of f(z) dz by sum_j w_j f(z_j)."""
    gamma, rho = 0.5 * (a + b), 0.5 * (b - a)
    t = 2.0 * np.pi * (np.arange(nq) + 0.5) / nq
    e = np.exp(1j * t)
    return gamma + rho * e, rho * e / nq


def contour_filter(C, V, a, b, nq):
    """Y = sum_j w_j (z_j I - C)^{-1} V, one dense solve per node."""
    C = np.asarray(C, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    n = C.shape[0]
    z, w = contour_points(a, b, nq)
    Y = np.zeros_like(V)
    for zj, wj in zip(z, w):
        Y += wj * np.linalg.solve(zj * np.eye(n) - C, V)
    return Y


def contour_filter_pencil(A, B, V, a, b, nq):
    """The same quadrature in the original pencil: sum_j w_j (z_j B - A)^{-1} B V.
    With A = L C L^H and B = L L^H this equals L^{-H} contour_filter(C, L^H V)."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    z, w = contour_points(a, b, nq)
    Y = np.zeros_like(V)
    BV = B @ V
    for zj, wj in zip(z, w):
        Y += wj * np.linalg.solve(zj * B - A, BV)
    return Y


def lu_nopivot(M):
    """Doolittle LU without row exchanges, M = L U with L unit lower
    triangular; returned packed (L strictly below the diagonal, U on and
    above).  For M = z I - C with C Hermitian and Im z != 0, -i M has
    Hermitian part Im(z) I, positive definite, so every leading block is
    nonsingular and no pivoting is needed."""
    F = np.array(M, dtype=np.complex128)
    n = F.shape[0]
    for k in range(n):
        F[k + 1:, k] /= F[k, k]
        F[k + 1:, k + 1:] -= np.outer(F[k + 1:, k], F[k, k + 1:])
    return F


def contour_solve(A, B, nev, X0, nq=16, tol=1e-10, nex=None, maxit=20, seed=0):
    """Lowest nev eigenpairs of A x = lambda B x by Rayleigh-Ritz on the
    contour-filtered block (plain FP64 reference of the method):

    1. Cholesky B = L L^H, C = L^{-1} A L^{-H}; block Y = [L^H X0, random]
       of width nb = nev + nex.
    2. Orthonormalise Y (QR), Rayleigh-Ritz: H = Y^H C Y = Z diag(theta) Z^H,
       Y <- Y Z.
    3. Stop when ||C y_i - theta_i y_i|| <= tol ||C||_2 for i < nev.
    4. Contour (chosen once, from the first Ritz values): b halfway between
       theta_{nev-1} and theta_nev, a = theta_0 - (b - theta_0) / 20.
    5. Y <- contour_filter(C, Y, a, b, nq); back to 2.
    Returns (lambda[nev], X (n x nev, B-orthonormal), iterations)."""
    A = np.asarray(A, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    n = A.shape[0]
    if nex is None:
        nex = max(16, int(np.ceil(0.15 * nev)))
    nb = min(n, nev + nex)
    L = np.linalg.cholesky(B)
    Linv = np.linalg.inv(L)
    C = Linv @ A @ Linv.conj().T
    C = 0.5 * (C + C.conj().T)
    normC = np.linalg.norm(C, 2)
    rng = np.random.default_rng(seed)
    Y = (rng.standard_normal((n, nb)) + 1j * rng.standard_normal((n, nb))) / np.sqrt(2.0)
    if X0 is not None:
        X0 = np.asarray(X0, dtype=np.complex128)
        k0 = min(X0.shape[1], nb)
        Y[:, :k0] = L.conj().T @ X0[:, :k0]
    ab = None
    for it in range(1, maxit + 1):
        Q, _ = np.linalg.qr(Y)
        H = Q.conj().T @ C @ Q
        theta, Z = np.linalg.eigh(0.5 * (H + H.conj().T))
        Y = Q @ Z
        R = C @ Y[:, :nev] - Y[:, :nev] * theta[:nev]
        if np.max(np.linalg.norm(R, axis=0)) <= tol * normC:
            break
        if ab is None:
            b = 0.5 * (theta[nev - 1] + theta[nev]) if nb > nev else theta[nev - 1] + 1.0
            ab = (theta[0] - 0.05 * (b - theta[0]), b)
        Y = contour_filter(C, Y, ab[0], ab[1], nq)
    X = np.linalg.solve(L.conj().T, Y[:, :nev])
    return theta[:nev], X, it
