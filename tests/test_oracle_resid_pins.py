"""Pins of the oracle's residual functions and its norm bound.

``oracle.residuals`` and ``oracle.pair_residual`` are the residual half of
every parity check (the per-pair residual ||A x_i - lambda_i B x_i||_2 of the
pencil of the paper's section 1, eq. (3), and the B-orthonormality
max |X^H B X - I|).  They are pinned here by values derived by hand, by exact
constructed pairs perturbed by a known amount, and by a known scaling of a
B-orthonormal block.  Each pin is then shown to be sensitive: copies of the
oracle's C source with a planted mistake (a zero result, a missing square
root, a dropped B, a mirrored triangle without the conjugate, the upper
triangle read instead of the lower, the identity not subtracted) are compiled
and must fail at least one pin.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sl

from paper_1007_4400_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SRC = os.path.join(os.path.dirname(HERE), "oracle", "gevp_oracle.c")


# --------------------------------------------------------------------------
# the functions under test, as thin wrappers over any build of the C source


class _Lib:
    def __init__(self, path):
        lib = ctypes.CDLL(path)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        lib.oref_residuals.argtypes = [I, P, I, P, I, I, P, P, I, P, P]
        lib.oref_residuals.restype = None
        lib.oref_pair_residual.argtypes = [I, P, I, P, I, D, P, P, P]
        lib.oref_pair_residual.restype = None
        self.lib = lib

    def residuals(self, A, B, lam, X):
        A, B, X = (np.asfortranarray(np.asarray(M, dtype=np.complex128)) for M in (A, B, X))
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        n, m = X.shape
        res = np.empty(m)
        orth = np.zeros(1)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self.lib.oref_residuals(n, p(A), n, p(B), n, m, p(lam), p(X), n, p(res), p(orth))
        return res, float(orth[0])

    def pair_residual(self, A, B, lam, x):
        A, B = (np.asfortranarray(np.asarray(M, dtype=np.complex128)) for M in (A, B))
        x = np.ascontiguousarray(x, dtype=np.complex128)
        r, q = np.zeros(1), np.zeros(1)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self.lib.oref_pair_residual(A.shape[0], p(A), A.shape[0], p(B), B.shape[0], float(lam), p(x),
                                    p(r), p(q))
        return float(r[0]), float(q[0])


@pytest.fixture(scope="module")
def real_lib(oracle_mod):
    return _Lib(oracle_mod._LIB_PATH)


def _planted(tmpdir, name, subs):
    """Compile a copy of the oracle source with the replacements `subs`
    (each old text must occur exactly once)."""
    src = open(ORACLE_SRC).read()
    for old, new in subs:
        assert src.count(old) == 1, f"{name}: pattern not unique in the oracle source: {old!r}"
        src = src.replace(old, new)
    c = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"{name}.so")
    open(c, "w").write(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"],
                   check=True)
    return _Lib(so)


# --------------------------------------------------------------------------
# the pins, as one checker returning the names of the pins that fail


def _hand_case():
    """2 x 2 pencil with garbage in the strict upper triangles (never read):
    A = [[2, 1-i], [1+i, 3]], B = diag(4, 1)."""
    A = np.array([[2.0, 100.0 + 7.0j], [1.0 + 1.0j, 3.0]])
    B = np.array([[4.0, -55.0 + 3.0j], [0.0, 1.0]])
    return A, B


def _pins(lib):
    failed = []
    A, B = _hand_case()
    x = np.array([1.0, 1.0j])
    # A x = [2 + (1-i) i, (1+i) + 3i] = [3 + i, 1 + 4i];  B x = [4, i]
    # lambda = 1: r = [-1 + i, 1 + 3i], |r|^2 = 2 + 10 = 12
    r, q = lib.pair_residual(A, B, 1.0, x)
    if abs(r - np.sqrt(12.0)) > 1e-14 * np.sqrt(12.0):
        failed.append("pair_hand_lambda1")
    # x^H B x = 4 + 1 = 5
    if abs(q - 5.0) > 1e-14:
        failed.append("pair_hand_xBx")
    # lambda = 0: r = A x, |r|^2 = 10 + 17 = 27
    r0, _ = lib.pair_residual(A, B, 0.0, x)
    if abs(r0 - np.sqrt(27.0)) > 1e-14 * np.sqrt(27.0):
        failed.append("pair_hand_lambda0")
    # two columns x / sqrt(5) (lambda 1) and y = e_2 (lambda 3):
    #   r_x = [-1 + i, 1 + 3i] / sqrt(5), |r_x| = sqrt(12 / 5)
    #   A y = [1 - i, 3], B y = [0, 1]: r_y = [1 - i, 0], |r_y| = sqrt(2)
    #   X^H B X = [[1, -i / sqrt(5)], [i / sqrt(5), 1]]: orth = 1 / sqrt(5)
    X = np.array([[1.0 / np.sqrt(5.0), 0.0], [1.0j / np.sqrt(5.0), 1.0]])
    res, orth = lib.residuals(A, B, np.array([1.0, 3.0]), X)
    if abs(res[0] - np.sqrt(12.0 / 5.0)) > 1e-14 or abs(res[1] - np.sqrt(2.0)) > 1e-14:
        failed.append("resid_hand")
    if abs(orth - 1.0 / np.sqrt(5.0)) > 1e-14:
        failed.append("orth_hand")

    # constructed exact pairs: A = L Q diag(lam) Q^H L^H, B = L L^H has the
    # eigenpairs (lam_i, L^{-H} q_i), B-orthonormal.  Shifting lambda by delta
    # leaves the residual -delta B x_i (up to rounding of the construction).
    wl = synth.scaled(synth.MEDIUM, 48)
    p, _ = synth.make_pencil(wl, 3)
    Xe = sl.solve_triangular(p.L.conj().T, p.Q, lower=False)
    lam = p.Lambda
    sel = np.argsort(lam)[:6]
    Xs, ls = Xe[:, sel], lam[sel]
    delta = 1e-3 * (1.0 + np.abs(ls))
    res, orth = lib.residuals(p.A, p.B, ls + delta, Xs)
    want = delta * np.linalg.norm(p.B @ Xs, axis=0)
    if np.max(np.abs(res - want) / want) > 1e-8:
        failed.append("resid_shifted_exact_pairs")
    if orth > 1e-12:
        failed.append("orth_exact_pairs")
    # one column scaled by (1 + eta): the (j, j) entry of X^H B X - I is
    # (1 + eta)^2 - 1, everything else stays at rounding level
    eta = 1e-3
    Xsc = Xs.copy()
    Xsc[:, 2] *= 1.0 + eta
    _, orth_s = lib.residuals(p.A, p.B, ls, Xsc)
    if abs(orth_s - ((1.0 + eta) ** 2 - 1.0)) > 1e-11:
        failed.append("orth_scaled_column")
    # the per-pair routine agrees with the block routine column by column
    for j in range(Xs.shape[1]):
        rj, qj = lib.pair_residual(p.A, p.B, ls[j] + delta[j], Xs[:, j])
        if abs(rj - res[j]) > 1e-12 * res[j] or abs(qj - 1.0) > 1e-12:
            failed.append(f"pair_vs_block_{j}")
            break
    return failed


def test_residual_pins_hold(real_lib):
    assert _pins(real_lib) == []


MUTANTS = {
    "resid_zero": [("res[c] = sqrt(s);", "res[c] = 0.0;")],
    "resid_no_sqrt": [("res[c] = sqrt(s);", "res[c] = s;")],
    "resid_drops_B": [("zc r = ax - lam[c] * bx;", "zc r = ax - lam[c] * x[i];")],
    "mirror_without_conj": [("F[IDX(i, j, n)] = conj(A[IDX(j, i, lda)]);",
                             "F[IDX(i, j, n)] = A[IDX(j, i, lda)];")],
    "reads_upper": [("F[IDX(i, j, n)] = conj(A[IDX(j, i, lda)]);",
                     "F[IDX(i, j, n)] = A[IDX(i, j, lda)];")],
    "orth_no_identity": [("if (a == b) s -= 1.0;", "(void)0;")],
    "pair_zero": [("*res = sqrt(s);", "*res = 0.0;")],
    "pair_no_sqrt": [("*res = sqrt(s);", "*res = s;")],
    "pair_drops_B": [("zc r = ax - lam * bx;", "zc r = ax - lam * x[i];")],
    "pair_mirror_without_conj": [
        ("zc a = (i >= j) ? A[IDX(i, j, lda)] : conj(A[IDX(j, i, lda)]);",
         "zc a = (i >= j) ? A[IDX(i, j, lda)] : A[IDX(j, i, lda)];")],
    "pair_reads_upper": [
        ("zc a = (i >= j) ? A[IDX(i, j, lda)] : conj(A[IDX(j, i, lda)]);",
         "zc a = A[IDX(i, j, lda)];")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    lib = _planted(str(tmp_path), name, MUTANTS[name])
    assert _pins(lib) != [], f"planted mistake {name} passed every pin"


# --------------------------------------------------------------------------
# the norm lower bound used to scale full-size residual checks


def _hermitian_with_spectrum(n, lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return (Q * lam) @ Q.conj().T


def test_norm2_lower_bound(oracle_mod):
    # ||A||_2 = 50 (the eigenvalue -50 dominates; the rest lie in [-30, 30])
    rng = np.random.default_rng(5)
    lam = np.r_[-50.0, rng.uniform(-30.0, 30.0, 159)]
    A = _hermitian_with_spectrum(160, lam, 6)
    est = oracle_mod.norm2_lower(A, iters=60)
    assert est <= 50.0 * (1 + 1e-12)
    assert est >= 50.0 * (1 - 1e-10)
    # a bound after very few steps is still a lower bound
    assert oracle_mod.norm2_lower(A, iters=2) <= 50.0 * (1 + 1e-12)


def test_norm2_lower_reads_lower_triangle(oracle_mod):
    lam = np.r_[20.0, np.linspace(-10.0, 10.0, 63)]
    A = _hermitian_with_spectrum(64, lam, 7)
    G = A.copy()
    iu = np.triu_indices(64, 1)
    G[iu] = 1e3 * (1 + 1j)  # garbage above the diagonal is never read
    G[np.diag_indices(64)] += 1e-3j  # nor the imaginary part of the diagonal
    assert abs(oracle_mod.norm2_lower(G, iters=80) - 20.0) <= 1e-9 * 20.0


def test_norm2_lower_diagonal_closed_form(oracle_mod):
    # a diagonal matrix: ||A||_2 = max |a_ii|
    d = np.array([3.0, -7.5, 1.0, 0.25, 7.0])
    assert abs(oracle_mod.norm2_lower(np.diag(d).astype(complex), iters=400) - 7.5) <= 1e-9
