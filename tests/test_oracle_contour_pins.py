"""Pins of the oracle's contour-integral (Sakurai-Sugiura) filter, the
candidate solver the paper names for the fast iterations (section 3).

Independent facts used:
* the nq-point trapezoidal rule on the circle with diameter [a, b] and nodes
  at angles 2 pi (j + 1/2) / nq turns the resolvent integral into the
  rational filter f(lambda) = 1 / (1 + t^nq), t = (lambda - gamma) / rho
  (geometric series of the node sums), so for C = Q diag(lambda) Q^H the
  filtered block is Q diag(f) exactly;
* the reduced form and the original-pencil form of the quadrature agree
  (A = L C L^H, B = L L^H);
* LU without row exchanges satisfies L U = M and coincides with LAPACK's
  partially pivoted LU wherever that picks no exchange;
* the seeded iteration reproduces LAPACK's generalized eigenvalues.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1007_4400_amd import synth


def _unitary(n, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(F)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


@pytest.mark.parametrize("nq", [4, 5, 8, 16, 24])
def test_rational_filter_closed_form(oracle_mod, nq):
    n = 60
    lam = np.linspace(-4.0, 6.0, n)  # inside, outside and near the circle's ends
    Q = _unitary(n, nq)
    C = (Q * lam) @ Q.conj().T
    a, b = -2.5, 1.5
    gamma, rho = 0.5 * (a + b), 0.5 * (b - a)
    t = (lam - gamma) / rho
    f = 1.0 / (1.0 + t ** nq)  # odd nq: a pole at t = -1, large values near it
    Y = oracle_mod.contour_filter(C, Q, a, b, nq)
    assert np.abs(Y - Q * f).max() <= 1e-13 * max(1.0, np.abs(f).max())
    # the filter separates: about 1 well inside, about 0 well outside
    assert f[np.abs(t) < 0.5].min() > 0.9 and f[np.abs(t) > 2.0].max() < 0.1


def test_nodes_and_weights(oracle_mod):
    z, w = oracle_mod.contour_points(-1.0, 3.0, 8)
    assert np.allclose(np.abs(z - 1.0), 2.0, atol=1e-15, rtol=0)
    assert np.all(np.abs(z.imag) > 0.5)  # no node on or near the real axis
    # sum_j w_j z_j^k / (2 pi i)-rule: integral of z^k over the circle is 0 for
    # k >= 0 and the rule is exact for |k| < nq; k = -1 about the centre gives 1
    assert abs(np.sum(w)) < 1e-15
    assert abs(np.sum(w / (z - 1.0)) - 1.0) < 1e-15


def test_pencil_form_matches_reduced_form(oracle_mod):
    wl = synth.scaled(synth.SMALL, 50)
    p, _ = synth.make_pencil(wl, 2)
    rng = np.random.default_rng(1)
    V = rng.standard_normal((50, 7)) + 1j * rng.standard_normal((50, 7))
    L = np.linalg.cholesky(p.B)
    Li = np.linalg.inv(L)
    C = Li @ p.A @ Li.conj().T
    Yr = np.linalg.solve(L.conj().T, oracle_mod.contour_filter(C, L.conj().T @ V, -2.5, -0.2, 8))
    Yp = oracle_mod.contour_filter_pencil(p.A, p.B, V, -2.5, -0.2, 8)
    assert np.abs(Yr - Yp).max() <= 1e-11 * np.abs(Yp).max()


def test_lu_nopivot_reconstructs(oracle_mod):
    n = 70
    Q = _unitary(n, 3)
    C = (Q * np.linspace(-3, 40, n)) @ Q.conj().T
    for z in (0.3 + 0.5j, -2.0 + 0.05j, 10.0 - 3.0j):
        M = z * np.eye(n) - C
        F = oracle_mod.lu_nopivot(M)
        Lf = np.tril(F, -1) + np.eye(n)
        U = np.triu(F)
        assert np.abs(Lf @ U - M).max() <= 1e-12 * np.abs(M).max() * n


def test_lu_nopivot_matches_lapack_without_exchanges(oracle_mod):
    rng = np.random.default_rng(4)
    n = 40
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M += np.diag(50.0 + 10j + rng.uniform(0, 1, n))  # diagonal dominance: no exchange
    P, Lr, Ur = sl.lu(M)
    assert np.array_equal(P, np.eye(n))
    F = oracle_mod.lu_nopivot(M)
    assert np.abs(np.tril(F, -1) + np.eye(n) - Lr).max() <= 1e-13
    assert np.abs(np.triu(F) - Ur).max() <= 1e-12 * np.abs(Ur).max()


@pytest.mark.parametrize("n,base", [(120, "small"), (200, "medium")])
def test_seeded_contour_solve_matches_lapack(oracle_mod, n, base):
    wl = synth.scaled(synth.SMALL if base == "small" else synth.MEDIUM, n)
    p, _ = synth.make_pencil(wl, 3)
    lam0, X0 = sl.eigh(p.A, p.B)
    A1 = p.A + 1e-3 * synth.unit_hermitian(np.random.default_rng(5), n)
    lam1 = sl.eigh(A1, p.B, eigvals_only=True)[:wl.nev]
    nb = wl.nev + max(16, int(np.ceil(0.15 * wl.nev)))
    lam, X, its = oracle_mod.contour_solve(A1, p.B, wl.nev, X0[:, :nb], nq=16)
    assert its <= 3
    assert np.max(np.abs(lam - lam1) / np.maximum(np.abs(lam1), 1.0)) <= 1e-10
    R = A1 @ X - (p.B @ X) * lam
    assert np.linalg.norm(R, axis=0).max() <= 1e-10 * np.linalg.norm(A1, 2)
    assert np.abs(X.conj().T @ p.B @ X - np.eye(wl.nev)).max() <= 1e-10
