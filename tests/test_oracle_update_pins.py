"""Pins of the oracle's thresholded partial update (section 2, paragraph
"Matrix generation": delta = largest entry change between adjacent SCF
Hamiltonians, entries whose change exceeds p_t * delta are updated).

What fixes the result independently of the oracle's own formula:
* exact lattice counts on a grid of exactly representable changes whose
  modulus depends on (i, j) asymmetrically (a transposed triangle, a dropped
  real or imaginary part, a wrong delta or a non-strict comparison all change
  the count),
* an exact tie at the threshold (strict comparison),
* the limiting thresholds p_t = 0 (everything that changed) and p_t >= 1
  (nothing), nesting of the masks across thresholds,
* a brute-force loop with complex abs() on tiny inputs,
* Weyl's inequality for the generalized eigenvalues of the truncated pencil.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

from paper_1007_4400_amd import synth


def _grid_pair(n):
    """A_cur = 0 and A_new with |A_new(i, j)| = (2i + j) / 128 (exact in
    binary), real for even i + j and imaginary for odd i + j."""
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    mag = (2 * i + j) / 128.0
    A_new = np.where((i + j) % 2 == 0, mag + 0j, 1j * mag)
    return np.zeros((n, n), dtype=np.complex128), A_new


def _lattice_count(n, c):
    """#{(i, j): 0 <= j <= i < n, 2i + j > c}, counted row by row: in row i
    the admissible j are max(0, floor(c - 2i) + 1) .. i."""
    total = 0
    for i in range(n):
        lo = max(0, math.floor(c - 2 * i) + 1)
        total += max(0, i - lo + 1)
    return total


@pytest.mark.parametrize("n,p_t", [(9, 0.3), (37, 0.1), (64, 0.55), (130, 0.9), (200, 0.05)])
def test_grid_closed_form_count(oracle_mod, n, p_t):
    A_cur, A_new = _grid_pair(n)
    out, mask, delta, updated = oracle_mod.threshold_update(A_cur, A_new, p_t)
    # the largest lower-triangle change sits at i = j = n - 1
    assert delta == 3 * (n - 1) / 128.0
    c = p_t * 3 * (n - 1)  # threshold on 2i + j
    assert updated == _lattice_count(n, c)
    # every updated entry takes the new value, the rest keep the old
    assert np.array_equal(out[mask], A_new[mask])
    assert np.all(out[~mask] == 0)


def test_grid_exact_tie_is_not_updated(oracle_mod):
    # n = 9: delta = 24/128; p_t = 0.5 puts the threshold at 2i + j = 12
    # exactly (squared values 144/16384 both sides, exact in binary)
    A_cur, A_new = _grid_pair(9)
    _, mask, _, updated = oracle_mod.threshold_update(A_cur, A_new, 0.5)
    i, j = np.nonzero(np.tril(np.ones((9, 9), dtype=bool)))
    on_tie = (2 * i + j) == 12
    assert on_tie.any()
    assert not mask[i[on_tie], j[on_tie]].any()
    assert updated == _lattice_count(9, 12.0)


def test_upper_triangle_is_ignored(oracle_mod):
    # a huge change in the strict upper triangle changes nothing
    A_cur, A_new = _grid_pair(40)
    A_big = A_new.copy()
    A_big[3, 30] = 1e6
    r1 = oracle_mod.threshold_update(A_cur, A_new, 0.2)
    r2 = oracle_mod.threshold_update(A_cur, A_big, 0.2)
    assert r1[2] == r2[2] and r1[3] == r2[3]
    assert np.array_equal(r1[1], r2[1])
    assert r2[0][3, 30] == 0


def _random_pair(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = 0.5 * (A + A.conj().T)
    E = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    E *= np.exp(-np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]) / (0.2 * n))
    return A, A + 1e-3 * 0.5 * (E + E.conj().T)


def test_limits_and_nesting(oracle_mod):
    A_cur, A_new = _random_pair(70, 3)
    low = np.tril(np.ones((70, 70), dtype=bool))
    out0, m0, _, c0 = oracle_mod.threshold_update(A_cur, A_new, 0.0)
    assert c0 == int(low.sum())  # every lower entry changed
    assert np.array_equal(out0[low], A_new[low])
    out1, m1, _, c1 = oracle_mod.threshold_update(A_cur, A_new, 1.0)
    assert c1 == 0 and np.array_equal(out1, A_cur)
    prev = m0
    for p in [0.01, 0.05, 0.1, 0.3, 0.6, 0.99]:
        _, m, _, _ = oracle_mod.threshold_update(A_cur, A_new, p)
        assert np.all(~m | prev)  # masks shrink as the threshold rises
        prev = m
    # no change at all: nothing is updated, delta = 0
    _, m, d, c = oracle_mod.threshold_update(A_cur, A_cur.copy(), 0.1)
    assert d == 0.0 and c == 0


def test_brute_force_tiny(oracle_mod):
    for seed in range(5):
        A_cur, A_new = _random_pair(6, 10 + seed)
        p_t = 0.25
        delta = 0.0
        for i in range(6):
            for j in range(i + 1):
                delta = max(delta, abs(A_new[i, j] - A_cur[i, j]))
        ref = A_cur.copy()
        count = 0
        for i in range(6):
            for j in range(i + 1):
                if abs(A_new[i, j] - A_cur[i, j]) > p_t * delta:
                    ref[i, j] = A_new[i, j]
                    count += 1
        out, mask, d, c = oracle_mod.threshold_update(A_cur, A_new, p_t)
        assert abs(d - delta) <= 1e-15 * delta
        assert c == count
        assert np.array_equal(out, ref)


def test_masked_update_reproduces_threshold_update(oracle_mod):
    A_cur, A_new = _random_pair(50, 7)
    out, mask, _, _ = oracle_mod.threshold_update(A_cur, A_new, 0.2)
    assert np.array_equal(oracle_mod.masked_update(A_cur, A_new, mask), out)
    # an all-true mask takes the whole lower triangle, never the upper
    full = oracle_mod.masked_update(A_cur, A_new, np.ones((50, 50), dtype=bool))
    low = np.tril(np.ones((50, 50), dtype=bool))
    assert np.array_equal(full[low], A_new[low]) and np.array_equal(full[~low], A_cur[~low])


def test_nonfinite_change_disables_update(oracle_mod):
    A_cur, A_new = _random_pair(20, 8)
    A_new[5, 2] = np.nan
    out, mask, d, c = oracle_mod.threshold_update(A_cur, A_new, 0.1)
    assert c == 0 and not mask.any() and math.isnan(d)
    assert np.array_equal(out, A_cur)


def _herm_from_lower(M):
    L = np.tril(M, -1)
    return L + L.conj().T + np.diag(M.diagonal().real)


@pytest.mark.parametrize("p_t", [0.05, 0.1, 0.3])
def test_weyl_bound_on_truncated_pencil(oracle_mod, p_t):
    """Skipping entries below p_t * delta perturbs the pencil by a Hermitian
    E with |E_ij| <= p_t * delta, so each generalized eigenvalue moves by at
    most ||E||_2 / lambda_min(B) (Weyl's inequality after Cholesky
    reduction)."""
    wl = synth.update_scaled(synth.UPDATE_SMALL, 120, steps=2)
    pen, _ = synth.make_pencil(synth.scaled(synth.SMALL, 120), 4)
    seq = list(synth.update_sequence(wl, 5, A0=pen.A))
    A_cur, A_new = seq[0], seq[1]
    out, mask, delta, _ = oracle_mod.threshold_update(A_cur, A_new, p_t)
    E = _herm_from_lower(out) - _herm_from_lower(A_new)
    assert np.max(np.abs(E)) <= p_t * delta
    lam_t = sl.eigh(_herm_from_lower(out), pen.B, eigvals_only=True)
    lam_n = sl.eigh(_herm_from_lower(A_new), pen.B, eigvals_only=True)
    bound = np.linalg.norm(E, 2) / np.linalg.eigvalsh(pen.B).min()
    assert np.max(np.abs(lam_t - lam_n)) <= bound * (1 + 1e-8) + 1e-12
    # and the bound is not vacuous here: some eigenvalue actually moved
    assert np.max(np.abs(lam_t - lam_n)) > 0


def test_update_sequence_fraction_falls():
    """The generator's stated behaviour: the share above threshold falls
    along the sequence and the frozen bands never change enough."""
    from oracle import oracle

    wl = synth.update_scaled(synth.UPDATE_LARGE, 512, steps=8)
    seq = synth.update_sequence(wl, 1)
    A_cur = next(seq)
    fr = []
    w = synth.update_weights(wl)
    for A_new in seq:
        A_cur, mask, _, c = oracle.threshold_update(A_cur, A_new, wl.p_t)
        fr.append(c / (wl.n * (wl.n + 1) / 2))
        fz = np.nonzero(w < 1)[0]
        assert not mask[np.ix_(fz, fz)].any()
    assert fr[0] > 0.4 and fr[-1] < 0.3 and fr[0] > fr[-1]
