"""Seeded input generator: determinism and the properties of the
construction (the stand-in for the paper's FLEUR pencil sequences)."""
import numpy as np
import pytest

from paper_1007_4400_amd import synth


def test_deterministic_per_seed():
    wl = synth.scaled(synth.MEDIUM, 128, steps=3)
    a = [A.copy() for A, _ in synth.sequence(wl, 5)]
    b = [A.copy() for A, _ in synth.sequence(wl, 5)]
    c = [A.copy() for A, _ in synth.sequence(wl, 6)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert not np.array_equal(a[0], c[0])


def test_hermitian_and_hpd():
    p, _ = synth.make_pencil(synth.SMALL, 0)
    assert np.array_equal(p.A, p.A.conj().T)
    assert np.array_equal(p.B, p.B.conj().T)
    assert np.linalg.eigvalsh(p.B).min() > 0


@pytest.mark.parametrize("n", [512, 1024])
def test_condition_of_b_near_1e2(n):
    wl = synth.scaled(synth.MEDIUM, n)
    p, _ = synth.make_pencil(wl, 0)
    assert 50 <= np.linalg.cond(p.B) <= 200


def test_split_spectrum_and_gap():
    p, _ = synth.make_pencil(synth.SMALL, 0)
    lam = np.sort(p.Lambda)
    assert np.all((lam[:16] >= -2) & (lam[:16] <= -0.5))
    assert np.all((lam[16:] >= 0) & (lam[16:] <= 50))


def test_cluster_spectrum_gaps():
    wl = synth.scaled(synth.MEDIUM, 1000)
    p, _ = synth.make_pencil(wl, 1)
    lam = np.sort(p.Lambda)
    low = lam[: wl.nev]
    assert low.min() >= -3 and low.max() <= 0
    assert np.min(np.diff(low)) >= 1e-4 * (1 - 1e-9)


def test_unit_perturbation_norm():
    rng = np.random.default_rng(0)
    H = synth.unit_hermitian(rng, 200)
    assert np.array_equal(H, H.conj().T)
    # 60 power steps give a lower estimate of ||H||_2, so the scaled norm is
    # at least 1 and within a few per cent of it
    nrm = np.linalg.norm(H, 2)
    assert 1.0 - 1e-12 <= nrm <= 1.05


def test_batched_workloads():
    wls = synth.batched_workloads()
    assert len(wls) == 32
    for wl, s in wls:
        assert 1500 <= wl.n <= 3000 and wl.nev == round(0.1 * wl.n)
        assert -0.5 <= wl.shift <= 0.5
    assert len({s for _, s in wls}) == 32
