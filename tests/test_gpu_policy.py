"""The cold / seeded / refresh schedule (section 2, paragraph "Eigenvectors
evolution") driving real solves: every step meets the parity bar against
the oracle, a sequence whose perturbations shrink stays on fast seeded
steps, and a large jump between steps triggers a full (cold) refresh."""
import numpy as np
import pytest

from paper_1007_4400_amd import synth
from paper_1007_4400_amd.policy import RestartPolicy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def h():
    from paper_1007_4400_amd import gevp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return gevp.Handle(0)


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda")


def _run(h, oracle_mod, mats, nev, policy):
    from paper_1007_4400_amd import gevp

    modes, X = [], None
    kx = h.block_size(mats[0][0].shape[0], nev)
    for k, (A, B) in enumerate(mats):
        mode = policy.next_mode()
        print(f"policy step {k}: {mode}", flush=True)
        o = gevp.make_opts(precision="bf16x3", seed_monitor=True)
        X0 = X if mode == "seeded" else None
        lam, X, _, info = h.solve(_dev(A), _dev(B), nev, X0=X0, tol=TOL, kx=kx, opts=o)
        res, orth = oracle_mod.residuals(A, B, lam.cpu().numpy()[:nev], X.cpu().numpy()[:, :nev])
        assert res.max() <= TOL * np.linalg.norm(A, 2) and orth <= 1e-9
        policy.record(mode, info)
        modes.append(mode)
    return modes


def test_policy_smooth_sequence_stays_seeded(h, oracle_mod):
    wl = synth.scaled(synth.MEDIUM, 300, nev=30)
    mats = list(synth.sequence(wl, 5, steps=6))
    modes = _run(h, oracle_mod, mats, wl.nev, RestartPolicy())
    assert modes == ["cold"] + ["seeded"] * 5


def test_policy_refreshes_after_a_jump(h, oracle_mod):
    wl = synth.scaled(synth.MEDIUM, 300, nev=30)
    mats = list(synth.sequence(wl, 6, steps=4))
    rng = np.random.default_rng(7)
    G = rng.standard_normal((300, 300)) + 1j * rng.standard_normal((300, 300))
    Hj = 0.5 * (G + G.conj().T)
    Hj *= 10.0 / np.linalg.norm(Hj, 2)
    A3, B = mats[3]
    mats.append((A3 + Hj, B))  # the spectrum moves by O(10): the seed is far off
    mats.append((A3 + Hj, B))
    modes = _run(h, oracle_mod, mats, wl.nev, RestartPolicy(max_sin_rms=0.3))
    assert modes[:5] == ["cold", "seeded", "seeded", "seeded", "seeded"]
    assert modes[5] == "cold"
