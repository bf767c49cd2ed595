"""Batched k-points (the paper, section 1: one independent pencil per Bloch
vector): uneven sizes solved concurrently on several streams must give the
same pairs as one-by-one solves (bitwise: each problem's arithmetic is the
same) and pass the oracle bar."""
import numpy as np
import pytest

from paper_1007_4400_amd import synth

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


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_batched_matches_single_and_oracle(h, oracle_mod, precision):
    from paper_1007_4400_amd import gevp

    wls = synth.batched_workloads(count=6, nmin=150, nmax=330, seed=3, steps=2)
    opts = gevp.make_opts(precision=precision, batch_streams=3)
    pencils = [synth.make_pencil(wl, s)[0] for wl, s in wls]
    probs = [{"A": _dev(p.A), "B": _dev(p.B), "nev": wl.nev} for p, (wl, _) in zip(pencils, wls)]
    print("batched", precision, [wl.n for wl, _ in wls], flush=True)
    out = h.solve_batched(probs, tol=TOL, opts=opts)
    for (lam, X, res, info), p, (wl, _) in zip(out, pencils, wls):
        lam1, X1, _, _ = h.solve(_dev(p.A), _dev(p.B), wl.nev, tol=TOL, opts=opts)
        assert torch.equal(lam, lam1) and torch.equal(X, X1)
        lam_ref, _ = oracle_mod.solve(p.A, p.B, wl.nev)
        ln = lam.cpu().numpy()
        assert np.max(np.abs(ln - lam_ref) / np.maximum(np.abs(lam_ref), 1)) <= TOL
        r, orth = oracle_mod.residuals(p.A, p.B, ln, X.cpu().numpy())
        assert r.max() <= TOL * np.linalg.norm(p.A, 2) and orth <= 1e-9


def test_batched_seeded_sequence(h, oracle_mod):
    from paper_1007_4400_amd import gevp

    wls = synth.batched_workloads(count=4, nmin=120, nmax=260, seed=5, steps=3)
    opts = gevp.make_opts(precision="bf16x3", batch_streams=4)
    seqs = [list(synth.sequence(wl, s)) for wl, s in wls]
    X = [None] * len(wls)
    for k in range(3):
        probs = [{"A": _dev(seq[k][0]), "B": _dev(seq[k][1]), "nev": wl.nev, "X0": X[i],
                  "kx": h.block_size(wl.n, wl.nev, opts)} for i, ((wl, _), seq) in enumerate(zip(wls, seqs))]
        out = h.solve_batched(probs, tol=TOL, opts=opts)
        for i, ((lam, Xi, res, info), (wl, _), seq) in enumerate(zip(out, wls, seqs)):
            A, B = seq[k]
            lam_ref, _ = oracle_mod.solve(A, B, wl.nev)
            ln = lam.cpu().numpy()[: wl.nev]
            assert np.max(np.abs(ln - lam_ref) / np.maximum(np.abs(lam_ref), 1)) <= TOL
            X[i] = Xi


def test_batched_seeded_with_contour_filter(h, oracle_mod):
    """The contour filter inside the batched solver's workers (one stream per
    worker: the quadrature nodes run in order there)."""
    from paper_1007_4400_amd import gevp

    wls = synth.batched_workloads(count=3, nmin=120, nmax=200, seed=7, steps=2)
    opts = gevp.make_opts(precision="fp64", filter="contour", batch_streams=3)
    seqs = [list(synth.sequence(wl, s)) for wl, s in wls]
    X = [None] * len(wls)
    for k in range(2):
        probs = [{"A": _dev(seq[k][0]), "B": _dev(seq[k][1]), "nev": wl.nev, "X0": X[i],
                  "kx": h.block_size(wl.n, wl.nev, opts)} for i, ((wl, _), seq) in enumerate(zip(wls, seqs))]
        out = h.solve_batched(probs, tol=TOL, opts=opts)
        for i, ((lam, Xi, res, info), (wl, _), seq) in enumerate(zip(out, wls, seqs)):
            A, B = seq[k]
            lam_ref, _ = oracle_mod.solve(A, B, wl.nev)
            ln = lam.cpu().numpy()[: wl.nev]
            assert np.max(np.abs(ln - lam_ref) / np.maximum(np.abs(lam_ref), 1)) <= TOL
            r, orth = oracle_mod.residuals(A, B, ln, Xi.cpu().numpy()[:, : wl.nev])
            assert r.max() <= TOL * np.linalg.norm(A, 2) and orth <= 1e-9
            assert (info["contour_applications"] >= 1) == (k > 0)
            X[i] = Xi


def test_autotune_batched_picks_and_caches(h, oracle_mod, tmp_path):
    """The autotuner times the batched call per stream count and split-K mode,
    keeps the fastest in the handle, and a JSON cache gives the same choice to
    a new handle without timing; tuned solves pass the oracle bar, and the
    configuration can be cleared and is validated."""
    from paper_1007_4400_amd import gevp

    wls = synth.batched_workloads(count=6, nmin=200, nmax=420, seed=5, steps=1)
    pencils = [synth.make_pencil(wl, s)[0] for wl, s in wls]
    probs = [{"A": _dev(p.A), "B": _dev(p.B), "nev": wl.nev} for p, (wl, _) in zip(pencils, wls)]
    opts = gevp.make_opts(precision="bf16x3")
    cache = str(tmp_path / "tuning.json")
    t = h.autotune_batched(probs, tol=TOL, opts=opts, cache=cache)
    print("tuning", t, flush=True)
    assert not t["cached"] and t["streams"] in (4, 6) and t["split_mode"] in (0, 1, 2)
    assert t["seconds"] > 0
    got = h.get_tuning()
    assert (got["streams"], got["split_mode"]) == (t["streams"], t["split_mode"])
    for (lam, X, _, info), p, (wl, _) in zip(h.solve_batched(probs, tol=TOL, opts=opts), pencils, wls):
        ln = lam.cpu().numpy()[: wl.nev]
        lo, _ = oracle_mod.solve(p.A, p.B, wl.nev)
        assert np.max(np.abs(ln - lo) / np.maximum(np.abs(lo), 1.0)) <= TOL
        r, orth = oracle_mod.residuals(p.A, p.B, ln, X.cpu().numpy()[:, : wl.nev])
        assert r.max() <= TOL * np.linalg.norm(p.A, 2) and orth <= 1e-9
    h2 = gevp.Handle(0)
    t2 = h2.autotune_batched(probs, tol=TOL, opts=opts, cache=cache)
    assert t2["cached"] and (t2["streams"], t2["split_mode"], t2["seconds"]) == \
        (t["streams"], t["split_mode"], t["seconds"])
    assert h2.get_tuning()["streams"] == t["streams"]
    h2.close()
    h.set_tuning(None)
    assert h.get_tuning() == {"streams": 0, "split_mode": 0, "seconds": 0.0}
    for bad in ({"streams": 17, "split_mode": 0}, {"streams": 4, "split_mode": 3},
                {"streams": -1, "split_mode": 0}):
        with pytest.raises(gevp.GevpError):
            h.set_tuning(bad)
