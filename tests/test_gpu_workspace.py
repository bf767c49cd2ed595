"""Caller-owned workspace (gevp_set_workspace): solves in a torch-allocated
buffer give the same results as solves in library-allocated memory, allocate
no device memory, and a buffer that is too small is reported before anything
is launched."""
import numpy as np
import pytest

from paper_1007_4400_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def gevp_mod():
    from paper_1007_4400_amd import gevp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return gevp


def _seq(n, nev, steps):
    wl = synth.scaled(synth.MEDIUM, n, nev=nev, steps=steps)
    out = []
    for A, B in synth.sequence(wl, 0):
        out.append((torch.from_numpy(np.asfortranarray(A)).cuda(),
                    torch.from_numpy(np.asfortranarray(B)).cuda()))
    return wl, out


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_torch_workspace_matches_library_memory(gevp_mod, precision):
    gevp = gevp_mod
    wl, seq = _seq(640, 64, 3)
    opts = gevp.make_opts(precision=precision)
    ref = gevp.Handle(0)
    h = gevp.Handle(0)
    kx = h.block_size(wl.n, wl.nev, opts)
    # the library-managed sequence first (it also loads every code object)
    refs, Xr = [], None
    for A, B in seq:
        lam_r, Xr, _, _ = ref.solve(A, B, wl.nev, X0=Xr, tol=TOL, kx=kx, opts=opts)
        refs.append(lam_r)
    nbytes = h.workspace_size(wl.n, wl.nev, opts)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h.set_workspace(buf)
    outs = [torch.empty(kx, dtype=torch.float64, device="cuda") for _ in seq]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    X = None
    for k, (A, B) in enumerate(seq):
        lam, X, _, info = h.solve(A, B, wl.nev, X0=X, tol=TOL, kx=kx, opts=opts)
        assert info["max_resid"] <= TOL
        outs[k].copy_(lam)
    torch.cuda.synchronize()
    for k, lam_r in enumerate(refs):
        err = ((outs[k][: wl.nev] - lam_r[: wl.nev]).abs() / lam_r[: wl.nev].abs().clamp(min=1)).max()
        assert err.item() <= 1e-12, (k, err.item())
    # the seeded steps used the second stream and the panel stream: none of
    # them allocated device memory (a library-managed handle takes >= 128 MiB
    # of split-K buffer per stream)
    assert free0 - torch.cuda.mem_get_info()[0] < 32 * 2 ** 20
    # back to library-managed memory: a cold solve of the last step agrees on
    # the wanted pairs (the guard Ritz values of a cold solve differ)
    h.set_workspace(None)
    lam2, _, _, info2 = h.solve(*seq[-1], wl.nev, tol=TOL, kx=kx, opts=opts)
    assert info2["max_resid"] <= TOL
    err = ((lam2[: wl.nev] - lam[: wl.nev]).abs() / lam[: wl.nev].abs().clamp(min=1)).max()
    assert err.item() <= TOL
    ref.close()
    h.close()


def test_too_small_workspace_is_reported(gevp_mod):
    gevp = gevp_mod
    wl, seq = _seq(512, 40, 1)
    h = gevp.Handle(0)
    need = h.workspace_size(wl.n, wl.nev)
    small = torch.empty(6 * 128 * 2 ** 20 + 4096, dtype=torch.uint8, device="cuda")
    assert small.numel() < need
    h.set_workspace(small)
    with pytest.raises(gevp.GevpError) as e:
        h.solve(*seq[0], wl.nev, tol=TOL)
    assert e.value.status == gevp.GEVP_ERR_WORKSPACE
    # a misaligned or undersized buffer is an argument error
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(gevp.GevpError):
        h.set_workspace(big[1:])
    with pytest.raises(gevp.GevpError):
        h.set_workspace(big[: 4096])
    h.set_workspace(big[: need])
    lam, X, _, info = h.solve(*seq[0], wl.nev, tol=TOL)
    assert info["max_resid"] <= TOL
    h.close()


def test_batched_in_torch_workspace(gevp_mod):
    gevp = gevp_mod
    wls = synth.batched_workloads(count=4, nmin=300, nmax=700, seed=2, steps=1)
    pencils = [synth.make_pencil(wl, s)[0] for wl, s in wls]
    h = gevp.Handle(0)
    ref = gevp.Handle(0)
    ns = [wl.n for wl, _ in wls]
    nevs = [wl.nev for wl, _ in wls]
    opts = gevp.make_opts(batch_streams=2)
    buf = torch.empty(h.workspace_size_batched(ns, nevs, opts), dtype=torch.uint8, device="cuda")
    h.set_workspace(buf)
    cases = [{"A": torch.from_numpy(np.asfortranarray(p.A)).cuda(),
              "B": torch.from_numpy(np.asfortranarray(p.B)).cuda(), "nev": wl.nev}
             for p, (wl, _) in zip(pencils, wls)]
    out = h.solve_batched(cases, tol=TOL, opts=opts)
    out_r = ref.solve_batched(cases, tol=TOL, opts=opts)
    for (lam, _, _, info), (lam_r, _, _, _) in zip(out, out_r):
        assert info["max_resid"] <= TOL
        assert ((lam - lam_r).abs() / lam_r.abs().clamp(min=1)).max().item() <= 1e-12
    h.close()
    ref.close()
