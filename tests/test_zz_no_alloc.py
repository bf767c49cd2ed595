"""gevp_backward_noalloc (the entry point for callers that cannot allocate)
against gevp_backward through the C ABI: two calls in a row, the second with
a smaller problem, element by element; a problem too large for its fixed
scratch array is rejected with nothing launched."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_1007_4400_amd import gevp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return gevp.Handle(0)


def _case(n, nev, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    X = torch.randn((nev, n), dtype=torch.complex128, device="cuda", generator=g).mT  # column-major
    lam = torch.randn(nev, dtype=torch.float64, device="cuda", generator=g)
    w = torch.rand(nev, dtype=torch.float64, device="cuda", generator=g)
    return X, lam, w


def _call(h, fn, X, lam, w):
    from paper_1007_4400_amd import gevp

    n, nev = X.shape
    dA = gevp.empty_colmajor(n, n, device="cuda")
    dB = gevp.empty_colmajor(n, n, device="cuda")
    dA.fill_(float("nan"))
    dB.fill_(float("nan"))
    vp = ctypes.c_void_p
    h._stream()
    s = fn(h.h, n, nev, vp(X.data_ptr()), X.stride(1), vp(lam.data_ptr()), vp(w.data_ptr()),
           vp(dA.data_ptr()), n, vp(dB.data_ptr()), n)
    return s, dA, dB


def test_noalloc_backward_matches_backward_twice(h):
    from paper_1007_4400_amd import gevp

    for n, nev, seed in ((700, 96, 1), (300, 40, 2)):  # the second call is smaller
        print(f"noalloc backward n={n} nev={nev}", flush=True)
        X, lam, w = _case(n, nev, seed)
        s_ref, dA_ref, dB_ref = _call(h, h.lib.gevp_backward, X, lam, w)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        s, dA, dB = _call(h, h.lib.gevp_backward_noalloc, X, lam, w)
        torch.cuda.synchronize()
        # only the two n x n outputs (torch's caching allocator) are new
        assert free0 - torch.cuda.mem_get_info()[0] <= 2 * 16 * n * n + (8 << 20)
        assert s_ref == gevp.GEVP_OK and s == gevp.GEVP_OK
        for got, ref in ((dA, dA_ref), (dB, dB_ref)):
            assert torch.isfinite(torch.view_as_real(got)).all()
            err = (got - ref).abs().max().item()
            assert err <= 1e-13 * max(ref.abs().max().item(), 1.0), err
        # and the definition, independently: dA = X diag(w) X^H
        Xh = X.cpu().numpy()
        wn, ln = w.cpu().numpy(), lam.cpu().numpy()
        GA = (Xh * wn) @ Xh.conj().T
        GB = -(Xh * (wn * ln)) @ Xh.conj().T
        assert np.max(np.abs(dA.cpu().numpy() - GA)) <= 1e-12 * np.max(np.abs(GA))
        assert np.max(np.abs(dB.cpu().numpy() - GB)) <= 1e-12 * np.max(np.abs(GB))


def test_noalloc_rejects_oversized_problem(h):
    from paper_1007_4400_amd import gevp

    # 4096 x 1024 complex128 = 64 MiB > the 32 MiB scratch array
    n, nev = 4096, 1024
    X = torch.zeros((nev, n), dtype=torch.complex128, device="cuda").mT
    lam = torch.zeros(nev, dtype=torch.float64, device="cuda")
    w = torch.zeros(nev, dtype=torch.float64, device="cuda")
    vp = ctypes.c_void_p
    s = h.lib.gevp_backward_noalloc(h.h, n, nev, vp(X.data_ptr()), n, vp(lam.data_ptr()),
                                    vp(w.data_ptr()), None, n, None, n)
    assert s == gevp.GEVP_ERR_WORKSPACE
