"""The Python binding checks every tensor before its pointer crosses the C
ABI: wrong dtype, shape or device raises ValueError with nothing launched,
and lazy conjugate views are materialised (the library reads stored values,
so an unresolved A.conj() would otherwise solve conj(A)).  CPU only: tensors
on the CPU are themselves one of the rejected cases."""
import pytest

torch = pytest.importorskip("torch")

from paper_1007_4400_amd import gevp  # noqa: E402


def _cpu(n=4, m=None, dtype=torch.complex128):
    return torch.zeros((n, m if m is not None else n), dtype=dtype)


@pytest.mark.parametrize("case", ["cpu", "c64", "nonsquare", "B_shape", "nev0", "nev_big",
                                  "X0_rows", "X0_dtype", "A_1d"])
def test_solve_args_rejected(case):
    A, B, X0, nev = _cpu(), _cpu(), None, 2
    if case == "c64":
        A = _cpu(dtype=torch.complex64)
    elif case == "nonsquare":
        A = _cpu(4, 3)
    elif case == "B_shape":
        B = _cpu(5)
    elif case == "nev0":
        nev = 0
    elif case == "nev_big":
        nev = 5
    elif case == "X0_rows":
        X0 = _cpu(3, 2)
    elif case == "X0_dtype":
        X0 = _cpu(4, 2, dtype=torch.float64)
    elif case == "A_1d":
        A = torch.zeros(16, dtype=torch.complex128)
    with pytest.raises(ValueError):
        gevp.check_solve_args(A, B, nev, X0, device=0)


def test_cpu_tensor_rejected_even_when_well_formed():
    with pytest.raises(ValueError, match="cuda:0"):
        gevp.check_solve_args(_cpu(), _cpu(), 2, None, device=0)


@pytest.mark.parametrize("case", ["w_short", "w_int", "lam_missing", "lam_short", "X_real"])
def test_backward_args_rejected(case):
    X, lam, w = _cpu(4, 3), torch.zeros(3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64)
    need_lam = True
    if case == "w_short":
        w = torch.zeros(2, dtype=torch.float64)
    elif case == "w_int":
        w = torch.zeros(3, dtype=torch.int64)
    elif case == "lam_missing":
        lam = None
    elif case == "lam_short":
        lam = torch.zeros(1, dtype=torch.float64)
    elif case == "X_real":
        X = torch.zeros((4, 3), dtype=torch.float64)
    with pytest.raises(ValueError):
        gevp.check_backward_args(X, lam, w, device=0, need_lam=need_lam)


def test_colmajor_resolves_conjugate_and_negative_views():
    M = torch.tensor([[1 + 2j, 3 - 1j], [0.5j, 2.0]], dtype=torch.complex128)
    for view, want in ((M.conj(), M.conj().resolve_conj()), (M.mH, M.mH.resolve_conj()),
                       (-M.conj(), (-M.conj()).resolve_conj().resolve_neg())):
        c = gevp.colmajor(view)
        assert not c.is_conj() and not c.is_neg()
        assert c.stride(0) == 1
        assert torch.equal(c, want)


def test_inplace_update_rejects_conjugate_view():
    A = torch.zeros((4, 4), dtype=torch.complex128).mT  # column-major
    with pytest.raises(ValueError):
        gevp._check_inplace(A.conj())
