"""Kernel-level parity of the HIP building blocks against plain definitions
(numpy complex128 products and solves, and the CPU oracle for the small
eigensolver), at sizes that span several 64-wide tiles plus ragged tails."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def h():
    from paper_1007_4400_amd import gevp

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return gevp.Handle(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("m,n,k", [(64, 64, 16), (70, 45, 33), (130, 200, 257), (1, 3, 1), (200, 150, 4000)])
def test_zgemm_ops(h, opA, opB, m, n, k):
    print(f"zgemm {opA}{opB} m={m} n={n} k={k}", flush=True)
    rng = np.random.default_rng(m * 1000 + n + k)
    A = _cn(rng, *((m, k) if opA == "N" else (k, m)))
    B = _cn(rng, *((k, n) if opB == "N" else (n, k)))
    C = _cn(rng, m, n)
    E = _cn(rng, m, n)
    g = rng.standard_normal(n)
    opa = A if opA == "N" else A.conj().T
    opb = B if opB == "N" else B.conj().T
    ref = 1.5 * opa @ opb - 0.25 * C + 0.75 * E * g[None, :]
    out = h.zgemm(opA, opB, _dev(A), _dev(B), alpha=1.5, beta=-0.25, C=_dev(C), gamma=0.75,
                  E=_dev(E), gcol=_dev(g))
    torch.cuda.synchronize()
    err = np.max(np.abs(_np(out) - ref)) / max(1.0, np.max(np.abs(ref)))
    assert err <= 1e-14 * np.sqrt(k) * 10


def test_zgemm_plain_and_inplace_beta(h):
    rng = np.random.default_rng(5)
    m, n, k = 300, 190, 410
    A, B, C = _cn(rng, m, k), _cn(rng, k, n), _cn(rng, m, n)
    Cd = h.zgemm("N", "N", _dev(A), _dev(B))
    Dd = _dev(C)
    from paper_1007_4400_amd import gevp

    Dd = gevp.colmajor(Dd)
    h.zgemm("N", "N", _dev(A), _dev(B), alpha=-1.0, beta=1.0, C=Dd, out=Dd)
    torch.cuda.synchronize()
    assert np.allclose(_np(Cd), A @ B, rtol=0, atol=1e-12)
    assert np.allclose(_np(Dd), C - A @ B, rtol=0, atol=1e-12)


# panel boundaries of the factorisation (384-wide panels of 64-wide blocks)
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("m,n,k", [(64, 948, 64), (50, 300, 200), (948, 64, 64), (300, 40, 500),
                                   (64, 70, 1024), (17, 5, 3)])
def test_zgemm_skinny_tiles(h, opA, opB, m, n, k):
    """Products with at most 64 rows or columns and a short K run on 64 x 16
    or 16 x 64 tiles (one wave each); ragged edges and the K limit included."""
    print(f"zgemm skinny {opA}{opB} m={m} n={n} k={k}", flush=True)
    rng = np.random.default_rng(m * 7 + n + k)
    A = _cn(rng, *((m, k) if opA == "N" else (k, m)))
    B = _cn(rng, *((k, n) if opB == "N" else (n, k)))
    C = _cn(rng, m, n)
    E = _cn(rng, m, n)
    g = rng.standard_normal(n)
    opa = A if opA == "N" else A.conj().T
    opb = B if opB == "N" else B.conj().T
    ref = -0.5 * opa @ opb + 2.0 * C - 0.25 * E * g[None, :]
    out = h.zgemm(opA, opB, _dev(A), _dev(B), alpha=-0.5, beta=2.0, C=_dev(C), gamma=-0.25,
                  E=_dev(E), gcol=_dev(g))
    torch.cuda.synchronize()
    scale = 0.5 * np.abs(opa) @ np.abs(opb) + 2.0 * np.abs(C) + 0.25 * np.abs(E * g[None, :])
    assert np.max(np.abs(_np(out) - ref) / scale) <= 1e-14 * np.sqrt(k) * 10


@pytest.mark.parametrize("side", ["L", "R"])
def test_zgemm_in_place_base_cases(h, side):
    """The base cases of the triangular solves overwrite one operand: the
    left one as X = X T (rows of 16, every column in one tile) and the right
    one as X = T X (columns of 16, every row in one tile)."""
    from paper_1007_4400_amd import gevp

    rng = np.random.default_rng(3)
    T = np.tril(_cn(rng, 64, 64))
    if side == "L":  # X (64 x 948) <- T X
        X = _cn(rng, 64, 948)
        Xd = gevp.colmajor(_dev(X))
        h.zgemm("N", "N", _dev(T), Xd, out=Xd)
        ref = T @ X
    else:  # X (948 x 64) <- X T^H
        X = _cn(rng, 948, 64)
        Xd = gevp.colmajor(_dev(X))
        h.zgemm("N", "C", Xd, _dev(T), out=Xd)
        ref = X @ T.conj().T
    torch.cuda.synchronize()
    assert np.max(np.abs(_np(Xd) - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("opA,opB", [("C", "N"), ("N", "C"), ("N", "N")])
@pytest.mark.parametrize("n,k", [(200, 70), (948, 8192), (130, 4000)])
def test_zgemm_lower_triangle_tiles(h, opA, opB, n, k):
    """Lower-triangle launches (Gram and projected matrices): the tiles that
    touch the lower triangle hold the product, the tiles entirely above the
    diagonal are left as they were.  (948, 8192) runs split-K."""
    from paper_1007_4400_amd import gevp

    print(f"zgemm lower {opA}{opB} n={n} k={k}", flush=True)
    rng = np.random.default_rng(n + k)
    A = _cn(rng, *((n, k) if opA == "N" else (k, n)))
    B = _cn(rng, *((k, n) if opB == "N" else (n, k)))
    D0 = _cn(rng, n, n)
    opa = A if opA == "N" else A.conj().T
    opb = B if opB == "N" else B.conj().T
    ref = opa @ opb
    out = h.zgemm_tri(opA, opB, _dev(A), _dev(B), gevp.colmajor(_dev(D0)), lower=True)
    torch.cuda.synchronize()
    got = _np(out)
    ti, tj = np.meshgrid(np.arange(n) // 64, np.arange(n) // 64, indexing="ij")
    computed = ti >= tj
    scale = np.abs(opa) @ np.abs(opb)
    assert np.max(np.abs(got - ref)[computed] / scale[computed]) <= 1e-14 * np.sqrt(k)
    assert np.array_equal(got[~computed], D0[~computed])


@pytest.mark.parametrize("opA", ["N", "C"])
@pytest.mark.parametrize("m,n,beta", [(300, 70, 0.0), (1000, 130, -0.5), (8192, 96, 0.0)])
def test_zgemm_upper_triangular_a(h, opA, m, n, beta):
    """upperA launches use only the upper triangle of op(A): whatever lies
    below its diagonal (here random values) reads as zero.  (8192, 96) runs
    split-K, with splits that lie entirely below a row block's diagonal."""
    print(f"zgemm upperA {opA} m={m} n={n}", flush=True)
    rng = np.random.default_rng(m + 7 * n)
    A = _cn(rng, m, m)
    B = _cn(rng, m, n)
    C = _cn(rng, m, n)
    opa = A if opA == "N" else A.conj().T
    ref = np.triu(opa) @ B + beta * C
    from paper_1007_4400_amd import gevp

    out = gevp.empty_colmajor(m, n, device=torch.device("cuda"))
    out = h.zgemm_tri(opA, "N", _dev(A), _dev(B), out, beta=beta,
                      C=_dev(C) if beta != 0.0 else None, upperA=True)
    torch.cuda.synchronize()
    scale = np.abs(np.triu(opa)) @ np.abs(B) + abs(beta) * np.abs(C)
    assert np.max(np.abs(_np(out) - ref) / scale) <= 1e-14 * np.sqrt(m)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 200, 333, 383, 384, 385, 769, 1000])
def test_potrf(h, n):
    print(f"potrf n={n}", flush=True)
    rng = np.random.default_rng(n)
    G = _cn(rng, n, n)
    M = G @ G.conj().T + n * np.eye(n)
    L, piv = h.potrf(_dev(M))
    torch.cuda.synchronize()
    assert piv == 0
    Lr = np.linalg.cholesky(M)
    assert np.max(np.abs(_np(L) - Lr)) <= 1e-12 * np.max(np.abs(Lr))


@pytest.mark.parametrize("n,bad", [(150, 97), (900, 700)])
def test_potrf_not_hpd_reports_pivot(h, n, bad):
    M = np.eye(n, dtype=complex)
    M[bad, bad] = -2.0
    _, piv = h.potrf(_dev(M))
    assert piv == bad + 1


@pytest.mark.parametrize("side,trans", [("L", "N"), ("L", "C"), ("R", "C")])
@pytest.mark.parametrize("n,m", [(64, 10), (150, 77), (257, 130)])
def test_trsm(h, side, trans, n, m):
    print(f"trsm {side}{trans} n={n} m={m}", flush=True)
    rng = np.random.default_rng(n + m)
    L = np.tril(_cn(rng, n, n)) * 0.1 + np.diag(2.0 + rng.random(n))
    R = _cn(rng, n, m) if side == "L" else _cn(rng, m, n)
    out = _np(h.trsm(side, trans, _dev(L), _dev(R)))
    if side == "L" and trans == "N":
        ref = np.linalg.solve(L, R)
    elif side == "L":
        ref = np.linalg.solve(L.conj().T, R)
    else:
        ref = R @ np.linalg.inv(L.conj().T)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 127, 128, 129, 130, 193, 301, 948])
def test_heev_vs_oracle(h, n, oracle_mod):
    print(f"heev n={n}", flush=True)
    rng = np.random.default_rng(n)
    G = _cn(rng, n, n)
    H = 0.5 * (G + G.conj().T)
    th, Z = h.heev(_dev(H))
    torch.cuda.synchronize()
    th, Z = _np(th), _np(Z)
    lam, _ = oracle_mod.solve(H, np.eye(n, dtype=complex), n)
    nrm = max(1.0, np.max(np.abs(lam)))
    assert np.max(np.abs(th - lam)) <= 1e-13 * nrm * max(1, np.sqrt(n))
    assert np.max(np.abs(H @ Z - Z * th[None, :])) <= 1e-12 * nrm * max(1, np.sqrt(n))
    assert np.max(np.abs(Z.conj().T @ Z - np.eye(n))) <= 1e-10


def test_heev_replayed_sequence(h):
    """The tridiagonalisation's launches are captured once per argument set
    and replayed: consecutive eigensolves of different matrices of one order
    (same workspace, so the same captured sequence) each match numpy's
    eigenvalues and give their own eigenvectors; a fresh handle (captures
    anew) gives bitwise the same results as the replays."""
    from paper_1007_4400_amd import gevp

    n = 300
    rng = np.random.default_rng(11)
    outs = []
    for r in range(3):
        G = _cn(rng, n, n)
        H = 0.5 * (G + G.conj().T) + r * np.eye(n)
        th, Z = h.heev(_dev(H))
        th, Z = _np(th), _np(Z)
        lam = np.linalg.eigvalsh(H)
        nrm = max(1.0, np.max(np.abs(lam)))
        assert np.max(np.abs(th - lam)) <= 1e-13 * nrm * np.sqrt(n)
        assert np.max(np.abs(H @ Z - Z * th[None, :])) <= 1e-12 * nrm * np.sqrt(n)
        outs.append((H, th, Z))
    h2 = gevp.Handle(0)
    th2, Z2 = h2.heev(_dev(outs[-1][0]))
    assert np.array_equal(_np(th2), outs[-1][1]) and np.array_equal(_np(Z2), outs[-1][2])
    h2.close()


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130, 1000, 2049])
def test_hemv_lower_tiles(h, n):
    """gevp_k_hemv (the Lanczos bounds' matrix-vector product) against a host
    product: y = H x for a random Hermitian H whose tiles strictly above the
    diagonal 64 x 64 blocks are overwritten with NaN (they must not be read),
    ragged orders included, and once with a padded leading dimension."""
    from paper_1007_4400_amd import gevp

    rng = np.random.default_rng(n)
    G = _cn(rng, n, n)
    H = 0.5 * (G + G.conj().T)
    x = _cn(rng, n, 1)[:, 0]
    ref = H @ x
    M = H.copy()
    for I in range((n + 63) // 64):
        for J in range(I + 1, (n + 63) // 64):
            M[I * 64:(I + 1) * 64, J * 64:(J + 1) * 64] = np.nan
    for pad in (0, 3) if n in (65, 1000) else (0,):
        Md = gevp.empty_colmajor(n + pad, n, device="cuda")
        Md.copy_(torch.from_numpy(np.vstack([M, np.zeros((pad, n), dtype=complex)])))
        y = h.hemv(Md[:n], torch.from_numpy(x).to("cuda"))
        yh = _np(y)
        assert np.all(np.isfinite(yh))
        err = np.max(np.abs(yh - ref)) / max(1.0, np.max(np.abs(ref)))
        assert err <= 1e-13 * max(1.0, np.sqrt(n)), (pad, err)


@pytest.mark.parametrize("kind", ["diagonal", "real_tridiagonal", "blocks"])
def test_heev_identity_reflectors(h, kind):
    """Matrices whose tridiagonalisation meets identity reflectors (tau = 0:
    nothing below the subdiagonal and a real subdiagonal entry): a real
    diagonal, a real tridiagonal, and a block-diagonal matrix of dense complex
    blocks and 1 x 1 blocks.  The back-transformation must leave those
    reflectors out; eigenpairs against numpy's."""
    n = 200
    rng = np.random.default_rng(5)
    if kind == "diagonal":
        H = np.diag(rng.standard_normal(n)).astype(complex)
    elif kind == "real_tridiagonal":
        H = np.diag(rng.standard_normal(n)) + np.diag(rng.standard_normal(n - 1), 1)
        H = (H + np.triu(H, 1).T).astype(complex)
    else:
        H = np.zeros((n, n), dtype=complex)
        i = 0
        for b in (37, 1, 1, 64, 1, 50, 1, 45):
            G = _cn(rng, b, b)
            H[i:i + b, i:i + b] = 0.5 * (G + G.conj().T)
            i += b
        assert i == n
    th, Z = h.heev(_dev(H))
    th, Z = _np(th), _np(Z)
    lam = np.linalg.eigvalsh(H)
    nrm = max(1.0, np.max(np.abs(lam)))
    assert np.max(np.abs(th - lam)) <= 1e-13 * nrm * np.sqrt(n)
    assert np.max(np.abs(H @ Z - Z * th[None, :])) <= 1e-12 * nrm * np.sqrt(n)
    assert np.max(np.abs(Z.conj().T @ Z - np.eye(n))) <= 1e-10


@pytest.mark.parametrize("n", [40, 300])
def test_heev_degenerate(h, oracle_mod, n):
    # repeated eigenvalues: an invariant subspace, not unique vectors
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(_cn(rng, n, n))
    ev = np.repeat(np.arange(n // 5, dtype=float), 5)
    H = (Q * ev) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    th, Z = h.heev(_dev(H))
    th, Z = _np(th), _np(Z)
    assert np.max(np.abs(th - ev)) <= 1e-12
    assert np.max(np.abs(H @ Z - Z * th[None, :])) <= 1e-11
    assert np.max(np.abs(Z.conj().T @ Z - np.eye(n))) <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("bf16x3", 1e-4)])
@pytest.mark.parametrize("n,m", [(64, 16), (200, 70), (333, 129), (520, 260), (1100, 300)])
def test_filter_gemm_low_precision(h, precision, tol, n, m):
    """One residual-correction filter step in low precision against the
    complex128 definition; the error bound is relative to the size of the
    terms (normwise), the rounding scale of each format."""
    print(f"filter gemm {precision} n={n} m={m}", flush=True)
    rng = np.random.default_rng(n + m)
    G0 = _cn(rng, n, n)
    C = 0.5 * (G0 + G0.conj().T) / np.sqrt(n)
    Gm = _cn(rng, n, m).astype(np.complex64)
    P = _cn(rng, n, m).astype(np.complex64)
    R = _cn(rng, n, m).astype(np.complex64)
    al, be, ga, de = (rng.standard_normal(m) for _ in range(4))
    ref = (C @ Gm.astype(complex)) * al + Gm * be + P * ga + R * de
    d = [torch.from_numpy(x).cuda() for x in (al, be, ga, de)]
    out = h.filter_gemm(precision, _dev(C), _dev(Gm), _dev(P), _dev(R), *d)
    torch.cuda.synchronize()
    out = _np(out)
    scale = np.abs(C) @ np.abs(Gm) * np.abs(al) + np.abs(Gm * be) + np.abs(P * ga) + np.abs(R * de)
    err = np.max(np.abs(out - ref) / scale)
    assert err <= tol, err
