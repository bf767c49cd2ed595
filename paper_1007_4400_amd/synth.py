"""Seeded synthetic SCF pencil sequences.

This module only builds inputs.  It holds none of the eigensolver's
arithmetic and imports neither the solver library nor the CPU oracle; both
sides are fed from here.

The paper's matrices come from FLEUR runs on two small metallic systems
(section 2, study setup) and are not available; these sequences stand in for
them.  Each sequence is a chain of correlated pencils (section 2, first
paragraph: the output of one iteration feeds the next): step 0 is a pencil
with a prescribed spectrum and every later step perturbs the Hamiltonian a
little, with a decaying perturbation size, as an SCF run settles.

Construction of one pencil (size n):

* B = L L^H with L = I + s * tril(G, -1), G complex Gaussian with E|g|^2 = 1.
* A = L Q diag(Lambda) Q^H L^H with Q Haar-unitary (QR of a complex Gaussian
  matrix with the phases of R's diagonal moved into Q), so that the exact
  eigenvalues of (A, B) are Lambda and the exact eigenvectors are
  L^{-H} Q (up to a phase per column).
* Step k >= 1: A_k = A_{k-1} + eps_k H_k, H_k = (G + G^H)/2 scaled by a
  60-step power-iteration estimate of its spectral norm (so ||H_k||_2 is 1 to
  within a few per cent); B stays fixed.

Spectra:

* ``"split"``  (the small oracle-scale case): the ``nev`` lowest values uniform
  in [-2, -0.5], the rest uniform in [0, 50].
* ``"cluster"`` (the larger cases): the ``nev`` lowest values in [-3, 0] with
  consecutive gaps of at least 1e-4 (sorted uniforms on [-3, -(nev-1)*1e-4]
  plus i * 1e-4), the rest uniform in [0, 50].

Random draws come from ``numpy.random.Generator(PCG64(seed))`` in the order
Lambda, L, Q, H_1, H_2, ...; the large device-side variant draws the same
quantities from a seeded ``torch.Generator`` on the GPU (a different but
equally deterministic stream) because a CPU QR of an 8192 x 8192 complex
matrix would take minutes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# named workloads (sizes and sequence parameters)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    nev: int
    steps: int
    spectrum: str  # "split" | "cluster"
    lscale: float  # off-diagonal scale s of L
    eps0: float  # eps_k = eps0 * decay**k
    decay: float
    shift: float = 0.0  # spectrum shift (batched k-point problems)


def _cluster_scale(n: int) -> float:
    # s = 1.1/sqrt(n) keeps cond(B) near 1e2 independent of n
    return 1.1 / math.sqrt(n)


SMALL = Workload("n256_nev16_split", 256, 16, 5, "split", 0.05, 1e-2, 0.5)
MEDIUM = Workload("n2048_nev205_cluster", 2048, 205, 20, "cluster", _cluster_scale(2048), 1e-2, 0.5)
LARGE = Workload("n8192_nev820_cluster", 8192, 820, 12, "cluster", _cluster_scale(8192), 5e-3, 0.6)
GRAD = Workload("n4096_nev410_cluster", 4096, 410, 1, "cluster", _cluster_scale(4096), 0.0, 1.0)


def scaled(wl: Workload, n: int, nev: Optional[int] = None, steps: Optional[int] = None) -> Workload:
    """The same construction at another size (cond(B) kept near 1e2 for the
    clustered spectra)."""
    nev = nev if nev is not None else max(1, round(wl.nev * n / wl.n))
    s = wl.lscale if wl.spectrum == "split" else _cluster_scale(n)
    return dataclasses.replace(wl, name=f"n{n}_nev{nev}_{wl.spectrum}", n=n, nev=nev,
                               steps=steps if steps is not None else wl.steps, lscale=s)


def eps(wl: Workload, k: int) -> float:
    return wl.eps0 * wl.decay ** k


# ---------------------------------------------------------------------------
# numpy (host) construction


def _cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def spectrum(wl: Workload, rng: np.random.Generator) -> np.ndarray:
    n, nev = wl.n, wl.nev
    if wl.spectrum == "split":
        low = rng.uniform(-2.0, -0.5, size=nev)
        high = rng.uniform(0.0, 50.0, size=n - nev)
    elif wl.spectrum == "cluster":
        gap = 1e-4
        u = np.sort(rng.uniform(-3.0, -(nev - 1) * gap, size=nev))
        low = u + gap * np.arange(nev)
        high = rng.uniform(0.0, 50.0, size=n - nev)
    else:
        raise ValueError(wl.spectrum)
    return np.concatenate([low, high]) + wl.shift


def haar_unitary(rng: np.random.Generator, n: int) -> np.ndarray:
    Z = _cgauss(rng, (n, n))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def unit_hermitian(rng: np.random.Generator, n: int, iters: int = 60) -> np.ndarray:
    G = _cgauss(rng, (n, n))
    H = 0.5 * (G + G.conj().T)
    # spectral norm by power iteration on H (deterministic start)
    v = np.ones(n, dtype=np.complex128) / math.sqrt(n)
    nrm = 1.0
    for _ in range(iters):
        w = H @ (H @ v)
        nrm = math.sqrt(np.linalg.norm(w))
        v = w / np.linalg.norm(w)
    return H / nrm


@dataclasses.dataclass
class Pencil:
    A: np.ndarray  # Hermitian, complex128
    B: np.ndarray  # Hermitian positive definite, complex128
    Lambda: np.ndarray  # exact eigenvalues of the step-0 pencil (unsorted)
    L: np.ndarray  # lower-triangular factor with B = L L^H
    Q: np.ndarray  # Haar unitary of the construction

    def exact_lowest(self, nev: int):
        """Exact lowest nev eigenvalues and eigenvectors (L^{-H} Q, B-orthonormal)
        of the step-0 pencil."""
        order = np.argsort(self.Lambda, kind="stable")[:nev]
        X = np.linalg.solve(self.L.conj().T, self.Q[:, order])
        return self.Lambda[order], X


def make_pencil(wl: Workload, seed: int) -> tuple[Pencil, np.random.Generator]:
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = spectrum(wl, rng)
    n = wl.n
    L = np.eye(n, dtype=np.complex128) + wl.lscale * np.tril(_cgauss(rng, (n, n)), -1)
    Q = haar_unitary(rng, n)
    M = L @ Q
    A = (M * lam[None, :]) @ M.conj().T
    A = 0.5 * (A + A.conj().T)
    B = L @ L.conj().T
    B = 0.5 * (B + B.conj().T)
    return Pencil(A, B, lam, L, Q), rng


def sequence(wl: Workload, seed: int, steps: Optional[int] = None) -> Iterator[tuple[np.ndarray, np.ndarray]]:
    """Yield (A_k, B) for k = 0 .. steps-1."""
    p, rng = make_pencil(wl, seed)
    A = p.A.copy()
    steps = wl.steps if steps is None else steps
    for k in range(steps):
        if k > 0:
            A = A + eps(wl, k) * unit_hermitian(rng, wl.n)
        yield A, p.B


# ---------------------------------------------------------------------------
# batched k-point problems


def batched_workloads(count: int = 32, nmin: int = 1500, nmax: int = 3000, seed: int = 0,
                      steps: int = 8) -> List[tuple[Workload, int]]:
    """Independent k-point problems with uneven sizes: n ~ U_int[nmin, nmax],
    nev = round(0.1 n), per-problem shift ~ U[-0.5, 0.5].  Returns
    (workload, seed) pairs; each problem has its own spawned seed."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.Generator(np.random.PCG64(ss))
    children = ss.spawn(count)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        shift = float(rng.uniform(-0.5, 0.5))
        wl = Workload(f"kpt{i}_n{n}", n, int(round(0.1 * n)), steps, "cluster",
                      _cluster_scale(n), 1e-2, 0.5, shift)
        out.append((wl, int(children[i].generate_state(1)[0])))
    return out


# ---------------------------------------------------------------------------
# device (torch) construction for the large sizes


def make_pencil_torch(wl: Workload, seed: int, device="cuda", qr_on_host=False, exact_nev=0):
    """The same construction with a seeded torch generator on ``device``.
    Returns (A, B, Lambda, L, gen) as torch tensors (row-major logical
    matrices, complex128) plus the generator for the perturbations.
    qr_on_host: factor the Gaussian matrix on the host (same draws, same
    construction; used where a device QR is unavailable).
    exact_nev > 0: also return the exact lowest eigenvalues and B-orthonormal
    eigenvectors L^{-H} Q(:, order) of the step-0 pencil (appended to the
    returned tuple)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n, nev = wl.n, wl.nev
    f64 = torch.float64
    if wl.spectrum == "split":
        low = torch.rand(nev, generator=g, device=device, dtype=f64) * 1.5 - 2.0
        high = torch.rand(n - nev, generator=g, device=device, dtype=f64) * 50.0
    else:
        gap = 1e-4
        u = torch.rand(nev, generator=g, device=device, dtype=f64)
        u = torch.sort(-3.0 + u * (3.0 - (nev - 1) * gap)).values
        low = u + gap * torch.arange(nev, device=device, dtype=f64)
        high = torch.rand(n - nev, generator=g, device=device, dtype=f64) * 50.0
    lam = torch.cat([low, high]) + wl.shift
    G = torch.randn(n, n, generator=g, device=device, dtype=torch.complex128)
    L = torch.eye(n, device=device, dtype=torch.complex128) + wl.lscale * torch.tril(G, -1)
    del G
    Z = torch.randn(n, n, generator=g, device=device, dtype=torch.complex128)
    if qr_on_host:
        Q, R = torch.linalg.qr(Z.cpu())
        Q, R = Q.to(device), R.to(device)
    else:
        Q, R = torch.linalg.qr(Z)
    del Z
    d = torch.diagonal(R)
    Q = Q * (d / d.abs())[None, :]
    del R
    exact = None
    if exact_nev:
        order = torch.argsort(lam)[:exact_nev]
        Xe = torch.linalg.solve_triangular(L.conj().T.contiguous(), Q[:, order].contiguous(), upper=True)
        exact = (lam[order], Xe)
    M = L @ Q
    del Q
    A = (M * lam[None, :].to(M.dtype)) @ M.conj().T.contiguous()
    del M
    A = 0.5 * (A + A.conj().T)
    B = L @ L.conj().T.contiguous()
    B = 0.5 * (B + B.conj().T)
    if exact_nev:
        return A, B, lam, L, g, exact
    return A, B, lam, L, g


def unit_hermitian_torch(n: int, g, device="cuda", iters: int = 60):
    import torch

    G = torch.randn(n, n, generator=g, device=device, dtype=torch.complex128)
    H = 0.5 * (G + G.conj().T)
    del G
    v = torch.ones(n, 1, device=device, dtype=torch.complex128) / math.sqrt(n)
    nrm = 1.0
    for _ in range(iters):
        w = H @ (H @ v)
        wn = torch.linalg.vector_norm(w).item()
        nrm = math.sqrt(wn)
        v = w / wn
    return H / nrm


# ---------------------------------------------------------------------------
# matrix-entry evolution (thresholded partial updates)
#
# Stand-in for the Hamiltonian differences between adjacent SCF iterations
# that the paper studies at fixed k-point (section 2, paragraph "Matrix
# generation", and its figure): wide areas of the difference stay below any
# threshold, rows and columns of unchanging entries form a cross, and the
# share of entries above a fixed threshold falls as the run settles.
#
# Step k >= 1 adds D_k = eps_k * (w w^T) o K_k o H_k to the Hamiltonian, where
# * w_i = 1, except ``frozen`` on the index bands listed in ``bands`` (the
#   rows and columns of the cross),
# * K_k(i, j) = exp(-|i - j| / l_k), l_k = width0 * n * width_decay**(k-1)
#   (the change reaches less far from the diagonal at later steps),
# * H_k Hermitian with entries of modulus uniform in [1/2, 1] and uniform
#   phase (drawn for the strict lower triangle and mirrored; real diagonal),
# * eps_k = eps0 * decay**(k-1).
# Step 0 is a Hermitian Gaussian matrix (or a given pencil's A).


@dataclasses.dataclass(frozen=True)
class UpdateWorkload:
    name: str
    n: int
    steps: int  # updates after step 0
    p_t: float  # variation threshold as a fraction of delta
    width0: float
    width_decay: float
    bands: tuple  # ((start, stop), ...) as fractions of n
    frozen: float
    eps0: float
    decay: float


# at p_t = 0.1 the share of lower-triangle entries above threshold falls
# from about 0.6 at step 1 to about 0.15 at step 12 (n = 1024 and 8192)
UPDATE_SMALL = UpdateWorkload("update_n300_pt0.1", 300, 4, 0.1, 0.3, 0.8,
                              ((0.30, 0.38), (0.70, 0.76)), 0.05, 1e-2, 0.85)
UPDATE_LARGE = UpdateWorkload("update_n8192_pt0.1", 8192, 12, 0.1, 0.3, 0.8,
                              ((0.30, 0.36), (0.62, 0.66), (0.85, 0.88)), 0.05, 1e-2, 0.85)


def update_scaled(wl: UpdateWorkload, n: int, steps: Optional[int] = None) -> UpdateWorkload:
    return dataclasses.replace(wl, name=f"update_n{n}_pt{wl.p_t:g}", n=n,
                               steps=steps if steps is not None else wl.steps)


def update_weights(wl: UpdateWorkload) -> np.ndarray:
    w = np.ones(wl.n)
    for a, b in wl.bands:
        w[int(round(a * wl.n)):int(round(b * wl.n))] = wl.frozen
    return w


def update_envelope(wl: UpdateWorkload, k: int) -> np.ndarray:
    """eps_k * (w w^T) o K_k as a real n x n array (k >= 1)."""
    w = update_weights(wl)
    ell = wl.width0 * wl.n * wl.width_decay ** (k - 1)
    idx = np.arange(wl.n)
    K = np.exp(-np.abs(idx[:, None] - idx[None, :]) / ell)
    return wl.eps0 * wl.decay ** (k - 1) * (w[:, None] * w[None, :]) * K


def _bounded_hermitian(mod: np.ndarray, phase: np.ndarray) -> np.ndarray:
    M = np.tril(mod * np.exp(1j * phase), -1)
    return M + M.conj().T + np.diag(mod.diagonal() * np.cos(phase.diagonal()))


def update_sequence(wl: UpdateWorkload, seed: int, A0: Optional[np.ndarray] = None):
    """Yields A_0, A_1, ..., A_steps (complex128, Hermitian)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    if A0 is None:
        G = _cgauss(rng, (wl.n, wl.n))
        A = 0.5 * (G + G.conj().T)
    else:
        A = np.array(A0, dtype=np.complex128)
    yield A.copy()
    for k in range(1, wl.steps + 1):
        mod = rng.uniform(0.5, 1.0, size=(wl.n, wl.n))
        phase = rng.uniform(0.0, 2.0 * math.pi, size=(wl.n, wl.n))
        A = A + update_envelope(wl, k) * _bounded_hermitian(mod, phase)
        yield A.copy()


def update_sequence_torch(wl: UpdateWorkload, seed: int, device="cuda", A0=None):
    """The same construction with a seeded torch generator on ``device``
    (a different but deterministic random stream).  Yields torch tensors."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = wl.n
    if A0 is None:
        G = torch.randn(n, n, generator=g, device=device, dtype=torch.complex128)
        A = 0.5 * (G + G.conj().T)
        del G
    else:
        A = A0.clone()
    yield A.clone()
    w = torch.as_tensor(update_weights(wl), device=device, dtype=torch.float64)
    idx = torch.arange(n, device=device, dtype=torch.float64)
    for k in range(1, wl.steps + 1):
        ell = wl.width0 * n * wl.width_decay ** (k - 1)
        env = torch.exp(-(idx[:, None] - idx[None, :]).abs() / ell)
        env *= w[:, None] * w[None, :] * (wl.eps0 * wl.decay ** (k - 1))
        mod = torch.rand(n, n, generator=g, device=device, dtype=torch.float64) * 0.5 + 0.5
        phase = torch.rand(n, n, generator=g, device=device, dtype=torch.float64) * (2.0 * math.pi)
        M = torch.tril(torch.polar(mod, phase), -1)
        H = M + M.conj().T
        del M
        H.diagonal().copy_(mod.diagonal() * torch.cos(phase.diagonal()))
        del mod, phase
        A = A + env * H
        del H, env
        yield A.clone()
