"""ctypes binding of ``libgevp.so`` (declared in ``include/gevp.h``).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels on the GPU.  Tensors are torch tensors on the handle's device; the
library reads matrices column-major, so inputs that are not already
column-major (``t.stride() == (1, n)``) are copied into that layout, and
outputs are returned as column-major views with the usual (rows, cols)
shape.  If the library is missing the binding raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgevp.so")

GEVP_OK, GEVP_ERR_INVALID, GEVP_ERR_NOT_HPD, GEVP_ERR_NOCONV = 0, 1, 2, 3
GEVP_ERR_HIP, GEVP_ERR_NONFINITE, GEVP_ERR_ALLOC, GEVP_ERR_SINGULAR = 4, 5, 6, 7
GEVP_ERR_WORKSPACE = 8
FILTER_CHEBYSHEV, FILTER_CONTOUR = 0, 1
FILTERS = {"chebyshev": FILTER_CHEBYSHEV, "contour": FILTER_CONTOUR}
FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
STAGES = ("stage", "chol", "reduce", "bounds", "filter", "qr", "rr", "final")


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("nex", ctypes.c_int), ("deg_init", ctypes.c_int),
        ("deg_max", ctypes.c_int), ("maxit", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
        ("seed", ctypes.c_ulonglong), ("skip_final_residual", ctypes.c_int),
        ("batch_streams", ctypes.c_int), ("seed_monitor", ctypes.c_int),
        ("filter", ctypes.c_int), ("contour_points", ctypes.c_int),
        ("lock_mode", ctypes.c_int), ("sweep_reduction", ctypes.c_int),
        ("reserved", ctypes.c_int * 2),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("lapack_info", ctypes.c_int64), ("outer_iters", ctypes.c_int), ("nconv", ctypes.c_int),
        ("block", ctypes.c_int), ("qr_fallbacks", ctypes.c_int), ("col_degrees", ctypes.c_int64),
        ("max_resid", ctypes.c_double), ("normA", ctypes.c_double), ("normB", ctypes.c_double),
        ("filter_flops", ctypes.c_double), ("ms", ctypes.c_double * 8),
        ("filter_kernel_ms", ctypes.c_double), ("filter_launches", ctypes.c_int64),
        ("seed_sin_rms", ctypes.c_double), ("seed_dev_mean", ctypes.c_double),
        ("seed_dev_max", ctypes.c_double), ("seed_reindexed", ctypes.c_int),
        ("contour_points", ctypes.c_int), ("contour_a", ctypes.c_double),
        ("contour_b", ctypes.c_double), ("contour_applications", ctypes.c_int),
        ("contour_columns", ctypes.c_int64), ("seed_dev_std", ctypes.c_double),
        ("gemm_kernel_ms", ctypes.c_double), ("gemm_flops", ctypes.c_double),
        ("gemm_launches", ctypes.c_int64), ("locked", ctypes.c_int),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "ms"}
        d["ms"] = {s: self.ms[i] for i, s in enumerate(STAGES)}
        return d


class Tuning(ctypes.Structure):
    """gevp_tuning: launch configuration of gevp_solve_batched."""
    _fields_ = [("streams", ctypes.c_int), ("split_mode", ctypes.c_int), ("seconds", ctypes.c_double),
                ("reserved", ctypes.c_int * 4)]

    def as_dict(self):
        return {"streams": self.streams, "split_mode": self.split_mode, "seconds": self.seconds}


class UpdateInfo(ctypes.Structure):
    _fields_ = [
        ("delta", ctypes.c_double), ("entries", ctypes.c_int64), ("updated", ctypes.c_int64),
        ("tiles", ctypes.c_int64), ("tiles_touched", ctypes.c_int64),
        ("tiles_copied", ctypes.c_int64), ("nonfinite", ctypes.c_int), ("reserved", ctypes.c_int),
        ("scan_ms", ctypes.c_double), ("apply_ms", ctypes.c_double),
        ("rechecked", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class GevpError(RuntimeError):
    def __init__(self, status: int, what: str, info: Optional[Info] = None):
        self.status = status
        self.info = info
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lib = None


def load():
    """Load libgevp.so (built by ``paper_1007_4400_amd.build``); raises if it
    is missing -- the product path has no CPU fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1007_4400_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, L, D, C = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_char
    lib.gevp_status_string.argtypes = [I]
    lib.gevp_status_string.restype = ctypes.c_char_p
    lib.gevp_create.argtypes = [ctypes.POINTER(P), I]
    lib.gevp_create.restype = I
    lib.gevp_set_stream.argtypes = [P, P]
    lib.gevp_set_stream.restype = I
    lib.gevp_set_profiling.argtypes = [P, I]
    lib.gevp_set_profiling.restype = I
    lib.gevp_destroy.argtypes = [P]
    lib.gevp_destroy.restype = None
    lib.gevp_block_size.argtypes = [ctypes.POINTER(Opts), L, L]
    lib.gevp_block_size.restype = L
    lib.gevp_workspace_size.argtypes = [P, ctypes.POINTER(Opts), L, L, ctypes.POINTER(ctypes.c_size_t)]
    lib.gevp_workspace_size.restype = I
    lib.gevp_workspace_size_batched.argtypes = [P, ctypes.POINTER(Opts), I, P, P,
                                                ctypes.POINTER(ctypes.c_size_t)]
    lib.gevp_workspace_size_batched.restype = I
    lib.gevp_set_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.gevp_set_workspace.restype = I
    lib.gevp_solve.argtypes = [P, ctypes.POINTER(Opts), L, P, L, P, L, P, L, L, L, D, L, P, P, L, P,
                               ctypes.POINTER(Info)]
    lib.gevp_solve.restype = I
    lib.gevp_solve_batched.argtypes = [P, ctypes.POINTER(Opts), I, P, P, P, P, P, P, P, P, P, D, P,
                                       P, P, P, P, P]
    lib.gevp_solve_batched.restype = I
    lib.gevp_autotune_batched.argtypes = [P, ctypes.POINTER(Opts), I, P, P, P, P, P, P, P, P, P, D,
                                          P, P, P, P, P, ctypes.POINTER(Tuning)]
    lib.gevp_autotune_batched.restype = I
    lib.gevp_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.gevp_set_tuning.restype = I
    lib.gevp_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.gevp_get_tuning.restype = I
    lib.gevp_backward.argtypes = [P, L, L, P, L, P, P, P, L, P, L]
    lib.gevp_backward.restype = I
    lib.gevp_backward_noalloc.argtypes = [P, L, L, P, L, P, P, P, L, P, L]
    lib.gevp_backward_noalloc.restype = I
    lib.gevp_k_zgemm.argtypes = [P, C, C, L, L, L, D, P, L, P, L, D, P, L, D, P, L, P, P, L]
    lib.gevp_k_zgemm.restype = I
    lib.gevp_k_zgemm_tri.argtypes = [P, C, C, L, L, L, D, P, L, P, L, D, P, L, P, L, I, I]
    lib.gevp_k_zgemm_tri.restype = I
    lib.gevp_k_filter_gemm.argtypes = [P, I, L, L, P, L, P, L, P, L, P, L, P, L, P, P, P, P]
    lib.gevp_k_filter_gemm.restype = I
    lib.gevp_k_hemv.argtypes = [P, L, P, L, P, P]
    lib.gevp_k_hemv.restype = I
    lib.gevp_k_potrf.argtypes = [P, L, P, L, ctypes.POINTER(L)]
    lib.gevp_k_potrf.restype = I
    lib.gevp_k_trsm.argtypes = [P, C, C, L, L, P, L, P, L]
    lib.gevp_k_trsm.restype = I
    lib.gevp_k_heev.argtypes = [P, L, P, L, P, P, L]
    lib.gevp_k_heev.restype = I
    lib.gevp_k_seed_monitor.argtypes = [P, L, P, L, ctypes.POINTER(D), ctypes.POINTER(I)]
    lib.gevp_k_seed_monitor.restype = I
    lib.gevp_k_lu_shifted.argtypes = [P, L, P, L, D, D, P, L, ctypes.POINTER(L)]
    lib.gevp_k_lu_shifted.restype = I
    lib.gevp_k_contour_filter.argtypes = [P, L, P, L, P, L, L, D, D, I, P, L]
    lib.gevp_k_contour_filter.restype = I
    lib.gevp_update_thresholded.argtypes = [P, L, P, L, P, L, D, P, L, ctypes.POINTER(UpdateInfo)]
    lib.gevp_update_thresholded.restype = I
    lib.gevp_update_masked.argtypes = [P, L, P, L, P, L, P, L]
    lib.gevp_update_masked.restype = I
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().gevp_status_string(int(s)).decode()


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Column-major (Fortran-order) version of a 2-D tensor; no copy when it
    already is one.  Lazy conjugate / negative views are materialised first,
    since the library reads the stored values."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    t = t.resolve_conj().resolve_neg()
    r, c = t.shape
    if t.stride(0) == 1 and (t.stride(1) >= max(r, 1) or c == 1):
        return t
    return t.mT.contiguous().mT


def _on_device(t: torch.Tensor, device: int, name: str):
    if t.device.type != "cuda" or (t.device.index if t.device.index is not None else
                                   torch.cuda.current_device()) != device:
        raise ValueError(f"{name} must be on cuda:{device} (got {t.device})")


def _check_mat(t, name: str, device: int, dtype=torch.complex128, rows=None, cols=None,
               square=False) -> torch.Tensor:
    """Validate a matrix argument before its pointer crosses the ABI: a
    torch tensor of the given dtype, 2-D, with the expected shape, on the
    handle's device.  Returns its column-major form."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dim() != 2:
        raise ValueError(f"{name} must be a matrix, got shape {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if square and t.shape[0] != t.shape[1]:
        raise ValueError(f"{name} must be square, got shape {tuple(t.shape)}")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} must have {rows} rows, got {t.shape[0]}")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name} must have {cols} columns, got {t.shape[1]}")
    _on_device(t, device, name)
    return colmajor(t)


def _check_vec(t, name: str, device: int, length: int, dtype=torch.float64) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dim() != 1:
        raise ValueError(f"{name} must be a 1-D torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.shape[0] < length:
        raise ValueError(f"{name} must hold at least {length} entries, got {t.shape[0]}")
    _on_device(t, device, name)
    return t.contiguous()


def check_solve_args(A, B, nev, X0, device: int):
    """Validation of gevp_solve's tensor arguments (raises ValueError)."""
    A = _check_mat(A, "A", device, square=True)
    n = A.shape[0]
    B = _check_mat(B, "B", device, rows=n, cols=n)
    if not 1 <= int(nev) <= n:
        raise ValueError(f"nev must be in [1, {n}], got {nev}")
    if X0 is not None:
        X0 = _check_mat(X0, "X0", device, rows=n)
    return A, B, X0


def check_backward_args(X, lam, w, device: int, need_lam: bool):
    X = _check_mat(X, "X", device)
    nev = X.shape[1]
    if isinstance(w, torch.Tensor) and w.is_floating_point():
        w = w.to(torch.float64)
    w = _check_vec(w, "w", device, nev)
    lam = _check_vec(lam, "lam", device, nev) if (need_lam or lam is not None) else None
    return X, lam, w


def empty_colmajor(rows: int, cols: int, dtype=torch.complex128, device=None) -> torch.Tensor:
    return torch.empty((cols, rows), dtype=dtype, device=device).mT


def _ld(t: torch.Tensor) -> int:
    return max(int(t.stride(1)), int(t.shape[0]), 1)


def make_opts(precision="fp64", nex=0, deg_init=0, deg_max=0, maxit=0, lanczos_steps=0, seed=0,
              skip_final_residual=False, batch_streams=0, seed_monitor=False, filter="chebyshev",
              contour_points=0, locking="hard", sweep_reduction=0) -> Opts:
    o = Opts()
    o.lock_mode = {"hard": 0, "soft": 1}[locking]
    o.sweep_reduction = int(sweep_reduction)
    o.filter = FILTERS[filter] if isinstance(filter, str) else int(filter)
    o.contour_points = int(contour_points)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.nex, o.deg_init, o.deg_max, o.maxit = nex, deg_init, deg_max, maxit
    o.lanczos_steps, o.seed = lanczos_steps, seed
    o.skip_final_residual = int(bool(skip_final_residual))
    o.batch_streams = int(batch_streams)
    o.seed_monitor = int(bool(seed_monitor))
    return o


def workspace_size(n, nev, opts: Optional[Opts] = None) -> int:
    """Bytes of device workspace gevp_solve needs for (n, nev, opts); needs
    no GPU (the query does not touch a handle)."""
    b = ctypes.c_size_t(0)
    s = load().gevp_workspace_size(None, ctypes.byref(opts or make_opts()), int(n), int(nev),
                                   ctypes.byref(b))
    if s != GEVP_OK:
        raise GevpError(s, "gevp_workspace_size")
    return int(b.value)


class Handle:
    """One library handle (workspace owner) on a CUDA/HIP device."""

    def __init__(self, device: int = 0, profiling: int = 0):
        lib = load()
        self.lib = lib
        self.device = device
        h = ctypes.c_void_p()
        s = lib.gevp_create(ctypes.byref(h), device)
        if s != GEVP_OK:
            raise GevpError(s, "gevp_create")
        self.h = h
        if profiling:
            lib.gevp_set_profiling(h, int(profiling))

    def set_profiling(self, flags: int):
        self.lib.gevp_set_profiling(self.h, int(flags))

    def close(self):
        if getattr(self, "h", None):
            self.lib.gevp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        st = torch.cuda.current_stream(self.device).cuda_stream
        self.lib.gevp_set_stream(self.h, ctypes.c_void_p(st))

    def block_size(self, n, nev, opts: Optional[Opts] = None) -> int:
        return int(self.lib.gevp_block_size(ctypes.byref(opts or make_opts()), n, nev))

    # ---------------------------------------------------------- workspace
    def workspace_size(self, n, nev, opts: Optional[Opts] = None) -> int:
        """Bytes of device workspace gevp_solve needs for (n, nev, opts)."""
        return workspace_size(n, nev, opts)

    def workspace_size_batched(self, ns, nevs, opts: Optional[Opts] = None) -> int:
        cnt = len(ns)
        b = ctypes.c_size_t(0)
        s = self.lib.gevp_workspace_size_batched(
            self.h, ctypes.byref(opts or make_opts()), cnt, (ctypes.c_int64 * cnt)(*ns),
            (ctypes.c_int64 * cnt)(*nevs), ctypes.byref(b))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_workspace_size_batched")
        return int(b.value)

    def set_workspace(self, buf: Optional[torch.Tensor]):
        """Work only in ``buf`` (a contiguous uint8 tensor on the handle's
        device, e.g. ``torch.empty(handle.workspace_size(n, nev), dtype=torch.uint8,
        device="cuda")``); the handle keeps a reference.  None returns to
        library-managed memory."""
        if buf is None:
            s = self.lib.gevp_set_workspace(self.h, None, 0)
            if s != GEVP_OK:
                raise GevpError(s, "gevp_set_workspace")
            self._ws = None
            return
        if not isinstance(buf, torch.Tensor) or buf.dtype != torch.uint8 or not buf.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor")
        _on_device(buf, self.device, "workspace")
        self._stream()
        s = self.lib.gevp_set_workspace(self.h, ctypes.c_void_p(buf.data_ptr()), buf.numel())
        if s != GEVP_OK:
            raise GevpError(s, "gevp_set_workspace")
        self._ws = buf

    # ------------------------------------------------------------------ solve
    def solve(self, A, B, nev, X0=None, tol=1e-10, kx=None, opts: Optional[Opts] = None,
              raise_on_noconv=True, want_resid=True):
        """Lowest ``nev`` eigenpairs of A x = lambda B x.  Returns
        (lam[kx], X[n, kx], resid[kx] or None, info dict).  With
        want_resid=False the per-column residuals are not returned and the
        final check covers the nev wanted pairs only (info max_resid)."""
        opts = opts or make_opts()
        A, B, X0 = check_solve_args(A, B, nev, X0, self.device)
        n = A.shape[0]
        kx = nev if kx is None else kx
        dev = A.device
        lam = torch.empty(kx, dtype=torch.float64, device=dev)
        X = empty_colmajor(n, kx, device=dev)
        res = torch.empty(kx, dtype=torch.float64, device=dev) if want_resid else None
        k0 = X0.shape[1] if X0 is not None else 0
        info = Info()
        self._stream()
        s = self.lib.gevp_solve(self.h, ctypes.byref(opts), n, _ptr(A), _ld(A), _ptr(B), _ld(B),
                                _ptr(X0), _ld(X0) if X0 is not None else n, k0, nev, float(tol), kx,
                                _ptr(lam), _ptr(X), _ld(X), _ptr(res), ctypes.byref(info))
        if s != GEVP_OK and not (s == GEVP_ERR_NOCONV and not raise_on_noconv):
            raise GevpError(s, "gevp_solve", info)
        d = info.as_dict()
        d["status"] = s
        return lam, X, res, d

    def _batched_args(self, problems):
        """Checked tensors, outputs and the ctypes arrays of a batched call."""
        cnt = len(problems)
        arr = lambda t, vals: (t * cnt)(*vals)
        checked = [check_solve_args(p["A"], p["B"], p["nev"], p.get("X0"), self.device)
                   for p in problems]
        As = [c[0] for c in checked]
        Bs = [c[1] for c in checked]
        X0s = [c[2] for c in checked]
        ns = [a.shape[0] for a in As]
        nevs = [p["nev"] for p in problems]
        kxs = [p.get("kx") or p["nev"] for p in problems]
        lams = [torch.empty(k, dtype=torch.float64, device=a.device) for k, a in zip(kxs, As)]
        Xs = [empty_colmajor(n, k, device=a.device) for n, k, a in zip(ns, kxs, As)]
        rs = [torch.empty(k, dtype=torch.float64, device=a.device) for k, a in zip(kxs, As)]
        L64, VP = ctypes.c_int64, ctypes.c_void_p
        args = (cnt, arr(L64, ns), arr(VP, [a.data_ptr() for a in As]),
                arr(L64, [_ld(a) for a in As]), arr(VP, [b.data_ptr() for b in Bs]),
                arr(L64, [_ld(b) for b in Bs]),
                arr(VP, [x.data_ptr() if x is not None else None for x in X0s]),
                arr(L64, [_ld(x) if x is not None else n for x, n in zip(X0s, ns)]),
                arr(L64, [x.shape[1] if x is not None else 0 for x in X0s]), arr(L64, nevs))
        outs = (arr(L64, kxs), arr(VP, [t.data_ptr() for t in lams]),
                arr(VP, [x.data_ptr() for x in Xs]), arr(L64, [_ld(x) for x in Xs]),
                arr(VP, [t.data_ptr() for t in rs]))
        keep = (As, Bs, X0s)  # the tensors the pointers refer to
        return args, outs, (lams, Xs, rs), keep

    def solve_batched(self, problems, tol=1e-10, opts: Optional[Opts] = None, raise_on_noconv=True):
        """Independent pencils solved concurrently.  ``problems`` is a list of
        dicts with keys A, B, nev and optional X0, kx.  Returns a list of
        (lam, X, resid, info dict)."""
        opts = opts or make_opts()
        args, outs, (lams, Xs, rs), keep = self._batched_args(problems)
        cnt = len(problems)
        infos = (Info * cnt)()
        self._stream()
        s = self.lib.gevp_solve_batched(self.h, ctypes.byref(opts), *args, float(tol), *outs, infos)
        del keep
        if s != GEVP_OK and not (s == GEVP_ERR_NOCONV and not raise_on_noconv):
            raise GevpError(s, "gevp_solve_batched")
        out = []
        for i in range(cnt):
            d = infos[i].as_dict()
            out.append((lams[i], Xs[i], rs[i], d))
        return out

    def autotune_batched(self, problems, tol=1e-10, opts: Optional[Opts] = None, cache=None):
        """Pick the batched launch configuration (streams, split-K mode) by
        timing gevp_solve_batched on these problems (gevp_autotune_batched)
        and keep it in the handle.  With ``cache`` (a JSON file path), a
        configuration stored for the same device, precision, problem sizes and
        tolerance is applied without timing, and a new one is stored.
        Returns the configuration as a dict."""
        import hashlib
        import json
        import os

        opts = opts or make_opts()
        sizes = sorted((int(p["A"].shape[0]), int(p["nev"])) for p in problems)
        key = "|".join([torch.cuda.get_device_name(self.device), str(int(opts.precision)),
                        f"{float(tol):.3e}", hashlib.sha1(json.dumps(sizes).encode()).hexdigest()])
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tuning(table[key])
                return dict(table[key], cached=True)
        args, outs, _, keep = self._batched_args(problems)
        best = Tuning()
        self._stream()
        s = self.lib.gevp_autotune_batched(self.h, ctypes.byref(opts), *args, float(tol), *outs,
                                           ctypes.byref(best))
        del keep
        if s not in (GEVP_OK, GEVP_ERR_NOCONV):
            raise GevpError(s, "gevp_autotune_batched")
        t = best.as_dict()
        if cache:
            table[key] = t
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return dict(t, cached=False)

    def set_tuning(self, t):
        """Apply a batched launch configuration (dict with streams, split_mode
        and optionally seconds), or clear it with None."""
        if t is None:
            s = self.lib.gevp_set_tuning(self.h, None)
        else:
            tt = Tuning(int(t["streams"]), int(t["split_mode"]), float(t.get("seconds", 0.0)))
            s = self.lib.gevp_set_tuning(self.h, ctypes.byref(tt))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_set_tuning")

    def get_tuning(self):
        t = Tuning()
        s = self.lib.gevp_get_tuning(self.h, ctypes.byref(t))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_get_tuning")
        return t.as_dict()

    def backward(self, X, lam, w, want_dA=True, want_dB=True):
        X, lam, w = check_backward_args(X, lam, w, self.device, need_lam=want_dB)
        n, nev = X.shape
        dA = empty_colmajor(n, n, device=X.device) if want_dA else None
        dB = empty_colmajor(n, n, device=X.device) if want_dB else None
        self._stream()
        s = self.lib.gevp_backward(self.h, n, nev, _ptr(X), _ld(X), _ptr(lam), _ptr(w), _ptr(dA),
                                   n, _ptr(dB), n)
        if s != GEVP_OK:
            raise GevpError(s, "gevp_backward")
        return dA, dB

    # ------------------------------------------------------------ kernels
    def zgemm(self, opA, opB, A, B, alpha=1.0, beta=0.0, C=None, gamma=0.0, E=None, gcol=None,
              out=None, m=None, n=None, k=None):
        if opA not in ("N", "C") or opB not in ("N", "C"):
            raise ValueError("opA and opB must be 'N' or 'C'")
        A = _check_mat(A, "A", self.device)
        B = _check_mat(B, "B", self.device)
        ka = A.shape[1] if opA == "N" else A.shape[0]
        kb = B.shape[0] if opB == "N" else B.shape[1]
        m = m if m is not None else (A.shape[0] if opA == "N" else A.shape[1])
        k = k if k is not None else ka
        n = n if n is not None else (B.shape[1] if opB == "N" else B.shape[0])
        if k > min(ka, kb) or m > (A.shape[0] if opA == "N" else A.shape[1]) or \
                n > (B.shape[1] if opB == "N" else B.shape[0]):
            raise ValueError("m, n, k exceed the operands' shapes")
        if out is None:
            out = empty_colmajor(m, n, device=A.device)
        out = _check_mat(out, "out", self.device)
        if out.shape[0] < m or out.shape[1] < n:
            raise ValueError("out is smaller than m x n")
        C = _check_mat(C, "C", self.device) if C is not None else None
        E = _check_mat(E, "E", self.device) if E is not None else None
        for t, nm in ((C, "C"), (E, "E")):
            if t is not None and (t.shape[0] < m or t.shape[1] < n):
                raise ValueError(f"{nm} is smaller than m x n")
        if gcol is not None:
            gcol = _check_vec(gcol, "gcol", self.device, n)
        self._stream()
        s = self.lib.gevp_k_zgemm(self.h, opA.encode(), opB.encode(), m, n, k, float(alpha),
                                  _ptr(A), _ld(A), _ptr(B), _ld(B), float(beta), _ptr(C),
                                  _ld(C) if C is not None else m, float(gamma), _ptr(E),
                                  _ld(E) if E is not None else m, _ptr(gcol), _ptr(out), _ld(out))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_zgemm")
        return out

    def zgemm_tri(self, opA, opB, A, B, out, alpha=1.0, beta=0.0, C=None, lower=False,
                  upperA=False):
        """The structured products (gevp_k_zgemm_tri): `out` is written in
        place (lower: only tiles touching the lower triangle)."""
        if opA not in ("N", "C") or opB not in ("N", "C"):
            raise ValueError("opA and opB must be 'N' or 'C'")
        A = _check_mat(A, "A", self.device)
        B = _check_mat(B, "B", self.device)
        out = _check_mat(out, "out", self.device)
        m = A.shape[0] if opA == "N" else A.shape[1]
        k = A.shape[1] if opA == "N" else A.shape[0]
        n = B.shape[1] if opB == "N" else B.shape[0]
        if (B.shape[0] if opB == "N" else B.shape[1]) != k or tuple(out.shape) != (m, n):
            raise ValueError("operand shapes do not agree")
        C = _check_mat(C, "C", self.device, rows=m, cols=n) if C is not None else None
        self._stream()
        s = self.lib.gevp_k_zgemm_tri(self.h, opA.encode(), opB.encode(), m, n, k, float(alpha),
                                      _ptr(A), _ld(A), _ptr(B), _ld(B), float(beta), _ptr(C),
                                      _ld(C) if C is not None else m, _ptr(out), _ld(out),
                                      int(bool(lower)), int(bool(upperA)))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_zgemm_tri")
        return out

    def filter_gemm(self, precision, C, G, P, R, alpha, beta, gamma, delta):
        """One low-precision filter step: D = alpha C G + beta G + gamma P + delta R
        (per-column coefficients); C complex128, G/P/R complex64."""
        C = _check_mat(C, "C", self.device, square=True)
        n = C.shape[0]
        G = _check_mat(G, "G", self.device, dtype=torch.complex64, rows=n)
        m = G.shape[1]
        P = _check_mat(P, "P", self.device, dtype=torch.complex64, rows=n, cols=m)
        R = _check_mat(R, "R", self.device, dtype=torch.complex64, rows=n, cols=m)
        D = empty_colmajor(n, m, dtype=torch.complex64, device=G.device)
        co = [_check_vec(x.to(torch.float64), nm, self.device, m)
              for x, nm in zip((alpha, beta, gamma, delta), ("alpha", "beta", "gamma", "delta"))]
        self._stream()
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        s = self.lib.gevp_k_filter_gemm(self.h, pr, n, m, _ptr(C), _ld(C), _ptr(G), _ld(G), _ptr(P),
                                        _ld(P), _ptr(R), _ld(R), _ptr(D), _ld(D), *[_ptr(x) for x in co])
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_filter_gemm")
        return D

    def hemv(self, M, x):
        """y = M x for a Hermitian M stored in full (gevp_k_hemv)."""
        M = _check_mat(M, "M", self.device, square=True)
        n = M.shape[0]
        x = _check_vec(x, "x", self.device, n, dtype=torch.complex128)[:n]
        x = x.resolve_conj().resolve_neg().contiguous()
        y = torch.empty_like(x)
        self._stream()
        s = self.lib.gevp_k_hemv(self.h, n, _ptr(M), _ld(M), _ptr(x), _ptr(y))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_hemv")
        return y

    def potrf(self, M):
        """In-place lower Cholesky on a column-major copy; returns (L, pivot)."""
        L = _check_mat(M, "M", self.device, square=True).clone()
        n = L.shape[0]
        piv = ctypes.c_int64(0)
        self._stream()
        s = self.lib.gevp_k_potrf(self.h, n, _ptr(L), _ld(L), ctypes.byref(piv))
        if s not in (GEVP_OK, GEVP_ERR_NOT_HPD):
            raise GevpError(s, "gevp_k_potrf")
        return L, int(piv.value)

    def trsm(self, side, trans, L, R):
        if side not in ("L", "R") or trans not in ("N", "C") or (side, trans) == ("R", "N"):
            raise ValueError("side/trans must be L/N, L/C or R/C")
        L = _check_mat(L, "L", self.device, square=True)
        n = L.shape[0]
        R = _check_mat(R, "R", self.device, rows=n if side == "L" else None,
                       cols=n if side == "R" else None).clone()
        m = R.shape[1] if side == "L" else R.shape[0]
        self._stream()
        s = self.lib.gevp_k_trsm(self.h, side.encode(), trans.encode(), n, m, _ptr(L), _ld(L),
                                 _ptr(R), _ld(R))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_trsm")
        return R

    def heev(self, H):
        H = _check_mat(H, "H", self.device, square=True).clone()
        n = H.shape[0]
        th = torch.empty(n, dtype=torch.float64, device=H.device)
        Z = empty_colmajor(n, n, device=H.device)
        self._stream()
        s = self.lib.gevp_k_heev(self.h, n, _ptr(H), _ld(H), _ptr(th), _ptr(Z), _ld(Z))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_heev")
        return th, Z


    def seed_monitor(self, M):
        """Seed monitor of a k x k cross-overlap M: returns (sin_rms, dev_mean,
        dev_max, reindexed, dev_std, match)."""
        M = _check_mat(M, "M", self.device, square=True)
        k = M.shape[0]
        st = (ctypes.c_double * 5)()
        match = (ctypes.c_int * k)()
        self._stream()
        s = self.lib.gevp_k_seed_monitor(self.h, k, _ptr(M), _ld(M), st, match)
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_seed_monitor")
        return st[0], st[1], st[2], int(st[3]), st[4], list(match)

    # ---- contour-integral filter pieces

    def lu_shifted(self, C, z):
        """Packed LU (no row exchanges) of z I - C; returns (LU, pivot) with
        pivot = 0 or the first failing pivot (1-based)."""
        C = _check_mat(C, "C", self.device, square=True)
        n = C.shape[0]
        LU = empty_colmajor(n, n, device=C.device)
        piv = ctypes.c_int64(0)
        self._stream()
        s = self.lib.gevp_k_lu_shifted(self.h, n, _ptr(C), _ld(C), float(complex(z).real),
                                       float(complex(z).imag), _ptr(LU), _ld(LU), ctypes.byref(piv))
        if s not in (GEVP_OK, GEVP_ERR_SINGULAR):
            raise GevpError(s, "gevp_k_lu_shifted")
        return LU, int(piv.value)

    def contour_filter(self, C, V, a, b, nq):
        """Y = sum_j w_j (z_j I - C)^{-1} V on the circle with diameter [a, b]."""
        C = _check_mat(C, "C", self.device, square=True)
        V = _check_mat(V, "V", self.device, rows=C.shape[0])
        n, m = V.shape
        Y = empty_colmajor(n, m, device=V.device)
        self._stream()
        s = self.lib.gevp_k_contour_filter(self.h, n, _ptr(C), _ld(C), _ptr(V), _ld(V), m, float(a),
                                           float(b), int(nq), _ptr(Y), _ld(Y))
        if s != GEVP_OK:
            raise GevpError(s, "gevp_k_contour_filter")
        return Y

    # ---- thresholded partial matrix update

    def update_thresholded(self, A, A_new, p_t, mask=None, want_info=True):
        """In place on A (complex128, column-major, n x n): lower entries whose
        change exceeds p_t * delta are taken from A_new.  mask: optional int32
        tensor from empty_mask(n) receiving the updated entries.  Returns the
        gevp_update_info fields as a dict (with "status"), or None when
        want_info is False (then the call is asynchronous)."""
        n = _check_inplace(A)
        _on_device(A, self.device, "A")
        A_new = _check_mat(A_new, "A_new", self.device, rows=n, cols=n)
        ldm = _check_mask(mask, n)
        if mask is not None:
            _on_device(mask, self.device, "mask")
        inf = UpdateInfo() if want_info else None
        self._stream()
        s = self.lib.gevp_update_thresholded(self.h, n, _ptr(A), _ld(A), _ptr(A_new), _ld(A_new),
                                             float(p_t), _ptr(mask), ldm,
                                             ctypes.byref(inf) if want_info else None)
        if s not in (GEVP_OK, GEVP_ERR_NONFINITE):
            raise GevpError(s, "gevp_update_thresholded")
        if not want_info:
            return None
        d = inf.as_dict()
        d["status"] = s
        return d

    def update_masked(self, A, S, mask):
        """In place on A: lower entries whose bit is set in mask (int32 words
        from empty_mask(n)) are taken from S."""
        n = _check_inplace(A)
        _on_device(A, self.device, "A")
        S = _check_mat(S, "S", self.device, rows=n, cols=n)
        if mask is None:
            raise ValueError("mask is required")
        ldm = _check_mask(mask, n)
        _on_device(mask, self.device, "mask")
        self._stream()
        s = self.lib.gevp_update_masked(self.h, n, _ptr(A), _ld(A), _ptr(S), _ld(S), _ptr(mask), ldm)
        if s != GEVP_OK:
            raise GevpError(s, "gevp_update_masked")


def mask_words(n: int) -> int:
    """uint32 words per column of an update mask."""
    return (n + 31) // 32


def empty_mask(n: int, device=None) -> torch.Tensor:
    """Update mask storage: row j of the (n, mask_words(n)) int32 tensor holds
    column j's bits (bit i % 32 of word i // 32 is entry (i, j))."""
    return torch.empty((n, mask_words(n)), dtype=torch.int32, device=device)


def _check_inplace(A) -> int:
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.dtype != torch.complex128:
        raise ValueError("A must be a complex128 n x n matrix")
    if A.stride(0) != 1 and A.shape[0] > 1:
        raise ValueError("A is updated in place and must be column-major")
    if A.is_conj() or A.is_neg():
        raise ValueError("A is updated in place and must not be a lazy conjugate or negative view")
    return int(A.shape[0])


def _check_mask(mask, n) -> int:
    if mask is None:
        return 1
    if mask.dtype != torch.int32 or mask.dim() != 2 or mask.shape[0] != n or mask.stride(1) != 1 \
            or mask.shape[1] < mask_words(n):
        raise ValueError("mask must be an int32 tensor shaped (n, >= ceil(n/32)), rows contiguous")
    return max(int(mask.stride(0)), mask_words(n), 1)


class GEVPFunction(torch.autograd.Function):
    """Differentiable lowest-eigenvalue solve: ``lam = GEVPFunction.apply(A, B,
    nev, X0, tol, opts, handle)``.  Only eigenvalue cotangents are supported
    (the gradient of a loss built from eigenvalues, e.g. an occupation-weighted
    eigenvalue sum).  The gradients are those of the Hermitian pencil the
    lower triangles define, as full Hermitian matrices:
    dL/dA = X diag(g) X^H, dL/dB = -X diag(g lam) X^H (first-order perturbation
    of B-orthonormal pairs, computed by gevp_backward on the GPU)."""

    @staticmethod
    def forward(ctx, A, B, nev, X0=None, tol=1e-10, opts=None, handle=None):
        h = handle or _default_handle(A.device)
        lam, X, _, info = h.solve(A.detach(), B.detach(), nev, X0=X0, tol=tol, opts=opts)
        ctx.save_for_backward(X, lam)
        ctx.h = h
        ctx.mark_non_differentiable()
        return lam

    @staticmethod
    def backward(ctx, glam):
        X, lam = ctx.saved_tensors
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dA, dB = ctx.h.backward(X, lam, glam.to(torch.float64), want_dA=need_a, want_dB=need_b)
        return dA, dB, None, None, None, None, None


_handles = {}


def _default_handle(device):
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _handles:
        _handles[idx] = Handle(idx)
    return _handles[idx]
