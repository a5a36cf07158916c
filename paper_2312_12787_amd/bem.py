"""Thin Python binding of the C ABI in include/bem.h (libbem_hip.so).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  PyTorch supplies device memory and the HIP stream.  There is
no CPU fallback: if the library or a GPU is missing, the calls raise.

Matrix convention: a device matrix with leading dimension ld is held in a
torch tensor T of shape (ncols, ld); the mathematical matrix is T.T[:nrows].
A block of vectors (one per right-hand side) is a tensor of shape (nrhs, ld).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BEM_LIB_PATH") or os.path.join(_HERE, "libbem_hip.so")

F64, F32, MIXED = 0, 1, 2
MAX_RESTART = 1990  # BEM_MAX_RESTART of include/bem.h
CALDERON, CALDERON_BETA1, CONVENTIONAL, CALDERON_ORIG = 0, 1, 2, 3
STATUS = {0: "BEM_OK", 1: "BEM_E_ARG", 2: "BEM_E_GEOMETRY", 3: "BEM_E_STATE", 4: "BEM_E_DEVICE",
          5: "BEM_E_NOMEM", 6: "BEM_E_NOCONV", 7: "BEM_E_NONFINITE"}
EXPORTS = ["bem_create", "bem_destroy", "bem_n_elements", "bem_order", "bem_sizes", "bem_geometry",
           "bem_geometry_update", "bem_assemble", "bem_rhs", "bem_matvec", "bem_matvec_noalloc", "bem_solve",
           "bem_solve_batch", "bem_farfield", "bem_nearfield",
           "bem_profile_enable", "bem_profile_read", "bem_tune", "bem_tune_export", "bem_tune_import",
           "bem_tune_reset", "bem_last_error"]


class BemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class bem_z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class bem_desc(C.Structure):
    _fields_ = [("n_dom", C.c_int), ("k", C.POINTER(bem_z)), ("n_if", C.c_int), ("n_nodes", C.POINTER(C.c_int)),
                ("closed", C.POINTER(C.c_int)), ("xy", C.POINTER(C.c_double)), ("dom_left", C.POINTER(C.c_int)),
                ("dom_right", C.POINTER(C.c_int)), ("quad", C.c_int), ("form", C.c_int),
                ("alpha", C.POINTER(bem_z)), ("beta", C.POINTER(bem_z)), ("bm_coef", C.POINTER(bem_z))]


class bem_solve_opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iter", C.c_int), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("max_refine", C.c_int), ("graph_steps", C.c_int)]


class bem_profile(C.Structure):
    _fields_ = [("assemble_launches", C.c_int), ("assemble_ms", C.c_double), ("matvec_launches", C.c_int),
                ("matvec_ms", C.c_double), ("residual_launches", C.c_int), ("residual_ms", C.c_double)]


class bem_tune_info(C.Structure):
    _fields_ = [("rt", C.c_int), ("u", C.c_int), ("splits", C.c_int), ("g3", C.c_int), ("candidates", C.c_int),
                ("best_ms", C.c_double), ("default_ms", C.c_double)]


class bem_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int), ("rel_residual", C.c_double)]


_lib = None


def lib():
    """Load libbem_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_2312_12787_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.bem_create.argtypes = [C.POINTER(bem_desc), C.POINTER(vp)]
        L.bem_destroy.argtypes = [vp]
        L.bem_destroy.restype = None
        L.bem_n_elements.argtypes = [vp]
        L.bem_order.argtypes = [vp]
        L.bem_sizes.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(sz), C.POINTER(sz), C.POINTER(sz)]
        L.bem_geometry.argtypes = [vp, vp, sz, vp]
        L.bem_geometry_update.argtypes = [vp, vp]
        L.bem_assemble.argtypes = [vp, C.c_int, vp, sz, vp]
        L.bem_rhs.argtypes = [vp, C.c_int, C.POINTER(C.c_double), vp, sz, vp]
        L.bem_matvec.argtypes = [vp, C.c_int, vp, sz, vp, sz, vp, sz, vp]
        L.bem_matvec_noalloc.argtypes = [vp, C.c_int, vp, sz, vp, sz, vp]
        L.bem_solve.argtypes = [vp, C.c_int, vp, sz, C.POINTER(bem_solve_opts), vp, sz, vp, sz,
                                C.POINTER(bem_solve_info), vp]
        L.bem_solve_batch.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(C.c_int), C.POINTER(vp), C.POINTER(sz),
                                      C.POINTER(bem_solve_opts), C.POINTER(vp), C.POINTER(sz), C.POINTER(vp),
                                      C.POINTER(sz), C.POINTER(C.POINTER(bem_solve_info)), vp]
        L.bem_farfield.argtypes = [vp, C.c_int, vp, sz, C.c_int, C.POINTER(C.c_double), vp, sz, vp, sz, vp]
        L.bem_nearfield.argtypes = [vp, C.c_int, vp, sz, C.POINTER(C.c_double), C.c_int, vp, vp, vp, sz, vp]
        L.bem_profile_enable.argtypes = [vp, C.c_int]
        L.bem_profile_read.argtypes = [vp, C.POINTER(bem_profile), C.c_int]
        L.bem_tune.argtypes = [vp, C.c_int, vp, sz, vp, sz, vp, sz, C.c_int, C.POINTER(bem_tune_info), vp]
        L.bem_tune_export.argtypes = [C.c_char_p, sz]
        L.bem_tune_export.restype = sz
        L.bem_tune_import.argtypes = [C.c_char_p]
        L.bem_tune_reset.argtypes = []
        L.bem_tune_reset.restype = None
        L.bem_last_error.restype = C.c_char_p
        for f in ["bem_tune", "bem_tune_import", "bem_create", "bem_sizes", "bem_geometry", "bem_geometry_update", "bem_assemble", "bem_rhs", "bem_matvec", "bem_matvec_noalloc",
                  "bem_solve", "bem_solve_batch", "bem_farfield", "bem_nearfield", "bem_profile_enable", "bem_profile_read"]:
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def tune_export() -> str:
    """The process's tuned launch-shape table as text (bem_tune_export)."""
    n = lib().bem_tune_export(None, 0)
    buf = C.create_string_buffer(n + 1)
    lib().bem_tune_export(buf, n + 1)
    return buf.value.decode()


def tune_import(text: str) -> None:
    """Add a table in tune_export's format (bem_tune_import)."""
    _check(lib().bem_tune_import(text.encode()))


def tune_reset() -> None:
    """Forget every tuned shape (bem_tune_reset)."""
    lib().bem_tune_reset()


def _check(status: int, allow=()):
    if status != 0 and status not in allow:
        raise BemError(status, lib().bem_last_error().decode())
    return status


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _zarr(vals):
    arr = (bem_z * len(vals))()
    for i, v in enumerate(vals):
        arr[i].re = complex(v).real
        arr[i].im = complex(v).imag
    return arr


def _zptr(v):
    if v is None:
        return None, None
    z = bem_z(complex(v).real, complex(v).imag)
    return z, C.pointer(z)


@dataclass
class SolveInfo:
    iters: np.ndarray
    restarts: np.ndarray
    converged: np.ndarray
    rel_residual: np.ndarray
    status: int


def make_desc(spec):
    """bem_desc of a problem statement (attributes k, interfaces with xy,
    closed, dom_left, dom_right, and quad, form, alpha, beta, bm_coef); returns
    (desc, keep) where keep holds the ctypes arrays desc points into."""
    ks = list(spec.k)
    n_nodes = [len(f.xy) for f in spec.interfaces]
    xy = np.ascontiguousarray(np.concatenate([np.asarray(f.xy, np.float64) for f in spec.interfaces]).ravel())
    keep = dict(k=_zarr(ks), nn=(C.c_int * len(n_nodes))(*n_nodes),
                cl=(C.c_int * len(n_nodes))(*[1 if f.closed else 0 for f in spec.interfaces]),
                dl=(C.c_int * len(n_nodes))(*[int(f.dom_left) for f in spec.interfaces]),
                dr=(C.c_int * len(n_nodes))(*[int(f.dom_right) for f in spec.interfaces]),
                xy=xy, alpha=_zptr(spec.alpha), beta=_zptr(spec.beta),
                bm=_zarr(spec.bm_coef) if spec.bm_coef is not None else None)
    d = bem_desc()
    d.n_dom = len(ks)
    d.k = C.cast(keep["k"], C.POINTER(bem_z))
    d.n_if = len(n_nodes)
    d.n_nodes = keep["nn"]
    d.closed = keep["cl"]
    d.xy = xy.ctypes.data_as(C.POINTER(C.c_double))
    d.dom_left = keep["dl"]
    d.dom_right = keep["dr"]
    d.quad = int(spec.quad)
    d.form = int(spec.form)
    d.alpha = keep["alpha"][1]
    d.beta = keep["beta"][1]
    d.bm_coef = C.cast(keep["bm"], C.POINTER(bem_z)) if keep["bm"] is not None else None
    return d, keep


class Problem:
    """A transmission problem on the GPU.

    ``spec`` needs the attributes k (per-domain wavenumbers), interfaces (each
    with xy, closed, dom_left, dom_right), quad, form, alpha, beta, bm_coef.
    """

    def __init__(self, spec, device: str = "cuda"):
        import torch
        L = lib()
        self.spec = spec
        self.device = torch.device(device)
        d, self._keep = make_desc(spec)
        h = C.c_void_p()
        _check(L.bem_create(C.byref(d), C.byref(h)))
        self._h = h
        self.N = L.bem_n_elements(h)
        self.n = L.bem_order(h)
        self.geom = None
        self.A = None
        self.prec = None
        self._work = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().bem_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- sizes
    def sizes(self, prec: int = F64, nrhs: int = 1, restart: int = 1):
        g, m, w = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(lib().bem_sizes(self._h, prec, nrhs, restart, C.byref(g), C.byref(m), C.byref(w)))
        return g.value, m.value, w.value

    def _workspace(self, nbytes: int):
        import torch
        if self._work is None or self._work.numel() < nbytes:
            self._work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._work

    # ---------------------------------------------------------------- steps
    def geometry(self, stream=None):
        import torch
        g, _, _ = self.sizes()
        self.geom = torch.empty(g, dtype=torch.uint8, device=self.device)
        _check(lib().bem_geometry(self._h, C.c_void_p(self.geom.data_ptr()), g, _stream(stream)))
        return self

    def geometry_update(self, stream=None):
        """Re-derive the device tables from the inputs already on the device."""
        _check(lib().bem_geometry_update(self._h, _stream(stream)))
        self.A = None
        self.prec = None
        return self

    def assemble(self, prec: int = F64, out=None, lda: Optional[int] = None, stream=None):
        """Assemble into `out` (allocated if None) and return the matrix tensor.
        MIXED: `out` is a uint8 buffer of sizes(MIXED)[1] bytes holding the
        FP64 matrix and its FP32 copy; the FP64 part is returned.  F64 / F32:
        `out` is (n, lda) (column-major, lda >= n); an lda that is a multiple
        of 8 (complex128) or 16 (complex64) entries starts every column on a
        128-byte line, which the products read faster when n is not one."""
        import torch
        if self.geom is None:
            self.geometry(stream)
        if prec == MIXED:
            _, mb, _ = self.sizes(MIXED)
            if out is None:
                out = torch.empty(mb, dtype=torch.uint8, device=self.device)
            assert out.dtype == torch.uint8 and out.numel() >= mb and out.is_contiguous()
            _check(lib().bem_assemble(self._h, prec, C.c_void_p(out.data_ptr()), self.n, _stream(stream)))
            self.A = out
            self.prec = prec
            return out[:16 * self.n * self.n].view(torch.complex128).view(self.n, self.n)
        lda = lda or self.n
        dt = torch.complex128 if prec == F64 else torch.complex64
        if out is None:
            out = torch.empty((self.n, lda), dtype=dt, device=self.device)
        assert out.dtype == dt and out.shape[1] == lda and out.shape[0] >= self.n and out.is_contiguous()
        _check(lib().bem_assemble(self._h, prec, C.c_void_p(out.data_ptr()), lda, _stream(stream)))
        self.A = out
        self.prec = prec
        return out

    def rhs(self, angles: Sequence[float], stream=None):
        import torch
        ang = np.ascontiguousarray(angles, dtype=np.float64)
        B = torch.empty((len(ang), self.n), dtype=torch.complex128, device=self.device)
        _check(lib().bem_rhs(self._h, len(ang), ang.ctypes.data_as(C.POINTER(C.c_double)),
                             C.c_void_p(B.data_ptr()), self.n, _stream(stream)))
        return B

    def mixed_f32(self):
        """The FP32 copy of a MIXED matrix, as a (n, n) complex64 view."""
        import torch
        assert self.prec == MIXED
        off = (16 * self.n * self.n + 255) // 256 * 256
        return self.A[off:off + 8 * self.n * self.n].view(torch.complex64).view(self.n, self.n)

    def matvec(self, X, stream=None):
        """Y = A X for X of shape (nrhs, n) in the matrix precision (complex128
        for MIXED: its FP64 matrix)."""
        import torch
        X = X.contiguous()
        nrhs = X.shape[0]
        Y = torch.empty_like(X)
        _, _, wb = self.sizes(self.prec if self.prec is not None else F64, min(nrhs, 64), 1)
        W = self._workspace(wb)
        _check(lib().bem_matvec(self._h, nrhs, C.c_void_p(X.data_ptr()), X.shape[1], C.c_void_p(Y.data_ptr()),
                                Y.shape[1], C.c_void_p(W.data_ptr()), W.numel(), _stream(stream)))
        return Y

    def matvec_noalloc(self, X, Y=None, stream=None):
        """Y = A X through bem_matvec_noalloc (no workspace: the library's own
        device scratch).  Y (same shape and dtype as X) is allocated here if
        None; pass it to keep the call free of allocations."""
        import torch
        X = X.contiguous()
        if Y is None:
            Y = torch.empty_like(X)
        _check(lib().bem_matvec_noalloc(self._h, X.shape[0], C.c_void_p(X.data_ptr()), X.shape[1],
                                        C.c_void_p(Y.data_ptr()), Y.shape[1], _stream(stream)))
        return Y

    def tune(self, nrhs: int, reps: int = 3, X=None, stream=None):
        """Autotune the launch shape of the products bem_solve runs for nrhs
        right-hand sides on this matrix (bem_tune); returns the chosen shape
        and the timings.  X: complex128 (nrhs, n), random if None."""
        import torch
        if X is None:
            g = torch.Generator(device="cpu").manual_seed(1234)
            X = torch.complex(torch.rand(nrhs, self.n, generator=g, dtype=torch.float64),
                              torch.rand(nrhs, self.n, generator=g, dtype=torch.float64)).to(self.A.device)
        X = X.contiguous()
        Y = torch.empty_like(X)
        _, _, wb = self.sizes(self.prec if self.prec is not None else F64, min(nrhs, 64), 1)
        W = self._workspace(wb)
        info = bem_tune_info()
        _check(lib().bem_tune(self._h, nrhs, C.c_void_p(X.data_ptr()), X.shape[1], C.c_void_p(Y.data_ptr()),
                              Y.shape[1], C.c_void_p(W.data_ptr()), W.numel(), reps, C.byref(info), _stream(stream)))
        return {"rt": info.rt, "u": info.u, "splits": info.splits, "g3": info.g3, "candidates": info.candidates,
                "best_ms": info.best_ms, "default_ms": info.default_ms}

    def solve(self, B, restart: int = 100, tol: float = 1e-10, max_iter: int = 10000, inner_tol: float = 0.0,
              max_refine: int = 0, X=None, stream=None, raise_on_noconv: bool = False, graph_steps: int = 0):
        """Solve A X = B (B complex128 of shape (nrhs, n)); returns (X, SolveInfo).
        graph_steps > 0 runs the Krylov steps as captured HIP graphs of that many
        steps (bem_solve_opts.graph_steps)."""
        import torch
        B = B.contiguous()
        nrhs = B.shape[0]
        if X is None:
            X = torch.empty_like(B)
        _, _, wb = self.sizes(self.prec if self.prec is not None else F64, nrhs, restart)
        W = self._workspace(wb)
        opts = bem_solve_opts(restart, max_iter, tol, inner_tol, max_refine, graph_steps)
        info = (bem_solve_info * nrhs)()
        st = lib().bem_solve(self._h, nrhs, C.c_void_p(B.data_ptr()), B.shape[1], C.byref(opts),
                             C.c_void_p(X.data_ptr()), X.shape[1], C.c_void_p(W.data_ptr()), W.numel(), info,
                             _stream(stream))
        _check(st, allow=() if raise_on_noconv else (6,))
        return X, SolveInfo(np.array([i.iters for i in info]), np.array([i.restarts for i in info]),
                            np.array([i.converged for i in info]), np.array([i.rel_residual for i in info]), st)

    def profile(self, enable: bool = True):
        """Turn the library's HIP-event timing of the main kernels on or off."""
        _check(lib().bem_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        pr = bem_profile()
        _check(lib().bem_profile_read(self._h, C.byref(pr), 1 if reset else 0))
        return dict(assemble_launches=pr.assemble_launches, assemble_ms=pr.assemble_ms,
                    matvec_launches=pr.matvec_launches, matvec_ms=pr.matvec_ms,
                    residual_launches=pr.residual_launches, residual_ms=pr.residual_ms)

    def farfield(self, X, dirs: Sequence[float], stream=None):
        import torch
        X = X.contiguous()
        d = np.ascontiguousarray(dirs, dtype=np.float64)
        F = torch.empty((X.shape[0], len(d)), dtype=torch.complex128, device=self.device)
        _check(lib().bem_farfield(self._h, X.shape[0], C.c_void_p(X.data_ptr()), X.shape[1], len(d),
                                  d.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(F.data_ptr()), len(d),
                                  None, 0, _stream(stream)))
        return F

    def nearfield(self, X, points, dom, angles: Optional[Sequence[float]] = None, stream=None):
        """Field at points (npts, 2) in domains dom (npts,) for solutions X of
        shape (nrhs, n): the total field at host-medium points when the
        incident angles are given, else the scattered field.  Returns a
        complex128 tensor of shape (nrhs, npts)."""
        import torch
        X = X.contiguous()
        pts = torch.as_tensor(points, dtype=torch.float64, device=self.device).reshape(-1, 2).contiguous()
        dm = torch.as_tensor(dom, dtype=torch.int32, device=self.device).reshape(-1).contiguous()
        npts = pts.shape[0]
        assert dm.numel() == npts
        U = torch.zeros((X.shape[0], max(npts, 1)), dtype=torch.complex128, device=self.device)
        ang = None
        if angles is not None:
            ang = np.ascontiguousarray(angles, dtype=np.float64)
            assert len(ang) == X.shape[0]
        _check(lib().bem_nearfield(self._h, X.shape[0], C.c_void_p(X.data_ptr()), X.shape[1],
                                   ang.ctypes.data_as(C.POINTER(C.c_double)) if ang is not None else None, npts,
                                   C.c_void_p(pts.data_ptr()), C.c_void_p(dm.data_ptr()), C.c_void_p(U.data_ptr()),
                                   U.shape[1], _stream(stream)))
        return U[:, :npts]


def solve_batch(problems, Bs, restart: int = 100, tol: float = 1e-10, max_iter: int = 10000, inner_tol: float = 0.0,
                max_refine: int = 0, stream=None):
    """bem_solve_batch: solve A_k X_k = B_k for up to 8 assembled problems at
    once (restart cycles in step, fused orthogonalisation launches); returns
    [(X_k, SolveInfo_k)].  Bs[k]: complex128 (nrhs_k, n_k)."""
    import torch
    npb = len(problems)
    Bs = [B.contiguous() for B in Bs]
    Xs = [torch.empty_like(B) for B in Bs]
    Ws = []
    for g, B in zip(problems, Bs):
        _, _, wb = g.sizes(g.prec if g.prec is not None else F64, B.shape[0], restart)
        Ws.append(g._workspace(wb))
    infos = [(bem_solve_info * B.shape[0])() for B in Bs]
    vp = C.c_void_p
    arr = lambda t, vals: (t * npb)(*vals)
    opts = bem_solve_opts(restart, max_iter, tol, inner_tol, max_refine, 0)
    info_ptrs = (C.POINTER(bem_solve_info) * npb)(*[C.cast(i, C.POINTER(bem_solve_info)) for i in infos])
    st = lib().bem_solve_batch(npb, arr(vp, [g._h.value for g in problems]), arr(C.c_int, [B.shape[0] for B in Bs]),
                               arr(vp, [B.data_ptr() for B in Bs]), arr(C.c_size_t, [B.shape[1] for B in Bs]),
                               C.byref(opts), arr(vp, [X.data_ptr() for X in Xs]),
                               arr(C.c_size_t, [X.shape[1] for X in Xs]), arr(vp, [W.data_ptr() for W in Ws]),
                               arr(C.c_size_t, [W.numel() for W in Ws]), info_ptrs, _stream(stream))
    _check(st, allow=(6,))
    return [(X, SolveInfo(np.array([i.iters for i in inf]), np.array([i.restarts for i in inf]),
                          np.array([i.converged for i in inf]), np.array([i.rel_residual for i in inf]), st))
            for X, inf in zip(Xs, infos)]
