"""ctypes binding of the C oracle (oracle/bem_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")

CALDERON, CALDERON_BETA1, CONVENTIONAL, CALDERON_ORIG = 0, 1, 2, 3


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(_LIB_PATH)
        L.or_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.or_hankel01.argtypes = [C.c_double, C.c_double, _dp]
        L.or_self_terms.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
        L.or_problem_new.restype = C.c_void_p
        L.or_problem_new.argtypes = [C.c_int, _dp, C.c_int, _ip, _ip, _dp, _ip, _ip, C.c_int, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_problem_free.argtypes = [C.c_void_p]
        L.or_n_elements.argtypes = [C.c_void_p]
        L.or_last_error.restype = C.c_char_p
        L.or_elements.argtypes = [C.c_void_p, _dp]
        L.or_normals.argtypes = [C.c_void_p, _dp]
        L.or_operator_entries.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.or_assemble.argtypes = [C.c_void_p, _dp]
        L.or_assemble_rows.argtypes = [C.c_void_p, C.c_int, _ip, _dp]
        L.or_rhs.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        L.or_matvec.argtypes = [C.c_int, _dp, _dp, _dp]
        L.or_matvec.restype = None
        L.or_lu_solve.argtypes = [C.c_int, _dp, C.c_int, _dp]
        L.or_gmres.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_double, C.c_int, _dp,
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_farfield.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, _dp, _dp]
        L.or_nearfield.argtypes = [C.c_void_p, C.c_int, _dp, C.c_void_p, C.c_int, _dp, _ip, _dp]
        _lib = L
    return _lib


def _cview(a: np.ndarray) -> np.ndarray:
    """complex128 array (any order given) -> float64 view of its memory."""
    return a.view(np.float64)


def gauss_legendre(q: int):
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().or_gauss_legendre(q, x, w):
        raise ValueError(lib().or_last_error().decode())
    return x, w


def hankel01(z: complex):
    out = np.zeros(4)
    if lib().or_hankel01(float(np.real(z)), float(np.imag(z)), out):
        raise ValueError(lib().or_last_error().decode())
    return complex(out[0], out[1]), complex(out[2], out[3])


def self_terms(k: complex, h: float):
    out = np.zeros(4)
    lib().or_self_terms(float(np.real(k)), float(np.imag(k)), float(h), out)
    return complex(out[0], out[1]), complex(out[2], out[3])


def _opt_complex(v):
    if v is None:
        return None, None
    arr = np.array([complex(v).real, complex(v).imag], dtype=np.float64)
    return arr, arr.ctypes.data_as(C.c_void_p)


class Problem:
    """Oracle view of a ``workloads.ProblemSpec``."""

    def __init__(self, spec):
        L = lib()
        k, n_nodes, closed, xy, dl, dr = spec.flat()
        self._keep = []
        a_arr, a_ptr = _opt_complex(spec.alpha)
        b_arr, b_ptr = _opt_complex(spec.beta)
        if spec.bm_coef is not None:
            c_arr = np.array([[complex(v).real, complex(v).imag] for v in spec.bm_coef], np.float64).ravel()
            c_ptr = c_arr.ctypes.data_as(C.c_void_p)
        else:
            c_arr, c_ptr = None, None
        self._keep += [a_arr, b_arr, c_arr]
        h = L.or_problem_new(len(spec.k), k, len(spec.interfaces), n_nodes, closed, xy, dl, dr,
                             int(spec.quad), int(spec.form), a_ptr, b_ptr, c_ptr)
        if not h:
            raise ValueError("oracle: " + L.or_last_error().decode())
        self._h = h
        self.spec = spec
        self.N = L.or_n_elements(h)
        self.n = 2 * self.N

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_problem_free(h)
            self._h = None

    def elements(self):
        out = np.zeros(9 * self.N)
        lib().or_elements(self._h, out)
        return out.reshape(self.N, 9)

    def normals(self):
        out = np.zeros(2 * self.N)
        lib().or_normals(self._h, out)
        return out.reshape(self.N, 2)

    def operator_entries(self, d: int, i: int, j: int):
        out = np.zeros(8)
        if lib().or_operator_entries(self._h, d, i, j, out):
            raise IndexError(lib().or_last_error().decode())
        return out.view(np.complex128)

    def assemble(self) -> np.ndarray:
        A = np.zeros((self.n, self.n), dtype=np.complex128, order="F")
        flat = A.reshape(-1, order="F").view(np.float64)
        if lib().or_assemble(self._h, flat):
            raise RuntimeError(lib().or_last_error().decode())
        return A

    def assemble_rows(self, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        out = np.zeros((len(rows), self.n), dtype=np.complex128)
        if lib().or_assemble_rows(self._h, len(rows), rows, _cview(out).reshape(-1)):
            raise IndexError(lib().or_last_error().decode())
        return out

    def rhs(self, angles) -> np.ndarray:
        angles = np.ascontiguousarray(angles, dtype=np.float64)
        B = np.zeros((self.n, len(angles)), dtype=np.complex128, order="F")
        lib().or_rhs(self._h, len(angles), angles, B.reshape(-1, order="F").view(np.float64))
        return B

    def farfield(self, X: np.ndarray, dirs) -> np.ndarray:
        X = np.asfortranarray(X.reshape(self.n, -1), dtype=np.complex128)
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        F = np.zeros((len(dirs), X.shape[1]), dtype=np.complex128, order="F")
        lib().or_farfield(self._h, X.shape[1], X.reshape(-1, order="F").view(np.float64), len(dirs), dirs,
                          F.reshape(-1, order="F").view(np.float64))
        return F

    def nearfield(self, X: np.ndarray, points, dom, angles=None) -> np.ndarray:
        """Field at points (npts, 2) of domains dom (npts,) for solutions X
        (2N, nrhs): total field at host-medium points when angles are given,
        else the scattered field; returns (npts, nrhs)."""
        X = np.asfortranarray(np.asarray(X, dtype=np.complex128).reshape(self.n, -1))
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
        dm = np.ascontiguousarray(dom, dtype=np.int32)
        ang = None if angles is None else np.ascontiguousarray(angles, dtype=np.float64)
        U = np.zeros((len(pts), X.shape[1]), dtype=np.complex128, order="F")
        st = lib().or_nearfield(self._h, X.shape[1], X.reshape(-1, order="F").view(np.float64),
                                None if ang is None else ang.ctypes.data_as(C.c_void_p), len(pts), pts.reshape(-1), dm,
                                U.reshape(-1, order="F").view(np.float64))
        if st:
            raise ValueError(lib().or_last_error().decode())
        return U


def matvec(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    A = np.asfortranarray(A, dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.zeros_like(x)
    lib().or_matvec(A.shape[0], A.reshape(-1, order="F").view(np.float64), x.view(np.float64), y.view(np.float64))
    return y


def lu_solve(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = np.array(A, dtype=np.complex128, order="F", copy=True)
    B2 = np.array(B.reshape(A.shape[0], -1), dtype=np.complex128, order="F", copy=True)
    if lib().or_lu_solve(A.shape[0], A.reshape(-1, order="F").view(np.float64), B2.shape[1],
                         B2.reshape(-1, order="F").view(np.float64)):
        raise np.linalg.LinAlgError("oracle LU: zero pivot")
    return B2.reshape(B.shape)


def gmres(A: np.ndarray, b: np.ndarray, restart: int, tol: float, max_it: int = 10000):
    """Returns (x, iterations, relative residual, converged)."""
    A = np.asfortranarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    it = C.c_int(0)
    rr = C.c_double(0.0)
    rc = lib().or_gmres(A.shape[0], A.reshape(-1, order="F").view(np.float64), b.view(np.float64), restart,
                        tol, max_it, x.view(np.float64), C.byref(it), C.byref(rr))
    return x, it.value, rr.value, rc == 0
