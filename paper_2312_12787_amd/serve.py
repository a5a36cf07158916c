"""Thin Python binding of the request server in include/bem_serve.h.

The server runs in the library (slot threads, HIP streams, arena admission);
this module marshals arguments, owns the device arena (a torch tensor) and
the host far-field buffers of pending requests.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from .bem import F32, F64, BemError, _check, bem_desc, bem_solve_opts, bem_z, lib, make_desc  # noqa: F401

SERVE_EXPORTS = ["bem_server_create", "bem_server_footprint", "bem_server_submit", "bem_server_poll",
                 "bem_server_stat", "bem_server_destroy"]


class bem_server_opts(C.Structure):
    _fields_ = [("slots", C.c_int), ("device", C.c_int), ("arena_dev", C.c_void_p), ("arena_bytes", C.c_size_t),
                ("prec", C.c_int), ("solve", bem_solve_opts), ("ndir", C.c_int), ("dirs", C.POINTER(C.c_double)),
                ("fuse", C.c_int)]


class bem_server_result(C.Structure):
    _fields_ = [("id", C.c_longlong), ("status", C.c_int), ("n", C.c_int), ("nrhs", C.c_int),
                ("iters_max", C.c_int), ("refine_max", C.c_int), ("rel_residual_max", C.c_double),
                ("footprint", C.c_size_t), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("message", C.c_char * 160)]


class bem_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("waiting", C.c_longlong), ("running", C.c_longlong),
                ("unpolled", C.c_longlong), ("arena_in_use", C.c_size_t), ("arena_high_water", C.c_size_t)]


def _serve_lib():
    L = lib()
    if not getattr(L, "_serve_ready", False):
        vp = C.c_void_p
        L.bem_server_create.argtypes = [C.POINTER(bem_server_opts), C.POINTER(vp)]
        L.bem_server_footprint.argtypes = [vp, C.POINTER(bem_desc), C.c_int, C.POINTER(C.c_size_t)]
        L.bem_server_submit.argtypes = [vp, C.POINTER(bem_desc), C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(bem_z), C.POINTER(C.c_longlong)]
        L.bem_server_poll.argtypes = [vp, C.POINTER(bem_server_result), C.c_int, C.POINTER(C.c_int), C.c_int]
        L.bem_server_stat.argtypes = [vp, C.POINTER(bem_server_stats)]
        L.bem_server_destroy.argtypes = [vp]
        for f in SERVE_EXPORTS:
            getattr(L, f).restype = C.c_int
        L._serve_ready = True
    return L


@dataclass
class Result:
    id: int
    status: int
    n: int
    nrhs: int
    iters_max: int
    refine_max: int
    rel_residual_max: float
    footprint: int
    t_submit: float
    t_admit: float
    t_done: float
    message: str
    far_field: np.ndarray   # (nrhs, ndir) complex128


class Server:
    """Continuous-batching solver service on one GPU.

    slots: requests in flight at once; arena_bytes: device memory the server
    sub-allocates per request (admission by footprint); prec: F32 (FP32 matrix
    and products with FP64 refinement) or F64; dirs: far-field directions
    returned for every right-hand side; graph_steps: Krylov steps per captured
    HIP graph in every request's solve (0: launched kernel by kernel); fuse: up
    to this many requests admitted together by a slot are solved as one batch
    with fused Krylov launches (1: one request per slot).
    """

    def __init__(self, arena_bytes: int, slots: int = 4, prec: int = F32, restart: int = 100, tol: float = 1e-8,
                 inner_tol: float = 1e-5, max_iter: int = 20000, max_refine: int = 0,
                 dirs: Sequence[float] = (0.0,), device: str = "cuda", graph_steps: int = 0, fuse: int = 1):
        import torch
        L = _serve_lib()
        self.device = torch.device(device)
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        self.dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        o = bem_server_opts()
        o.slots = int(slots)
        o.device = int(idx)
        o.arena_dev = self.arena.data_ptr()
        o.arena_bytes = self.arena.numel()
        o.prec = int(prec)
        o.solve = bem_solve_opts(int(restart), int(max_iter), float(tol), float(inner_tol), int(max_refine),
                                int(graph_steps))
        o.ndir = len(self.dirs)
        o.dirs = self.dirs.ctypes.data_as(C.POINTER(C.c_double))
        o.fuse = int(fuse)
        h = C.c_void_p()
        _check(L.bem_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._out: Dict[int, np.ndarray] = {}

    def footprint(self, spec, nrhs: int) -> int:
        d, _keep = make_desc(spec)
        b = C.c_size_t()
        _check(_serve_lib().bem_server_footprint(self._h, C.byref(d), int(nrhs), C.byref(b)))
        return b.value

    def submit(self, spec, angles: Sequence[float]) -> int:
        d, _keep = make_desc(spec)
        ang = np.ascontiguousarray(angles, dtype=np.float64)
        out = np.empty((len(ang), len(self.dirs)), dtype=np.complex128)
        rid = C.c_longlong()
        _check(_serve_lib().bem_server_submit(self._h, C.byref(d), len(ang), ang.ctypes.data_as(C.POINTER(C.c_double)),
                                              out.ctypes.data_as(C.POINTER(bem_z)), C.byref(rid)))
        self._out[rid.value] = out
        return rid.value

    def poll(self, wait_ms: int = 0, max_results: int = 256) -> List[Result]:
        buf = (bem_server_result * max_results)()
        cnt = C.c_int()
        _check(_serve_lib().bem_server_poll(self._h, buf, max_results, C.byref(cnt), int(wait_ms)))
        res = []
        for r in buf[:cnt.value]:
            res.append(Result(r.id, r.status, r.n, r.nrhs, r.iters_max, r.refine_max, r.rel_residual_max,
                              r.footprint, r.t_submit, r.t_admit, r.t_done, r.message.decode(errors="replace"),
                              self._out.pop(r.id)))
        return res

    def drain(self) -> List[Result]:
        """Wait for every submitted request; return their results."""
        out = []
        while self._out:
            out.extend(self.poll(wait_ms=-1))
        return out

    def stats(self) -> dict:
        st = bem_server_stats()
        _check(_serve_lib().bem_server_stat(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in bem_server_stats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _serve_lib().bem_server_destroy(h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
