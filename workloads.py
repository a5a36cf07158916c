"""Seeded synthetic inputs for the collocation BEM of arXiv 2312.12787.

This module only produces INPUTS: boundary polylines, wavenumbers, incident
angles, solver settings and request streams.  It holds none of the method's
arithmetic (no element geometry, kernels, quadrature or solves), so the CPU
oracle and the HIP path can both take their inputs from here without sharing
any of the computation.

Orientation convention used by every generator: an interface's normal is the
LEFT normal of its direction of travel.  It points INTO ``dom_left`` and OUT
of ``dom_right``.  The host medium is domain 0 and must be a ``dom_right``
(Sec. 2: the normal is directed from the host medium; Sec. 6: for the
multi-material sketch the normals point into Omega_2).  A counter-clockwise
outer boundary therefore has ``dom_left`` = scatterer, ``dom_right`` = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

CALDERON = 0          # eq. (calderon_bieb) beta=-alpha / eq. (3dom_calderon_bie)
CALDERON_BETA1 = 1    # eq. (calderon_bie1)
CONVENTIONAL = 2      # eq. (naive_bie) / eq. (3dom_conv_bie)
CALDERON_ORIG = 3     # eq. (3dom_calderon_bie0)


@dataclass
class Interface:
    xy: np.ndarray            # (n_nodes, 2) float64 node coordinates
    closed: bool              # closed curve: last element joins node n-1 to node 0
    dom_left: int             # domain the normal points into
    dom_right: int            # domain the normal leaves


@dataclass
class ProblemSpec:
    k: List[complex]                      # wavenumber of each domain; k[0] real > 0
    interfaces: List[Interface]
    quad: int = 8                         # Gauss-Legendre points per element
    form: int = CALDERON
    alpha: Optional[complex] = None       # None: -i/k0
    beta: Optional[complex] = None        # None: -alpha (Calderon forms) or 1
    bm_coef: Optional[List[complex]] = None  # None: alpha/eps_d per domain
    name: str = ""

    @property
    def n_elements(self) -> int:
        return sum(len(f.xy) if f.closed else len(f.xy) - 1 for f in self.interfaces)

    @property
    def order(self) -> int:
        return 2 * self.n_elements

    # flat arrays in the layout both C interfaces take
    def flat(self):
        k = np.array([[complex(v).real, complex(v).imag] for v in self.k], dtype=np.float64).ravel()
        n_nodes = np.array([len(f.xy) for f in self.interfaces], dtype=np.int32)
        closed = np.array([1 if f.closed else 0 for f in self.interfaces], dtype=np.int32)
        xy = np.ascontiguousarray(np.concatenate([np.asarray(f.xy, np.float64) for f in self.interfaces]).ravel())
        dl = np.array([f.dom_left for f in self.interfaces], dtype=np.int32)
        dr = np.array([f.dom_right for f in self.interfaces], dtype=np.int32)
        return k, n_nodes, closed, xy, dl, dr


# --------------------------------------------------------------------------
# boundary curves
# --------------------------------------------------------------------------
def circle_nodes(n: int, radius: float = 1.0, clockwise: bool = False, center=(0.0, 0.0)) -> np.ndarray:
    """Inscribed regular n-gon, vertex 0 at angle 0 (Sec. 7: the unit circle is
    approximated by its inscribed polygon)."""
    t = 2.0 * np.pi * np.arange(n) / n
    if clockwise:
        t = -t
    return np.stack([center[0] + radius * np.cos(t), center[1] + radius * np.sin(t)], axis=1)


def kite_nodes(n: int) -> np.ndarray:
    """Kite x(t) = (cos t + 0.65 cos 2t - 0.65, 1.5 sin t) at t_j = 2 pi j / n (CCW)."""
    t = 2.0 * np.pi * np.arange(n) / n
    return np.stack([np.cos(t) + 0.65 * np.cos(2 * t) - 0.65, 1.5 * np.sin(t)], axis=1)


def perturbed_circle_nodes(n: int, amps: Sequence[float], phases: Sequence[float]) -> np.ndarray:
    """r(t) = 1 + sum_{m=2..6} a_m cos(m t + phi_m) at t_j = 2 pi j / n (CCW)."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = np.ones_like(t)
    for m, (a, p) in enumerate(zip(amps, phases), start=2):
        r += a * np.cos(m * t + p)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def square_nodes(per_side: int, side: float = 1.0) -> np.ndarray:
    """Square of the given side, centred at 0, ``per_side`` equal elements per
    side, CCW starting at the lower-left corner (Sec. 4 check)."""
    h = side / per_side
    s = side / 2.0
    pts = []
    for i in range(per_side):
        pts.append((-s + i * h, -s))
    for i in range(per_side):
        pts.append((s, -s + i * h))
    for i in range(per_side):
        pts.append((s - i * h, s))
    for i in range(per_side):
        pts.append((-s, s - i * h))
    return np.array(pts, dtype=np.float64)


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------
def single_material(nodes: np.ndarray, k0: float, k1: complex, quad: int = 8, form: int = CALDERON,
                    name: str = "", **kw) -> ProblemSpec:
    """A scatterer (domain 1) bounded by the CCW closed curve ``nodes`` in the
    host medium (domain 0)."""
    return ProblemSpec(k=[complex(k0), complex(k1)],
                       interfaces=[Interface(np.asarray(nodes, np.float64), True, 1, 0)],
                       quad=quad, form=form, name=name, **kw)


def disk(n: int, k0: float, k1: complex, radius: float = 1.0, **kw) -> ProblemSpec:
    return single_material(circle_nodes(n, radius), k0, k1, name=f"disk{n}", **kw)


def kite(n: int, k0: float, k1: complex, **kw) -> ProblemSpec:
    return single_material(kite_nodes(n), k0, k1, name=f"kite{n}", **kw)


def concentric(n_outer: int, n_inner: int, k: Sequence[complex], r_outer: float = 2.0,
               r_inner: float = 1.0, quad: int = 8, form: int = CALDERON) -> ProblemSpec:
    """Concentric disks (Sec. 7.2): Omega_2 = annulus (domain 1), Omega_3 =
    inner disk (domain 2).  Normals point into Omega_2 on both circles, so the
    inner circle is traversed clockwise."""
    outer = Interface(circle_nodes(n_outer, r_outer), True, 1, 0)
    inner = Interface(circle_nodes(n_inner, r_inner, clockwise=True), True, 1, 2)
    return ProblemSpec(k=[complex(v) for v in k], interfaces=[outer, inner], quad=quad, form=form,
                       name=f"concentric{n_outer}+{n_inner}")


def graded_params(length: float, h: float, grade_start: bool, grade_end: bool, hmin_ratio: float = 16.0,
                  ratio: float = 1.5) -> np.ndarray:
    """Node parameters in [0, length]: element size h in the middle, refined
    geometrically (sizes h/hmin_ratio, x ratio, ...) toward the graded ends."""
    ramp = []
    size = h / hmin_ratio
    while size < h:
        ramp.append(size)
        size *= ratio
    ramp = np.array(ramp)
    left = ramp if grade_start else np.array([])
    right = ramp[::-1] if grade_end else np.array([])
    middle_len = length - left.sum() - right.sum()
    if middle_len <= h:  # too short to grade: uniform
        n = max(1, int(round(length / h)))
        return np.linspace(0.0, length, n + 1)
    n_mid = max(1, int(round(middle_len / h)))
    mid = np.full(n_mid, middle_len / n_mid)
    sizes = np.concatenate([left, mid, right])
    t = np.concatenate([[0.0], np.cumsum(sizes)])
    t[-1] = length
    return t


def sectors(k: Sequence[complex], h: float = 1.0 / 800, graded: bool = True, angles_deg=(90.0, 210.0, 330.0),
            quad: int = 8, form: int = CALDERON, hmin_ratio: float = 16.0) -> ProblemSpec:
    """Unit disk split into three 120-degree sectors (domains 1, 2, 3; sector s
    spans [theta_s, theta_s + 120 deg)) in the host medium (domain 0).  Six
    open interfaces: the three arcs (normal into the sector, leaving the host)
    and the three radii at theta_s from the centre outwards (normal into
    sector s, leaving sector s-1).  Junctions: the centre and the three outer
    triple points; with graded=True the elements shrink geometrically (ratio
    1.5, down to h/16) toward every junction."""
    th = [np.deg2rad(a) for a in angles_deg]
    ifs = []
    for s_ in range(3):
        t = graded_params(2 * np.pi / 3, h, graded, graded, hmin_ratio)
        phi = th[s_] + t
        xy = np.stack([np.cos(phi), np.sin(phi)], axis=1)
        xy[0] = [np.cos(th[s_]), np.sin(th[s_])]
        xy[-1] = [np.cos(th[(s_ + 1) % 3]), np.sin(th[(s_ + 1) % 3])]
        ifs.append(Interface(xy, False, s_ + 1, 0))
    for s_ in range(3):
        t = graded_params(1.0, h, graded, graded, hmin_ratio)
        xy = np.stack([t * np.cos(th[s_]), t * np.sin(th[s_])], axis=1)
        xy[0] = [0.0, 0.0]
        xy[-1] = [np.cos(th[s_]), np.sin(th[s_])]
        ifs.append(Interface(xy, False, s_ + 1, (s_ - 1) % 3 + 1))
    return ProblemSpec(k=[complex(v) for v in k], interfaces=ifs, quad=quad, form=form, name="sectors")


def split_disk(n: int, k: Sequence[complex], quad: int = 8, form: int = CALDERON) -> ProblemSpec:
    """Unit disk split by its vertical diameter (Sec. 7.2, junction example:
    two triple points at (0, +-1)): left half = domain 1, right half =
    domain 2.  3n/8 elements on each half circle (counter-clockwise, normal
    into the disk) and n/4 on the diameter (upwards, normal into the left
    half)."""
    n_arc = max(1, int(round(3 * n / 8)))
    n_line = max(1, n - 2 * n_arc)
    def arc(a0, a1):
        t = np.linspace(a0, a1, n_arc + 1)
        return np.stack([np.cos(t), np.sin(t)], axis=1)
    left = arc(0.5 * np.pi, 1.5 * np.pi)
    right = arc(1.5 * np.pi, 2.5 * np.pi)
    for xy in (left, right):  # exact junction coordinates
        xy[0] = [0.0, np.sign(xy[0, 1])]
        xy[-1] = [0.0, np.sign(xy[-1, 1])]
    line = np.stack([np.zeros(n_line + 1), np.linspace(-1.0, 1.0, n_line + 1)], axis=1)
    ifs = [Interface(left, False, 1, 0), Interface(right, False, 2, 0), Interface(line, False, 1, 2)]
    return ProblemSpec(k=[complex(v) for v in k], interfaces=ifs, quad=quad, form=form, name=f"split_disk{n}")


def equispaced_angles(n: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n) / n


# --------------------------------------------------------------------------
# the benchmark workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    problems: List[ProblemSpec]
    angles: np.ndarray
    restart: int
    tol: float
    far_dirs: np.ndarray = field(default_factory=lambda: equispaced_angles(360))
    precision: str = "f64"       # "f32": FP32 matrix and products, FP64 refinement
    inner_tol: float = 1e-5      # inner (FP32-product) GMRES tolerance of the mixed path


def workload_disk256() -> Workload:
    """Unit disk as a 256-gon, k0 = 1, k1 = 2, 8-point Gauss, angle 0, GMRES(50), 1e-10."""
    return Workload("disk256_k1-2", [disk(256, 1.0, 2.0)], np.array([0.0]), 50, 1e-10)


def workload_kite4096(n: int = 4096) -> Workload:
    """Kite with N = 4096 elements (8192 x 8192 complex128), k0 = 20 with
    k1 = 30 and with lossy k1 = 30 + 0.3i, 16 equispaced incident angles,
    GMRES(100) to 1e-10."""
    return Workload(f"kite{n}_k20-30_x16", [kite(n, 20.0, 30.0), kite(n, 20.0, 30.0 + 0.3j)],
                    equispaced_angles(16), 100, 1e-10)


def workload_sectors(h: float = 1.0 / 800) -> Workload:
    """Unit disk in three 120-degree sectors, k0 = 10, k = 12, 18, 9 + 0.5i,
    junctions at the centre and the outer triple points, graded elements,
    modified Calderon formulation, FP64."""
    spec = sectors([10.0, 12.0, 18.0, 9.0 + 0.5j], h=h)
    return Workload(f"sectors{spec.n_elements}_k10-12-18-9+0.5i", [spec], np.array([0.0]), 100, 1e-10)


def workload_kite16384_fp32(n: int = 16384, k1: complex = 30.0) -> Workload:
    """Precision path: the kite refined to N = 16384 (32768 x 32768 complex64
    matrix), k0 = 20, k1 = 30, 64 equispaced angles as one block, GMRES(100)
    with FP32 products inside FP64 residual refinement to 1e-8 (far field
    within 1e-6 of the FP64 solution at 360 directions)."""
    return Workload(f"kite{n}_k20-{k1:g}_x64_mixed", [kite(n, 20.0, k1)], equispaced_angles(64), 100, 1e-8,
                    precision="f32")


def request_stream(n_requests: int = 2000, rate: float = 20.0, seed: int = 0, n_range=(512, 8192),
                   k0_range=(1.0, 50.0), ratio_range=(1.2, 3.0), max_rhs: int = 32):
    """Served-path request stream: Poisson arrivals at `rate` per second,
    Fourier-perturbed circles r(t) = 1 + sum_{m=2..6} a_m cos(m t + phi_m) with
    a_m ~ U(0, 0.08), phi_m ~ U(0, 2 pi), N log-uniform in n_range, k0 ~ U(k0_range),
    k1 / k0 ~ U(ratio_range) (real), 1..max_rhs incident angles ~ U(0, 2 pi).
    One SeedSequence child per request, so request i does not depend on n_requests."""
    ss = np.random.SeedSequence(seed)
    rng_t = np.random.default_rng(ss.spawn(1)[0])
    gaps = rng_t.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    out = []
    for i, child in enumerate(ss.spawn(n_requests)):
        rng = np.random.default_rng(child)
        amps = rng.uniform(0.0, 0.08, size=5)
        phases = rng.uniform(0.0, 2 * np.pi, size=5)
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        k0 = float(rng.uniform(*k0_range))
        ratio = float(rng.uniform(*ratio_range))
        nrhs = int(rng.integers(1, max_rhs + 1))
        angles = rng.uniform(0.0, 2 * np.pi, size=nrhs)
        spec = single_material(perturbed_circle_nodes(n, amps, phases), k0, k0 * ratio,
                               name=f"req{i}")
        out.append(dict(arrival=float(t[i]), spec=spec, angles=angles))
    return out


def stream_like_request(n: int, k0: float, ratio: float, nrhs: int, seed: int):
    """One request shaped like those of request_stream (a perturbed circle
    with a_m ~ U(0, 0.08), phi_m ~ U(0, 2 pi), nrhs angles ~ U(0, 2 pi)) with
    its size and wavenumbers fixed by the caller, e.g. at the ends of the
    stream's ranges."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, 0.08, size=5)
    phases = rng.uniform(0.0, 2 * np.pi, size=5)
    angles = rng.uniform(0.0, 2 * np.pi, size=nrhs)
    spec = single_material(perturbed_circle_nodes(n, amps, phases), k0, k0 * ratio, name=f"req_n{n}_k{k0:g}")
    return dict(arrival=0.0, spec=spec, angles=angles)
