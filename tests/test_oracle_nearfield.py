"""Pins of the oracle's near field (Sec. 7.1: the total field at field
points), independent of its own arithmetic:
  * the paper's error measure against the Mie series (eq. (2dom_anal)) falls
    like N^-1 on the disk at omega = 5, eps2 = 2;
  * extinction: each domain's representation formula vanishes outside that
    domain (the host's at interior points, the inclusion's at exterior ones);
  * element integrals at points close to an element (down to 1e-6 of its
    length) against 30-digit adaptive quadrature (mpmath);
  * far from the scatterer the near field tends to the far field.
"""
import mpmath
import numpy as np

import oracle as O
import workloads as W
from closed_forms import mie_nearfield, paper_grid, real_part_error

K0, K1 = 5.0, 5.0 * np.sqrt(2.0)  # omega = 5, eps2 = 2 (Sec. 7.1)


def _solve(spec, ang):
    po = O.Problem(spec)
    X = np.linalg.solve(po.assemble(), po.rhs(ang))
    return po, X


def _disk_domains(pts):
    return (np.hypot(pts[:, 0], pts[:, 1]) < 1.0).astype(np.int32)


def test_nearfield_error_against_mie_falls_like_one_over_n():
    pts = paper_grid(11)
    dom = _disk_domains(pts)
    ua = mie_nearfield(K0, K1, 1.0, 0.0, pts)
    errs = []
    for n in (64, 128, 256):
        po, X = _solve(W.disk(n, K0, K1), [0.0])
        U = po.nearfield(X, pts, dom, angles=[0.0])[:, 0]
        errs.append(real_part_error(U, ua))
    print("near-field error vs Mie", errs)
    assert errs[2] < 2e-2
    for a, b in zip(errs, errs[1:]):
        assert 1.6 < a / b < 2.6


def test_extinction_of_each_representation_outside_its_domain():
    """Green's formula of the host medium is zero inside the scatterer (with the
    incident wave included) and the inclusion's is zero outside: O(h) for the
    discrete solution, halving when N doubles."""
    inside = np.array([[0.1, 0.2], [-0.4, 0.3], [0.5, -0.5], [0.0, -0.8]])
    outside = np.array([[1.5, 0.2], [-2.0, 1.0], [0.3, -1.7], [1.2, 1.2]])
    res = []
    for n in (128, 256):
        po, X = _solve(W.disk(n, K0, K1), [0.7])
        host_at_inside = po.nearfield(X, inside, np.zeros(len(inside), np.int32), angles=[0.7])[:, 0]
        incl_at_outside = po.nearfield(X, outside, np.ones(len(outside), np.int32))[:, 0]
        res.append((np.abs(host_at_inside).max(), np.abs(incl_at_outside).max()))
    print("extinction residuals", res)
    assert res[1][0] < 2e-2 and res[1][1] < 2e-2
    assert res[0][0] / res[1][0] > 1.6 and res[0][1] / res[1][1] > 1.6


def test_close_point_element_integrals_against_mpmath():
    """S_j(x) and D_j(x) for points at distances 1e-6 h .. 0.3 h from element j
    (above its middle and near an end node), read through the near field with
    unit boundary data on that element, against mpmath quadrature split at the
    foot of the perpendicular."""
    mpmath.mp.dps = 30
    spec = W.disk(16, 3.0, 4.0)
    po = O.Problem(spec)
    el = po.elements()  # per element: ax ay bx by cx cy tx ty h
    j = 5
    ax, ay, _, _, _, _, tx, ty, h = el[j]
    nx, ny = -ty, tx  # left normal
    k = 3.0
    for along, dist in [(0.5, 1e-6), (0.5, 1e-3), (0.3, 0.05), (0.02, 1e-4), (-0.01, 2e-3), (0.97, 0.3)]:
        side = -1.0  # outward side of the circle: the host medium, where the normal points away
        x = ax + along * h * tx + side * dist * h * nx
        y = ay + along * h * ty + side * dist * h * ny
        for col in ("w", "u"):
            X = np.zeros((po.n, 1), dtype=np.complex128)
            X[j if col == "u" else po.N + j, 0] = 1.0
            got = po.nearfield(X, [[x, y]], [0])[0, 0]

            def kern(s):
                yx, yy = ax + s * tx, ay + s * ty
                rx, ry = x - yx, y - yy
                r = mpmath.sqrt(rx * rx + ry * ry)
                if col == "w":
                    return 0.25j * mpmath.hankel1(0, k * r)
                return -(0.25j * k * mpmath.hankel1(1, k * r) * (rx * nx + ry * ny) / r)

            foot = min(max(along * h, 0.0), h)
            pts = [0.0, foot, h] if 0.0 < foot < h else [0.0, h]
            ref = complex(mpmath.quad(kern, pts))
            print(col, along, dist, got, ref)
            assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-3)


def test_nearfield_tends_to_the_far_field():
    po, X = _solve(W.kite(120, 4.0, 6.0), [0.3])
    dirs = np.array([0.0, 1.0, 2.5, 4.0])
    F = po.farfield(X, dirs)[:, 0]
    gaps = []
    for R in (200.0, 400.0):
        pts = R * np.stack([np.cos(dirs), np.sin(dirs)], axis=1)
        U = po.nearfield(X, pts, np.zeros(len(dirs), np.int32))[:, 0]
        approx = np.exp(1j * 4.0 * R) / np.sqrt(R) * F
        gaps.append(np.abs(U - approx).max() / np.abs(approx).max())
    print("near vs far field gaps", gaps)
    assert gaps[1] < 5e-3 and 1.6 < gaps[0] / gaps[1] < 2.4
