"""Oracle pins for several materials with junction points (Sec. 6 recipe,
Sec. 7.2): a disk cut into three 120-degree sectors meeting at the centre and
at three triple points on the circle."""
import numpy as np

import oracle as O
import workloads as W
from closed_forms import mie_farfield, rel_err


def _solve(spec, angles):
    P = O.Problem(spec)
    X = O.lu_solve(P.assemble(), P.rhs(angles))
    return P, X


def test_equal_sectors_reproduce_the_single_disk_mie_series():
    """Three sectors of one material (k = 3) inside k0 = 2: the radii carry no
    jump, so the far field is the Mie series of the homogeneous disk, to O(h);
    halving h halves the error."""
    dirs = W.equispaced_angles(120)
    ref = mie_farfield(2.0, 3.0, 1.0, 0.0, dirs)
    errs = []
    for h in (1 / 24, 1 / 48):
        P, X = _solve(W.sectors([2.0, 3.0, 3.0, 3.0], h=h, graded=False), [0.0])
        errs.append(rel_err(P.farfield(X, dirs)[:, 0], ref))
    assert errs[1] < 1.5e-2
    assert 1.6 < errs[0] / errs[1] < 2.6


def test_index_matched_sectors_are_invisible():
    dirs = W.equispaced_angles(60)
    P, X = _solve(W.sectors([2.0, 2.0, 2.0, 2.0], h=1 / 30), [0.4])
    F = P.farfield(X, dirs)
    scale = np.abs(mie_farfield(2.0, 3.0, 1.0, 0.0, dirs)).max()
    assert np.abs(F).max() < 5e-3 * scale


def test_sectors_optical_theorem_and_formulations():
    """Lossless sectors: energy balance of the far field to O(h).  The
    conventional form (eq. (3dom_conv_bie)) and the original Calderon form
    (eq. (3dom_calderon_bie0)) hold the same equations in another order and
    scaling, so their solutions agree to rounding; the modified form (eq.
    (3dom_calderon_bie)) replaces interior equations by Burton-Miller ones
    (Sec. 7.2), so its far field agrees to O(h): the gap halves with h."""
    dirs = W.equispaced_angles(360)
    th = 0.7
    k = [2.0, 2.6, 3.4, 2.2]
    gaps = []
    for h in (1 / 15, 1 / 30):
        sols = {}
        for form in (W.CALDERON, W.CALDERON_ORIG, W.CONVENTIONAL):
            P, X = _solve(W.sectors(k, h=h, form=form), [th])
            sols[form] = (P, X)
        assert rel_err(sols[W.CONVENTIONAL][1], sols[W.CALDERON_ORIG][1]) < 1e-10
        Fm = sols[W.CALDERON][0].farfield(sols[W.CALDERON][1], dirs)
        Fo = sols[W.CALDERON_ORIG][0].farfield(sols[W.CALDERON_ORIG][1], dirs)
        gaps.append(rel_err(Fm, Fo))
    assert gaps[1] < 5e-3 and 1.7 < gaps[0] / gaps[1] < 3.0
    P, X = sols[W.CALDERON]
    F = P.farfield(X, np.concatenate([dirs, [th]]))[:, 0]
    lhs = np.sum(np.abs(F[:-1]) ** 2) * 2 * np.pi / len(dirs)
    rhs = -np.sqrt(8 * np.pi / k[0]) * (np.exp(1j * np.pi / 4) * F[-1]).real
    assert abs(lhs - rhs) < 2e-2 * lhs


def test_sectors_geometry_and_junctions():
    spec = W.sectors([10.0, 12.0, 18.0, 9.0 + 0.5j])
    assert 7000 < spec.n_elements < 8200
    P = O.Problem(W.sectors([10.0, 12.0, 18.0, 9.0 + 0.5j], h=1 / 20))
    el = P.elements()
    h = el[:, 8]
    # graded toward the junctions: shortest element h/16, neighbour ratio <= 1.5 (+ rounding)
    assert abs(h.min() - (1 / 20) / 16) < 1e-6 * (1 / 20) / 16  # chords of the arcs are a hair shorter
    for f in W.sectors([1.0, 2.0, 3.0, 4.0], h=1 / 20).interfaces:
        d = np.hypot(*np.diff(f.xy, axis=0).T)
        assert np.max(np.maximum(d[1:] / d[:-1], d[:-1] / d[1:])) < 1.5 + 1e-6


def test_concentric_disks_converge_to_the_layered_cylinder_series():
    """Sec. 7.2 geometry (radii 2 and 1, eps = 1, 2, 3 at omega = 1.5): the far
    field of every formulation converges to the concentric-cylinder series
    (solved per order from the transmission conditions at both radii) like
    N^-1, and the formulations agree with each other to O(h)."""
    from closed_forms import layered_mie_farfield
    w = 1.5
    k = [w, w * np.sqrt(2.0), w * np.sqrt(3.0)]
    dirs = W.equispaced_angles(36)
    Fa = layered_mie_farfield(k, [2.0, 1.0], 0.0, dirs)
    for form in (W.CALDERON, W.CALDERON_ORIG, W.CONVENTIONAL):
        errs = []
        for n in (40, 80, 160):
            po = O.Problem(W.concentric(2 * n, n, k, form=form))
            X = np.linalg.solve(po.assemble(), po.rhs([0.0]))
            errs.append(rel_err(po.farfield(X, dirs)[:, 0], Fa))
        print("form", form, "far-field error vs layered series", errs)
        assert errs[-1] < 8e-3
        for a, b in zip(errs, errs[1:]):
            assert 1.6 < a / b < 2.6


def test_split_disk_geometry_and_equal_halves():
    """Disk split by a vertical diameter (junction example of Sec. 7.2): with
    both halves of the same material it is the one-disk problem again
    (far field against the Mie series, O(h))."""
    k0, k1 = 2.0, 3.0
    spec = W.split_disk(200, [k0, k1, k1])
    assert spec.n_elements == 200
    el = O.Problem(spec).elements()
    assert np.allclose(np.hypot(el[:150, 4], el[:150, 5]), 1.0, atol=1e-3)  # arc midpoints
    assert np.allclose(el[150:, 4], 0.0)                                     # diameter midpoints
    dirs = W.equispaced_angles(24)
    po = O.Problem(spec)
    X = np.linalg.solve(po.assemble(), po.rhs([0.3]))
    err = rel_err(po.farfield(X, dirs)[:, 0], mie_farfield(k0, k1, 1.0, 0.3, dirs))
    print("split disk with equal halves: far-field error vs Mie", err)
    assert err < 1e-2
