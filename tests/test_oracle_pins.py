"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test ties one part of the oracle to something other than itself: values
printed in the paper (tests/golden/paper_printed_values.json), closed forms
(Mie series, Laplace limit, Gauss exactness), library routines used as black
boxes (mpmath Hankel functions and adaptive quadrature), invariants (optical
theorem, reciprocity, translation, circulant structure) and brute force.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest

import oracle as O
import workloads as W
from closed_forms import mie_farfield, rel_err

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


# ---------------------------------------------------------------- Gauss rule
@pytest.mark.parametrize("q", [1, 2, 5, 8, 10, 16])
def test_gauss_legendre_exact_on_polynomials(q):
    """q-point Gauss-Legendre integrates x^p exactly for p <= 2q-1 (Sec. 7 rule)."""
    x, w = O.gauss_legendre(q)
    assert np.all(np.diff(x) > 0)
    assert np.allclose(x, -x[::-1], atol=1e-15)
    for p in range(2 * q):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, x ** p) - exact) < 5e-15
    # not exact one degree higher (checks it really is a q-point rule)
    p = 2 * q
    assert abs(np.dot(w, x ** p) - 2.0 / (p + 1)) > 1e-12


# ---------------------------------------------------------------- Hankel
HANKEL_POINTS = [1e-5, 1e-3, 0.05, 0.7, 1.0, 3.3, 6.0, 7.999, 8.001, 11.0, 17.5, 24.99, 25.01,
                 37.0, 90.0, 420.0, 2 + 0.4j, 7.9 + 1.0j, 8.1 + 0.2j, 14 + 0.9j, 24 + 2j, 30 + 0.3j,
                 95 + 0.95j, 0.02 + 0.01j, 4.5 + 0.25j, 1e-3j + 1e-3]
# the largest argument of a lossy wavenumber the library accepts (10 degrees), in every regime
ARG10 = complex(np.cos(np.deg2rad(10.0)), np.sin(np.deg2rad(10.0)))
HANKEL_POINTS += [r * ARG10 for r in (0.5, 5.0, 7.9, 8.1, 12.0, 24.9, 25.1, 60.0, 150.0)]


@pytest.mark.parametrize("z", HANKEL_POINTS)
def test_hankel_against_mpmath(z):
    """H0^(1), H1^(1) against mpmath at 60 digits (library used as a black box;
    the digits cover the cancellation between J and Y at Im z up to 26)."""
    mpmath.mp.dps = 60
    h0, h1 = O.hankel01(z)
    r0 = complex(mpmath.hankel1(0, z))
    r1 = complex(mpmath.hankel1(1, z))
    assert abs(h0 - r0) <= 1e-15 * abs(r0)
    assert abs(h1 - r1) <= 1e-15 * abs(r1)


def test_hankel_wronskian_real_axis():
    """J1 Y0 - J0 Y1 = 2/(pi x) for real x (J = Re H, Y = Im H)."""
    for x in np.geomspace(1e-3, 300, 57):
        h0, h1 = O.hankel01(x)
        wr = h1.real * h0.imag - h0.real * h1.imag
        assert abs(wr - 2 / (np.pi * x)) < 2e-15 * max(1.0, abs(2 / (np.pi * x))) * (1 + abs(h0) * abs(h1) * x)


def test_hankel_rejects_lower_half_plane():
    with pytest.raises(ValueError):
        O.hankel01(1.0 - 0.1j)
    with pytest.raises(ValueError):
        O.hankel01(0.0)


# ---------------------------------------------------------------- self terms
@pytest.mark.parametrize("k,h", [(1.0, 0.1), (30.0, 2.3e-3), (30 + 0.3j, 2.3e-3), (20.0, 0.05),
                                 (150.0, 0.017), (9 + 0.5j, 0.01)])
def test_self_term_S_against_adaptive_quadrature(k, h):
    """S_ii = int_{-h/2}^{h/2} (i/4) H0(k|s|) ds by mpmath's adaptive quadrature
    (endpoint log singularity handled by tanh-sinh)."""
    mpmath.mp.dps = 25
    S, _ = O.self_terms(k, h)
    ref = complex(2 * mpmath.quad(lambda s: 0.25j * mpmath.hankel1(0, k * s), [0, h / 2]))
    assert abs(S - ref) < 1e-14 * abs(ref)


def test_self_term_N_laplace_limit():
    """k -> 0: the finite part of the hypersingular self term of a flat element
    tends to the Laplace value -2/(pi h)."""
    for h in [0.1, 0.01, 1.0]:
        _, N = O.self_terms(1e-6, h)
        assert abs(N - (-2 / (np.pi * h))) < 1e-6 * 2 / (np.pi * h)


def test_self_term_N_matches_finite_part_quadrature():
    """N_ii as the Hadamard finite part.  On a flat element with x at its
    midpoint (rh.n = 0) the kernel of eq. (ddtmp) is (ik/4) H1(k|s|)/|s|; its
    finite part is int [K(s) - 1/(2 pi s^2)] ds - 2/(pi h).  The regular
    remainder is integrated by mpmath on [delta, h/2] and on [0, delta] from
    the leading terms of the ascending series of H1 (error O(delta^3))."""
    for k, h in [(2.0, 0.3), (30.0, 0.01), (5 + 0.2j, 0.2)]:
        mpmath.mp.dps = 50
        _, N = O.self_terms(k, h)
        delta = mpmath.mpf(h) * mpmath.mpf("1e-7")

        def kern(s):
            return 0.25j * k * mpmath.hankel1(1, k * s) / s - 1 / (2 * mpmath.pi * s * s)

        reg = mpmath.quad(kern, [delta, h / 2])
        tail = (1j * k * k / 8) * (delta + (2j / mpmath.pi) * delta * (mpmath.log(k * delta / 2) - 1)
                                   - (1j / mpmath.pi) * (1 - 2 * mpmath.euler) * delta)
        ref = complex(2 * (reg + tail)) - 2 / (np.pi * h)
        assert abs(N - ref) < 1e-14 * abs(ref)


# ---------------------------------------------------------------- operator entries
def _brute_entries(P, d, i, j, k):
    """Adaptive quadrature (mpmath) of the four kernels over element j seen
    from the centre of element i: the plain definition, no Gauss rule and no
    integration by parts."""
    mpmath.mp.dps = 25
    el = P.elements()
    nrm = P.normals()
    ax, ay, bx, by, cx, cy, tx, ty, h = el[j]
    xi, yi = el[i][4], el[i][5]
    nxi, nyi = nrm[i]
    nxj, nyj = nrm[j]

    def integ(which):
        def f(s):
            yx, yy = cx + s * tx, cy + s * ty
            rx, ry = xi - yx, yi - yy
            r = mpmath.sqrt(rx * rx + ry * ry)
            H0 = mpmath.hankel1(0, k * r)
            H1 = mpmath.hankel1(1, k * r)
            if which == 0:
                return 0.25j * H0
            if which == 1:
                return 0.25j * k * H1 * (rx * nxj + ry * nyj) / r
            if which == 2:
                return -0.25j * k * H1 * (rx * nxi + ry * nyi) / r
            rnx = (rx * nxi + ry * nyi) / r
            rny = (rx * nxj + ry * nyj) / r
            return 0.25j * k * (H1 * (nxi * nxj + nyi * nyj) / r + (k * H0 - 2 * H1 / r) * rnx * rny)
        return complex(mpmath.quad(f, [-h / 2, 0, h / 2]))

    return np.array([integ(w) for w in range(4)])


@pytest.mark.parametrize("form_k", [(1.0, 2.0), (20.0, 30.0 + 0.3j)])
def test_entries_against_brute_force(form_k):
    """Far and adjacent pairs on a kite: S, D, D* by 8-point Gauss and N by the
    tangential-derivative identity against adaptive quadrature of the kernels
    of eqs. (stmp)-(ddtmp) (the N kernel written out in full)."""
    k0, k1 = form_k
    P = O.Problem(W.kite(64, k0, k1))
    for d, k in [(0, k0), (1, k1)]:
        for (i, j, tol) in [(0, 32, 1e-13), (5, 20, 1e-13), (10, 11, 1e-7), (40, 38, 1e-9)]:
            got = P.operator_entries(d, i, j)
            ref = _brute_entries(P, d, i, j, k)
            scale = np.abs(ref).max()
            # S, D, D* carry the Gauss error (adjacent pairs: ~1e-8); N is exact
            # up to the Gauss error of its S part times k^2
            assert np.all(np.abs(got - ref) <= tol * scale + 1e-15), (i, j, got, ref)


# ---------------------------------------------------------------- assembled matrix
def test_circulant_structure_on_regular_polygon():
    """On the inscribed regular N-gon every block is circulant and S, D, D*
    blocks symmetric (rotation and reflection symmetry), to rounding."""
    N = 48
    P = O.Problem(W.disk(N, 1.5, 2.5))
    A = P.assemble()
    for (r0, c0) in [(0, 0), (0, N), (N, 0), (N, N)]:
        B = A[r0:r0 + N, c0:c0 + N]
        first = B[0]
        for i in range(1, N):
            assert np.allclose(B[i], np.roll(first, i), rtol=0, atol=1e-13 * np.abs(first).max())
        assert np.allclose(B, B.T, rtol=0, atol=1e-13 * np.abs(B).max())


def test_calderon_square_printed_values():
    """Sec. 4: -SN and -NS approximate I/4 on the unit square; the paper prints
    the element-wise maximum errors 5.394e-2 and 6.213e-2 (k = 1.5, 100
    elements per side).  Reproduced within 1% (the paper's own regularisation
    of N is only cited, so exact equality is not expected)."""
    g = GOLDEN["calderon_square"]
    nodes = W.square_nodes(g["per_side"], g["side"])
    P = O.Problem(W.single_material(nodes, g["k"], g["k"] * 1.5))
    n = P.N
    S = np.zeros((n, n), complex)
    Nm = np.zeros((n, n), complex)
    for i in range(n):
        for j in range(n):
            e = P.operator_entries(0, i, j)
            S[i, j] = e[0]
            Nm[i, j] = e[3]
    q = np.eye(n) / 4
    e1 = np.abs(-S @ Nm - q).max()
    e2 = np.abs(-Nm @ S - q).max()
    assert abs(e1 - g["max_abs_minus_SN_minus_quarter_I"]) < 0.01 * g["max_abs_minus_SN_minus_quarter_I"]
    assert abs(e2 - g["max_abs_minus_NS_minus_quarter_I"]) < 0.01 * g["max_abs_minus_NS_minus_quarter_I"]


def test_single_material_clusters():
    """Sec. 5 / 7.1: for N = 100, omega = 1, eps_2 = 2 the eigenvalues of
    A_{-alpha}^2 gather at alpha^2 (1 + eps_2)/4 = -3/4 (eq. (A_-alpha^2)); the
    diagonal blocks of A_1^2 at (1 - alpha eps_2)/4 and alpha (alpha - eps_2)/4
    = +-1/4 + i/2 (eq. (A_1^2)); the conventional square spreads far out."""
    g = GOLDEN["single_material_clusters"]
    k0 = g["omega"]
    k1 = g["omega"] * math.sqrt(g["eps2"])
    N = g["N"]
    A = O.Problem(W.disk(N, k0, k1, form=W.CALDERON)).assemble()
    ev = np.linalg.eigvals(A @ A)
    pred = complex(*g["beta_minus_alpha_point"])
    assert np.mean(np.abs(ev - pred) < 0.2) > 0.85
    assert np.abs(ev).max() < 3.0
    A1 = O.Problem(W.disk(N, k0, k1, form=W.CALDERON_BETA1)).assemble()
    A12 = A1 @ A1
    for blk, p in [(A12[:N, :N], complex(*g["beta1_points"][0])), (A12[N:, N:], complex(*g["beta1_points"][1]))]:
        e = np.linalg.eigvals(blk)
        assert abs(np.median(e.real) - p.real) < 0.05 and abs(np.median(e.imag) - p.imag) < 0.1
    Ac = O.Problem(W.disk(N, k0, k1, form=W.CONVENTIONAL)).assemble()
    assert np.abs(np.linalg.eigvals(Ac @ Ac)).max() > 50.0


def test_concentric_largest_eigenvalues():
    """Sec. 7.2 prints the largest-magnitude eigenvalues of A^2 for the
    concentric disks: -5.9178 + 3.9583i (modified, eq. (3dom_calderon_bie)) and
    2.1706 - 2.4538i (eq. (3dom_calderon_bie0)).  The modified one is matched to
    the printed digits; the original one to 1% (its imaginary part differs in
    the third digit, see the design notes)."""
    g = GOLDEN["concentric_largest_eigenvalues"]
    k = [g["omega"] * math.sqrt(e) for e in g["eps"]]
    for form, key, tol in [(W.CALDERON, "modified", 2e-4), (W.CALDERON_ORIG, "beta_minus_alpha_orig", 0.01)]:
        A = O.Problem(W.concentric(g["n_outer"], g["n_inner"], k, form=form)).assemble()
        ev = np.linalg.eigvals(A @ A)
        lam = ev[np.argmax(np.abs(ev))]
        ref = complex(*g[key])
        assert abs(lam - ref) < tol * abs(ref), (key, lam, ref)


# ---------------------------------------------------------------- solution
def test_mie_far_field_first_order_convergence():
    """Sec. 7.1: constant elements converge like N^-1.  Far field of the
    Calderon system (eq. (calderon_bieb), beta = -alpha) against the Mie series."""
    dirs = W.equispaced_angles(360)
    ref = mie_farfield(1.0, 2.0, 1.0, 0.0, dirs)
    errs = []
    for N in (64, 128, 256):
        P = O.Problem(W.disk(N, 1.0, 2.0))
        X = O.lu_solve(P.assemble(), P.rhs([0.0]))
        errs.append(rel_err(P.farfield(X, dirs)[:, 0], ref))
    assert errs[-1] < 2.5e-3
    for a, b in zip(errs, errs[1:]):
        assert 1.7 < a / b < 2.6


@pytest.mark.parametrize("form", [W.CALDERON, W.CALDERON_BETA1, W.CONVENTIONAL])
def test_all_forms_same_solution(form):
    """Row scaling and ordering do not change the solution (Sec. 5)."""
    dirs = W.equispaced_angles(90)
    P0 = O.Problem(W.disk(96, 3.0, 4.5 + 0.2j))
    X0 = O.lu_solve(P0.assemble(), P0.rhs([0.7]))
    P = O.Problem(W.disk(96, 3.0, 4.5 + 0.2j, form=form))
    X = O.lu_solve(P.assemble(), P.rhs([0.7]))
    assert rel_err(X, X0) < 1e-11
    assert rel_err(P.farfield(X, dirs), P0.farfield(X0, dirs)) < 1e-11


def test_optical_theorem_lossless_and_lossy():
    """Energy balance of the far field (derived from the radiation condition):
    int |F|^2 = -sqrt(8 pi/k0) Re(e^{i pi/4} F(theta_inc)) when nothing absorbs;
    with Im k1 > 0 the right side exceeds the left."""
    dirs = W.equispaced_angles(720)
    for k1, lossy in [(2.5, False), (2.5 + 0.3j, True)]:
        P = O.Problem(W.kite(192, 1.5, k1))
        th = 0.4
        X = O.lu_solve(P.assemble(), P.rhs([th]))
        F = P.farfield(X, np.concatenate([dirs, [th]]))[:, 0]
        lhs = np.sum(np.abs(F[:-1]) ** 2) * 2 * np.pi / len(dirs)
        rhs = -np.sqrt(8 * np.pi / 1.5) * (np.exp(1j * np.pi / 4) * F[-1]).real
        if lossy:
            assert rhs - lhs > 0.05 * lhs
        else:
            assert abs(lhs - rhs) < 3e-3 * lhs


def test_reciprocity():
    """F(xh; d) = F(-d; -xh) for the kite (non-symmetric scatterer); the
    discrete defect is O(h): it halves when N doubles."""
    defects = []
    for n in (96, 192):
        P = O.Problem(W.kite(n, 2.0, 3.0))
        A = P.assemble()
        a1, a2 = 0.3, 2.1
        X = O.lu_solve(A, P.rhs([a1, a2 + np.pi]))
        F12 = P.farfield(X[:, :1], [a2])[0, 0]
        F21 = P.farfield(X[:, 1:], [a1 + np.pi])[0, 0]
        defects.append(abs(F12 - F21) / abs(F12))
    assert defects[1] < 0.02
    assert 1.7 < defects[0] / defects[1] < 2.4


def test_index_matched_inclusion_scatters_nothing():
    """eps_2 = 1: the exact solution is u = u_in, F = 0; discretely F = O(h)."""
    dirs = W.equispaced_angles(60)
    P = O.Problem(W.disk(128, 2.0, 2.0))
    X = O.lu_solve(P.assemble(), P.rhs([0.0]))
    F = P.farfield(X, dirs)
    ref = mie_farfield(2.0, 3.0, 1.0, 0.0, dirs)
    assert np.abs(F).max() < 1e-2 * np.abs(ref).max()


def test_translation_multiplies_solution_by_phase():
    """Translating the scatterer by c multiplies u and w by e^{i k0 d.c}."""
    nodes = W.kite_nodes(80)
    c = np.array([0.37, -0.81])
    k0, th = 2.5, 0.9
    d = np.array([np.cos(th), np.sin(th)])
    P1 = O.Problem(W.single_material(nodes, k0, 3.3))
    P2 = O.Problem(W.single_material(nodes + c, k0, 3.3))
    X1 = O.lu_solve(P1.assemble(), P1.rhs([th]))
    X2 = O.lu_solve(P2.assemble(), P2.rhs([th]))
    assert rel_err(X2, X1 * np.exp(1j * k0 * d @ c)) < 1e-11


# ---------------------------------------------------------------- solvers
def test_lu_against_numpy_and_gmres_against_lu():
    P = O.Problem(W.kite(100, 4.0, 6.0 + 0.1j))
    A = P.assemble()
    B = P.rhs([0.0, 1.0])
    X = O.lu_solve(A, B)
    assert rel_err(X, np.linalg.solve(A, B)) < 1e-12
    cond = np.linalg.cond(A)
    for r in range(2):
        x, it, rr, ok = O.gmres(A, B[:, r], 30, 1e-12)
        assert ok and rr <= 1e-12
        assert rel_err(x, X[:, r]) < 10 * cond * 1e-12
    y = O.matvec(A, X[:, 0])
    assert rel_err(y, B[:, 0]) < 1e-12


def test_gmres_iterations_flat_for_calderon_growing_for_conventional():
    """Sec. 7.1: the iteration count of the Calderon system stays constant in N
    while the conventional one grows."""
    its = {}
    for form in (W.CALDERON, W.CONVENTIONAL):
        for N in (64, 256):
            P = O.Problem(W.disk(N, 5.0, 5.0 * math.sqrt(2.0), form=form))
            _, it, _, ok = O.gmres(P.assemble(), P.rhs([0.0])[:, 0], 2000, 1e-8, 4000)
            assert ok
            its[(form, N)] = it
    assert abs(its[(W.CALDERON, 256)] - its[(W.CALDERON, 64)]) <= 2
    assert its[(W.CONVENTIONAL, 256)] > its[(W.CONVENTIONAL, 64)] + 5
    assert its[(W.CALDERON, 256)] < its[(W.CONVENTIONAL, 256)]


def test_problem_validation():
    with pytest.raises(ValueError):
        O.Problem(W.disk(16, -1.0, 2.0))
    spec = W.disk(16, 1.0, 2.0)
    spec.interfaces[0].dom_left, spec.interfaces[0].dom_right = 0, 1
    with pytest.raises(ValueError):
        O.Problem(spec)
    spec = W.disk(16, 1.0, 2.0)
    spec.interfaces[0].xy[3] = spec.interfaces[0].xy[2]
    with pytest.raises(ValueError):
        O.Problem(spec)
