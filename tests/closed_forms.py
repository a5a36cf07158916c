"""Closed-form references used to pin the oracle (scipy / mpmath as black boxes).

Mie series for a penetrable circular cylinder (Sec. 7.1, eq. (2dom_anal)).
The paper leaves a_n, b_n to the transmission conditions (2.2)-(2.3); with
c_n = i^n e^{-i n theta_inc} the incident coefficients, x0 = k0 R, x1 = k1 R and
tau = k1 / (eps k0) = k0 / k1 for eps = (k1/k0)^2:
    a_n = -c_n [J_n'(x0) J_n(x1) - tau J_n(x0) J_n'(x1)]
              / [H_n'(x0) J_n(x1) - tau H_n(x0) J_n'(x1)],
and the far field of the scattered part with u_sc ~ e^{i k0 r}/sqrt(r) F:
    F(theta) = sqrt(2/(pi k0)) e^{-i pi/4} sum_n a_n (-i)^n e^{i n theta};
inside, b_n = (c_n J_n(x0) + a_n H_n(x0)) / J_n(x1) (continuity of u).
"""
import numpy as np
import scipy.special as sp


def mie_coefficients(k0, k1, R, theta_inc, nmax=30):
    x0, x1 = k0 * R, k1 * R
    tau = k0 / k1
    ns = np.arange(-nmax, nmax + 1)
    c = (1j ** ns) * np.exp(-1j * ns * theta_inc)
    J0, J0p = sp.jv(ns, x0), sp.jvp(ns, x0)
    H0, H0p = sp.hankel1(ns, x0), sp.h1vp(ns, x0)
    J1, J1p = sp.jv(ns, x1), sp.jvp(ns, x1)
    a = -c * (J0p * J1 - tau * J0 * J1p) / (H0p * J1 - tau * H0 * J1p)
    b = (c * J0 + a * H0) / J1
    return ns, a, b


def mie_farfield(k0, k1, R, theta_inc, dirs, nmax=30):
    ns, a, _ = mie_coefficients(k0, k1, R, theta_inc, nmax)
    dirs = np.asarray(dirs, dtype=np.float64)
    F = (a[None, :] * ((-1j) ** ns)[None, :] * np.exp(1j * np.outer(dirs, ns))).sum(axis=1)
    return np.sqrt(2.0 / (np.pi * k0)) * np.exp(-1j * np.pi / 4) * F


def layered_mie_coefficients(k, radii, theta_inc, nmax=40):
    """Concentric cylinders (Sec. 7.2): k = [k0, k_shell, k_core], radii =
    [R_outer, R_inner]; eps_d = (k_d/k0)^2.  Per order n the four unknowns
    [a_n, b_n, d_n, e_n] of
        host  : c_n J_n(k0 r) + a_n H_n(k0 r),
        shell : b_n J_n(k1 r) + d_n H_n(k1 r),
        core  : e_n J_n(k2 r),
    from continuity of u and of (1/eps) du/dr at both radii."""
    k0, k1, k2 = (complex(v) for v in k)
    R1, R2 = radii
    e1, e2 = (k1 / k0) ** 2, (k2 / k0) ** 2
    ns = np.arange(-nmax, nmax + 1)
    out = np.zeros((len(ns), 4), dtype=np.complex128)
    for i, n in enumerate(ns):
        c = (1j ** n) * np.exp(-1j * n * theta_inc)
        J, Jp, H, Hp = sp.jv, sp.jvp, sp.hankel1, sp.h1vp
        M = np.array([
            [H(n, k0 * R1), -J(n, k1 * R1), -H(n, k1 * R1), 0.0],
            [k0 * Hp(n, k0 * R1), -(k1 / e1) * Jp(n, k1 * R1), -(k1 / e1) * Hp(n, k1 * R1), 0.0],
            [0.0, J(n, k1 * R2), H(n, k1 * R2), -J(n, k2 * R2)],
            [0.0, (k1 / e1) * Jp(n, k1 * R2), (k1 / e1) * Hp(n, k1 * R2), -(k2 / e2) * Jp(n, k2 * R2)]],
            dtype=np.complex128)
        rhs = np.array([-c * J(n, k0 * R1), -c * k0 * Jp(n, k0 * R1), 0.0, 0.0], dtype=np.complex128)
        out[i] = np.linalg.solve(M, rhs)
    return ns, out


def layered_mie_farfield(k, radii, theta_inc, dirs, nmax=40):
    ns, co = layered_mie_coefficients(k, radii, theta_inc, nmax)
    k0 = float(np.real(k[0]))
    dirs = np.asarray(dirs, dtype=np.float64)
    F = (co[None, :, 0] * ((-1j) ** ns)[None, :] * np.exp(1j * np.outer(dirs, ns))).sum(axis=1)
    return np.sqrt(2.0 / (np.pi * k0)) * np.exp(-1j * np.pi / 4) * F


def mie_nearfield(k0, k1, R, theta_inc, points, nmax=50):
    """Total field of eq. (2dom_anal) at points (npts, 2): u_in + sum a_n H_n(k0 r) e^{in theta}
    outside the circle of radius R, sum b_n J_n(k1 r) e^{in theta} inside."""
    ns, a, b = mie_coefficients(k0, k1, R, theta_inc, nmax)
    pts = np.asarray(points, dtype=np.float64)
    r = np.hypot(pts[:, 0], pts[:, 1])
    th = np.arctan2(pts[:, 1], pts[:, 0])
    e = np.exp(1j * np.outer(th, ns))
    out = np.exp(1j * k0 * (np.cos(theta_inc) * pts[:, 0] + np.sin(theta_inc) * pts[:, 1])) \
        + (a[None, :] * sp.hankel1(ns[None, :], k0 * r[:, None]) * e).sum(axis=1)
    inn = (b[None, :] * sp.jv(ns[None, :], k1 * r[:, None]) * e).sum(axis=1)
    return np.where(r >= R, out, inn)


def paper_grid(m=101, half=2.99):
    """The m x m field points equally spaced in [-half, half]^2 (Sec. 7.1: 101 x 101 in [-2.99, 2.99]^2)."""
    t = np.linspace(-half, half, m)
    X, Y = np.meshgrid(t, t, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def real_part_error(num, ana):
    """Relative l2 error between the real parts (Sec. 7.1)."""
    return float(np.sqrt(np.sum(np.real(num - ana) ** 2) / np.sum(np.real(ana) ** 2)))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
