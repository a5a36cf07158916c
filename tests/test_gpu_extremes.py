"""Parity at the ends of the ranges the library is used over.

* The served stream draws k0 up to 50 and k1/k0 up to 3 (|k r| up to about
  420, about three elements per interior wavelength at N = 512).  Requests at
  the top of that range are checked against the oracle: FP64 entries (all of
  them at N = 512 and N = 1000, sampled rows at N = 8192), the FP64 solution
  and far field, and the far field the mixed-precision server returns
  (1e-6, the served path's target).
* Lossy media are accepted up to arg k = 10 degrees (the device's
  large-argument Hankel form is validated to 1.7e-12 relative there); an
  assembly at that bound is checked against the oracle.

The oracle's rows are assembled in parallel worker processes (oracle_pool);
the oracle itself is unchanged.  Tolerances:
  * entries: 1e-13 of the largest entry for real wavenumbers (both sides
    evaluate the same formulas; the phases k r differ by k times the rounding
    of r, ~3e-14 at k = 150), 4e-12 at the lossy bound (1.7e-12 per Hankel
    value, plus the same rounding);
  * FP64 solutions solved to 1e-12 against the oracle's LU solution:
    kappa * 1e-12 for the solution (reported with kappa), 1e-10 for the far
    field;
  * served mixed-precision far fields: 1e-6 (relative 2-norm over 360
    directions, per right-hand side).
"""
import numpy as np
import pytest

import oracle as O
import oracle_pool as OP
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DIRS = W.equispaced_angles(360)


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_12787_amd as P
    from paper_2312_12787_amd import serve as S
    return P, S


def _say(*a):
    print(*a, flush=True)


def _rel_rows(a, b):
    """max over rows (right-hand sides) of ||a_r - b_r|| / ||b_r||"""
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


def _served(S, P, prec, req, tol=1e-8, restart=300):
    with S.Server(24 << 30, slots=1, prec=prec, tol=tol, restart=restart, dirs=DIRS) as srv:
        srv.submit(req["spec"], req["angles"])
        (res,) = srv.drain()
    assert res.status == 0, res.message
    return res


@pytest.mark.parametrize("n_el,ratio,seed", [(512, 3.0, 21), (1000, 3.0, 22)], ids=["N512", "N1000"])
def test_stream_top_of_range_against_oracle_lu(n_el, ratio, seed):
    """k0 = 50, k1 = 150: every FP64 entry, the FP64 solution and far field
    against the oracle's LU solution, and the mixed-precision served far field."""
    P, S = _gpu()
    req = W.stream_like_request(n_el, 50.0, ratio, 4, seed)
    spec, ang = req["spec"], req["angles"]
    _say("request N", n_el, "k", spec.k, "angles", len(ang))
    g = P.Problem(spec)
    A = g.assemble(P.F64).T[:g.n].cpu().numpy()
    Ao = OP.assemble(spec)
    ea = np.abs(A - Ao).max() / np.abs(Ao).max()
    po = O.Problem(spec)
    Bo = po.rhs(ang)
    Xo = np.linalg.solve(Ao, Bo)
    kappa = np.linalg.cond(Ao)
    Fo = po.farfield(Xo, DIRS).T
    X, info = g.solve(g.rhs(ang), restart=300, tol=1e-12, max_iter=20000)
    ex = np.linalg.norm(X.cpu().numpy().T - Xo) / np.linalg.norm(Xo)
    ef = _rel_rows(g.farfield(X, DIRS).cpu().numpy(), Fo)
    _say("  entries", ea, "kappa", kappa, "FP64 iters", info.iters.tolist(), "solution", ex, "far field", ef)
    assert ea < 1e-13
    assert info.converged.all() and ex < max(1e-10, kappa * 1e-12) and ef < 1e-10
    res = _served(S, P, P.MIXED, req)
    em = _rel_rows(res.far_field, Fo)
    _say("  served mixed: iters", res.iters_max, "refinement steps", res.refine_max, "far field", em)
    assert em < 1e-6


def test_stream_largest_request_sampled_oracle_rows():
    """N = 8192 (16384 x 16384), k0 = 50, k1 = 150: sampled FP64 rows (first,
    last and ragged tiles of both equation blocks) against the oracle's; the
    FP64 solution's residual on those oracle rows; the mixed-precision served
    far field against the FP64 one."""
    P, S = _gpu()
    req = W.stream_like_request(8192, 50.0, 3.0, 2, 23)
    spec, ang = req["spec"], req["angles"]
    g = P.Problem(spec)
    n = g.n
    A_t = g.assemble(P.F64)
    rows = np.array([0, 1, 255, 256, 4097, 8191, 8192, 8193, 12000, 16127, 16128, 16383], dtype=np.int32)
    Ao = OP.assemble_rows(spec, rows)
    Ag = A_t[:, torch.as_tensor(rows, device=A_t.device).long()].T.cpu().numpy()
    ea = np.abs(Ag - Ao).max() / np.abs(Ao).max()
    X, info = g.solve(g.rhs(ang), restart=300, tol=1e-12, max_iter=20000)
    F64 = g.farfield(X, DIRS).cpu().numpy()
    Bo = O.Problem(spec).rhs(ang)
    res = Bo[rows] - Ao @ X.cpu().numpy().T
    rms_b = np.linalg.norm(Bo, axis=0) / np.sqrt(n)
    rr = float(np.max(np.abs(res) / rms_b))
    _say("N 8192 k0 50 k1 150: sampled entries", ea, "FP64 iters", info.iters.tolist(),
         "residual on oracle rows / rms(b)", rr)
    assert ea < 1e-13
    # tol 1e-12 bounds the rms of the residual rows by 1e-12 rms(b); the
    # matrices differ by < 1e-13 of the largest entry
    assert info.converged.all() and rr < 2e-10
    del A_t
    g.A = None
    torch.cuda.empty_cache()
    res_m = _served(S, P, P.MIXED, req)
    em = _rel_rows(res_m.far_field, F64)
    _say("  served mixed: iters", res_m.iters_max, "refinement steps", res_m.refine_max, "far field vs FP64", em)
    assert em < 1e-6


def test_lossy_bound_assembly_and_solve():
    """arg k1 just below 10 degrees (the largest the library accepts): entries
    against the oracle within the validated accuracy of the large-argument
    Hankel form there, and the solution against the oracle's LU solution."""
    P, _ = _gpu()
    t10 = np.tan(np.deg2rad(10.0))
    spec = W.kite(300, 20.0, 30.0 * (1.0 + 0.9999 * t10 * 1j))
    g = P.Problem(spec)
    A = g.assemble(P.F64).T[:g.n].cpu().numpy()
    Ao = OP.assemble(spec)
    ea = np.abs(A - Ao).max() / np.abs(Ao).max()
    po = O.Problem(spec)
    ang = [0.0, 1.3]
    Xo = np.linalg.solve(Ao, po.rhs(ang))
    kappa = np.linalg.cond(Ao)
    X, info = g.solve(g.rhs(ang), restart=200, tol=1e-12)
    ex = np.linalg.norm(X.cpu().numpy().T - Xo) / np.linalg.norm(Xo)
    ef = _rel_rows(g.farfield(X, DIRS).cpu().numpy(), po.farfield(Xo, DIRS).T)
    _say("arg k1 = 10 deg: entries", ea, "kappa", kappa, "solution", ex, "far field", ef)
    assert ea < 4e-12
    assert info.converged.all() and ex < max(1e-10, kappa * 4e-12) and ef < 1e-10
