#!/usr/bin/env python3
"""Paper-reproduction sweeps on the GPU path (Sec. 7): GMRES iteration counts
of the conventional and the Calderon-preconditioned formulations against the
number of elements N, the angular frequency omega and the material constants.

Experiments (Sec. 7; omega = k0, k_d = omega sqrt(eps_d), eps_1 = 1):
  single_N      unit disk (inscribed N-gon), omega = 5, eps2 = 2, N = 100 .. 1600   (Sec. 7.1, iterations vs N)
  single_omega  unit disk, N = 600, eps2 = 2, omega sweep                          (Sec. 7.1, left of the omega / eps figure)
  single_eps    unit disk, N = 600, omega = 5, eps2 sweep                          (Sec. 7.1, right)
  conc_N        concentric disks (radii 2 and 1, eps = 1, 2, 3), omega = 1, 2N/3 + N/3 elements  (Sec. 7.2)
  conc_omega    concentric disks, 1200 + 600 elements, eps = 1, 2, 3, omega sweep
  conc_eps      concentric disks, 1200 + 600 elements, omega = 5, eps2 = 1/eps3, 0 < eps3 <= 10
  split_N       disk split by its vertical diameter (two triple points), 3N/4 + N/4 elements, omega = 1
  split_omega   split disk, N = 1066, eps = 1, 2, 3, omega sweep
  split_eps     split disk, N = 1066, omega = 5, eps2 = 1/eps3 sweep
  spectra       eigenvalues of A^2 (Sec. 5 and 7.2): unit disk, N = 100, omega = 1,
                eps2 = 2 (beta = -alpha, beta = 1, conventional); concentric disks,
                200 + 100 elements, omega = 1 (modified, original, conventional)

Single material: conventional (eq. (naive_bie)), Calderon beta = 1
(eq. (calderon_bie1)) and beta = -alpha (eq. (calderon_bieb)).  Several
materials: conventional (eq. (3dom_conv_bie)), original (eq.
(3dom_calderon_bie0)) and modified (eq. (3dom_calderon_bie)).  GMRES from
x0 = 0 to a relative residual of 1e-8, incident angle 0, without restart up to
1990 Krylov vectors (the library's largest restart length, BEM_MAX_RESTART; a
longer run restarts), at most 5000 steps (more: reported as None), FP64.

Usage: python sweeps.py [--exp NAME ...] [--quick]   (one JSON line per experiment)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SINGLE_FORMS = {"conventional": 2, "calderon_beta1": 1, "calderon_beta_minus_alpha": 0}
MULTI_FORMS = {"conventional": 2, "calderon_orig": 3, "calderon_mod": 0}


def iterations(spec, tol=1e-8, max_iter=5000):
    """GMRES iterations of one FP64 solve on the GPU (incident angle 0); a
    solve still above tol after max_iter steps is reported as None."""
    import paper_2312_12787_amd as P
    g = P.Problem(spec)
    g.assemble(P.F64)
    B = g.rhs([0.0])
    X, info = g.solve(B, restart=min(g.n, P.MAX_RESTART), tol=tol, max_iter=max_iter)
    return int(info.iters[0]), bool(info.converged[0])


def _sweep(name, values, make, forms, label):
    rows = []
    t0 = time.perf_counter()
    for v in values:
        row = {label: v}
        for fname, form in forms.items():
            it, ok = iterations(make(v, form))
            row[fname] = it if ok else None
        rows.append(row)
        print(f"{name}: {row}", file=sys.stderr, flush=True)
    return {"experiment": name, "parameter": label, "rows": rows, "seconds": time.perf_counter() - t0}


def single_N(Ns=(100, 200, 400, 800, 1600), omega=5.0, eps2=2.0):
    import workloads as W
    return _sweep("single_N", Ns, lambda n, f: W.disk(n, omega, omega * np.sqrt(eps2), form=f), SINGLE_FORMS, "N")


def single_omega(omegas=tuple(np.arange(1.0, 10.5, 0.5)), N=600, eps2=2.0):
    import workloads as W
    return _sweep("single_omega", omegas, lambda w, f: W.disk(N, w, w * np.sqrt(eps2), form=f), SINGLE_FORMS,
                  "omega")


def single_eps(eps=tuple(np.arange(1.5, 10.5, 0.5)), N=600, omega=5.0):
    import workloads as W
    return _sweep("single_eps", eps, lambda e, f: W.disk(N, omega, omega * np.sqrt(e), form=f), SINGLE_FORMS,
                  "eps2")


def _conc(n_total, omega, eps2, eps3, form):
    import workloads as W
    k = [omega, omega * np.sqrt(eps2), omega * np.sqrt(eps3)]
    return W.concentric(2 * n_total // 3, n_total // 3, k, form=form)


def conc_N(Ns=(150, 300, 600, 1200), omega=1.0):
    return _sweep("conc_N", Ns, lambda n, f: _conc(n, omega, 2.0, 3.0, f), MULTI_FORMS, "N")


def conc_omega(omegas=tuple(np.arange(1.0, 10.5, 1.0)), N=1800):
    return _sweep("conc_omega", omegas, lambda w, f: _conc(N, w, 2.0, 3.0, f), MULTI_FORMS, "omega")


def conc_eps(eps3=(0.25, 0.5, 1.5, 2.0, 4.0, 6.0, 8.0, 10.0), N=1800, omega=5.0):
    return _sweep("conc_eps", eps3, lambda e, f: _conc(N, omega, 1.0 / e, e, f), MULTI_FORMS, "eps3")


def _split(n, omega, eps2, eps3, form):
    import workloads as W
    return W.split_disk(n, [omega, omega * np.sqrt(eps2), omega * np.sqrt(eps3)], form=form)


def split_N(Ns=(200, 400, 800, 1600), omega=1.0):
    return _sweep("split_N", Ns, lambda n, f: _split(n, omega, 2.0, 3.0, f), MULTI_FORMS, "N")


def split_omega(omegas=tuple(np.arange(1.0, 10.5, 1.0)), N=1066):
    return _sweep("split_omega", omegas, lambda w, f: _split(N, w, 2.0, 3.0, f), MULTI_FORMS, "omega")


def split_eps(eps3=(0.25, 0.5, 1.5, 2.0, 4.0, 6.0, 8.0, 10.0), N=1066, omega=5.0):
    return _sweep("split_eps", eps3, lambda e, f: _split(N, omega, 1.0 / e, e, f), MULTI_FORMS, "eps3")


def _gpu_matrix(spec):
    """The matrix assembled on the GPU (FP64), as a numpy (n, n) array."""
    import paper_2312_12787_amd as P
    g = P.Problem(spec)
    A = g.assemble(P.F64)
    return A.T.cpu().numpy()


def spectra(N=100, n_outer=200, n_inner=100, omega=1.0):
    """Eigenvalues of A^2 of GPU-assembled matrices (numpy.linalg.eigvals on
    the host): per form, the largest magnitude, the spread, and for the
    single-material beta = -alpha form the share within 0.2 of its predicted
    accumulation point alpha^2 (1 + eps2)/4 = -3/4 (eq. (A_-alpha^2))."""
    import workloads as W
    t0 = time.perf_counter()
    rows = []
    eps2 = 2.0
    alpha = -1j / omega
    single = {"calderon_beta_minus_alpha": W.CALDERON, "calderon_beta1": W.CALDERON_BETA1,
              "conventional": W.CONVENTIONAL}
    for name, form in single.items():
        A = _gpu_matrix(W.disk(N, omega, omega * np.sqrt(eps2), form=form))
        ev = np.linalg.eigvals(A @ A)
        row = {"case": "single", "form": name, "n": A.shape[0], "max_abs": float(np.abs(ev).max()),
               "largest": [float(ev[np.argmax(np.abs(ev))].real), float(ev[np.argmax(np.abs(ev))].imag)]}
        if form == W.CALDERON:
            pred = alpha ** 2 * (1 + eps2) / 4
            row["share_within_0.2_of_pred"] = float(np.mean(np.abs(ev - pred) < 0.2))
            row["predicted_point"] = [pred.real, pred.imag]
        rows.append(row)
        print(f"spectra: {row}", file=sys.stderr, flush=True)
    k = [omega, omega * np.sqrt(2.0), omega * np.sqrt(3.0)]
    multi = {"modified": W.CALDERON, "original": W.CALDERON_ORIG, "conventional": W.CONVENTIONAL}
    for name, form in multi.items():
        A = _gpu_matrix(W.concentric(n_outer, n_inner, k, form=form))
        ev = np.linalg.eigvals(A @ A)
        lam = ev[np.argmax(np.abs(ev))]
        row = {"case": "concentric", "form": name, "n": A.shape[0], "max_abs": float(np.abs(ev).max()),
               "largest": [float(lam.real), float(lam.imag)], "min_abs": float(np.abs(ev).min())}
        rows.append(row)
        print(f"spectra: {row}", file=sys.stderr, flush=True)
    return {"experiment": "spectra", "parameter": "form", "rows": rows, "seconds": time.perf_counter() - t0}


EXPERIMENTS = {f.__name__: f for f in (single_N, single_omega, single_eps, conc_N, conc_omega, conc_eps, split_N,
                                       split_omega, split_eps, spectra)}
QUICK = {"single_N": dict(Ns=(100, 200, 400, 800)), "single_omega": dict(omegas=(1.0, 3.0, 5.0, 7.0, 9.0)),
         "single_eps": dict(eps=(2.0, 4.0, 8.0)), "conc_N": dict(Ns=(150, 300, 600)),
         "conc_omega": dict(omegas=(2.0, 5.0, 8.0)), "conc_eps": dict(eps3=(0.5, 2.0, 8.0)),
         "split_N": dict(Ns=(200, 400, 800)), "split_omega": dict(omegas=(2.0, 5.0, 8.0)),
         "split_eps": dict(eps3=(0.5, 2.0, 8.0)), "spectra": {}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--exp", nargs="*", default=list(EXPERIMENTS), choices=list(EXPERIMENTS))
    ap.add_argument("--quick", action="store_true", help="a few points per sweep")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    for name in args.exp:
        res = EXPERIMENTS[name](**(QUICK[name] if args.quick else {}))
        print(json.dumps(res, default=float), flush=True)


if __name__ == "__main__":
    main()
