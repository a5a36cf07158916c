"""Launch-shape autotuning of the solve's products (bem_tune) on the GPU.

* The chosen shape is the fastest timed (never slower than the built-in one
  in the same run) and is what later products of its class run with.
* Products with the tuned shape equal those with the built-in shape to
  rounding (only the column-split summation order differs): 1e-13 relative.
* Solves after tuning still match the oracle's FP64 LU solution: 1e-10 for
  the FP64 path, 1e-6 for the mixed path (the targets of the untuned path).
* The vector kernel (up to 4 right-hand sides) is tuned as its own class.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_12787_amd as P
    P.tune_reset()
    return P


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _x(nrhs, n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.complex(torch.randn(nrhs, n, generator=g, dtype=torch.float64),
                         torch.randn(nrhs, n, generator=g, dtype=torch.float64)).cuda()


@pytest.mark.parametrize("nrhs", [16, 40, 2])
def test_tuned_products_equal_builtin_products(nrhs):
    P = _gpu()
    try:
        g = P.Problem(W.kite(1500, 8.0, 12.0))
        g.assemble(P.F64)
        X = _x(nrhs, g.n, 7)
        Y0 = g.matvec(X).cpu().numpy()
        info = g.tune(nrhs, reps=2)
        print("tuned", nrhs, info, flush=True)
        assert info["candidates"] >= 2 and info["best_ms"] <= info["default_ms"]
        table = P.tune_export().strip().splitlines()[1:]
        assert len(table) == 1
        t = [int(v) for v in table[0].split()]
        assert t[:2] == [3, 0 if nrhs <= 4 else (min(nrhs, 64) + 15) // 16]
        assert t[3:] == [info["rt"], info["u"], info["splits"], info["g3"]]
        Y1 = g.matvec(X).cpu().numpy()
        assert _rel(Y1, Y0) < 1e-13
    finally:
        P.tune_reset()


def test_solves_after_tuning_match_the_oracle():
    P = _gpu()
    try:
        spec = W.kite(400, 6.0, 9.0 + 0.2j)
        ang = W.equispaced_angles(16)
        po = O.Problem(spec)
        Xo = np.linalg.solve(po.assemble(), po.rhs(ang)).T
        g = P.Problem(spec)
        g.assemble(P.F64)
        print("FP64", g.tune(16, reps=2), flush=True)
        X, info = g.solve(g.rhs(ang), restart=60, tol=1e-12)
        assert info.converged.all()
        e64 = _rel(X.cpu().numpy(), Xo)
        g.assemble(P.MIXED)
        print("mixed", g.tune(16, reps=2), flush=True)
        Xm, infom = g.solve(g.rhs(ang), restart=60, tol=1e-8, inner_tol=1e-4, max_refine=20)
        assert infom.converged.all()
        em = _rel(Xm.cpu().numpy(), Xo)
        print("error vs oracle: FP64", e64, "mixed", em, flush=True)
        assert e64 < 1e-10 and em < 1e-6
    finally:
        P.tune_reset()


@pytest.mark.parametrize("nrhs", [64, 3])
def test_tuned_fp32_products_equal_builtin_products(nrhs):
    """FP32 matrix: the class of FP32 products (FP32 matrix and sums) is tuned
    by bem_tune on the solve's product (FP64 vectors) and then used by
    bem_matvec's FP32 products as well; only the split-K summation order
    changes, so the products agree to FP32 rounding (1e-5 relative in the
    2-norm, entries of both signs)."""
    P = _gpu()
    try:
        g = P.Problem(W.kite(1500, 8.0, 12.0))
        g.assemble(P.F32)
        X = _x(nrhs, g.n, 11).to(torch.complex64)
        Y0 = g.matvec(X).cpu().numpy().astype(np.complex128)
        info = g.tune(nrhs, reps=2)
        print("tuned FP32", nrhs, info, flush=True)
        t = [int(v) for v in P.tune_export().strip().splitlines()[1].split()]
        assert t[0] == 0 and t[3:] == [info["rt"], info["u"], info["splits"], info["g3"]]
        Y1 = g.matvec(X).cpu().numpy().astype(np.complex128)
        assert _rel(Y1, Y0) < 1e-5
    finally:
        P.tune_reset()
