"""The allocation-free product bem_matvec_noalloc (its partial sums in the
library's own device scratch) against bem_matvec (partial sums in a caller
workspace), called through the C ABI.

Same kernels, launch shapes and summation order, so the products are
bit-identical (the bar is the one of the workspace product itself).  Two
calls in a row, the second on a smaller input (fewer rows and right-hand
sides, a different kernel) that reuses the scratch the first left behind;
an FP32 matrix; and the size limit, refused from the host."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_12787_amd as P
    return P


def _x(nrhs, n, seed, dtype):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.complex(torch.randn(nrhs, n, generator=g, dtype=torch.float64),
                      torch.randn(nrhs, n, generator=g, dtype=torch.float64))
    return X.to(dtype).cuda()


def _noalloc(P, g, X):
    Y = torch.full_like(X, complex(3.0, -3.0))
    st = P.lib().bem_matvec_noalloc(g._h, X.shape[0], C.c_void_p(X.data_ptr()), X.shape[1], C.c_void_p(Y.data_ptr()),
                                    Y.shape[1], C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, Y


def test_noalloc_product_equals_workspace_product_two_calls_in_a_row():
    P = _gpu()
    cases = [(W.kite(1200, 8.0, 12.0), 16, "F64"),   # matrix-core product, n = 2400
             (W.disk(300, 2.0, 3.0 + 0.1j), 3, "F64"),  # vector product, smaller n and nrhs
             (W.kite(700, 6.0, 9.0), 20, "F32"),        # FP32 matrix, two groups of 16
             (W.disk(130, 1.0, 2.0), 1, "F32")]
    for spec, nrhs, prec in cases:
        g = P.Problem(spec)
        g.assemble(getattr(P, prec))
        dt = torch.complex128 if prec == "F64" else torch.complex64
        X = _x(nrhs, g.n, g.n + nrhs, dt)
        st, Y = _noalloc(P, g, X)
        assert P.STATUS[st] == "BEM_OK", P.lib().bem_last_error().decode()
        Yr = g.matvec(X)
        torch.cuda.synchronize()
        d = float((Y - Yr).abs().max())
        print(spec.name, prec, "n", g.n, "nrhs", nrhs, "max |Y_noalloc - Y_matvec|", d, flush=True)
        assert torch.equal(Y, Yr)


def test_noalloc_product_refuses_more_than_its_scratch():
    P = _gpu()
    g = P.Problem(W.kite(2048, 8.0, 12.0))
    g.assemble(P.F64)
    X = _x(64, g.n, 5, torch.complex128)
    st, Y = _noalloc(P, g, X)
    msg = P.lib().bem_last_error().decode()
    print(P.STATUS[st], msg, flush=True)
    assert P.STATUS[st] == "BEM_E_ARG" and "scratch" in msg
    assert bool((Y == complex(3.0, -3.0)).all())  # nothing written
    st, Y = _noalloc(P, g, X[:8])  # a smaller product on the same problem still runs
    assert P.STATUS[st] == "BEM_OK"
    assert torch.equal(Y, g.matvec(X[:8]))
