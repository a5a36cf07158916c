"""Graph-captured Krylov steps (bem_solve_opts.graph_steps) on the GPU.

The captured segments hold the same kernels, with the same arguments and in
the same order, as the kernel-by-kernel solve, and every reduction of the path
has a fixed order: the solution must be bit-identical and the iteration
counts equal, whatever the segment length.  The extra products the host
enqueues past the last stop only touch scratch vectors.

* Several solves in a row replay the captured segments, with eager work of
  the program in between; every replay equals the eager solve.
* Restarted solves replay the segments in every cycle.
* A change of restart length, matrix precision, matrix buffer or tuned
  product shapes captures again, and the result equals the eager solve of the
  new configuration.
* The mixed path (FP32 products, FP64 refinement) and the request server
  give the same results with and without graphs.
"""
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


def _angles(nrhs):
    return [2 * np.pi * r / nrhs for r in range(nrhs)]


def _same(P, g, B, restart, steps, X0, info0, tol=1e-10, reps=2):
    """Solve `reps` times with graphs of `steps` steps, with an eager product
    between the calls, and compare each result with the eager solve."""
    for rep in range(reps):
        X, info = g.solve(B, restart=restart, tol=tol, graph_steps=steps)
        torch.cuda.synchronize()
        print(f"  graph_steps={steps} rep={rep} iters={info.iters.tolist()}", flush=True)
        assert np.array_equal(info.iters, info0.iters), (info.iters, info0.iters)
        assert np.array_equal(info.converged, info0.converged)
        assert torch.equal(X, X0), float((X - X0).abs().max())
        g.matvec(X0 if g.prec != P.F32 else X0.to(torch.complex64))  # eager work between replays


CASES = [
    ("disk256", lambda: W.disk(256, 1.0, 2.0), "F64", 1, 50, (1, 4, 16)),
    ("kite600_restarted", lambda: W.kite(600, 8.0, 12.0), "F64", 3, 20, (4, 7)),
    ("kite600_block16", lambda: W.kite(600, 8.0, 12.0), "F64", 16, 30, (8,)),
    ("kite600_mixed", lambda: W.kite(600, 8.0, 12.0), "MIXED", 5, 25, (4, 16)),
    ("disk300_f32", lambda: W.disk(300, 3.0, 4.5), "F32", 2, 40, (5,)),
]


@pytest.mark.parametrize("name,spec,prec,nrhs,restart,steps", CASES, ids=[c[0] for c in CASES])
def test_graph_solves_equal_kernel_by_kernel_solves(name, spec, prec, nrhs, restart, steps):
    P = _gpu()
    print(f"case {name}: prec {prec} nrhs {nrhs} restart {restart} steps {steps}", flush=True)
    g = P.Problem(spec())
    g.assemble(getattr(P, prec))
    B = g.rhs(_angles(nrhs))
    tol = 1e-10 if prec == "F64" else 1e-8
    X0, info0 = g.solve(B, restart=restart, tol=tol)
    X0 = X0.clone()
    torch.cuda.synchronize()
    print(f"  eager iters={info0.iters.tolist()} restarts={info0.restarts.tolist()}", flush=True)
    assert info0.converged.all()
    for s in steps:
        _same(P, g, B, restart, s, X0, info0, tol=tol)


def test_graphs_are_captured_again_after_changes():
    P = _gpu()
    P.tune_reset()
    try:
        g = P.Problem(W.kite(500, 6.0, 9.0))
        g.assemble(P.F64)
        B = g.rhs(_angles(4))
        print("restart 30 then 25", flush=True)
        for restart in (30, 25):
            X0, i0 = g.solve(B, restart=restart)
            X0 = X0.clone()
            _same(P, g, B, restart, 4, X0, i0, reps=1)
        print("matrix in a new buffer, other wavenumbers", flush=True)
        keep = g.A  # the old buffer stays allocated, so the new one has another address
        g2 = P.Problem(W.kite(500, 7.0, 10.0))
        g2.assemble(P.F64)
        g.assemble(P.F64, out=torch.empty_like(g2.A))
        assert g.A.data_ptr() != keep.data_ptr()
        X0, i0 = g.solve(B, restart=25)
        X0 = X0.clone()
        _same(P, g, B, 25, 4, X0, i0, reps=1)
        print("precision F64 -> MIXED", flush=True)
        g.assemble(P.MIXED)
        X0, i0 = g.solve(B, restart=25, tol=1e-8)
        X0 = X0.clone()
        _same(P, g, B, 25, 4, X0, i0, tol=1e-8, reps=1)
        print("tuned product shapes", flush=True)
        g.assemble(P.F64)
        X0, i0 = g.solve(B, restart=25)
        X0 = X0.clone()
        _same(P, g, B, 25, 4, X0, i0, reps=1)
        info = g.tune(4, reps=2)
        print("  tuned", info, flush=True)
        Xt, it = g.solve(B, restart=25)
        Xt = Xt.clone()
        _same(P, g, B, 25, 4, Xt, it, reps=1)
    finally:
        P.tune_reset()


def test_graph_steps_out_of_range_is_an_argument_error():
    P = _gpu()
    g = P.Problem(W.disk(64, 1.0, 2.0))
    g.assemble(P.F64)
    B = g.rhs([0.0])
    for s in (-1, 17):
        with pytest.raises(P.BemError) as e:
            g.solve(B, restart=20, graph_steps=s)
        assert e.value.status == 1


def test_served_results_with_graphs_equal_kernel_by_kernel():
    P = _gpu()
    from paper_2312_12787_amd import serve as S
    reqs = W.request_stream(8, seed=3, n_range=(64, 500), k0_range=(1.0, 10.0), max_rhs=10)
    dirs = W.equispaced_angles(36)
    out = {}
    for steps, slots in ((0, 1), (6, 3)):
        with S.Server(1 << 30, slots=slots, prec=P.MIXED, dirs=dirs, graph_steps=steps) as srv:
            ids = {srv.submit(r["spec"], r["angles"]): i for i, r in enumerate(reqs)}
            for res in srv.drain():
                assert res.status == 0, res.message
                out[(steps, ids[res.id])] = res.far_field
    for i in range(len(reqs)):
        assert np.array_equal(out[(6, i)], out[(0, i)]), i
