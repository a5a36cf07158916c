"""Fused multi-instance solves (bem_solve_batch, and the request server's
fused batches): several problems' restart cycles run in step, each Krylov
step launching every problem's product and one fused set of
orthogonalisation kernels for all of them.

Each problem's arithmetic runs in the same order alone or fused, so the
solutions, iteration counts and far fields are bit-identical to bem_solve on
the problem alone (FP64, FP32 and mixed precision; vector and matrix-core
products; problems that stop early, problems that do not converge); the
fused server's far fields equal the one-request server's bit for bit and the
oracle's LU solution within 1e-6."""
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
    from paper_2312_12787_amd import serve as S
    return P, S


# different sizes, wavenumbers and right-hand-side counts (vector and matrix-core products)
CASES = [(W.kite(200, 5.0, 7.5), [0.1, 0.7]),
         (W.disk(150, 3.0, 6.0 + 0.2j), [0.3 * r for r in range(16)]),
         (W.stream_like_request(260, 9.0, 2.0, 5, 3)["spec"], [0.2 * r for r in range(5)]),
         (W.kite(90, 2.0, 3.0), [1.1])]


@pytest.mark.parametrize("prec", ["F64", "MIXED", "F32"])
def test_batch_equals_each_problem_alone(prec):
    P, _ = _gpu()
    pr = getattr(P, prec)
    tol = 1e-10 if prec == "F64" else 1e-8
    probs, Bs, alone = [], [], []
    for spec, ang in CASES:
        g = P.Problem(spec)
        g.assemble(pr)
        B = g.rhs(ang)
        X, info = g.solve(B, restart=30, tol=tol, inner_tol=1e-5 if prec != "F64" else 0.0)
        alone.append((X.clone(), info))
        probs.append(g)
        Bs.append(B)
    out = P.solve_batch(probs, Bs, restart=30, tol=tol, inner_tol=1e-5 if prec != "F64" else 0.0)
    torch.cuda.synchronize()
    for k, ((Xa, ia), (Xb, ib)) in enumerate(zip(alone, out)):
        print(prec, "problem", k, "n", probs[k].n, "nrhs", Bs[k].shape[0], "iters alone", ia.iters.tolist(),
              "fused", ib.iters.tolist(), "restarts", ia.restarts.tolist(), flush=True)
        assert ia.converged.all() and ib.converged.all()
        assert np.array_equal(ia.iters, ib.iters) and np.array_equal(ia.restarts, ib.restarts)
        assert torch.equal(Xa, Xb)
        assert np.array_equal(ia.rel_residual, ib.rel_residual)


def test_batch_against_oracle_and_nonconvergence():
    """A fused batch's solutions match the oracle's LU solutions (1e-10); a
    budget too small for one problem gives it BEM_E_NOCONV columns while the
    others of the batch converge."""
    P, _ = _gpu()
    probs, Bs, ref = [], [], []
    for spec, ang in CASES[:3]:
        g = P.Problem(spec)
        g.assemble(P.F64)
        probs.append(g)
        Bs.append(g.rhs(ang))
        po = O.Problem(spec)
        ref.append(np.linalg.solve(po.assemble(), po.rhs(ang)).T)
    out = P.solve_batch(probs, Bs, restart=40, tol=1e-12)
    for (X, info), Xo in zip(out, ref):
        e = np.linalg.norm(X.cpu().numpy() - Xo) / np.linalg.norm(Xo)
        print("fused vs oracle LU", e, "iters", info.iters.tolist(), flush=True)
        assert info.converged.all() and e < 1e-10
    # a step budget between the problems' needs: the one needing the fewest steps converges, the others stop
    it_budget = [int(o[1].iters.max()) for o in out]
    out2 = P.solve_batch(probs, Bs, restart=40, tol=1e-12, max_iter=min(it_budget[:2]) + 1)
    conv = [bool(o[1].converged.all()) for o in out2]
    print("budget", min(it_budget[:2]) + 1, "converged", conv, "status", out2[0][1].status, flush=True)
    assert out2[0][1].status == 6 and not all(conv)


@pytest.mark.parametrize("prec", ["MIXED", "F64"])
def test_fused_server_equals_one_request_server(prec):
    P, S = _gpu()
    pr = getattr(P, prec)
    reqs = W.request_stream(14, seed=9, n_range=(64, 700), k0_range=(1.0, 12.0), max_rhs=16)
    dirs = W.equispaced_angles(72)
    alone = {}
    with S.Server(1 << 30, slots=1, prec=pr, dirs=dirs) as srv:
        for i, r in enumerate(reqs):
            srv.submit(r["spec"], r["angles"])
            (res,) = srv.drain()
            assert res.status == 0, res.message
            alone[i] = res.far_field
    with S.Server(4 << 30, slots=2, prec=pr, dirs=dirs, fuse=4) as srv:
        ids = {srv.submit(r["spec"], r["angles"]): i for i, r in enumerate(reqs)}
        fused = srv.drain()
    batches = {}
    for o in fused:
        batches.setdefault(o.t_admit, []).append(o.id)
    print(prec, "batch sizes", sorted(len(v) for v in batches.values()), flush=True)
    assert max(len(v) for v in batches.values()) > 1
    for o in fused:
        assert o.status == 0, o.message
        assert np.array_equal(o.far_field, alone[ids[o.id]])
    # and the fused results against the oracle on the first three requests
    for o in fused:
        i = ids[o.id]
        if i >= 3:
            continue
        r = reqs[i]
        po = O.Problem(r["spec"])
        Fo = po.farfield(np.linalg.solve(po.assemble(), po.rhs(r["angles"])), dirs).T
        e = float(np.max(np.linalg.norm(o.far_field - Fo, axis=1) / np.linalg.norm(Fo, axis=1)))
        print("request", i, "fused far field vs oracle LU", e, flush=True)
        assert e < 1e-6
