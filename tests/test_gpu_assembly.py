"""The split assembly writes every entry, on geometries where the far/near
division of the source elements matters.

The far-element launch covers the full grid of (row tile, column chunk)
workgroups; the near-element launch only the pairs the host lists as within
the series radius.  Every matrix starts filled with NaN, so an entry neither
launch wrote would show; each is compared with the oracle's matrix
(FP64 path: 5e-13 of max|A|; FP32 path: 1e-6 of max|A|), and the FP32 copy of
a MIXED assembly is the FP64 matrix rounded to FP32, bit for bit.  Cases:
every element near (small k), almost every element far (large k), a
non-convex curve (the kite's concave side comes back within the radius),
Gauss rules of 8, 10 and 5 points (the kernels built for 8 and 10 points and
the general one), graded junction meshes with elements down to h/16 (three sectors), and the
disk split by a diameter.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ("disk200_k0.5-1_all_near", lambda: W.disk(200, 0.5, 1.0)),
    ("disk300_k50-80_mostly_far", lambda: W.disk(300, 50.0, 80.0 + 1.0j)),
    ("kite700_k20-30", lambda: W.kite(700, 20.0, 30.0)),
    ("kite500_k12-18+0.5i_q10", lambda: W.kite(500, 12.0, 18.0 + 0.5j, quad=10)),
    ("kite300_k8-12+0.3i_q5", lambda: W.kite(300, 8.0, 12.0 + 0.3j, quad=5)),
    ("sectors_graded_h1/40", lambda: W.sectors([10.0, 12.0, 18.0, 9.0 + 0.5j], h=1.0 / 40)),
    ("split_disk400", lambda: W.split_disk(400, [6.0, 6.0 * np.sqrt(2.0), 6.0 * np.sqrt(3.0)])),
]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_12787_amd as P
    return P


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_every_entry_written_and_equal_to_the_oracle(name, make):
    P = _gpu()
    spec = make()
    g = P.Problem(spec)
    n = g.n
    print("case", name, "N", spec.n_elements, flush=True)
    Ao = O.Problem(spec).assemble()
    scale = np.abs(Ao).max()
    A64 = torch.full((n, n), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    g.assemble(P.F64, out=A64)
    A = A64.T.cpu().numpy()
    assert np.isfinite(A).all()
    e64 = np.abs(A - Ao).max() / scale
    A32 = torch.full((n, n), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
    g.assemble(P.F32, out=A32)
    B = A32.T.cpu().numpy()
    assert np.isfinite(B).all()
    e32 = np.abs(B.astype(np.complex128) - Ao).max() / scale
    _, mb, _ = g.sizes(P.MIXED)
    buf = torch.empty(mb, dtype=torch.uint8, device="cuda")
    buf.view(torch.float32)[: mb // 4].fill_(float("nan"))
    Am = g.assemble(P.MIXED, out=buf)
    Am32 = g.mixed_f32()
    assert torch.isfinite(torch.view_as_real(Am)).all() and torch.isfinite(torch.view_as_real(Am32)).all()
    same = torch.equal(Am.to(torch.complex64), Am32)
    print(f"  FP64 {e64:.2e}  FP32 {e32:.2e}  MIXED copy = FP64 rounded: {same}", flush=True)
    assert e64 < 5e-13 and e32 < 1e-6 and same
