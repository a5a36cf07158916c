"""The C-ABI library (no GPU needed): it loads, exports every function that
include/bem.h and include/bem_serve.h declare, and its host-only paths (validation, planning, sizes,
call-order errors) behave as documented.  No call here launches device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(bem_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_2312_12787_amd as P
    from paper_2312_12787_amd.serve import SERVE_EXPORTS
    L = P.lib()
    names = _declared()
    assert "bem_solve" in names and "bem_assemble" in names and "bem_server_submit" in names
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(P.EXPORTS + SERVE_EXPORTS) == names


def test_server_option_validation_before_any_device_work():
    """bem_server_create rejects bad options from the host, before it selects
    a device or creates a stream."""
    import paper_2312_12787_amd as P
    from paper_2312_12787_amd import serve as S
    L = S._serve_lib()
    dirs = np.zeros(4)

    def opts(**kw):
        o = S.bem_server_opts()
        o.slots, o.device, o.arena_dev, o.arena_bytes, o.prec = 4, 0, 1 << 20, 1 << 30, P.F32
        o.solve = P.bem.bem_solve_opts(100, 1000, 1e-8, 1e-5, 0)
        o.ndir, o.dirs = 4, dirs.ctypes.data_as(C.POINTER(C.c_double))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    for bad in (dict(slots=0), dict(slots=17), dict(arena_dev=None), dict(arena_dev=(1 << 20) + 8),
                dict(ndir=0), dict(ndir=5000), dict(prec=7), dict(dirs=None), dict(fuse=9), dict(fuse=-1)):
        h = C.c_void_p()
        st = L.bem_server_create(C.byref(opts(**bad)), C.byref(h))
        assert P.STATUS[st] == "BEM_E_ARG", bad
        assert h.value is None
    o = opts()
    o.solve = P.bem.bem_solve_opts(0, 1000, 1e-8, 1e-5, 0)
    assert P.STATUS[L.bem_server_create(C.byref(o), C.byref(C.c_void_p()))] == "BEM_E_ARG"
    assert "solve options" in L.bem_last_error().decode()


def _problem(spec):
    import paper_2312_12787_amd as P
    return P.Problem(spec, device="cpu")


def test_create_validation_errors():
    import paper_2312_12787_amd as P
    cases = []
    s = W.disk(16, -1.0, 2.0)
    cases.append((s, "BEM_E_ARG"))
    s = W.disk(16, 1.0, 2.0 - 0.1j)
    cases.append((s, "BEM_E_ARG"))
    s = W.disk(16, 1.0, 2.0)
    s.interfaces[0].dom_left, s.interfaces[0].dom_right = 0, 1
    cases.append((s, "BEM_E_GEOMETRY"))
    s = W.disk(16, 1.0, 2.0)
    s.interfaces[0].dom_left = 5
    cases.append((s, "BEM_E_GEOMETRY"))
    s = W.disk(16, 1.0, 2.0)
    s.interfaces[0].xy[4] = s.interfaces[0].xy[3]
    cases.append((s, "BEM_E_GEOMETRY"))
    s = W.single_material(W.circle_nodes(2), 1.0, 2.0)
    cases.append((s, "BEM_E_GEOMETRY"))
    s = W.disk(16, 1.0, 1.0j)  # eps = -1 (accumulation point at 0) needs arg k = 90 deg: refused as such
    cases.append((s, "BEM_E_ARG"))
    s = W.disk(16, 1.0, 2.0, quad=17)
    cases.append((s, "BEM_E_ARG"))
    s = W.disk(16, 1.0, 2.0)
    s.k[1] = complex(np.nan, 0)
    cases.append((s, "BEM_E_ARG"))
    for spec, code in cases:
        with pytest.raises(P.BemError, match=code):
            _problem(spec)


def test_sizes_and_order():
    import paper_2312_12787_amd as P
    g = _problem(W.concentric(30, 17, [1.0, 2.0, 3.0]))
    assert g.N == 47 and g.n == 94
    geom, mat, work = g.sizes(P.F64, 5, 20)
    assert mat == 94 * 94 * 16
    assert g.sizes(P.F32, 5, 20)[1] == 94 * 94 * 8
    assert geom > 47 * 128 and work > 21 * 5 * 94 * 16
    # an open interface has one element fewer than nodes
    spec = W.ProblemSpec(k=[1.0, 2.0, 3.0], interfaces=[
        W.Interface(W.circle_nodes(20), True, 1, 0),
        W.Interface(np.array([[-0.5, 0.0], [0.0, 0.0], [0.5, 0.0]]), False, 1, 2)])
    assert _problem(spec).N == 22
    with pytest.raises(P.BemError, match="BEM_E_ARG"):
        g.sizes(P.F64, 0, 20)
    # restart lengths up to BEM_MAX_RESTART (the step block's LDS holds a cycle)
    assert P.MAX_RESTART == int(re.search(r"#define BEM_MAX_RESTART (\d+)",
                                          open(os.path.join(ROOT, "include", "bem.h")).read()).group(1))
    assert g.sizes(P.F64, 1, P.MAX_RESTART)[2] > g.sizes(P.F64, 1, 1000)[2]
    with pytest.raises(P.BemError, match="BEM_E_ARG"):
        g.sizes(P.F64, 1, P.MAX_RESTART + 1)


def test_call_order_errors_before_any_device_work():
    """bem_assemble / bem_rhs / bem_solve / bem_farfield before bem_geometry
    return BEM_E_STATE from the host, without touching a device."""
    import paper_2312_12787_amd as P
    L = P.lib()
    g = _problem(W.disk(16, 1.0, 2.0))
    st = L.bem_assemble(g._h, P.F64, C.c_void_p(16), g.n, None)
    assert P.STATUS[st] == "BEM_E_STATE"
    ang = np.zeros(1)
    st = L.bem_rhs(g._h, 1, ang.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(16), g.n, None)
    assert P.STATUS[st] == "BEM_E_STATE"
    assert "bem_geometry" in L.bem_last_error().decode()
    st = L.bem_geometry_update(g._h, None)
    assert P.STATUS[st] == "BEM_E_STATE"
    st = L.bem_matvec(g._h, 1, C.c_void_p(16), g.n, C.c_void_p(16), g.n, C.c_void_p(16), 1 << 20, None)
    assert P.STATUS[st] == "BEM_E_STATE"
    st = L.bem_tune(g._h, 16, C.c_void_p(16), g.n, C.c_void_p(16), g.n, C.c_void_p(16), 1 << 20, 3, None, None)
    assert P.STATUS[st] == "BEM_E_STATE"


def test_tuning_table_text_round_trip_on_the_host():
    """bem_tune_import / bem_tune_export / bem_tune_reset are host-only: a
    valid table survives a round trip, a malformed line or an invalid shape
    (row tiles 3, 2-4 groups without the 3-product form, splits 0) is refused
    without changing the table, the reset empties it, and work sizes do not
    depend on the table."""
    import paper_2312_12787_amd as P
    P.tune_reset()
    g = _problem(W.disk(600, 1.0, 2.0))
    sizes = g.sizes(P.F64, 16, 30)
    assert P.tune_export().strip().splitlines()[1:] == []
    text = "# comment\n3 1 11 1 4 4 0\n0 4 15 2 2 8 1\n3 0 11 0 0 16 0\n"
    P.tune_import(text)
    rows = sorted(P.tune_export().strip().splitlines()[1:])
    assert rows == sorted(["3 1 11 1 4 4 0", "0 4 15 2 2 8 1", "3 0 11 0 0 16 0"])
    for bad in ["3 1 11 3 4 4 0\n", "3 2 11 1 4 4 0\n", "3 1 11 1 4 0 0\n", "3 1 11 1 4\n", "x\n", "2 1 11 1 4 4 0\n"]:
        with pytest.raises(P.BemError, match="BEM_E_ARG"):
            P.tune_import(bad)
    assert sorted(P.tune_export().strip().splitlines()[1:]) == rows
    assert g.sizes(P.F64, 16, 30) == sizes
    P.tune_reset()
    assert P.tune_export().strip().splitlines()[1:] == []


def test_phase_range_is_checked_on_the_host():
    """bem_create refuses max |k| times the boundary's diameter >= 2^29 (the
    device reduces phases k r by pi/2 exactly only below 2^30)."""
    import paper_2312_12787_amd as P
    # unit disk: bounding-box diagonal 2 sqrt(2); 2^29 = 5.37e8
    _problem(W.disk(16, 1.0e8, 1.8e8))  # 5.09e8: accepted
    with pytest.raises(P.BemError, match="2\\^29"):
        _problem(W.disk(16, 1.0e8, 2.0e8))  # 5.66e8


def test_lossy_wavenumber_argument_is_bounded_on_the_host():
    """bem_create accepts lossy media up to arg k = 10 degrees (the device's
    large-argument Hankel form is validated to 1.7e-12 there) and refuses a
    larger argument with BEM_E_ARG."""
    import paper_2312_12787_amd as P
    t10 = np.tan(np.deg2rad(10.0))
    _problem(W.disk(16, 1.0, 30.0 + 0.3j))
    _problem(W.disk(16, 1.0, 30.0 * (1.0 + 0.999999 * t10 * 1j)))
    _problem(W.sectors([10.0, 12.0, 18.0, 9.0 + 0.5j], h=1 / 10))
    for k1 in (30.0 * (1.0 + 1.000001 * t10 * 1j), 2.0 + 2.0j, -1.0 + 0.1j):
        with pytest.raises(P.BemError, match="arg k"):
            _problem(W.disk(16, 1.0, k1))
