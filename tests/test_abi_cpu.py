"""The C-ABI library loads and exports every entry point declared in
include/cntr.h; host-side validation rejects bad arguments before any device
work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1911_01211_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "cntr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:cntr_status|const char\*)\s+(cntr_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 12
    L = _abi.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(_abi.SYMBOLS)
    assert L.cntr_version().decode().startswith("cntr")


def _grid(**kw):
    base = dict(nt=10, ntau=20, d=2, sig=-1, k=5, beta=1.0, h=0.1, mu=0.0)
    base.update(kw)
    return _abi.Grid(*(base[k] for k in ("nt", "ntau", "d", "sig", "k", "beta", "h", "mu")))


@pytest.mark.parametrize("kw", [dict(k=0), dict(k=6), dict(d=0), dict(d=9), dict(ntau=11),
                                dict(nt=4), dict(sig=0), dict(h=0.0), dict(beta=-1.0)])
def test_invalid_grids_are_rejected(kw):
    L = _abi.lib()
    g = (_abi.Grid * 1)(_grid(**kw))
    gf = (_abi.GF * 1)(_abi.GF(1, 1, 1, 1))
    eps = (C.c_void_p * 1)(1)
    rc = L.cntr_dyson_step(6, 1, g, gf, gf, eps, None)
    assert rc == -1, (kw, rc)
    assert "cntr_dyson_step" in L.cntr_last_error().decode()


def test_shape_and_order_errors():
    L = _abi.lib()
    g = (_abi.Grid * 1)(_grid())
    gf = (_abi.GF * 1)(_abi.GF(1, 1, 1, 1))
    nul = (_abi.GF * 1)(_abi.GF(None, 1, 1, 1))
    eps = (C.c_void_p * 1)(1)
    assert L.cntr_dyson_step(6, 1, g, nul, gf, eps, None) == -2
    assert L.cntr_dyson_step(11, 1, g, gf, gf, eps, None) == -3
    assert L.cntr_dyson_step(-1, 1, g, gf, gf, eps, None) == -3
    assert L.cntr_dyson_step(6, 0, g, gf, gf, eps, None) == -2
    g2 = (_abi.Grid * 2)(_grid(), _grid(d=3))
    gf2 = (_abi.GF * 2)(_abi.GF(1, 1, 1, 1), _abi.GF(1, 1, 1, 1))
    eps2 = (C.c_void_p * 2)(1, 1)
    assert L.cntr_dyson_step(6, 2, g2, gf2, gf2, eps2, None) == -2
    assert L.cntr_convolution(-2, 1, g, gf, gf, gf, gf, gf, None, None) == -3
    assert L.cntr_extrapolate(2, 1, g, gf, None) == -3


def test_adjoint_sweep_validation():
    """cntr_adjoint_sweep rejects bad arguments on the host, before any
    device work: null contour pointers, missing eps_bar, and the second-Born
    mode without its Sigmabar / U_bar accumulators."""
    L = _abi.lib()
    g = (_abi.Grid * 1)(_grid())
    gf = (_abi.GF * 1)(_abi.GF(1, 1, 1, 1))
    nul = (_abi.GF * 1)(_abi.GF(1, None, 1, 1))
    p1 = (C.c_void_p * 1)(1)
    pn = (C.c_void_p * 1)(None)
    conv = C.c_double(0.0)
    args = lambda G=gf, S=gf, Gb=gf, Sb=None, U=None, Ub=None, eb=p1, n=1, gr=g: (
        n, gr, G, S, p1, U, 0.5, Gb, Sb, eb, Ub, 4, 0.0, C.byref(conv), None)
    assert L.cntr_adjoint_sweep(*args(G=nul)) == -2
    assert L.cntr_adjoint_sweep(*args(Gb=nul)) == -2
    assert L.cntr_adjoint_sweep(*args(eb=pn)) == -2
    assert "eps_bar" in L.cntr_last_error().decode()
    assert L.cntr_adjoint_sweep(*args(U=p1)) == -2           # second-Born mode needs Sigmabar, U_bar
    assert "second-Born" in L.cntr_last_error().decode()
    assert L.cntr_adjoint_sweep(*args(U=p1, Sb=gf)) == -2
    assert L.cntr_adjoint_sweep(*args(U=p1, Sb=nul, Ub=p1)) == -2
    assert L.cntr_adjoint_sweep(*args(n=0)) == -2
    bad = (_abi.Grid * 1)(_grid(k=7))
    assert L.cntr_adjoint_sweep(*args(gr=bad)) == -1


def test_order_checks_track_the_last_completed_slice():
    """With CNTR_CHECK_ORDER a step whose inputs are not complete is refused
    on the host (Tab. dyson: the step at tstp needs slices -1..tstp-1)."""
    L = _abi.lib()
    g = (_abi.Grid * 1)(_grid(nt=10))
    gf = (_abi.GF * 1)(_abi.GF(11, 12, 13, 14))
    eps = (C.c_void_p * 1)(1)
    assert L.cntr_set_checks(1) == 0
    try:
        assert L.cntr_dyson_step(5, 1, g, gf, gf, eps, None) == -3  # unknown instance
        assert "slice" in L.cntr_last_error().decode()
        assert L.cntr_mark_slices(1, gf, 6) == 0
        assert L.cntr_dyson_step(8, 1, g, gf, gf, eps, None) == -3  # slice 7 missing
        assert L.cntr_mark_slices(1, gf, 7) == 0
        assert L.cntr_dyson_step(8, 1, g, gf, gf, eps, None) != -3  # passes the check (then needs a device)
        assert L.cntr_mark_slices(1, gf, -2) == 0
        assert L.cntr_dyson_step(8, 1, g, gf, gf, eps, None) == -3
        assert L.cntr_set_checks(8) == -1
    finally:
        assert L.cntr_set_checks(0) == 0
    # checks off: no tracking
    assert L.cntr_dyson_step(5, 1, g, gf, gf, eps, None) != -3
