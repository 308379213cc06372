"""Host-side checks of libhelm27 (no GPU calls): exported symbols and the
FP64 table builder against the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import table as T
from paper_2108_08730_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(helm27_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(L.lib, n)]
    assert not missing, missing


def _lib_table(gmin, gmax, dg, lam, n_angles=5, step=10.0, order=1):
    h = C.c_void_p()
    opts = L.TableOpts(n_angles, step, order)
    L.check(L.lib.helm27_build_table(None, gmin, gmax, dg, lam, C.byref(opts), C.byref(h)))
    n = C.c_int()
    L.check(L.lib.helm27_table_weights(h, None, C.byref(n), None, None))
    w = np.zeros((n.value, 7))
    L.check(L.lib.helm27_table_weights(h, w.ctypes.data_as(C.POINTER(C.c_double)), None, None, None))
    L.lib.helm27_table_destroy(h)
    return w


def test_table_matches_oracle_default():
    """Banded Givens QR (library) vs dense LAPACK least squares (oracle) on the
    default table G in [3, 20] step 0.05, lambda = 1e-3: agree to 1e-9."""
    _, W = T.build_table(3.0, 20.0, 0.05, 1e-3)
    w_or = T.complete_weights(W)
    w_lib = _lib_table(3.0, 20.0, 0.05, 1e-3)
    assert w_lib.shape == w_or.shape
    assert np.max(np.abs(w_lib - w_or)) < 1e-9


def test_table_build_is_deterministic():
    """The per-G block reductions run on several host threads (one per 64+
    G values, at most 8): repeated builds of a table large enough to use them
    are bit-identical, and it matches the oracle's dense least squares."""
    a = _lib_table(3.0, 40.0, 0.05, 1e-3)
    b = _lib_table(3.0, 40.0, 0.05, 1e-3)
    assert a.shape == (741, 7)
    assert np.array_equal(a, b)
    w_or = T.complete_weights(T.build_table(3.0, 40.0, 0.05, 1e-3)[1])
    assert np.max(np.abs(a - w_or)) < 1e-9


@pytest.mark.parametrize("gmin,gmax,dg,lam,order,tol", [(2.5, 45.0, 0.1, 1e-2, 1, 1e-9),
                                                       (3.0, 8.0, 0.25, 1e-4, 2, 1e-7),
                                                       (3.0, 6.0, 0.5, 0.0, 1, 1e-10)])
def test_table_matches_oracle_other_grids(gmin, gmax, dg, lam, order, tol):
    """Other G ranges, smoothing orders and lambda = 0 (minimum-norm per G).
    The tolerance follows the conditioning of each problem (both solutions
    satisfy the normal equations to ~1e-15)."""
    Gs, W = T.build_table(gmin, gmax, dg, lam, diff="first" if order == 1 else "second")
    w_lib = _lib_table(gmin, gmax, dg, lam, order=order)
    assert np.max(np.abs(w_lib - T.complete_weights(W))) < tol
    if lam > 0:
        assert T.table_normal_residual(Gs, w_lib[:, [0, 1, 3, 4, 5]], lam,
                                       diff="first" if order == 1 else "second") < 1e-12


@pytest.mark.parametrize("anchor", [False, True])
@pytest.mark.parametrize("glist", [[4.0], [4.0, 6.0, 8.0, 10.0]])
def test_fixed_weights_match_oracle(glist, anchor):
    """G4 / Gm weights, library (Jacobi SVD) vs oracle (LAPACK gelsd): the
    minimum-norm least-squares solution, or the one closest to a given weight
    vector (here the oracle table's entry at G = 4)."""
    g = np.array(glist, np.float64)
    near = None
    if anchor:
        Gs, W = T.build_table(3.0, 6.0, 0.05, 1e-3)
        near = np.ascontiguousarray(W[20])
    h = C.c_void_p()
    L.check(L.lib.helm27_fit_fixed(None, g.ctypes.data_as(C.POINTER(C.c_double)), len(g), None,
                                   near.ctypes.data_as(C.POINTER(C.c_double)) if anchor else None, C.byref(h)))
    w = np.zeros((1, 7))
    L.check(L.lib.helm27_table_weights(h, w.ctypes.data_as(C.POINTER(C.c_double)), None, None, None))
    L.lib.helm27_table_destroy(h)
    w_or = T.complete_weights(T.fit_fixed(glist, near=near))
    assert np.max(np.abs(w[0] - w_or)) < 1e-10


def test_table_errors():
    h = C.c_void_p()
    assert L.lib.helm27_build_table(None, -1.0, 20.0, 0.05, 1e-3, None, C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 3.0, 2.0, 0.05, 1e-3, None, C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 3.0, 20.0, 0.0, 1e-3, None, C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 3.0, 20.0, 0.05, -1.0, None, C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 1.0, 1e6, 1.0, 1e-3, None, C.byref(h)) == L.EINVAL
    # 1/G axis: s_min may be 0 but not negative; lambda = 0 (decoupled fits) needs the G axis
    opts = L.TableOpts(5, 10.0, 1, L.SPACING_INVG)
    assert L.lib.helm27_build_table(None, -0.1, 0.4, 0.001, 1e-3, C.byref(opts), C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 0.0, 0.4, 0.001, 0.0, C.byref(opts), C.byref(h)) == L.EINVAL
    assert L.lib.helm27_build_table(None, 3.0, 20.0, 0.05, 1e-3, C.byref(L.TableOpts(5, 10.0, 1, 7)),
                                    C.byref(h)) == L.EINVAL


def test_table_from_weights_roundtrip():
    w5 = np.array([[0.5, 0.3, 0.6, 0.04, 0.01], [0.2, 0.7, 0.62, 0.035, 0.018]])
    h = C.c_void_p()
    L.check(L.lib.helm27_table_from_weights(None, L.SPACING_G, 4.0, 1.0, 2,
                                            w5.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
    w = np.zeros((2, 7))
    n = C.c_int()
    g0 = C.c_double()
    dg = C.c_double()
    L.check(L.lib.helm27_table_weights(h, w.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n), C.byref(g0),
                                       C.byref(dg)))
    L.lib.helm27_table_destroy(h)
    assert n.value == 2 and g0.value == 4.0 and dg.value == 1.0
    assert np.allclose(w, T.complete_weights(w5), rtol=0, atol=1e-15)


def test_strerror():
    for code in (L.OK, L.EINVAL, L.ENOCONV, L.ERANGE, L.EADMIT):
        assert len(L.lib.helm27_strerror(code)) > 0


def test_inverse_axis_table_matches_oracle():
    """The table on the paper's own axis, 1/G from 0 to 0.4 by 0.001 (Sec. 2.2,
    figure caption): the library's banded QR against the oracle's dense
    least squares on the same stacked problem, to 1e-9 (as on the G axis)."""
    S, W = T.build_table(0.0, 0.4, 0.001, 1e-3, spacing="invG")
    opts = L.TableOpts(5, 10.0, 1, L.SPACING_INVG)
    h = C.c_void_p()
    L.check(L.lib.helm27_build_table(None, 0.0, 0.4, 0.001, 1e-3, C.byref(opts), C.byref(h)))
    n = C.c_int()
    sp = C.c_int()
    v0 = C.c_double()
    dv = C.c_double()
    L.check(L.lib.helm27_table_axis(h, C.byref(sp), C.byref(v0), C.byref(dv), C.byref(n)))
    assert sp.value == L.SPACING_INVG and n.value == 401 and v0.value == 0.0 and dv.value == 0.001
    w = np.zeros((401, 7))
    L.check(L.lib.helm27_table_weights(h, w.ctypes.data_as(C.POINTER(C.c_double)), None, None, None))
    L.lib.helm27_table_destroy(h)
    ref = T.complete_weights(W)
    assert np.max(np.abs(w - ref)) <= 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_fit_fixed_binding():
    """The binding's fit_fixed passes the anchor through: the one-entry table
    equals the oracle's anchored fit."""
    from paper_2108_08730_amd import api
    Gs, W = T.build_table(3.0, 6.0, 0.05, 1e-3)
    ctx = api.Context.__new__(api.Context)
    ctx._h = None
    t = api.Context.fit_fixed(ctx, [4.0], near=W[20])
    w7, g0, dg = t.weights()
    assert w7.shape == (1, 7) and g0 == 4.0
    assert np.max(np.abs(w7[0] - T.complete_weights(T.fit_fixed([4.0], near=W[20])))) < 1e-10
