"""GPU parity of the table-axis options against the oracle.

* The paper's own table axis, uniform in s = 1/G (Sec. 2.2, figure caption
  of the dispersion curves: 1/G from 0 to 0.4 by 0.001): the per-point index
  bit-exact (nearest s = (f h)/c, ties upward, clamped), FP64 apply <= 1e-12
  and FP32 apply <= 1e-5 against the oracle's CSR.
* HELM27_EXTEND_TABLE: a table that does not reach the model's G range is
  widened on its own axis grid until no row clamps.  The widened weights
  match the oracle's table built over the same axis to 1e-9 (the library /
  oracle table agreement), the index is bit-exact, and the FP64 apply matches
  the oracle's CSR to 1e-8 (a relative weight difference of 1e-9 moves each
  27-term row by at most ~1e-9 times the sum of its terms' magnitudes, a few
  times its value).
* Coarse multigrid levels rediscretise at G / 2^l: without widening their
  out-of-table rows are counted; with it they get their own tables and none
  clamps; both solves are certified by the oracle's FP64 residual.
"""
import numpy as np
import pytest

from oracle import operator as O
from oracle import solve as S
from oracle import table as T
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2108_08730_amd import api
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    return api.Context(0)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def inv_table():
    S_, W = T.build_table(0.0, 0.4, 0.001, 1e-3, spacing="invG")
    return S_, W, T.complete_weights(W)


@pytest.mark.parametrize("f", [6.0, 25.0])
def test_invg_axis_index_and_apply(ctx, inv_table, f):
    """77 x 37 x 19 random field, PML (4, 3, 2), h = 25 m: at 6 Hz every G is
    in the table (G 10..43), at 25 Hz the slowest rows (G < 2.5) clamp to the
    s = 0.4 entry."""
    _, W, W7 = inv_table
    dims, npml, h = (77, 37, 19), (4, 3, 2), 25.0
    c = synth.random_field_model(dims, h, seed=11)
    tab = ctx.table_from_weights(0.0, 0.001, W, spacing="invG")
    assert tab.axis() == ("invG", 0.0, 0.001, 401)
    op = ctx.assemble(tab, c, h, f, npml=npml, store=("c128",))
    idx, ncl = O.select_index(c, f, h, 0.0, 0.001, 401, spacing="invG")
    assert np.array_equal(op.index().astype(np.int64), idx.ravel())
    assert op.info()["n_clamped"] == ncl
    assert (ncl > 0) == (f == 25.0)
    A = O.assemble(c, f, h, npml, O.row_weights("GA", idx, W7))
    u = synth.random_vectors(int(np.prod(dims)), 2, seed=3)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()
    y64s = op.apply(ud, variant="stored").cpu().numpy()
    y32 = op.apply(ud.to(torch.complex64)).cpu().numpy()
    for r in range(2):
        assert _relerr(y64[r], y_ref[r]) <= 1e-12
        assert _relerr(y64s[r], y_ref[r]) <= 1e-12
        assert _relerr(y32[r], y_ref[r]) <= 1e-5


@pytest.mark.parametrize("spacing,v0,v1,dv", [("G", 3.0, 20.0, 0.05), ("invG", 0.05, 0.3, 0.001)])
def test_extend_table_to_model_range(ctx, spacing, v0, v1, dv):
    """A 40 x 34 x 30 random field at 8 Hz (G 7.5..32.5) against a table that
    does not reach G 32.5 (G axis [3, 20]) or G 7.5 (1/G axis [0.05, 0.3],
    i.e. G 3.3..20): without widening rows clamp; with it none does, the
    axis keeps its grid, and weights, index and apply match the oracle's table
    built over the widened axis."""
    dims, npml, f, h = (40, 34, 30), (4, 4, 3), 8.0, 25.0
    c = synth.random_field_model(dims, h, seed=6)
    tab = ctx.build_table(v0, v1, dv, 1e-3, spacing=spacing)
    plain = ctx.assemble(tab, c, h, f, npml=npml)
    assert plain.info()["n_clamped"] > 0
    op = ctx.assemble(tab, c, h, f, npml=npml, extend_table=True, store=("c128",))
    info = op.info()
    assert info["n_clamped"] == 0
    a0, n = info["table_min"], info["n_g"]
    assert info["table_step"] == dv and info["table_spacing"] == (0 if spacing == "G" else 1)
    k = round((v0 - a0) / dv)
    assert abs(a0 - (v0 - k * dv)) <= 1e-12 and k >= 0 and n > round((v1 - v0) / dv) + 1
    _, W = T.build_table(a0, a0 + (n - 1) * dv, dv, 1e-3, spacing=spacing)
    W7 = T.complete_weights(W)
    assert W7.shape[0] == n
    assert np.max(np.abs(op.table_weights() - W7)) <= 1e-9 * max(1.0, np.max(np.abs(W7)))
    idx, ncl = O.select_index(c, f, h, a0, dv, n, spacing=spacing)
    assert ncl == 0
    assert np.array_equal(op.index().astype(np.int64), idx.ravel())
    A = O.assemble(c, f, h, npml, O.row_weights("GA", idx, W7))
    u = synth.random_vectors(int(np.prod(dims)), 1, seed=5)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    assert _relerr(op.apply(ud).cpu().numpy()[0], y_ref[0]) <= 1e-8
    assert _relerr(op.apply(ud, variant="stored").cpu().numpy()[0], y_ref[0]) <= 1e-8


def test_coarse_levels_get_widened_tables(ctx):
    """48 x 40 x 36 random field at 6 Hz (G 16.1..43.3) with a G-axis table
    over [5, 50]: the fine rows are all in the table; the third multigrid
    level (G / 4 from 4.06) is not.  With the default coarse weights the solve
    reports its clamped coarse rows; with mg_coarse_table = 1 the coarse levels
    get tables of their own and nothing clamps.  Both solves reach 1e-7
    certified by the oracle's FP64 residual."""
    dims, npml, f, h = (48, 40, 36), 6, 6.0, 25.0
    c = synth.random_field_model(dims, h, seed=9)
    tab = ctx.build_table(5.0, 50.0, 0.05, 1e-3)
    src = [(24, 20, 9), (14, 22, 10)]
    _, W = T.build_table(5.0, 50.0, 0.05, 1e-3)
    W7 = T.complete_weights(W)
    idx, ncl = O.select_index(c, f, h, 5.0, 0.05, len(W7))
    assert ncl == 0
    A = O.assemble(c, f, h, npml, O.row_weights("GA", idx, W7))
    b = S.point_source_rhs(dims, h, src)
    res = {}
    for ext in (False, True):
        op = ctx.assemble(tab, c, h, f, npml=npml, extend_table=ext)
        assert op.info()["n_clamped"] == 0 and op.info()["n_g"] == len(W7)
        u, st = op.solve(src, tol=1e-7, mg_levels=3, mg_coarse_table=int(ext))
        assert st["converged"] == 1 and st["mg_levels"] == 3
        assert np.all(S.relative_residual(A, u.cpu().numpy().T, b) <= 1.01e-7)
        res[ext] = st
    assert res[False]["coarse_clamped"] > 0 and res[False]["coarse_tables"] == 0
    assert res[True]["coarse_clamped"] == 0 and res[True]["coarse_tables"] >= 1
