"""Adjoint (transposed) applies and solves, and several frequencies solved
at once, against the oracle.

Waveform inversion (the paper's purpose, Sec. 1) needs, per frequency, the
forward solve A u = s and the adjoint solve A^T lambda = r (A^H = conj A^T
conj).  A^T is applied from the stored coefficients read transposed
(HELM27_STORED_T); the oracle's reference is the plain transpose of its CSR.
Bars: FP64 <= 1e-12, FP32 <= 1e-5; the bilinear identity
<A u, v> = <u, A^T v> between the GPU's forward (recompute) and transposed
applies to 1e-12; adjoint solves certified by the oracle's FP64 residual of
A^T; each frequency of a batched solve bit-identical to its lone solve.
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


@pytest.fixture(scope="module")
def oracle_table():
    Gs, W = T.build_table(3.0, 20.0, 0.05, 1e-3)
    return Gs, W, T.complete_weights(W)


@pytest.fixture(scope="module")
def table(ctx, oracle_table):
    return ctx.table_from_weights(3.0, 0.05, oracle_table[1])


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle(c, f, h, npml, W7, mass_form="b"):
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(W7))
    return O.assemble(c, f, h, npml, O.row_weights("GA", idx, W7), mass_form=mass_form)


@pytest.mark.parametrize("mass_form", ["b", "a"])
@pytest.mark.parametrize("dims,npml,f", [((77, 37, 19), (4, 3, 2), 6.0), ((20, 5, 6), (2, 2, 2), 5.0)])
def test_transposed_apply(ctx, table, oracle_table, mass_form, dims, npml, f):
    h = 25.0
    c = synth.random_field_model(dims, h, seed=13)
    c[c.shape[0] // 2:] *= np.float32(1.25)
    op = ctx.assemble(table, c, h, f, npml=npml, mass_form=mass_form, store=("c64", "c128"))
    A = _oracle(c, f, h, npml, oracle_table[2], mass_form)
    N = int(np.prod(dims))
    u = synth.random_vectors(N, 2, seed=3)
    v = synth.random_vectors(N, 2, seed=4)
    yt_ref = (A.T @ v.T).T
    assert _relerr(yt_ref[0], (A @ v.T).T[0]) > 1e-6   # the adaptive operator is not symmetric
    vd = torch.from_numpy(v).cuda()
    yt64 = op.apply(vd, variant="stored_t").cpu().numpy()
    yt32 = op.apply(vd.to(torch.complex64), variant="stored_t").cpu().numpy()
    for r in range(2):
        assert _relerr(yt64[r], yt_ref[r]) <= 1e-12
        assert _relerr(yt32[r], yt_ref[r]) <= 1e-5
    # <A u, v> = <u, A^T v> (bilinear), forward from the recompute kernel
    Au = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    for r in range(2):
        lhs = np.sum(Au[r] * v[r])
        rhs = np.sum(u[r] * yt64[r])
        assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(np.abs(Au[r]) ** 2) * np.sum(np.abs(v[r]) ** 2))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_adjoint_solve_certified(ctx, table, oracle_table, precision):
    """A^T x = b for two point sources on a heterogeneous 16 x 14 x 12 model
    (PML 3) at 6 Hz (c 1600..2800 m/s, G 10.7..18.7, so the rows' weights
    differ): certified by the oracle's FP64 residual of A^T and compared with
    its direct solve; the forward solution of the same sources differs."""
    dims, npml, f, h = (16, 14, 12), 3, 6.0, 25.0
    c = synth.smooth_random_model(dims, h, seed=4)
    op = ctx.assemble(table, c, h, f, npml=npml, store=("c64", "c128"))
    src = [(7, 6, 5), (8, 7, 4)]
    u, st = op.solve(src, tol=1e-10, precision=precision, transpose=1)
    assert st["converged"] == 1
    A = _oracle(c, f, h, npml, oracle_table[2])
    b = S.point_source_rhs(dims, h, src)
    ud = u.cpu().numpy()
    assert np.all(S.relative_residual(A.T.tocsr(), ud.T, b) <= 1.01e-10)
    ref = S.solve(A.T.tocsr(), b).T
    fwd = S.solve(A, b).T
    for k in range(2):
        assert _relerr(ud[k], ref[k]) < 1e-8
        assert _relerr(fwd[k], ref[k]) > 1e-6


def test_adjoint_solve_needs_stored_coefficients(ctx, table):
    from paper_2108_08730_amd import _lib as L
    c = synth.homogeneous((12, 12, 12), 2000.0)
    op = ctx.assemble(table, c, 25.0, 6.0, npml=2)
    with pytest.raises(L.Helm27Error) as e:
        op.solve([(6, 6, 6)], transpose=1)
    assert e.value.status == L.EINVAL


def test_solve_many_frequencies_equal_lone_solves(ctx, table, oracle_table):
    """One 40 x 34 x 30 random-field model at 4, 6 and 8 Hz, two sources each,
    solved together (one stream per frequency, overlapping on the device):
    every frequency's solution is bit-identical to its lone solve and
    certified by the oracle."""
    from paper_2108_08730_amd import api
    dims, npml, h = (40, 34, 30), 5, 25.0
    c = synth.random_field_model(dims, h, seed=7)
    freqs = (4.0, 6.0, 8.0)
    ops = [ctx.assemble(table, c, h, f, npml=npml) for f in freqs]
    srcs = [[(20, 17, 8), (12, 17, 9)]] * 3
    us, sts = api.solve_many(ops, srcs, tol=1e-8)
    for op, f, u, st, sl in zip(ops, freqs, us, sts, srcs):
        assert st["converged"] == 1
        u1, st1 = op.solve(sl, tol=1e-8)
        assert st1["inner_iters"] == st["inner_iters"]
        assert torch.equal(u, u1)
        A = _oracle(c, f, h, npml, oracle_table[2])
        b = S.point_source_rhs(dims, h, sl)
        assert np.all(S.relative_residual(A, u.cpu().numpy().T, b) <= 1.01e-8)
