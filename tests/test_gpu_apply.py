"""GPU parity of the assembly and apply path against the oracle.

Bars:
* table index and CSR column indices: bit-exact;
* FP64 apply (recompute and stored) and exported CSR values: relative error
  <= 1e-12 against the oracle's CSR;
* FP32 apply: relative L2 error <= 1e-5 per right-hand side.  Derivation: a
  row is a 27-term sum; with FP32 coefficients and accumulation the rounding
  error of a term is ~27 eps_32 |a_i u_i| (eps_32 = 6e-8), and for random
  inputs sum |a_i u_i| / |y_i| ~ 5, giving ~1e-5 in the worst row and ~1e-7
  typically.
"""
import math

import numpy as np
import pytest

from oracle import operator as O
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
    # both sides assemble with the oracle's weights, so apply parity is not
    # blurred by the (separately tested, <= 1e-9) table-solver difference
    _, W, _ = oracle_table
    return ctx.table_from_weights(3.0, 0.05, W)


def _oracle_rows(c, f, h, npml, W7, mode="GA", rows=None):
    idx, _ = O.select_index(c, f, h, 3.0, 0.05, len(W7))
    nz, ny, nx = c.shape
    w = O.row_weights(mode, idx, W7, fixed_w=W7[0], dims=(nx, ny, nz))
    if rows is None:
        return O.assemble(c, f, h, npml, w)
    return O.assemble_rows(c, f, h, npml, w[rows], rows)


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [
    # dims (nx, ny, nz), npml, model, f, h
    ((5, 4, 3), (1, 1, 0), "gradient", 5.0, 25.0),
    ((77, 37, 19), (4, 3, 2), "random", 6.0, 25.0),
    ((66, 10, 9), (0, 0, 0), "random", 6.0, 25.0),
    ((20, 5, 6), (2, 2, 2), "gradient", 5.0, 25.0),
    ((131, 70, 11), (8, 8, 3), "random", 8.0, 25.0),
    # box of 2 x 62 + 12 columns: both 8-column x strips take 6 of the
    # leftover columns into their 14-column lane groups (as 77 x 37 x 19 does
    # on one side)
    ((152, 12, 10), (8, 3, 2), "random", 6.0, 25.0),
]


def _model(kind, dims, h, seed=11):
    if kind == "gradient":
        return synth.gradient_z(dims, h, 1500.0, 0.7)
    return synth.random_field_model(dims, h, seed=seed)


@pytest.mark.parametrize("dims,npml,kind,f,h", CASES)
def test_index_bit_exact(ctx, table, oracle_table, dims, npml, kind, f, h):
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    idx_o, ncl = O.select_index(c, f, h, 3.0, 0.05, len(oracle_table[0]))
    assert np.array_equal(op.index().astype(np.int64), idx_o.ravel())
    assert op.info()["n_clamped"] == ncl


def test_index_bit_exact_near_ties(ctx, table):
    """Velocities a few ulps either side of the table midpoints."""
    f, h = 5.0, 25.0
    k = np.arange(0, 340)
    mids = (3.0 + (k + 0.5) * 0.05) * f * h
    c = np.concatenate([np.nextafter(mids.astype(np.float32), np.float32(0)), mids.astype(np.float32),
                        np.nextafter(mids.astype(np.float32), np.float32(1e9))])
    n = 27 * ((len(c) + 26) // 27)
    c = np.resize(c, n).reshape(-1, 3, 9)
    op = ctx.assemble(table, c, h, f, npml=0)
    idx_o, _ = O.select_index(c, f, h, 3.0, 0.05, 341)
    assert np.array_equal(op.index().astype(np.int64), idx_o.ravel())


@pytest.mark.parametrize("dims,npml,kind,f,h", CASES[:4])
def test_csr_export_matches_oracle(ctx, table, oracle_table, dims, npml, kind, f, h):
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    ip, ind, val = op.csr()
    ipo, indo, valo, _ = O.assemble_csr(c, f, h, npml, O.row_weights(
        "GA", O.select_index(c, f, h, 3.0, 0.05, 341)[0], oracle_table[2]))
    assert np.array_equal(ip, ipo) and np.array_equal(ind, indo)
    assert np.max(np.abs(val - valo)) <= 1e-12 * np.max(np.abs(valo))


@pytest.mark.parametrize("dims,npml,kind,f,h", CASES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_apply_fp64_and_fp32_match_oracle(ctx, table, oracle_table, dims, npml, kind, f, h, nrhs):
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml, store=("c64", "c128"))
    A = _oracle_rows(c, f, h, npml, oracle_table[2])
    N = int(np.prod(dims))
    u = synth.random_vectors(N, nrhs, seed=7)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()
    y64s = op.apply(ud, variant="stored").cpu().numpy()
    y32 = op.apply(ud.to(torch.complex64)).cpu().numpy()
    y32s = op.apply(ud.to(torch.complex64), variant="stored").cpu().numpy()
    for r in range(nrhs):
        assert _relerr(y64[r], y_ref[r]) <= 1e-12
        assert _relerr(y64s[r], y_ref[r]) <= 1e-12
        assert _relerr(y32[r], y_ref[r]) <= 1e-5
        assert _relerr(y32s[r], y_ref[r]) <= 1e-5


@pytest.mark.parametrize("mode", ["GAm", "fixed"])
def test_apply_weight_modes(ctx, table, oracle_table, mode):
    dims, npml, f, h = (40, 23, 12), (3, 3, 2), 6.0, 25.0
    c = _model("random", dims, h, seed=5)
    op = ctx.assemble(table, c, h, f, npml=npml, weights=mode)
    A = _oracle_rows(c, f, h, npml, oracle_table[2], mode=mode)
    u = synth.random_vectors(int(np.prod(dims)), 2, seed=8)
    y_ref = (A @ u.T).T
    y64 = op.apply(torch.from_numpy(u).cuda()).cpu().numpy()
    for r in range(2):
        assert _relerr(y64[r], y_ref[r]) <= 1e-12


def test_apply_full_size_gradient_sampled(ctx, table, oracle_table):
    """101^3 vertical gradient (h = 25 m, f = 5 Hz, 10-node PML): FP64 and
    FP32 apply on sampled rows (random interior rows, every PML corner and
    face class) against the oracle's rows, in the launch shape used for timing."""
    dims, npml, f, h = (101, 101, 101), 10, 5.0, 25.0
    c = synth.gradient_z(dims, h, 1500.0, 0.7)
    op = ctx.assemble(table, c, h, f, npml=npml)
    idx_o, _ = O.select_index(c, f, h, 3.0, 0.05, 341)
    assert np.array_equal(op.index().astype(np.int64), idx_o.ravel())
    N = 101 ** 3
    rng = np.random.default_rng(0)
    special = []
    for z in (0, 5, 10, 11, 50, 89, 90, 95, 100):
        for y in (0, 9, 10, 11, 50, 90, 100):
            for x in (0, 1, 10, 11, 50, 63, 64, 65, 90, 91, 100):
                special.append(x + 101 * (y + 101 * z))
    rows = np.unique(np.concatenate([rng.integers(0, N, 1500), special]))
    w = O.row_weights("GA", idx_o, oracle_table[2])
    A = O.assemble_rows(c, f, h, npml, w[rows], rows)
    u = synth.random_vectors(N, 2, seed=9)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()[:, rows]
    y32 = op.apply(ud.to(torch.complex64)).cpu().numpy()[:, rows]
    for r in range(2):
        assert _relerr(y64[r], y_ref[r]) <= 1e-12
        assert _relerr(y32[r], y_ref[r]) <= 1e-5


def test_apply_many_rhs_block_tiles_sampled(ctx, table, oracle_table):
    """64^3 random field, 6-node PML, 32 right-hand sides in one launch
    (2^23 point-RHS pairs: the launch takes the block-tile kernel with two
    rows per wavefront and 16-plane chunks): FP64 and FP32 applies on sampled
    rows of every right-hand side against the oracle, and each right-hand
    side equal to its own single-RHS launch (per-wavefront tiles) to FP32
    rounding."""
    dims, npml, f, h = (64, 64, 64), 6, 8.0, 25.0
    c = synth.random_field_model(dims, h, seed=31)
    op = ctx.assemble(table, c, h, f, npml=npml)
    N = int(np.prod(dims))
    nrhs = 32
    assert N * nrhs >= 2 ** 23
    idx_o, _ = O.select_index(c, f, h, 3.0, 0.05, 341)
    rows = np.unique(np.random.default_rng(4).integers(0, N, 400))
    w = O.row_weights("GA", idx_o, oracle_table[2])
    A = O.assemble_rows(c, f, h, npml, w[rows], rows)
    u = synth.random_vectors(N, nrhs, seed=12)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()
    u32 = ud.to(torch.complex64)
    y32 = op.apply(u32).cpu().numpy()
    for r in range(nrhs):
        assert _relerr(y64[r, rows], y_ref[r]) <= 1e-12
        assert _relerr(y32[r, rows], y_ref[r]) <= 1e-5
    for r in (0, 17, 31):
        y1 = op.apply(u32[r:r + 1].contiguous()).cpu().numpy()[0]
        assert _relerr(y32[r], y1) <= 1e-5


def test_apply_large_single_rhs_sampled(ctx, table, oracle_table):
    """256 x 256 x 128 random field (2^23 points), 8-node PML, one
    right-hand side: the launch takes the block-tile kernel with one row per
    wavefront and 32-plane chunks; FP64 and FP32 sampled rows against the
    oracle."""
    dims, npml, f, h = (256, 256, 128), 8, 8.0, 25.0
    c = synth.random_field_model(dims, h, seed=41)
    op = ctx.assemble(table, c, h, f, npml=npml)
    N = int(np.prod(dims))
    assert N >= 2 ** 23
    idx_o, _ = O.select_index(c, f, h, 3.0, 0.05, 341)
    rows = np.unique(np.random.default_rng(6).integers(0, N, 1200))
    w = O.row_weights("GA", idx_o, oracle_table[2])
    A = O.assemble_rows(c, f, h, npml, w[rows], rows)
    u = synth.random_vectors(N, 1, seed=14)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()[:, rows]
    y32 = op.apply(ud.to(torch.complex64)).cpu().numpy()[:, rows]
    assert _relerr(y64[0], y_ref[0]) <= 1e-12
    assert _relerr(y32[0], y_ref[0]) <= 1e-5


def test_apply_non_temporal_instances_sampled(ctx, table, oracle_table):
    """Launches whose vectors exceed the last-level cache run the kernel
    instances with non-temporal stores (several RHS groups) or non-temporal
    stores and per-point data (one group): 320 x 320 x 170 random field
    (17.4 M points), one RHS in FP32 and FP64, four RHS one per wavefront and
    four per wavefront; sampled rows against the oracle, and every RHS equal
    to its single-RHS launch to rounding."""
    dims, npml, f, h = (320, 320, 170), 8, 8.0, 25.0
    c = synth.random_field_model(dims, h, seed=43)
    op = ctx.assemble(table, c, h, f, npml=npml)
    N = int(np.prod(dims))
    assert 2 * N * 8 >= 256 << 20
    idx_o, _ = O.select_index(c, f, h, 3.0, 0.05, 341)
    rows = np.unique(np.random.default_rng(8).integers(0, N, 1500))
    w = O.row_weights("GA", idx_o, oracle_table[2])
    A = O.assemble_rows(c, f, h, npml, w[rows], rows)
    u = synth.random_vectors(N, 4, seed=15)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    u32 = ud.to(torch.complex64)
    y64 = op.apply(ud[:1].contiguous()).cpu().numpy()[0, rows]
    assert _relerr(y64, y_ref[0]) <= 1e-12
    y1 = op.apply(u32[:1].contiguous()).cpu().numpy()[0]
    assert _relerr(y1[rows], y_ref[0]) <= 1e-5
    for nb in (1, 4):
        op.set_rhs_block(nb)
        y4 = op.apply(u32).cpu().numpy()
        for r in range(4):
            assert _relerr(y4[r, rows], y_ref[r]) <= 1e-5
        assert _relerr(y4[0], y1) <= 1e-6


def test_apply_large_random_field_sampled(ctx, table, oracle_table):
    """201 x 201 x 101 heterogeneous model, 8-node PML, f = 8 Hz, 4 right-hand
    sides: sampled rows against the oracle."""
    dims, npml, f, h = (201, 201, 101), 8, 8.0, 25.0
    c = synth.random_field_model(dims, h, seed=21)
    op = ctx.assemble(table, c, h, f, npml=npml)
    idx_o, ncl = O.select_index(c, f, h, 3.0, 0.05, 341)
    assert np.array_equal(op.index().astype(np.int64), idx_o.ravel())
    N = int(np.prod(dims))
    rows = np.unique(np.random.default_rng(1).integers(0, N, 1500))
    w = O.row_weights("GA", idx_o, oracle_table[2])
    A = O.assemble_rows(c, f, h, npml, w[rows], rows)
    u = synth.random_vectors(N, 4, seed=10)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    y64 = op.apply(ud).cpu().numpy()[:, rows]
    y32 = op.apply(ud.to(torch.complex64)).cpu().numpy()[:, rows]
    for r in range(4):
        assert _relerr(y64[r], y_ref[r]) <= 1e-12
        assert _relerr(y32[r], y_ref[r]) <= 1e-5


@pytest.mark.parametrize("dims,npml,kind,f,h", [CASES[1], CASES[4]])
def test_apply_tile_shapes_agree(ctx, table, oracle_table, dims, npml, kind, f, h):
    """Every rows-per-wavefront choice of the tuner matches the oracle, the
    choices agree with each other to rounding, and one choice repeated is bit
    for bit the same; the tuner returns one of them."""
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    A = _oracle_rows(c, f, h, npml, oracle_table[2])
    N = int(np.prod(dims))
    u = synth.random_vectors(N, 2, seed=12)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        outs = []
        for ry in (1, 2, 3, 4):
            op.set_tuning("c64" if dt == torch.complex64 else "c128", ry)
            outs.append(op.apply(ud.to(dt)).cpu().numpy())
        again = op.apply(ud.to(dt)).cpu().numpy()
        assert np.array_equal(again, outs[-1])
        for o in outs:
            for r in range(2):
                assert _relerr(o[r], y_ref[r]) <= tol
                assert _relerr(o[r], outs[0][r]) <= tol
    assert op.tune(2, "c64") in (1, 2, 3, 4)


@pytest.mark.parametrize("dims,npml,kind,f,h", [CASES[1], CASES[4]])
def test_apply_zchunks_bit_identical(ctx, table, oracle_table, dims, npml, kind, f, h):
    """The z chunk of the work items (automatic, 2, 3, 7, the whole depth)
    changes only which wavefront computes a plane: every choice matches the
    oracle, the choices agree with each other to rounding (the unrolled z
    steps may fuse multiply-adds differently), and a repeated launch is bit
    for bit the same."""
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    A = _oracle_rows(c, f, h, npml, oracle_table[2])
    u = synth.random_vectors(int(np.prod(dims)), 2, seed=14)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        outs = []
        for zc in (0, 2, 3, 7, dims[2]):
            op.set_zchunk(zc)
            outs.append(op.apply(ud.to(dt)).cpu().numpy())
        again = op.apply(ud.to(dt)).cpu().numpy()
        assert np.array_equal(again, outs[-1])
        for o in outs:
            for r in range(2):
                assert _relerr(o[r], y_ref[r]) <= tol
                assert _relerr(o[r], outs[0][r]) <= tol
    op.set_zchunk(0)
    from paper_2108_08730_amd import _lib as L
    with pytest.raises(L.Helm27Error):
        op.set_zchunk(1)


@pytest.mark.parametrize("dims,npml,kind,f,h", [CASES[1], CASES[3], CASES[4]])
def test_kernel_variants_agree(ctx, table, oracle_table, dims, npml, kind, f, h):
    """The wavefront-per-tile kernel (alone and with box rows shared across
    the block in LDS) and the LDS-tiled kernel all match the oracle, for every
    rows-per-wavefront choice of the shared variant."""
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    A = _oracle_rows(c, f, h, npml, oracle_table[2])
    u = synth.random_vectors(int(np.prod(dims)), 2, seed=13)
    y_ref = (A @ u.T).T
    ud = torch.from_numpy(u).cuda()
    for v in (0, 1, 2):
        op.set_kernel_variant(v)
        for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
            for ry in ((1, 2, 3, 4) if v == 2 else (2,)):
                op.set_tuning("c64" if dt == torch.complex64 else "c128", ry)
                y = op.apply(ud.to(dt)).cpu().numpy()
                for r in range(2):
                    assert _relerr(y[r], y_ref[r]) <= tol
    op.set_tuning("c64", 2)
    op.set_tuning("c128", 1)
    op.set_kernel_variant(0)


def test_apply_rejects_bad_arguments(ctx, table):
    from paper_2108_08730_amd import _lib as L
    import ctypes as C
    c = synth.homogeneous((8, 8, 8), 2000.0)
    op = ctx.assemble(table, c, 20.0, 10.0, npml=2)
    u = torch.zeros((1, 512), dtype=torch.complex64, device="cuda")
    # same buffer in and out
    assert L.lib.helm27_apply(op.handle, C.c_void_p(u.data_ptr()), C.c_void_p(u.data_ptr()), 1, L.C64,
                              L.RECOMPUTE, None) == L.EINVAL
    # stored variant without stored coefficients
    y = torch.zeros_like(u)
    assert L.lib.helm27_apply(op.handle, C.c_void_p(u.data_ptr()), C.c_void_p(y.data_ptr()), 1, L.C64,
                              L.STORED, None) == L.EINVAL
    assert L.lib.helm27_apply(op.handle, C.c_void_p(u.data_ptr()), C.c_void_p(y.data_ptr()), 0, L.C64,
                              L.RECOMPUTE, None) == L.EINVAL


@pytest.mark.parametrize("on_device", [False, True])
def test_assemble_validates_velocity(ctx, table, on_device):
    """The model's range and validity are found on the device: G range from
    the exact float min / max, and a zero, negative, infinite or NaN velocity
    anywhere in the grid is rejected, from a host array or a device tensor."""
    from paper_2108_08730_amd import _lib as L
    dims, f, h = (30, 22, 17), 6.0, 25.0
    c = synth.random_field_model(dims, h, seed=8)
    src = torch.from_numpy(c).cuda() if on_device else c
    info = ctx.assemble(table, src, h, f, npml=3).info()
    assert info["g_min_model"] == float(c.min()) / (f * h)
    assert info["g_max_model"] == float(c.max()) / (f * h)
    for bad in (0.0, -1500.0, float("inf"), float("nan")):
        cb = c.copy()
        cb[9, 13, 21] = bad
        srcb = torch.from_numpy(cb).cuda() if on_device else cb
        with pytest.raises(L.Helm27Error) as e:
            ctx.assemble(table, srcb, h, f, npml=3)
        assert e.value.status == L.EINVAL


@pytest.mark.parametrize("dims,npml,kind,f,h", CASES)
def test_apply_rhs_block_match_oracle(ctx, table, oracle_table, dims, npml, kind, f, h):
    """Two and four right-hand sides per box wavefront (block tiles, one row
    per wavefront, coefficients formed once per point for the group) for 2, 5
    and 8 right-hand sides (last groups of 1 to 4 members), with automatic and
    explicit z chunks and both work-item orders: every right-hand side
    matches the oracle and the one-right-hand-side-per-wavefront launch to
    FP32 rounding, and the two orders agree bit for bit."""
    c = _model(kind, dims, h)
    op = ctx.assemble(table, c, h, f, npml=npml)
    A = _oracle_rows(c, f, h, npml, oracle_table[2])
    N = int(np.prod(dims))
    for nrhs in (2, 5, 8):
        u = synth.random_vectors(N, nrhs, seed=20 + nrhs)
        y_ref = (A @ u.T).T
        u32 = torch.from_numpy(u).cuda().to(torch.complex64)
        op.set_rhs_block(1)
        base = op.apply(u32).cpu().numpy()
        for nb in (2, 4):
            op.set_rhs_block(nb)
            for zc in (0, 3):
                op.set_zchunk(zc)
                outs = []
                for order in (1, 2):
                    op.set_rhs_order(order)
                    outs.append(op.apply(u32).cpu().numpy())
                # the item order changes only which wavefront computes a tile
                assert np.array_equal(outs[0], outs[1]), (nrhs, nb, zc)
                y = outs[0]
                for r in range(nrhs):
                    assert _relerr(y[r], y_ref[r]) <= 1e-5, (nrhs, nb, zc, r)
                    assert _relerr(y[r], base[r]) <= 1e-5, (nrhs, nb, zc, r)
        op.set_rhs_block(0)
        op.set_rhs_order(0)
        op.set_zchunk(0)
