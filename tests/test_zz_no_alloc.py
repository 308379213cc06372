"""The no-allocation index selection against helm27_assemble's index.

helm27_select_index_noalloc writes, with no device allocation, the per-point
table index that helm27_assemble stores (paper Sec. 3.1: each row takes the
table entry of its local G = c/(f h), nearest entry, ties upward), keeping
its partial counts in a file-scope device array of the library.  Checked
through the C ABI: two calls in a row, the second on a smaller input (the
array keeps the first call's records), each bit-exact against the index
helm27_assemble exports, with the same clamp count and model G range; a
call beyond the array's capacity and a host pointer are refused.
"""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _noalloc(L, ctx, tab, vel_dev, h, f, idx_dev, stats=True):
    st = L.IndexStats()
    rc = L.lib.helm27_select_index_noalloc(ctx.handle, tab.handle, C.c_void_p(vel_dev.data_ptr()),
                                           vel_dev.numel(), h, f, C.c_void_p(idx_dev.data_ptr()),
                                           C.byref(st) if stats else None, None)
    return rc, st


def test_noalloc_index_matches_assemble_two_calls():
    from paper_2108_08730_amd import _lib as L
    from paper_2108_08730_amd import api
    assert torch.cuda.is_available(), "the GPU tests need a GPU"
    ctx = api.Context(0)
    tab = ctx.build_table(3.0, 20.0, 0.05, 1e-3)
    # first call: 64 x 48 x 40 random field at 8 Hz (G below and above the
    # table, so some points clamp); second call: a smaller 20 x 17 x 9 model
    # a third call on the 1/G table axis (smaller still)
    tab_inv = ctx.build_table(0.0, 0.4, 0.001, 1e-3, spacing="invG")
    cases = [((64, 48, 40), 25.0, 8.0, 3, tab), ((20, 17, 9), 20.0, 6.0, 5, tab), ((12, 10, 8), 25.0, 30.0, 7, tab_inv)]
    for dims, h, f, seed, tab in cases:
        c = synth.random_field_model(dims, h, seed=seed)
        vel = torch.from_numpy(c).cuda().reshape(-1)
        idx = torch.full((vel.numel(),), -1, dtype=torch.int16, device="cuda")
        rc, st = _noalloc(L, ctx, tab, vel, h, f, idx)
        assert rc == L.OK, rc
        op = ctx.assemble(tab, c, h, f, npml=2)
        ref = op.index()
        got = idx.cpu().numpy().view(np.uint16)
        assert np.array_equal(got, ref.astype(np.uint16))
        info = op.info()
        assert st.n_clamped == info["n_clamped"]
        assert st.n_invalid == 0
        assert st.g_min_model == info["g_min_model"] and st.g_max_model == info["g_max_model"]
        if seed == 3:   # G reaches above the table's 20: some points clamp
            assert st.n_clamped > 0


def test_noalloc_index_rejects_bad_inputs():
    from paper_2108_08730_amd import _lib as L
    from paper_2108_08730_amd import api
    ctx = api.Context(0)
    tab = ctx.build_table(3.0, 20.0, 0.05, 1e-3)
    c = synth.random_field_model((16, 12, 10), 25.0, seed=2)
    vel = torch.from_numpy(c).cuda().reshape(-1)
    idx = torch.zeros(vel.numel(), dtype=torch.int16, device="cuda")
    # more points than the scratch array covers: refused before any launch
    rc = L.lib.helm27_select_index_noalloc(ctx.handle, tab.handle, C.c_void_p(vel.data_ptr()), (1 << 28) + 1,
                                           25.0, 6.0, C.c_void_p(idx.data_ptr()), None, None)
    assert rc == L.EINVAL
    # a host velocity array is refused
    rc = L.lib.helm27_select_index_noalloc(ctx.handle, tab.handle, c.ctypes.data_as(C.c_void_p), c.size,
                                           25.0, 6.0, C.c_void_p(idx.data_ptr()), None, None)
    assert rc == L.EINVAL
    # an invalid velocity is reported (and the index of the others still written)
    cb = c.copy()
    cb[3, 4, 5] = -1.0
    vb = torch.from_numpy(cb).cuda().reshape(-1)
    rc, st = _noalloc(L, ctx, tab, vb, 25.0, 6.0, idx)
    assert rc == L.EINVAL and st.n_invalid == 1
    # without stats the call only enqueues; after a sync the index is there
    rc, _ = _noalloc(L, ctx, tab, vel, 25.0, 6.0, idx, stats=False)
    assert rc == L.OK
    torch.cuda.synchronize()
    op = ctx.assemble(tab, c, 25.0, 6.0, npml=2)
    assert np.array_equal(idx.cpu().numpy().view(np.uint16), op.index().astype(np.uint16))
