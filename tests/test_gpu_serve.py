"""Serving loop on the GPU: results in a concurrent mix equal the same
requests solved alone; admission by HBM footprint; tickets and timestamps."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TABLE = (2.5, 60.0, 0.05, 1e-3)


def _requests():
    # (dims, h, f, npml, sources, seed)
    return [
        ((32, 30, 28), 25.0, 6.0, 5, [(16, 15, 8)], 1),
        ((40, 36, 30), 25.0, 5.0, 6, [(10, 18, 8), (30, 18, 8)], 2),
        ((28, 28, 28), 30.0, 4.0, 5, [(14, 14, 10)], 3),
        ((36, 32, 30), 25.0, 7.0, 6, [(12, 16, 9), (18, 16, 9), (24, 16, 9)], 4),
        ((30, 34, 26), 25.0, 6.0, 5, [(15, 17, 8)], 5),
        ((44, 40, 32), 25.0, 5.0, 6, [(22, 20, 8), (20, 20, 10)], 6),
    ]


@pytest.fixture(scope="module")
def ctx():
    from paper_2108_08730_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


def test_mix_equals_alone(ctx):
    from paper_2108_08730_amd import api
    reqs = _requests()
    vels = [synth.random_field_model(d, h, seed=s) for d, h, f, p, src, s in reqs]
    srv = api.Server(ctx, max_slots=3, table=TABLE, tol=1e-8)
    tickets = []
    for (d, h, f, p, src, s), v in zip(reqs, vels):
        tickets.append(srv.submit(v, h, f, src, npml=p, model_key=s))
    results = [srv.wait(t) for t, _ in tickets]
    mix = [out.cpu().numpy() for _, out in tickets]
    srv.stop()
    for r in results:
        assert r["status"] == 0 and r["converged"] == 1
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
    # each request alone, same table and options, on the plain API
    tab = ctx.build_table(*TABLE)
    for k, ((d, h, f, p, src, s), v) in enumerate(zip(reqs, vels)):
        op = ctx.assemble(tab, v, h, f, npml=p)
        u, st = op.solve(src, tol=1e-8)
        a = u.cpu().numpy()
        assert st["converged"] == 1
        assert np.linalg.norm(mix[k] - a) <= 1e-12 * np.linalg.norm(a)


def test_admission_by_footprint(ctx):
    """A budget that holds one request at a time: every request still
    completes, and admissions do not overlap."""
    from paper_2108_08730_amd import api
    small = api.Context(0, hbm_budget=60 << 20)
    srv = api.Server(small, max_slots=3, table=TABLE, tol=1e-6)
    d, h, f = (40, 40, 40), 25.0, 6.0
    v = synth.random_field_model(d, h, seed=7)
    tk = [srv.submit(v, h, f, [(20, 20, 10)], npml=6) for _ in range(3)]
    res = sorted((srv.wait(t) for t, _ in tk), key=lambda r: r["t_start"])
    srv.stop()
    for r in res:
        assert r["status"] == 0
    for a, b in zip(res, res[1:]):
        assert b["t_start"] >= a["t_done"] - 1e-3


def test_oversize_request_rejected(ctx):
    from paper_2108_08730_amd import api
    from paper_2108_08730_amd import _lib as L
    small = api.Context(0, hbm_budget=32 << 20)
    srv = api.Server(small, max_slots=1, table=TABLE)
    v = synth.homogeneous((96, 96, 96), 2000.0)
    with pytest.raises(L.Helm27Error) as e:
        srv.submit(v, 20.0, 10.0, [(48, 48, 48)], npml=8)
    assert e.value.status == L.EADMIT
    with pytest.raises(L.Helm27Error) as e:
        srv.submit(v, 20.0, 10.0, [(2, 48, 48)], npml=8)
    assert e.value.status == L.ERANGE
    assert L.lib.helm27_serve_poll(small.handle, 12345, None) == L.ENOTFOUND
    srv.stop()


def test_operator_reuse_same_result(ctx):
    """Two requests on the same model key reuse the resident operator and give
    the same answer as a fresh operator."""
    from paper_2108_08730_amd import api
    srv = api.Server(ctx, max_slots=1, table=TABLE, tol=1e-7)
    d, h, f = (34, 32, 30), 25.0, 6.0
    v = synth.random_field_model(d, h, seed=8)
    t1, o1 = srv.submit(v, h, f, [(17, 16, 9)], npml=5, model_key=99)
    srv.wait(t1)
    t2, o2 = srv.submit(v, h, f, [(17, 16, 9)], npml=5, model_key=99)
    r2 = srv.wait(t2)
    srv.stop()
    assert r2["status"] == 0
    assert torch.equal(o1, o2)


def test_served_results_certified_by_oracle(ctx):
    """Every result the request loop returns solves its own problem: the
    oracle assembles each request's operator with its own table (the server's
    table agrees with it to 1e-9) and its FP64 residual of the served
    solution meets the tolerance (1e-8 plus the table difference's share,
    1e-9)."""
    from paper_2108_08730_amd import api
    from oracle import operator as O
    from oracle import solve as S
    from oracle import table as T
    reqs = _requests()[:4]
    vels = [synth.random_field_model(d, h, seed=s) for d, h, f, p, src, s in reqs]
    srv = api.Server(ctx, max_slots=3, table=TABLE, tol=1e-8)
    tickets = [srv.submit(v, h, f, src, npml=p, model_key=s)
               for (d, h, f, p, src, s), v in zip(reqs, vels)]
    results = [srv.wait(t) for t, _ in tickets]
    outs = [out.cpu().numpy() for _, out in tickets]
    srv.stop()
    Gs, W = T.build_table(*TABLE)
    W7 = T.complete_weights(W)
    for (d, h, f, p, src, s), v, r, u in zip(reqs, vels, results, outs):
        assert r["status"] == 0 and r["converged"] == 1
        idx, _ = O.select_index(v, f, h, TABLE[0], TABLE[2], len(Gs))
        A = O.assemble(v, f, h, p, O.row_weights("GA", idx, W7))
        b = S.point_source_rhs(d, h, src)
        assert np.all(S.relative_residual(A, u.T, b) <= 1e-8 * 1.01 + 1e-9)


def test_request_split_into_rhs_chunks(ctx):
    """A request with more right-hand sides than a solve may take (here the
    cap max_chunk_rhs = 3; by default half the HBM budget decides) is solved
    in chunks of right-hand sides on one operator: 7 sources -> 3 + 3 + 1.
    Every right-hand side is certified by the oracle's FP64 residual and
    agrees with the same sources solved in one batch to the tolerance."""
    from paper_2108_08730_amd import api
    from oracle import operator as O
    from oracle import solve as S
    from oracle import table as T
    d, h, f, p = (40, 36, 30), 25.0, 5.0, 6
    v = synth.random_field_model(d, h, seed=12)
    src = [(x, 18, 8) for x in (8, 12, 16, 20, 24, 28, 31)]
    srv = api.Server(ctx, max_slots=2, table=TABLE, tol=1e-8, max_chunk_rhs=3)
    t, out = srv.submit(v, h, f, src, npml=p)
    r = srv.wait(t)
    srv.stop()
    assert r["status"] == 0 and r["converged"] == 1
    u = out.cpu().numpy()
    Gs, W = T.build_table(*TABLE)
    idx, _ = O.select_index(v, f, h, TABLE[0], TABLE[2], len(Gs))
    A = O.assemble(v, f, h, p, O.row_weights("GA", idx, T.complete_weights(W)))
    b = S.point_source_rhs(d, h, src)
    assert np.all(S.relative_residual(A, u.T, b) <= 1e-8 * 1.01 + 1e-9)
    tab = ctx.build_table(*TABLE)
    op = ctx.assemble(tab, v, h, f, npml=p)
    ub, st = op.solve(src, tol=1e-8)
    ub = ub.cpu().numpy()
    for k in range(len(src)):
        assert np.linalg.norm(u[k] - ub[k]) <= 1e-6 * np.linalg.norm(ub[k])
