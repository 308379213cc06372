#!/usr/bin/env python3
"""Benchmark of the wavelength-adaptive 27-point Helmholtz hot path on one GPU.

Headline (the JSON line's `value`): throughput of the matrix-free adaptive
27-point apply y = A u (complex FP32, coefficients recomputed from the
per-point table index and velocity) on the large single-frequency workload:
a 400 x 400 x 200 seeded random-field model (background 1500 -> 4500 m/s with
depth, Gaussian random field, four dipping interfaces, a 3500 m/s body,
clipped to [1500, 6500] m/s), h = 25 m, f = 10 Hz (G 6 .. 26), 8-node PML,
16 right-hand sides in one launch.  One step = one such apply; `value` is
points x right-hand sides per second.  The tile shape is the one the
library's autotuner (helm27_tune) picks for this launch.

Next to it: the roofline of that launch (algorithmic bytes per launch over
its average duration from HIP events on the stream it runs on, against the
8 TB/s HBM peak) with the counter-measured traffic from profiles/, the
single-RHS, fixed-weight and stored-coefficient applies of the same model,
the whole-path solve step (table + assembly + solve to 1e-6) on the 101^3
vertical-gradient workload (solves/s, p50/p99), the serving mix, and the
oracle's CSR SpMV on a slab of the same model on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "27-pt apply Gpts/s (frac HBM peak); solves/s + p50/p99 latency @ resid 1e-6"
HBM_PEAK_GBS = 8000.0

LARGE = dict(name="rf400x16", dims=(400, 400, 200), h=25.0, freq=10.0, npml=8, seed=3, nrhs=16,
             table=(5.0, 30.0, 0.05, 1e-3))
GRADIENT = dict(name="gradz101", dims=(101, 101, 101), h=25.0, freq=5.0, npml=10, c0=1500.0, a=0.7,
                src=(50, 50, 11), tol=1e-6, table=(3.0, 30.0, 0.05, 1e-3))


def _ensure_lib():
    lib = os.path.join(ROOT, "paper_2108_08730_amd", "libhelm27.so")
    if not os.path.exists(lib):
        from paper_2108_08730_amd.build import build
        build()


def measured_traffic(key, shape=None):
    """HBM bytes per launch of the apply kernel from the committed
    hardware-counter summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy
    of known size), or None when the kernel sources changed since the
    counters were taken or the launch runs a tile shape that was not
    profiled (an entry holds one shape, or several under "by_shape")."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wave27_apply_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        for src, digest in rec["sources_sha256"].items():
            with open(os.path.join(ROOT, src), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != digest:
                    return None
        entry = rec[key]
        for e in entry.get("by_shape", [entry]):
            if shape is None or e.get("shape") in (None, shape):
                return float(e["traffic_bytes"])
        return None
    except (OSError, KeyError, ValueError):
        return None


def timed_applies(op, torch, u, y, steps, warmup_s=0.05, variant="recompute"):
    """Average seconds per helm27_apply over `steps` launches, bracketed by
    HIP events on the stream the kernels run on (and device synchronisation
    on both sides), after at least 5 launches and `warmup_s` of warm-up."""
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    k = 0
    while k < 5 or time.perf_counter() - t0 < warmup_s:
        op.apply(u, y, variant=variant, stream=stream)
        k += 1
        if k % 5 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        op.apply(u, y, variant=variant, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def alg_bytes(N, nrhs, vb=8, variant="recompute"):
    """Algorithmic bytes of one apply: the per-point operator data (u16 table
    index + f32 velocity, or 27 stored complex coefficients) read once, each
    right-hand side read once and each output written once."""
    per_point = (2 + 4) if variant == "recompute" else 27 * vb
    return (per_point + 2 * vb * nrhs) * N


def shape_of(op):
    d = op.info()
    return {k: d[k] for k in ("auto_tile", "kernel_variant", "rows_fp32", "zchunk", "rhs_block", "rhs_order")}


def copy_shape(src, dst):
    """Give operator `dst` the explicit tile shape of `src`."""
    s = shape_of(src)
    dst.set_kernel_variant(s["kernel_variant"])
    dst.set_tuning("c64", s["rows_fp32"])
    dst.set_zchunk(s["zchunk"])
    dst.set_rhs_block(s["rhs_block"])
    dst.set_rhs_order(s["rhs_order"])


def calibration_copy(torch, mib=256):
    """A plain device copy of known size, the reference for hardware byte counters."""
    calib = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    calib_dst = torch.empty_like(calib)
    for _ in range(3):
        calib_dst.copy_(calib)
    torch.cuda.synchronize()


def large_model(synth, dims=None, seed=None):
    wl = LARGE
    return synth.random_field_model(dims or wl["dims"], wl["h"], seed=wl["seed"] if seed is None else seed)


def apply_only(args, torch, api, synth):
    """One apply configuration on the large model family (profiling entry):
    --grid, --nrhs, --apply-dtype, --apply-variant; --tune runs the autotuner
    first (as the headline does)."""
    wl = LARGE
    dims = tuple(int(v) for v in args.grid.split(","))
    c = large_model(synth, dims)
    ctx = api.Context(0)
    tab = ctx.build_table(*wl["table"])
    store = () if args.apply_variant == "recompute" else (args.apply_dtype,)
    op = ctx.assemble(tab, torch.from_numpy(c).cuda(), wl["h"], wl["freq"], npml=wl["npml"], store=store)
    dt = torch.complex64 if args.apply_dtype == "c64" else torch.complex128
    if args.tune:
        op.tune(args.nrhs, args.apply_dtype)
    elif args.shape:
        v, rows, zc, nb, order = (int(t) for t in args.shape.split(","))
        op.set_kernel_variant(v)
        op.set_tuning(args.apply_dtype, rows)
        op.set_zchunk(zc)
        op.set_rhs_block(nb)
        op.set_rhs_order(order)
    calibration_copy(torch)
    g = torch.Generator(device="cuda").manual_seed(1)
    u = torch.randn((args.nrhs, op.N), dtype=dt, device="cuda", generator=g)
    y = torch.empty_like(u)
    sec = timed_applies(op, torch, u, y, args.apply_reps, variant=args.apply_variant)
    alg = alg_bytes(op.N, args.nrhs, 8 if dt == torch.complex64 else 16, args.apply_variant)
    print(json.dumps({"grid": list(dims), "nrhs": args.nrhs, "dtype": args.apply_dtype,
                      "variant": args.apply_variant, "shape": shape_of(op), "apply_us": sec * 1e6,
                      "gpts": op.N * args.nrhs / sec / 1e9, "alg_bytes": alg, "GBs": alg / sec / 1e9,
                      "frac": alg / sec / 1e9 / HBM_PEAK_GBS}), flush=True)


def solve_only(args, torch, api, synth):
    """One multi-RHS solve on the random-field model family (sources on a
    surface line, relative residual 1e-6, mixed precision); one JSON line
    with the solver statistics."""
    dims = tuple(int(v) for v in args.grid.split(","))
    h, npml = 25.0, 8
    ctx = api.Context(0)
    tv = tuple(float(v) for v in args.table.split(","))
    tab = ctx.build_table(tv[0], tv[1], tv[2], tv[3], spacing=args.table_spacing)
    c = synth.random_field_model(dims, h, seed=args.model_seed)
    op = ctx.assemble(tab, torch.from_numpy(c).cuda(), h, args.freq, npml=npml, extend_table=args.extend_table)
    info = op.info()
    xs = np.linspace(npml + 2, dims[0] - npml - 3, args.nrhs).astype(int)
    src = [(int(x), dims[1] // 2, npml + 2) for x in xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    extra = {} if args.mg_levels is None else {"mg_levels": args.mg_levels}
    extra["mg_coarse_table"] = args.mg_coarse_table
    if args.max_outer is not None:
        extra["max_outer"] = args.max_outer
    if args.restart is not None:
        extra["restart"] = args.restart
    u, st = op.solve(src, tol=1e-6, max_inner=args.max_inner, verbose=1, **extra)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    print(json.dumps({"grid": list(dims), "nrhs": args.nrhs, "freq": args.freq, "h": h, "npml": npml,
                      "g_range": [info["g_min_model"], info["g_max_model"]], "solve_s": sec,
                      "rhs_per_s": args.nrhs / sec, "inner_iters": st["inner_iters"],
                      "outer_iters": st["outer_iters"], "max_relres": st["max_relres"],
                      "converged": bool(st["converged"]), "mg_levels": st["mg_levels"],
                      "coarse_clamped": st["coarse_clamped"], "coarse_tables": st["coarse_tables"],
                      "table": [args.table, args.table_spacing, bool(args.extend_table)],
                      "mg_coarse_table": args.mg_coarse_table}), flush=True)


def solve_large(torch, api, synth, ctx, c_dev):
    """The large single-frequency configuration solved once: the 400x400x200
    random-field model at 10 Hz with 16 surface sources as one multi-RHS
    batch, mixed precision to relative residual 1e-6 (FP64 residual on the
    device), table G in [2.5, 60]."""
    wl = LARGE
    tab = ctx.build_table(2.5, 60.0, 0.05, 1e-3)
    op = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"])
    src = synth.surface_sources(wl["dims"], wl["nrhs"], 9, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, st = op.solve(src, tol=1e-6, max_inner=6000)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    del u, op
    torch.cuda.empty_cache()
    return {"workload": "rf400x16 solve: 400x400x200 random field, f=10 Hz, 16 surface sources in one batch, "
                        "GMRES(28) + shifted-Laplacian multigrid, FP64 refinement, rel. residual 1e-6",
            "seconds": sec, "rhs_per_s": wl["nrhs"] / sec, "inner_iters": st["inner_iters"],
            "outer_iters": st["outer_iters"], "max_relres": st["max_relres"], "converged": bool(st["converged"]),
            "mg_levels": st["mg_levels"]}


def solve_steps(args, torch, api, synth, ctx):
    """The whole path on the 101^3 vertical gradient: table build (host FP64),
    assembly from the device-resident velocity, solve for one source to
    relative residual 1e-6; solves/s and p50/p99 step latency."""
    wl = GRADIENT
    dims, h, f, npml = wl["dims"], wl["h"], wl["freq"], wl["npml"]
    c_dev = torch.from_numpy(synth.gradient_z(dims, h, wl["c0"], wl["a"])).cuda()
    phases = {"table": [], "assemble": [], "solve": []}

    def step():
        t0 = time.perf_counter()
        tab = ctx.build_table(*wl["table"])
        t1 = time.perf_counter()
        op = ctx.assemble(tab, c_dev, h, f, npml=npml)
        t2 = time.perf_counter()
        u, st = op.solve([wl["src"]], tol=wl["tol"])
        t3 = time.perf_counter()
        phases["table"].append(t1 - t0)
        phases["assemble"].append(t2 - t1)
        phases["solve"].append(t3 - t2)
        return st

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    for v in phases.values():
        v.clear()
    lat = []
    st = None
    t_start = time.perf_counter()
    for _ in range(args.solve_steps):
        t0 = time.perf_counter()
        st = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    total = time.perf_counter() - t_start
    lat_ms = np.array(lat) * 1e3
    # error of the timed (mixed-precision, 1e-6) solution against an FP64 solve
    # of the same system to 1e-11 (untimed)
    tab = ctx.build_table(*wl["table"])
    op = ctx.assemble(tab, c_dev, h, f, npml=npml)
    um, _ = op.solve([wl["src"]], tol=wl["tol"])
    ur, st_r = op.solve([wl["src"]], tol=1e-11, precision="fp64", max_inner=3000)
    err = float(torch.linalg.vector_norm(um - ur) / torch.linalg.vector_norm(ur))
    del op, um, ur
    return {"workload": "gradz101: 101^3 grid, c(z)=1500+0.7z m/s, h=25 m, f=5 Hz (G 12..26), 10-node PML, "
                        "1 point source at (50,50,11), rel. residual 1e-6; step = table + assembly + solve",
            "solves_per_s": args.solve_steps / total, "steps": args.solve_steps,
            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "inner_iters": st["inner_iters"], "outer_iters": st["outer_iters"], "relres": st["max_relres"],
            "converged": bool(st["converged"]),
            "error_vs_fp64_solve": err, "fp64_reference_relres": st_r["max_relres"],
            "phase_ms": {k: float(np.mean(v) * 1e3) for k, v in phases.items()}}


def batched_small_grids(torch, api, synth, ctx, reps=50):
    """Eight small grids of the serving mix (64^3, 96^3 and 128^2 x 64 models,
    h = 1500 / (4 f), 4 right-hand sides each): eight helm27_apply launches
    one after another against one helm27_apply_many, complex FP32, timed with
    HIP events on the launching stream."""
    specs = [((64, 64, 64), 10.0), ((96, 96, 96), 7.5), ((128, 128, 64), 5.0), ((64, 64, 64), 6.0),
             ((96, 96, 96), 4.0), ((64, 64, 64), 8.0), ((128, 128, 64), 9.0), ((96, 96, 96), 3.0)]
    tab = ctx.build_table(2.5, 60.0, 0.05, 1e-3)
    ops, us, ys = [], [], []
    g = torch.Generator(device="cuda").manual_seed(5)
    for k, (dims, f) in enumerate(specs):
        h = 1500.0 / (4.0 * f)
        c = synth.random_field_model(dims, h, seed=100 + k)
        op = ctx.assemble(tab, c, h, f, npml=8)
        ops.append(op)
        us.append(torch.randn((4, op.N), dtype=torch.complex64, device="cuda", generator=g))
        ys.append(torch.empty_like(us[-1]))
    stream = torch.cuda.current_stream()

    def run(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    def singles():
        for op, u, y in zip(ops, us, ys):
            op.apply(u, y, stream=stream)

    t_single = run(singles)
    t_fused = run(lambda: api.apply_many(ops, us, ys, stream=stream))
    pts = sum(op.N * 4 for op in ops)
    return {"grids": [list(d) for d, _ in specs], "rhs_per_grid": 4,
            "separate_launches_us": t_single * 1e6, "fused_launch_us": t_fused * 1e6,
            "fused_gpts": pts / t_fused / 1e9, "speedup": t_single / t_fused}


def serving(args, torch, api, synth):
    """Serving mix: Poisson arrivals of solve requests over seeded random-field
    models (frequencies 2.5-10 Hz, h = 1500 / (4 f) so the smallest G is about
    4, grids 64^3 / 96^3 / 128^2 x 64, 1-16 surface sources each), served by
    the request loop (mixed precision, all of a request's sources as one
    multi-RHS solve, up to 4 requests on the device at once, admission by
    HBM footprint); first all submitted at once (the loop's capacity, the
    like-for-like throughput), then with the Poisson arrivals (latency under
    load); then the same requests as plain FP64 single-RHS solves one after
    another.  All reach relative residual 1e-6."""
    reqs = synth.serving_requests(args.serve_requests, seed=11, rate_hz=args.serve_rate,
                                  dims_choices=((64, 64, 64), (96, 96, 96), (128, 128, 64)), nrhs_max=16)
    models = [synth.random_field_model(r["dims"], r["h"], seed=r["model_seed"] % 1000003) for r in reqs]
    srcs = [synth.surface_sources(r["dims"], r["nrhs"], 9, 10) for r in reqs]
    table = (2.5, 60.0, 0.05, 1e-3)
    ctx = api.Context(0)

    def run(arrivals):
        srv = api.Server(ctx, max_slots=4, table=table, tol=1e-6)
        t0 = time.perf_counter()
        tickets = []
        for r, v, sr, ta in zip(reqs, models, srcs, arrivals):
            wait = t0 + ta - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(v, r["h"], r["freq"], sr, npml=8, model_key=r["id"] + 1)[0])
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
        srv.stop()
        return wall, res

    wall_cap, res_cap = run([0.0] * len(reqs))
    wall, res = run([r["t_arrival"] for r in reqs])
    lat = np.array([(x["t_done"] - x["t_submit"]) * 1e3 for x in res])
    lat_cap = np.array([(x["t_done"] - x["t_submit"]) * 1e3 for x in res_cap])
    nrhs_tot = int(sum(r["nrhs"] for r in reqs))
    ok = all(x["status"] == 0 and x["converged"] == 1 for x in res + res_cap)
    tab = ctx.build_table(*table)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    worst = 0.0
    ok64 = True
    for r, v, sr in zip(reqs, models, srcs):
        op = ctx.assemble(tab, v, r["h"], r["freq"], npml=8)
        for s1 in sr:
            _, st = op.solve([s1], tol=1e-6, precision="fp64")
            ok64 = ok64 and st["converged"] == 1
            worst = max(worst, st["max_relres"])
        del op
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t1
    return {
        "requests": len(reqs), "rhs": nrhs_tot, "arrival_rate_hz": args.serve_rate,
        "mixed_multi_rhs_capacity": {"rhs_per_s": nrhs_tot / wall_cap, "requests_per_s": len(reqs) / wall_cap,
                                     "wall_s": wall_cap, "p50_ms": float(np.percentile(lat_cap, 50)),
                                     "p99_ms": float(np.percentile(lat_cap, 99))},
        "mixed_multi_rhs_serving": {"rhs_per_s": nrhs_tot / wall, "requests_per_s": len(reqs) / wall,
                                    "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
                                    "p99_ms": float(np.percentile(lat, 99)), "all_converged": ok,
                                    "max_relres": max(x["max_relres"] for x in res + res_cap)},
        "fp64_single_rhs": {"rhs_per_s": nrhs_tot / wall64, "wall_s": wall64, "all_converged": ok64,
                            "max_relres": worst},
        "speedup_rhs_per_s": (nrhs_tot / wall_cap) / (nrhs_tot / wall64),
        "note": "speedup: the loop's capacity pass (all requests submitted at once) against the FP64 "
                "single-RHS solves back to back; the Poisson pass's wall time includes waiting for arrivals",
    }


def serving_config4(args, torch, api, synth):
    """The serving-mix configuration at full shape: seeded random-field models,
    frequencies uniform in 2.5-10 Hz, h = 1500 / (4 f) (smallest G = 4), grids
    64^3, 96^3, 128^3, 192^2 x 96 and 256^2 x 128, 1-128 surface sources per
    request (log-uniform).  Pass 1 submits every request at once and measures
    the capacity (requests/s); pass 2 replays the same requests with Poisson
    arrivals at `--serve-load` (0.7) of that capacity and reports p50/p99
    latency (submit to done).  Requests too large for half the HBM budget
    are solved in chunks of right-hand sides.  The FP64 single-RHS baseline
    solves the first source of the first `--serve-fp64-sample` requests one
    at a time."""
    n = args.serve_requests
    dims_choices = ((64, 64, 64), (96, 96, 96), (128, 128, 128), (192, 192, 96), (256, 256, 128))
    reqs = synth.serving_requests(n, seed=21, rate_hz=1.0, dims_choices=dims_choices, nrhs_max=128)
    models = []
    for k, r in enumerate(reqs):
        models.append(synth.random_field_model(r["dims"], r["h"], seed=r["model_seed"] % 1000003))
        print(f"serving: model {k + 1}/{n} {r['dims']}", file=sys.stderr, flush=True)
    srcs = [synth.surface_sources(r["dims"], r["nrhs"], 9, 10) for r in reqs]
    table = (2.5, 60.0, 0.05, 1e-3)
    # admission budget 200 GiB: the outputs (complex128 [nrhs][N] per request,
    # allocated at submission) live outside it
    ctx = api.Context(0, hbm_budget=200 << 30)

    def run(arrivals):
        srv = api.Server(ctx, max_slots=4, table=table, tol=1e-6)
        t0 = time.perf_counter()
        tickets = []
        for r, v, sr, ta in zip(reqs, models, srcs, arrivals):
            wait = t0 + ta - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(v, r["h"], r["freq"], sr, npml=8, model_key=0))
        res = []
        for k, (t, out) in enumerate(tickets):
            res.append(srv.wait(t, timeout=3600.0))
            del out
            print(f"serving: request {k + 1}/{n} done after {time.perf_counter() - t0:.1f} s "
                  f"(status {res[-1]['status']}, {res[-1]['inner_iters']} steps)", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        srv.stop()
        torch.cuda.empty_cache()
        lat = np.array([(x["t_done"] - x["t_submit"]) * 1e3 for x in res])
        return wall, lat, res

    nrhs_tot = int(sum(r["nrhs"] for r in reqs))
    wall1, lat1, res1 = run([0.0] * n)
    cap = n / wall1
    rate = args.serve_load * cap
    rng = np.random.Generator(np.random.PCG64(22))
    arr = np.cumsum(rng.exponential(1.0 / rate, n))
    wall2, lat2, res2 = run(list(arr))
    ok = all(x["status"] == 0 and x["converged"] == 1 for x in res1 + res2)
    # FP64 single-RHS baseline on a sample
    tab = ctx.build_table(*table)
    t64, n64, worst = 0.0, 0, 0.0
    for r, v, sr in list(zip(reqs, models, srcs))[:args.serve_fp64_sample]:
        op = ctx.assemble(tab, v, r["h"], r["freq"], npml=8)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st = op.solve([sr[0]], tol=1e-6, precision="fp64", max_inner=6000)
        torch.cuda.synchronize()
        t64 += time.perf_counter() - t1
        print(f"serving: fp64 sample {n64 + 1} {r['dims']} {time.perf_counter() - t1:.1f} s", file=sys.stderr,
              flush=True)
        n64 += 1
        worst = max(worst, st["max_relres"])
        del op
    # the mixed-precision single-RHS solve of the same sample, for the like-for-like per-RHS ratio
    t32 = 0.0
    for r, v, sr in list(zip(reqs, models, srcs))[:args.serve_fp64_sample]:
        op = ctx.assemble(tab, v, r["h"], r["freq"], npml=8)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        op.solve([sr[0]], tol=1e-6)
        torch.cuda.synchronize()
        t32 += time.perf_counter() - t1
        del op
    return {
        "requests": n, "rhs": nrhs_tot, "grids": [list(d) for d in dims_choices],
        "nrhs_per_request": [r["nrhs"] for r in reqs], "grid_points": [int(np.prod(r["dims"])) for r in reqs],
        "capacity_pass": {"wall_s": wall1, "requests_per_s": cap, "rhs_per_s": nrhs_tot / wall1,
                          "p50_ms": float(np.percentile(lat1, 50)), "p99_ms": float(np.percentile(lat1, 99))},
        "poisson_pass": {"load": args.serve_load, "rate_hz": rate, "wall_s": wall2, "requests_per_s": n / wall2,
                         "rhs_per_s": nrhs_tot / wall2, "p50_ms": float(np.percentile(lat2, 50)),
                         "p99_ms": float(np.percentile(lat2, 99)), "max_ms": float(lat2.max())},
        "all_converged": ok, "max_relres": max(x["max_relres"] for x in res1 + res2),
        "fp64_single_rhs_sample": {"solves": n64, "s_per_rhs": t64 / max(1, n64), "max_relres": worst},
        "mixed_single_rhs_sample": {"solves": n64, "s_per_rhs": t32 / max(1, n64)},
        "served_rhs_per_s_over_fp64_single": (nrhs_tot / wall1) * (t64 / max(1, n64)),
    }


HOMOG_SMALL = dict(n=25, c=2000.0, h=20.0, freq=10.0, npml=6, table=(3.0, 20.0, 0.05, 1e-3))


def synth_homogeneous(n, c):
    import synth
    return synth.homogeneous((n, n, n), c)


def solve_homog_small(torch, api, ctx, reps=20):
    """The small homogeneous point-source problem of the oracle's direct-solve
    baseline, solved on the GPU (mixed precision to relative residual 1e-8,
    table build and assembly included in each step)."""
    w = HOMOG_SMALL
    n = w["n"]
    c = synth_homogeneous(n, w["c"])
    src = [(n // 2,) * 3]

    def step():
        tab = ctx.build_table(*w["table"])
        op = ctx.assemble(tab, c, w["h"], w["freq"], npml=w["npml"])
        _, st = op.solve(src, tol=1e-8)
        return st

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    return {"workload": f"{n}^3 homogeneous, f={w['freq']:.0f} Hz, centre source, rel. residual 1e-8",
            "seconds": sec, "solves_per_s": 1.0 / sec, "inner_iters": st["inner_iters"],
            "max_relres": st["max_relres"]}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(c_large, seconds=10.0, planes=6):
    """The oracle on the host: its own weight table (dense least squares,
    FP64), its own CSR assembly of a slab of `planes` z-planes from the
    middle of the large model (same h, f, table and x/y PML), then the scipy
    CSR SpMV y = A U with the workload's 16 right-hand sides (complex128)
    repeated for about `seconds`."""
    from oracle import operator as O
    from oracle import table as T
    wl = LARGE
    gmin, gmax, dg, lam = wl["table"]
    Gs, W = T.build_table(gmin, gmax, dg, lam)
    W7 = T.complete_weights(W)
    nz = c_large.shape[0]
    z0 = nz // 2 - planes // 2
    cs = np.ascontiguousarray(c_large[z0:z0 + planes])
    idx, _ = O.select_index(cs, wl["freq"], wl["h"], gmin, dg, len(Gs))
    A = O.assemble(cs, wl["freq"], wl["h"], (wl["npml"], wl["npml"], 0), O.row_weights("GA", idx, W7))
    A = A.tocsr()
    rng = np.random.default_rng(0)
    U = rng.standard_normal((A.shape[0], wl["nrhs"])) + 1j * rng.standard_normal((A.shape[0], wl["nrhs"]))
    A @ U
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds or n < 3:
        A @ U
        n += 1
    dt = (time.perf_counter() - t0) / n
    # the oracle's direct solve (SuperLU, single-threaded) of a small
    # homogeneous point-source problem, the GPU leg "solve_homog25" solves
    # the same system
    from oracle import solve as S
    n3, hs, fs = HOMOG_SMALL["n"], HOMOG_SMALL["h"], HOMOG_SMALL["freq"]
    cs3 = synth_homogeneous(n3, HOMOG_SMALL["c"])
    Gs3, Wt3 = T.build_table(*HOMOG_SMALL["table"])
    idx3, _ = O.select_index(cs3, fs, hs, HOMOG_SMALL["table"][0], HOMOG_SMALL["table"][2], len(Gs3))
    A3 = O.assemble(cs3, fs, hs, HOMOG_SMALL["npml"], O.row_weights("GA", idx3, T.complete_weights(Wt3)))
    b3 = S.point_source_rhs((n3, n3, n3), hs, [(n3 // 2,) * 3])
    t1 = time.perf_counter()
    S.solve(A3, b3)
    t_solve = time.perf_counter() - t1
    return dict(value=A.shape[0] * wl["nrhs"] / dt / 1e9, unit="Gpts/s", cores=1, kind="oracle",
                solve={"workload": f"{n3}^3 homogeneous c={HOMOG_SMALL['c']:.0f} m/s, h={hs:.0f} m, f={fs:.0f} Hz, "
                                   f"{HOMOG_SMALL['npml']}-node PML, centre source (N = {len(Gs3)}-entry table)",
                       "method": "oracle sparse direct solve (scipy SuperLU, single-threaded)",
                       "seconds": t_solve, "solves_per_s": 1.0 / t_solve, "cores": 1},
                sample=f"oracle CSR SpMV (scipy, complex128, single-threaded) of its own assembly of a "
                       f"{cs.shape[2]}x{cs.shape[1]}x{planes} slab (z-planes {z0}..{z0 + planes - 1}) of the "
                       f"400x400x200 model with its own table, 16 right-hand sides, {n} repeats in "
                       f"{dt * n:.1f} s; points x RHS per second",
                nproc=os.cpu_count(), cpu_model=cpu_model())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed 16-RHS applies")
    ap.add_argument("--warmup", type=int, default=5, help="untimed applies before the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large-solve", action="store_true",
                    help="skip the 400x400x200 x 16 solve (about a minute)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--solve-steps", type=int, default=10, help="timed 101^3 solve steps (0: skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline apply (no single-RHS / fixed / stored applies)")
    ap.add_argument("--apply-only", action="store_true",
                    help="time only one apply on --grid of the large model family")
    ap.add_argument("--grid", type=str, default="400,400,200")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--tune", action="store_true", help="--apply-only: autotune the tile shape first")
    ap.add_argument("--shape", type=str, default="",
                    help="--apply-only: explicit tile shape 'variant,rows,zchunk,rhs_block,rhs_order'")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--apply-dtype", choices=("c64", "c128"), default="c64")
    ap.add_argument("--apply-variant", choices=("recompute", "stored"), default="recompute")
    ap.add_argument("--solve-only", action="store_true",
                    help="one multi-RHS solve on --grid with --nrhs surface sources at --freq")
    ap.add_argument("--freq", type=float, default=10.0)
    ap.add_argument("--max-inner", type=int, default=3000)
    ap.add_argument("--max-outer", type=int, default=None,
                    help="--solve-only: refinement steps (with a small --max-inner: a truncated solve to profile)")
    ap.add_argument("--restart", type=int, default=None, help="--solve-only: GMRES restart length")
    ap.add_argument("--table", type=str, default="2.5,60,0.05,1e-3",
                    help="--solve-only: table v_min,v_max,dv,lambda (G, or s = 1/G with --table-spacing invG)")
    ap.add_argument("--table-spacing", choices=("G", "invG"), default="G")
    ap.add_argument("--model-seed", type=int, default=1, help="--solve-only: random-field model seed")
    ap.add_argument("--extend-table", action="store_true",
                    help="--solve-only: widen the table (and the coarse levels' tables) to the model's G range")
    ap.add_argument("--mg-levels", type=int, default=None)
    ap.add_argument("--mg-coarse-table", type=int, default=0,
                    help="--solve-only: 1 = coarse levels take tables widened for their own G range")
    ap.add_argument("--serve-requests", type=int, default=16, help="serving-mix requests (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="serving-mix Poisson arrival rate (1/s)")
    ap.add_argument("--serve-config4", action="store_true",
                    help="only the full-shape serving mix: grids to 256^2 x 128, 1-128 sources, capacity pass "
                         "then Poisson arrivals at --serve-load of capacity (use --serve-requests 32)")
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-fp64-sample", type=int, default=6)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver has no multi-GPU "
              f"path (sources and frequencies would be split across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    _ensure_lib()
    import torch
    from paper_2108_08730_amd import api
    import synth

    if args.apply_only:
        apply_only(args, torch, api, synth)
        return
    if args.solve_only:
        solve_only(args, torch, api, synth)
        return
    if args.serve_config4:
        print(json.dumps({"serving_config4": serving_config4(args, torch, api, synth)}), flush=True)
        return

    t_bench = time.perf_counter()
    wl = LARGE
    nrhs = wl["nrhs"]
    c_host = large_model(synth)
    c_dev = torch.from_numpy(c_host).cuda()
    ctx = api.Context(0)
    tab = ctx.build_table(*wl["table"])
    op = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"])
    N = op.N
    info = op.info()
    g = torch.Generator(device="cuda").manual_seed(1)
    u = torch.randn((nrhs, N), dtype=torch.complex64, device="cuda", generator=g)
    y = torch.empty_like(u)
    t_tune = time.perf_counter()
    op.tune(nrhs, "c64")
    t_tune = time.perf_counter() - t_tune
    shape = shape_of(op)

    # headline: W untimed, K timed applies, synchronised on both sides
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        op.apply(u, y, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        op.apply(u, y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sec = e0.elapsed_time(e1) * 1e-3 / args.steps
    alg = alg_bytes(N, nrhs)
    achieved = alg / sec / 1e9
    out = {
        "metric": METRIC,
        "value": N * nrhs / sec / 1e9,
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "rf400x16: 400x400x200 seeded random-field model (1500-6500 m/s), h=25 m, f=10 Hz "
                        f"(G {info['g_min_model']:.2f}..{info['g_max_model']:.2f}), 8-node PML, 16 right-hand "
                        "sides per apply; step = one adaptive 27-point apply y = A u, complex FP32, "
                        "coefficients recomputed from the per-point table index and velocity",
            "table": {"g_min": wl["table"][0], "g_max": wl["table"][1], "dg": wl["table"][2],
                      "lambda": wl["table"][3], "n_clamped": info["n_clamped"]},
            "tile_shape": dict(shape, tuned_s=t_tune),
        },
        "wall_s_timed": wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(wl["name"], shape),
                     "kernel": "wave27_kernel (recompute FP32, box and PML frame in one launch), 16 RHS",
                     "alg_bytes_per_launch": alg,
                     "alg_bytes_per_point": "6 (u16 index + f32 velocity) + 16 per right-hand side"},
    }
    if not args.no_extras:
        ext = {}
        # the same launch shape with fixed (non-adaptive) weights: the paper's
        # claim that the adaptive stencil costs nothing extra, on the HBM-bound shape
        op_f = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"], weights="fixed")
        copy_shape(op, op_f)
        sf = timed_applies(op_f, torch, u, y, args.steps)
        ext["fixed_weights_16rhs"] = {"us": sf * 1e6, "gpts": N * nrhs / sf / 1e9,
                                      "adaptive_over_fixed_time": sec / sf}
        del op_f
        # single right-hand side (automatic shape)
        op1 = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"])
        u1 = u[:1].contiguous()
        y1 = torch.empty_like(u1)
        s1 = timed_applies(op1, torch, u1, y1, 4 * args.steps)
        a1 = alg_bytes(N, 1)
        ext["single_rhs"] = {"us": s1 * 1e6, "gpts": N / s1 / 1e9, "GBs": a1 / s1 / 1e9,
                             "frac": a1 / s1 / 1e9 / HBM_PEAK_GBS, "alg_bytes": a1,
                             "traffic": measured_traffic("large_400x400x200", shape_of(op1))}
        del op1, u1, y1
        # stored coefficients (27 complex FP32 per point), one right-hand side
        op_s = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"], store=("c64",))
        u1 = u[:1].contiguous()
        y1 = torch.empty_like(u1)
        ss = timed_applies(op_s, torch, u1, y1, 20, variant="stored")
        a_s = alg_bytes(N, 1, variant="stored")
        ext["stored_single_rhs"] = {"us": ss * 1e6, "gpts": N / ss / 1e9, "GBs": a_s / ss / 1e9,
                                    "frac": a_s / ss / 1e9 / HBM_PEAK_GBS, "alg_bytes": a_s}
        del op_s, u1, y1
        # complex-FP64 recompute apply, one right-hand side (6 + 32 B per point)
        op_d = ctx.assemble(tab, c_dev, wl["h"], wl["freq"], npml=wl["npml"])
        ud = u[:1].to(torch.complex128).contiguous()
        yd = torch.empty_like(ud)
        sd = timed_applies(op_d, torch, ud, yd, 4 * args.steps)
        a_d = alg_bytes(N, 1, vb=16)
        ext["fp64_single_rhs"] = {"us": sd * 1e6, "gpts": N / sd / 1e9, "GBs": a_d / sd / 1e9,
                                  "frac": a_d / sd / 1e9 / HBM_PEAK_GBS, "alg_bytes": a_d}
        del op_d, ud, yd
        ext["batched_small_grids"] = batched_small_grids(torch, api, synth, ctx)
        out["apply_variants"] = ext
    del op, u, y
    torch.cuda.empty_cache()

    def leg(name):
        print(f"bench: {name} ({time.perf_counter() - t_bench:.0f} s)", file=sys.stderr, flush=True)

    if args.solve_steps > 0:
        leg("101^3 solve steps")
        out["solve_gradz101"] = solve_steps(args, torch, api, synth, ctx)
    leg("25^3 solve")
    out["solve_homog25"] = solve_homog_small(torch, api, ctx)
    if not args.no_large_solve:
        leg("400x400x200 x 16 solve")
        out["solve_rf400x16"] = solve_large(torch, api, synth, ctx, c_dev)
    if args.serve_requests > 0:
        leg("serving mix")
        out["serving"] = serving(args, torch, api, synth)
    if not args.no_cpu_baseline:
        leg("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(c_host, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
