#!/usr/bin/env python3
"""Benchmark of the wavelength-adaptive 27-point Helmholtz path on one GPU.

One step = one pass of the whole path over the workload: build the weight
table (host, FP64), assemble the operator from the device-resident velocity
(per-point table index), and solve for the source to a relative residual of
1e-6 (complex-FP32 GMRES with multigrid preconditioning and FP64 iterative
refinement).  Workload: 101^3 grid, vertical gradient c(z) = 1500 + 0.7 z m/s,
h = 25 m, f = 5 Hz (G from 12 to 26), 10-node PML, one source near the top.

Printed (one JSON line): solves/s over the timed steps, p50/p99 step latency,
the apply throughput of the recompute stencil (Gpts/s) and its HBM roofline
fraction measured with HIP events on the stream it runs on, and the oracle's
CSR SpMV on the host cores as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "27-pt apply Gpts/s (frac HBM peak); solves/s + p50/p99 latency @ resid 1e-6"
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(name="gradz101", dims=(101, 101, 101), h=25.0, freq=5.0, npml=10, c0=1500.0, a=0.7,
                src=(50, 50, 11), tol=1e-6, table=(3.0, 30.0, 0.05, 1e-3))


def measured_traffic(key):
    """HBM bytes per launch of the apply kernel from the committed hardware-counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or
    None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "wave27_apply_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
        for src, digest in rec["sources_sha256"].items():
            with open(os.path.join(ROOT, src), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != digest:
                    return None
        return float(rec[key]["traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def _ensure_lib():
    lib = os.path.join(ROOT, "paper_2108_08730_amd", "libhelm27.so")
    if not os.path.exists(lib):
        from paper_2108_08730_amd.build import build
        build()


def apply_timing(op, torch, nrhs=1, reps=200, dtype=None, variant="recompute"):
    """Average duration of helm27_apply over `reps` launches bracketed by HIP
    events on the stream the kernels run on, and the algorithmic bytes of one
    launch (recompute: idx u16 + c f32 per point; stored: 27 complex
    coefficients per point; plus u in and y out per right-hand side)."""
    dtype = dtype or torch.complex64
    stream = torch.cuda.current_stream()
    u = torch.randn((nrhs, op.N), dtype=dtype, device="cuda")
    y = torch.empty_like(u)
    # warm-up: at least 5 launches and 50 ms (clocks and caches settle)
    t0 = time.perf_counter()
    k = 0
    while k < 5 or time.perf_counter() - t0 < 0.05:
        op.apply(u, y, variant=variant, stream=stream)
        k += 1
        if k % 5 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        op.apply(u, y, variant=variant, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    vb = 8 if dtype == torch.complex64 else 16
    per_point = (2 + 4) if variant == "recompute" else 27 * vb
    alg_bytes = (per_point + 2 * vb * nrhs) * op.N
    return sec, alg_bytes


def large_apply(ctx, torch, synth, dims, nrhs=1, reps=50, dtype="c64", variant="recompute"):
    """Apply on a large grid (working set well beyond the 256 MB MALL): seeded
    random-field model, h = 25 m, f = 10 Hz, 8-node PML."""
    h, f, npml = 25.0, 10.0, 8
    c = synth.random_field_model(dims, h, seed=3)
    tab = ctx.build_table(2.5, 60.0, 0.05, 1e-3)
    store = () if variant == "recompute" else (dtype,)
    op = ctx.assemble(tab, torch.from_numpy(c).cuda(), h, f, npml=npml, store=store)
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    sec, alg = apply_timing(op, torch, nrhs=nrhs, reps=reps, dtype=dt, variant=variant)
    achieved = alg / sec / 1e9
    return {"grid": list(dims), "nrhs": nrhs, "dtype": dtype, "variant": variant, "apply_us": sec * 1e6,
            "gpts": op.N * nrhs / sec / 1e9, "alg_bytes": alg, "GBs": achieved, "frac": achieved / HBM_PEAK_GBS}


def calibration_copy(torch, mib=256):
    """A plain device copy of known size, the reference for hardware byte counters."""
    calib = torch.empty(mib << 18, dtype=torch.float32, device="cuda")
    calib_dst = torch.empty_like(calib)
    for _ in range(3):
        calib_dst.copy_(calib)
    torch.cuda.synchronize()


def apply_only(args, torch, api, synth):
    dims = tuple(int(v) for v in args.grid.split(","))
    ctx = api.Context(0)
    calibration_copy(torch)
    print(json.dumps(large_apply(ctx, torch, synth, dims, args.nrhs, args.apply_reps, args.apply_dtype,
                                 args.apply_variant)), flush=True)


def solve_only(args, torch, api, synth):
    """One multi-RHS solve on the heterogeneous random-field model (the
    family of the 201x201x101 x 64-source and 400x400x200 x 16-source
    configurations): sources on a surface line, relative residual 1e-6,
    mixed precision; prints one JSON line with the solver statistics."""
    dims = tuple(int(v) for v in args.grid.split(","))
    h, npml = 25.0, 8
    ctx = api.Context(0)
    tab = ctx.build_table(2.5, 60.0, 0.05, 1e-3)
    c = synth.random_field_model(dims, h, seed=1)
    op = ctx.assemble(tab, torch.from_numpy(c).cuda(), h, args.freq, npml=npml)
    info = op.info()
    xs = np.linspace(npml + 2, dims[0] - npml - 3, args.nrhs).astype(int)
    src = [(int(x), dims[1] // 2, npml + 2) for x in xs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, st = op.solve(src, tol=1e-6, max_inner=args.max_inner, verbose=1)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    print(json.dumps({"grid": list(dims), "nrhs": args.nrhs, "freq": args.freq, "h": h, "npml": npml,
                      "g_range": [info["g_min_model"], info["g_max_model"]], "solve_s": sec,
                      "rhs_per_s": args.nrhs / sec, "inner_iters": st["inner_iters"],
                      "outer_iters": st["outer_iters"], "max_relres": st["max_relres"],
                      "converged": bool(st["converged"])}), flush=True)


def serving(args, torch, api, synth):
    """Serving mix: Poisson arrivals of solve requests over seeded random-field
    models (frequencies 2.5-10 Hz, h = 1500 / (4 f) so the smallest G is about
    4, grids 64^3 / 96^3 / 128^2 x 64, 1-16 surface sources each), served by
    the request loop (mixed precision, all of a request's sources as one
    multi-RHS solve, up to 4 requests on the device at once, admission by
    HBM footprint); then the same requests as plain FP64 single-RHS solves
    one after another.  Both reach relative residual 1e-6."""
    reqs = synth.serving_requests(args.serve_requests, seed=11, rate_hz=args.serve_rate,
                                  dims_choices=((64, 64, 64), (96, 96, 96), (128, 128, 64)), nrhs_max=16)
    models = [synth.random_field_model(r["dims"], r["h"], seed=r["model_seed"] % 1000003) for r in reqs]
    srcs = [synth.surface_sources(r["dims"], r["nrhs"], 9, 10) for r in reqs]
    table = (2.5, 60.0, 0.05, 1e-3)
    ctx = api.Context(0)
    srv = api.Server(ctx, max_slots=4, table=table, tol=1e-6)
    t0 = time.perf_counter()
    tickets = []
    for r, v, sr in zip(reqs, models, srcs):
        wait = t0 + r["t_arrival"] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(v, r["h"], r["freq"], sr, npml=8, model_key=r["id"] + 1)[0])
    res = [srv.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    srv.stop()
    lat = np.array([(x["t_done"] - x["t_submit"]) * 1e3 for x in res])
    nrhs_tot = int(sum(r["nrhs"] for r in reqs))
    ok = all(x["status"] == 0 and x["converged"] == 1 for x in res)
    # the same requests as plain FP64 single-RHS solves, one after another
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
        "mixed_multi_rhs_serving": {"rhs_per_s": nrhs_tot / wall, "requests_per_s": len(reqs) / wall,
                                    "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
                                    "p99_ms": float(np.percentile(lat, 99)), "all_converged": ok,
                                    "max_relres": max(x["max_relres"] for x in res)},
        "fp64_single_rhs": {"rhs_per_s": nrhs_tot / wall64, "wall_s": wall64, "all_converged": ok64,
                            "max_relres": worst},
        "speedup_rhs_per_s": (nrhs_tot / wall) / (nrhs_tot / wall64),
        "note": "serving wall time includes waiting for Poisson arrivals; FP64 baseline runs back to back",
    }


def cpu_baseline(c, W7, seconds=10.0):
    """The oracle (scipy CSR, FP64) on the host: assemble the same operator
    once, then repeat the SpMV y = A u for about `seconds`."""
    from oracle import operator as O
    from oracle import table as T  # noqa: F401
    wl = WORKLOAD
    gmin, gmax, dg, lam = wl["table"]
    idx, _ = O.select_index(c, wl["freq"], wl["h"], gmin, dg, len(W7))
    A = O.assemble(c, wl["freq"], wl["h"], wl["npml"], O.row_weights("GA", idx, W7))
    u = np.random.default_rng(0).standard_normal(A.shape[0]) + 0j
    A @ u
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        A @ u
        n += 1
    dt = (time.perf_counter() - t0) / n
    return dict(value=A.shape[0] / dt / 1e9, unit="Gpts/s", cores=1, kind="oracle",
                sample=f"scipy CSR SpMV (complex128, single-threaded) of the 101^3 operator, "
                       f"{n} repeats in {seconds:.0f} s after one assembly; compare with apply_gpts")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--apply-reps", type=int, default=200)
    ap.add_argument("--apply-only", action="store_true",
                    help="time only the FP32 apply on --grid (seeded random-field model, h=25 m, f=10 Hz, 8-node PML)")
    ap.add_argument("--grid", type=str, default="400,400,200")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--apply-dtype", choices=("c64", "c128"), default="c64")
    ap.add_argument("--apply-variant", choices=("recompute", "stored"), default="recompute")
    ap.add_argument("--no-large", action="store_true", help="skip the 400x400x200 apply roofline")
    ap.add_argument("--solve-only", action="store_true",
                    help="one multi-RHS solve on --grid with --nrhs surface sources at --freq")
    ap.add_argument("--freq", type=float, default=10.0)
    ap.add_argument("--max-inner", type=int, default=3000)
    ap.add_argument("--serve-requests", type=int, default=16, help="serving-mix requests (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="serving-mix Poisson arrival rate (1/s)")
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

    wl = WORKLOAD
    dims, h, f, npml = wl["dims"], wl["h"], wl["freq"], wl["npml"]
    c_host = synth.gradient_z(dims, h, wl["c0"], wl["a"])
    c_dev = torch.from_numpy(c_host).cuda()
    ctx = api.Context(0)
    gmin, gmax, dg, lam = wl["table"]

    phases = {"table": [], "assemble": [], "solve": []}

    def step():
        t0 = time.perf_counter()
        tab = ctx.build_table(gmin, gmax, dg, lam)
        t1 = time.perf_counter()
        op = ctx.assemble(tab, c_dev, h, f, npml=npml)
        t2 = time.perf_counter()
        u, st = op.solve([wl["src"]], tol=wl["tol"])
        t3 = time.perf_counter()
        phases["table"].append(t1 - t0)
        phases["assemble"].append(t2 - t1)
        phases["solve"].append(t3 - t2)
        return op, u, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for v in phases.values():
        v.clear()
    lat = []
    stats = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        op, u, stats = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start

    calibration_copy(torch, 64)

    # apply roofline on the workload's operator (launch shape of the solve's matvec)
    tab = ctx.build_table(gmin, gmax, dg, lam)
    op = ctx.assemble(tab, c_dev, h, f, npml=npml)
    sec, alg = apply_timing(op, torch, nrhs=1, reps=args.apply_reps)
    achieved = alg / sec / 1e9
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": "gradz101: 101^3 grid, c(z)=1500+0.7z m/s, h=25 m, f=5 Hz (G 12..26), 10-node PML, "
                        "1 point source at (50,50,11), rel. residual 1e-6",
            "table": {"g_min": gmin, "g_max": gmax, "dg": dg, "lambda": lam},
            "solver": "FP64 refinement around complex-FP32 GMRES(28) + shifted-Laplacian multigrid V-cycle (3 levels at this size), replayed from a hipGraph",
            "precision": "complex FP32 stencil/Krylov, FP64 residual and Givens",
        },
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "solve": {"inner_iters": stats["inner_iters"], "outer_iters": stats["outer_iters"],
                  "relres": stats["max_relres"], "converged": bool(stats["converged"])},
        "phase_ms": {k: float(np.mean(v) * 1e3) for k, v in phases.items()},
        "apply_gpts": op.N / sec / 1e9,
        "apply_us": sec * 1e6,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("gradz101"),
                     "kernel": "helm27_apply recompute FP32, 1 RHS (wave27 kernel, box and PML frame in one launch)",
                     "alg_bytes_per_launch": alg},
    }
    # the same apply with fixed (non-adaptive) weights and with stored coefficients
    variants = {"recompute_adaptive": {"gpts": op.N / sec / 1e9, "us": sec * 1e6}}
    op_f = ctx.assemble(tab, c_dev, h, f, npml=npml, weights="fixed")
    sf, _ = apply_timing(op_f, torch, nrhs=1, reps=args.apply_reps)
    variants["recompute_fixed_weights"] = {"gpts": op.N / sf / 1e9, "us": sf * 1e6}
    del op_f
    op_s = ctx.assemble(tab, c_dev, h, f, npml=npml, store=("c64",))
    ss, alg_s = apply_timing(op_s, torch, nrhs=1, reps=args.apply_reps, variant="stored")
    variants["stored_c64"] = {"gpts": op.N / ss / 1e9, "us": ss * 1e6, "alg_bytes": alg_s,
                              "GBs": alg_s / ss / 1e9, "frac": alg_s / ss / 1e9 / HBM_PEAK_GBS}
    del op_s
    out["apply_variants"] = variants
    del op, tab
    if not args.no_large:
        out["roofline_large"] = dict(large_apply(ctx, torch, synth, (400, 400, 200), reps=50), bound="hbm",
                                     peak=HBM_PEAK_GBS, unit="GB/s",
                                     traffic=measured_traffic("large_400x400x200"))
        out["roofline_stored_large"] = dict(large_apply(ctx, torch, synth, (400, 400, 200), reps=20,
                                                        variant="stored"), bound="hbm", peak=HBM_PEAK_GBS,
                                            unit="GB/s")
    if args.serve_requests > 0:
        out["serving"] = serving(args, torch, api, synth)
    if not args.no_cpu_baseline:
        W7 = ctx.build_table(gmin, gmax, dg, lam).weights()[0]
        out["cpu_baseline"] = cpu_baseline(c_host, W7, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
