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


def _ensure_lib():
    lib = os.path.join(ROOT, "paper_2108_08730_amd", "libhelm27.so")
    if not os.path.exists(lib):
        from paper_2108_08730_amd.build import build
        build()


def apply_timing(op, torch, nrhs=1, reps=200, dtype=None):
    """Average duration of helm27_apply (recompute) over `reps` launches
    bracketed by HIP events on the stream the kernels run on."""
    dtype = dtype or torch.complex64
    stream = torch.cuda.current_stream()
    u = torch.randn((nrhs, op.N), dtype=dtype, device="cuda")
    y = torch.empty_like(u)
    for _ in range(5):
        op.apply(u, y, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        op.apply(u, y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    vb = 8 if dtype == torch.complex64 else 16
    alg_bytes = (2 + 4 + 2 * vb * nrhs) * op.N        # idx u16 + c f32 + u in + y out
    return sec, alg_bytes


def apply_only(args, torch, api, synth):
    """FP32 recompute apply on a large grid (working set well beyond the 256 MB
    MALL): seeded random-field model, h = 25 m, f = 10 Hz, 8-node PML."""
    dims = tuple(int(v) for v in args.grid.split(","))
    h, f, npml = 25.0, 10.0, 8
    c = synth.random_field_model(dims, h, seed=3)
    ctx = api.Context(0)
    tab = ctx.build_table(2.5, 60.0, 0.05, 1e-3)
    op = ctx.assemble(tab, torch.from_numpy(c).cuda(), h, f, npml=npml)
    calib = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    calib_dst = torch.empty_like(calib)
    for _ in range(3):
        calib_dst.copy_(calib)
    torch.cuda.synchronize()
    del calib, calib_dst
    dt = torch.complex64 if args.apply_dtype == "c64" else torch.complex128
    sec, alg = apply_timing(op, torch, nrhs=args.nrhs, reps=args.apply_reps, dtype=dt)
    achieved = alg / sec / 1e9
    print(json.dumps({"grid": dims, "nrhs": args.nrhs, "dtype": args.apply_dtype, "apply_us": sec * 1e6,
                      "gpts": op.N * args.nrhs / sec / 1e9, "alg_bytes": alg,
                      "GBs": achieved, "frac": achieved / HBM_PEAK_GBS}), flush=True)


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded path is a design "
              f"described in DESIGN.md and is not built", file=sys.stderr)
        sys.exit(2)

    _ensure_lib()
    import torch
    from paper_2108_08730_amd import api
    import synth

    if args.apply_only:
        apply_only(args, torch, api, synth)
        return

    wl = WORKLOAD
    dims, h, f, npml = wl["dims"], wl["h"], wl["freq"], wl["npml"]
    c_host = synth.gradient_z(dims, h, wl["c0"], wl["a"])
    c_dev = torch.from_numpy(c_host).cuda()
    ctx = api.Context(0)
    gmin, gmax, dg, lam = wl["table"]

    def step():
        tab = ctx.build_table(gmin, gmax, dg, lam)
        op = ctx.assemble(tab, c_dev, h, f, npml=npml)
        u, st = op.solve([wl["src"]], tol=wl["tol"])
        return op, u, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
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

    # calibration for hardware byte counters: a plain device copy of known size
    calib = torch.empty(16 << 20, dtype=torch.float32, device="cuda")
    calib_dst = torch.empty_like(calib)
    for _ in range(3):
        calib_dst.copy_(calib)
    torch.cuda.synchronize()

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
            "solver": "FP64 refinement around complex-FP32 GMRES(30) + 4-level shifted-Laplacian multigrid",
            "precision": "complex FP32 stencil/Krylov, FP64 residual and Givens",
        },
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "solve": {"inner_iters": stats["inner_iters"], "outer_iters": stats["outer_iters"],
                  "relres": stats["max_relres"], "converged": bool(stats["converged"])},
        "apply_gpts": op.N / sec / 1e9,
        "apply_us": sec * 1e6,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "helm27_apply recompute FP32, 1 RHS (plain-box + PML-frame launches)",
                     "alg_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        W7 = tab.weights()[0]
        out["cpu_baseline"] = cpu_baseline(c_host, W7, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
