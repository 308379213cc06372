"""Thin Python binding over the helm27 C ABI (marshalling only).

Every step of the path runs in libhelm27 (host C++ and HIP kernels); PyTorch
only provides device memory and the stream handle.
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Sequence

import numpy as np

from . import _lib as L

_WEIGHTS = {"GA": L.WEIGHTS_GA, "fixed": L.WEIGHTS_FIXED, "GAm": L.WEIGHTS_GAM}


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    if stream is None:
        torch = _torch()
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


_SPACING = {"G": L.SPACING_G, "invG": L.SPACING_INVG}


class Table:
    def __init__(self, handle):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def weights(self):
        """(w7 [n_g, 7], g_min, dg)."""
        n = C.c_int()
        g0 = C.c_double()
        dg = C.c_double()
        L.check(L.lib.helm27_table_weights(self._h, None, C.byref(n), C.byref(g0), C.byref(dg)), "table_weights")
        w = np.zeros((n.value, 7), np.float64)
        L.check(L.lib.helm27_table_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_double)), None, None, None))
        return w, g0.value, dg.value

    def axis(self):
        """(spacing "G" | "invG", first abscissa, step, entries)."""
        sp, v0, dv, n = C.c_int(), C.c_double(), C.c_double(), C.c_int()
        L.check(L.lib.helm27_table_axis(self._h, C.byref(sp), C.byref(v0), C.byref(dv), C.byref(n)), "table_axis")
        return ("G" if sp.value == L.SPACING_G else "invG"), v0.value, dv.value, n.value

    def close(self):
        if self._h:
            L.lib.helm27_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    def __init__(self, handle, ctx):
        self._h = handle
        self._ctx = ctx     # keep the context alive
        d = L.OpDesc()
        L.check(L.lib.helm27_op_info(handle, C.byref(d)), "op_info")
        self.nx, self.ny, self.nz = d.nx, d.ny, d.nz
        self.N = d.nx * d.ny * d.nz
        self.h, self.freq = d.h, d.freq

    @property
    def handle(self):
        return self._h

    def table_weights(self):
        """Weights [n_g, 7] of the table the operator uses (widened under extend_table)."""
        n = self.info()["n_g"]
        w = np.zeros((n, 7), np.float64)
        L.check(L.lib.helm27_op_table_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_double))), "op_table_weights")
        return w

    def info(self):
        d = L.OpDesc()
        L.check(L.lib.helm27_op_info(self._h, C.byref(d)), "op_info")
        return {f: getattr(d, f) for f, _ in L.OpDesc._fields_}

    def index(self):
        out = np.zeros(self.N, np.uint16)
        L.check(L.lib.helm27_export_index(self._h, out.ctypes.data_as(C.c_void_p)), "export_index")
        return out

    def csr(self):
        nnz = C.c_int64()
        L.check(L.lib.helm27_export_csr(self._h, C.byref(nnz), None, None, None), "export_csr")
        indptr = np.zeros(self.N + 1, np.int64)
        indices = np.zeros(nnz.value, np.int64)
        vals = np.zeros(nnz.value, np.complex128)
        L.check(L.lib.helm27_export_csr(self._h, C.byref(nnz), indptr.ctypes.data_as(C.c_void_p),
                                        indices.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p)),
                "export_csr")
        return indptr, indices, vals

    def apply(self, u, y=None, variant="recompute", stream=None):
        """y = A u for a device tensor u of shape [nrhs, N] (or [N]), complex64 or
        complex128."""
        torch = _torch()
        if u.dim() == 1:
            u = u.view(1, -1)
        assert u.is_cuda and u.is_contiguous() and u.shape[1] == self.N
        if u.dtype == torch.complex64:
            dt = L.C64
        elif u.dtype == torch.complex128:
            dt = L.C128
        else:
            raise TypeError(u.dtype)
        if y is None:
            y = torch.empty_like(u)
        var = {"recompute": L.RECOMPUTE, "stored": L.STORED, "stored_t": L.STORED_T}[variant]
        L.check(L.lib.helm27_apply(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(y.data_ptr()), u.shape[0], dt,
                                   var, _stream_handle(stream)), "apply")
        return y

    def set_tuning(self, dtype, rows_per_wave):
        dt = L.C64 if dtype in ("c64", L.C64) else L.C128
        L.check(L.lib.helm27_set_tuning(self._h, dt, rows_per_wave), "set_tuning")

    def set_kernel_variant(self, variant):
        L.check(L.lib.helm27_set_kernel_variant(self._h, variant), "set_kernel_variant")

    def set_zchunk(self, zchunk):
        """z planes per work item of the wavefront kernel (0 = automatic)."""
        L.check(L.lib.helm27_set_zchunk(self._h, zchunk), "set_zchunk")

    def set_rhs_block(self, nb):
        """Right-hand sides per box wavefront of FP32 launches: 1, 2, 4, or 0 (automatic)."""
        L.check(L.lib.helm27_set_rhs_block(self._h, nb), "set_rhs_block")

    def set_attenuation(self, Q):
        """Constant-Q attenuation, complex velocity c (1 - i/(2Q)); Q = 0: none."""
        L.check(L.lib.helm27_set_attenuation(self._h, float(Q)), "set_attenuation")

    def set_rhs_order(self, order):
        """Multi-RHS work-item order: 2 right-hand side slowest, 1 fastest, 0 automatic."""
        L.check(L.lib.helm27_set_rhs_order(self._h, order), "set_rhs_order")

    def tune(self, nrhs=1, dtype="c64", stream=None):
        dt = L.C64 if dtype in ("c64", L.C64) else L.C128
        best = C.c_int()
        L.check(L.lib.helm27_tune(self._h, nrhs, dt, _stream_handle(stream), C.byref(best)), "tune")
        return best.value

    def solve(self, sources: Sequence[Sequence[int]], amps=None, out=None, stream=None, **opts):
        """Solve for point sources (i, j, k); returns (u [nrhs, N] complex128
        device tensor, stats dict)."""
        torch = _torch()
        n = len(sources)
        src = np.zeros((n, 5), np.float64)
        for s, p in enumerate(sources):
            src[s, :3] = p
            a = 1.0 if amps is None else amps[s]
            src[s, 3] = np.real(a)
            src[s, 4] = np.imag(a)
        if out is None:
            out = torch.empty((n, self.N), dtype=torch.complex128, device="cuda")
        o = solve_opts(**opts)
        st = L.SolveStats()
        status = L.lib.helm27_solve(self._h, src.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(out.data_ptr()),
                                    n, C.byref(o), C.byref(st), _stream_handle(stream))
        stats = {f: getattr(st, f) for f, _ in L.SolveStats._fields_}
        stats["status"] = status
        if status not in (L.OK, L.ENOCONV):
            L.check(status, "solve")
        return out, stats

    def solve_rhs(self, b, out=None, stream=None, **opts):
        torch = _torch()
        if b.dim() == 1:
            b = b.view(1, -1)
        assert b.is_cuda and b.dtype == torch.complex128 and b.is_contiguous()
        if out is None:
            out = torch.empty_like(b)
        o = solve_opts(**opts)
        st = L.SolveStats()
        status = L.lib.helm27_solve_rhs(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr()), b.shape[0],
                                        C.byref(o), C.byref(st), _stream_handle(stream))
        stats = {f: getattr(st, f) for f, _ in L.SolveStats._fields_}
        stats["status"] = status
        if status not in (L.OK, L.ENOCONV):
            L.check(status, "solve_rhs")
        return out, stats

    def close(self):
        if self._h:
            L.lib.helm27_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_many(ops, sources, **opts):
    """helm27_solve_many: ops[k] (distinct operators, e.g. one model at several
    frequencies) with point sources sources[k]; returns ([u_k], [stats_k])."""
    torch = _torch()
    n = len(ops)
    srcs, outs = [], []
    for op, sl in zip(ops, sources):
        a = np.zeros((len(sl), 5), np.float64)
        for s, p in enumerate(sl):
            a[s, :3] = p
            a[s, 3] = 1.0
        srcs.append(a)
        outs.append(torch.empty((len(sl), op.N), dtype=torch.complex128, device="cuda"))
    P = C.c_void_p
    h_ops = (P * n)(*[op.handle for op in ops])
    h_src = (C.POINTER(C.c_double) * n)(*[a.ctypes.data_as(C.POINTER(C.c_double)) for a in srcs])
    h_n = (C.c_int * n)(*[a.shape[0] for a in srcs])
    h_u = (P * n)(*[P(o.data_ptr()) for o in outs])
    o = solve_opts(**opts)
    st = (L.SolveStats * n)()
    status = L.lib.helm27_solve_many(h_ops, n, h_src, h_n, h_u, C.byref(o), st)
    if status not in (L.OK, L.ENOCONV):
        L.check(status, "solve_many")
    stats = [{f: getattr(st[k], f) for f, _ in L.SolveStats._fields_} for k in range(n)]
    return outs, stats


def apply_many(ops, us, ys=None, stream=None):
    """helm27_apply_many: y_k = A_k u_k for every operator in fused launches.
    us[k]: device tensor [nrhs_k, N_k] (or [N_k]), all complex64 or all
    complex128; returns the list of outputs."""
    torch = _torch()
    n = len(ops)
    us = [u.view(1, -1) if u.dim() == 1 else u for u in us]
    if len(us) != n:
        raise ValueError("one input per operator")
    dts = {u.dtype for u in us}
    if len(dts) != 1 or not dts <= {torch.complex64, torch.complex128}:
        raise TypeError("inputs must all be complex64 or all complex128")
    for op, u in zip(ops, us):
        assert u.is_cuda and u.is_contiguous() and u.shape[1] == op.N
    if ys is None:
        ys = [torch.empty_like(u) for u in us]
    dt = L.C64 if us[0].dtype == torch.complex64 else L.C128
    P = C.c_void_p
    h_ops = (P * n)(*[op.handle for op in ops])
    h_u = (P * n)(*[P(u.data_ptr()) for u in us])
    h_y = (P * n)(*[P(y.data_ptr()) for y in ys])
    h_n = (C.c_int * n)(*[u.shape[0] for u in us])
    L.check(L.lib.helm27_apply_many(h_ops, n, h_u, h_y, h_n, dt, _stream_handle(stream)), "apply_many")
    return ys


def _check_device_velocity(vel):
    """A device velocity is read in place as float32 [nz][ny][nx]."""
    torch = _torch()
    if vel.dtype != torch.float32 or not vel.is_contiguous() or vel.dim() != 3:
        raise TypeError("device velocity must be a contiguous float32 tensor of shape [nz, ny, nx]")


def solve_opts(**kw):
    o = L.SolveOpts()
    L.lib.helm27_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "precision":
            v = {"mixed": L.C64, "fp64": L.C128, L.C64: L.C64, L.C128: L.C128}[v]
        setattr(o, k, v)
    return o


class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = C.c_void_p()
        L.check(L.lib.helm27_create(C.byref(h), device, hbm_budget), "create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def build_table(self, g_min=3.0, g_max=20.0, dg=0.05, lam=1e-3, n_angles=5, angle_step_deg=10.0,
                    diff_order=1, spacing="G") -> Table:
        """spacing "G": abscissae G = g_min + i dg; "invG": s = 1/G = g_min + i dg."""
        opts = L.TableOpts(n_angles, angle_step_deg, diff_order, _SPACING[spacing])
        h = C.c_void_p()
        L.check(L.lib.helm27_build_table(self._h, g_min, g_max, dg, lam, C.byref(opts), C.byref(h)), "build_table")
        return Table(h)

    def fit_fixed(self, g_list, near=None, n_angles=5, angle_step_deg=10.0) -> Table:
        """Non-adaptive weights fitted jointly over g_list (helm27_fit_fixed):
        a one-entry table for assemble(weights="fixed").  near (five free
        weights) picks the least-squares solution closest to it when the fit
        is rank deficient (a single G), else the minimum-norm one."""
        g = np.ascontiguousarray(np.asarray(g_list, np.float64).ravel())
        opts = L.TableOpts(n_angles, angle_step_deg, 1, 0)
        nr = None
        if near is not None:
            nr = np.ascontiguousarray(np.asarray(near, np.float64).ravel()[:5])
        h = C.c_void_p()
        L.check(L.lib.helm27_fit_fixed(self._h, g.ctypes.data_as(C.POINTER(C.c_double)), g.size, C.byref(opts),
                                       nr.ctypes.data_as(C.POINTER(C.c_double)) if nr is not None else None,
                                       C.byref(h)), "fit_fixed")
        return Table(h)

    def table_from_weights(self, g_min, dg, w5, spacing="G") -> Table:
        w5 = np.ascontiguousarray(np.asarray(w5, np.float64).reshape(-1, 5))
        h = C.c_void_p()
        L.check(L.lib.helm27_table_from_weights(self._h, _SPACING[spacing], g_min, dg, w5.shape[0],
                                                w5.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)),
                "table_from_weights")
        return Table(h)

    def assemble(self, table: Table, vel, h: float, freq: float, npml=8, R=1e-3, c_ref=0.0,
                 weights="GA", store: Iterable[str] = (), extend_table=False, mass_form="b") -> Operator:
        """vel: numpy float32 [nz, ny, nx] or a device tensor of that shape."""
        if hasattr(vel, "data_ptr"):
            _check_device_velocity(vel)
            nz, ny, nx = vel.shape
            ptr = C.c_void_p(vel.data_ptr())
            keep = vel
        else:
            keep = np.ascontiguousarray(vel, dtype=np.float32)
            nz, ny, nx = keep.shape
            ptr = keep.ctypes.data_as(C.c_void_p)
        if np.isscalar(npml):
            npml = (int(npml),) * 3
        p = L.Pml((C.c_int * 3)(*npml), R, c_ref)
        flags = _WEIGHTS[weights]
        for s in store:
            flags |= {"c64": L.STORE_C64, "c128": L.STORE_C128}[s]
        if extend_table:
            flags |= L.EXTEND_TABLE
        if mass_form == "a":
            flags |= L.MASS_A
        elif mass_form != "b":
            raise ValueError(mass_form)
        hnd = C.c_void_p()
        L.check(L.lib.helm27_assemble(self._h, table.handle, ptr, nx, ny, nz, h, freq, C.byref(p), flags,
                                      C.byref(hnd)), "assemble")
        del keep
        return Operator(hnd, self)

    def close(self):
        if self._h:
            L.lib.helm27_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop over a context (helm27_serve_*): submit solves at any time,
    poll or wait for their results."""

    def __init__(self, ctx: Context, max_slots=4, table=(2.5, 60.0, 0.05, 1e-3), max_cached_ops=8, max_chunk_rhs=0,
                 **solve):
        o = L.ServeOpts()
        L.lib.helm27_serve_opts_default(C.byref(o))
        o.max_slots = max_slots
        o.table_gmin, o.table_gmax, o.table_dg, o.table_lambda = table
        o.max_cached_ops = max_cached_ops
        o.max_chunk_rhs = max_chunk_rhs
        so = solve_opts(**solve)
        o.solve = so
        self._ctx = ctx
        self._keep = {}
        L.check(L.lib.helm27_serve_start(ctx.handle, C.byref(o)), "serve_start")
        self._running = True

    def submit(self, vel, h, freq, sources, amps=None, npml=8, R=1e-3, c_ref=0.0, model_key=0, out=None):
        """vel: numpy float32 [nz, ny, nx] or device tensor; returns (ticket,
        out tensor [nrhs, N] complex128 that receives the solution)."""
        torch = _torch()
        if hasattr(vel, "data_ptr"):
            _check_device_velocity(vel)
            nz, ny, nx = vel.shape
            vptr = C.cast(C.c_void_p(vel.data_ptr()), C.POINTER(C.c_float))
        else:
            vel = np.ascontiguousarray(vel, dtype=np.float32)
            nz, ny, nx = vel.shape
            vptr = vel.ctypes.data_as(C.POINTER(C.c_float))
        n = len(sources)
        src = np.zeros((n, 5), np.float64)
        for s, p in enumerate(sources):
            src[s, :3] = p
            a = 1.0 if amps is None else amps[s]
            src[s, 3], src[s, 4] = np.real(a), np.imag(a)
        if out is None:
            out = torch.empty((n, nx * ny * nz), dtype=torch.complex128, device="cuda")
        if np.isscalar(npml):
            npml = (int(npml),) * 3
        req = L.Request()
        req.vel = vptr
        req.nx, req.ny, req.nz = nx, ny, nz
        req.h, req.freq = h, freq
        req.pml = L.Pml((C.c_int * 3)(*npml), R, c_ref)
        req.src = src.ctypes.data_as(C.POINTER(C.c_double))
        req.nrhs = n
        req.model_key = model_key
        req.out = C.c_void_p(out.data_ptr())
        t = C.c_uint64()
        L.check(L.lib.helm27_serve_submit(self._ctx.handle, C.byref(req), C.byref(t)), "serve_submit")
        self._keep[t.value] = out
        return t.value, out

    @staticmethod
    def _res(r):
        d = {f: getattr(r, f) for f, _ in L.Result._fields_ if f != "stats"}
        d.update({f: getattr(r.stats, f) for f, _ in L.SolveStats._fields_})
        return d

    def poll(self, ticket):
        r = L.Result()
        st = L.lib.helm27_serve_poll(self._ctx.handle, ticket, C.byref(r))
        if st == L.EAGAIN:
            return None
        L.check(st, "serve_poll")
        self._keep.pop(ticket, None)   # the library no longer writes the output
        return self._res(r)

    def wait(self, ticket, timeout=600.0):
        r = L.Result()
        L.check(L.lib.helm27_serve_wait(self._ctx.handle, ticket, C.byref(r), timeout), "serve_wait")
        self._keep.pop(ticket, None)   # the library no longer writes the output
        return self._res(r)

    def stop(self):
        if self._running:
            L.check(L.lib.helm27_serve_stop(self._ctx.handle), "serve_stop")
            self._running = False
            self._keep.clear()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
