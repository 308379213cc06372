// Krylov solve of [M + S] p = s (paper Sec. 2.1 / 3.1) on the GPU.
//
// The paper factorises the impedance matrix with a sparse direct solver; this
// solver is matrix-free and iterative:
//   * outer loop in FP64: r = b - A u with the FP64 stencil, stop when every
//     right-hand side has ||r|| / ||b|| <= tol, else solve A e = r / ||r||
//     approximately and update u += ||r|| e (iterative refinement);
//   * inner solve: restarted GMRES(m) in the inner precision (complex FP32 by
//     default), right-preconditioned, classical Gram-Schmidt with one
//     reorthogonalisation (CGS2), Hessenberg / Givens / triangular solve in
//     FP64 on the device, all right-hand sides advancing together;
//   * preconditioner: one V-cycle of geometric multigrid on the complex-shifted
//     operator S + (a + i b) k^2 M (a = 0.5, b = 1 by default), rediscretised on
//     every level (velocity injected, h doubled, the same weight table and the
//     same physical PML), damped-Jacobi smoothing with the same stencil kernel,
//     full-weighting restriction and trilinear prolongation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "krylov.h"

namespace h27 {

struct SolverState {
    // hierarchy (levels 1..L-1 owned here; level 0 is the operator's grid)
    int levels = 0;
    int req_levels = -1;             // levels asked for when the hierarchy was built
    int req_coarse_table = 0;        // coarse-table choice it was built with
    std::vector<GridOp> coarse;
    int64_t coarse_clamped = 0;      // coarse rows outside their table
    int coarse_tables = 0;           // coarse levels with their own widened table
    double last_est = 0;             // last inner solve: Givens residual estimate / its rhs norm (max over RHS)
    // workspace
    int nrhs = 0, m = 0, prec = 0;   // prec = sizeof(real) of the inner precision
    int64_t N = 0;
    std::vector<void*> bufs;         // every allocation, freed together
    void* V = nullptr;               // (m+1) x [nrhs][N]
    void* w = nullptr;
    void* e = nullptr;
    void* rin = nullptr;
    void* tmp = nullptr;
    std::vector<void*> X, T, B, Rr;  // per level
    // per level, one value per point: omega D^-1 of the shifted operator (the
    // first damped-Jacobi sweep from zero is dinv * b); null where the level
    // runs without the wavefront kernel.  Keyed by shift, omega, precision.
    std::vector<void*> Dv;
    bool dv_ok = false;
    double dv_key[3] = {0, 0, 0};
    void* vy = nullptr;              // dinv * vin, the V-cycle graph's first iterate
    void* arena = nullptr;           // the workspace's one device allocation (in bufs)
    size_t arena_size = 0, arena_used = 0;
    bool arena_plan = false;
    double2* r64 = nullptr;
    double* d_partial = nullptr;
    int max_blocks = 1024;
    double2* d_hcol = nullptr;
    double2* d_htmp = nullptr;
    double* d_nrm = nullptr;
    double* d_n0 = nullptr;          // ||w|| before / after the first Gram-Schmidt pass
    double* d_n1 = nullptr;
    double* d_beta = nullptr;
    double* d_est = nullptr;
    // residual estimates copied to pinned host memory each Arnoldi step, two
    // slots [2][nrhs] so the host checks step j - 1 while step j runs, then
    // one slot [nrhs] for the restart residual norms (checked after the
    // cycle's first step is queued)
    double* h_est = nullptr;
    hipEvent_t est_ev[2] = {nullptr, nullptr};
    hipEvent_t beta_ev = nullptr;
    double* d_rn = nullptr;
    double* d_bn = nullptr;
    double2* d_H = nullptr;
    double* d_cs = nullptr;
    double2* d_sn = nullptr;
    double2* d_g = nullptr;
    double2* d_y = nullptr;
    int64_t* d_lin = nullptr;
    double2* d_amp = nullptr;
    int src_cap = 0;
    double2* d_b = nullptr;          // point-source right-hand sides [src_cap][N]
    // captured V-cycle (hipGraph): reads vin, leaves its result in vgraph_out
    void* vin = nullptr;
    hipGraphExec_t vgraph = nullptr;
    void* vgraph_out = nullptr;
    double gkey_d[3] = {0, 0, 0};
    int gkey_i[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool graph_failed = false;
};

static void drop_graph(SolverState* S) {
    if (S->vgraph) hipGraphExecDestroy(S->vgraph);
    S->vgraph = nullptr;
    S->vgraph_out = nullptr;
}

static void free_workspace(SolverState* S) {
    drop_graph(S);
    S->vin = nullptr;
    if (S->h_est) hipHostFree(S->h_est);
    S->h_est = nullptr;
    S->Dv.clear();
    S->dv_ok = false;
    S->vy = nullptr;
    S->arena = nullptr;
    S->arena_size = S->arena_used = 0;
    for (void* p : S->bufs) hipFree(p);
    S->bufs.clear();
    S->X.clear();
    S->T.clear();
    S->B.clear();
    S->Rr.clear();
    S->nrhs = S->m = S->prec = 0;
}

static void free_hierarchy(SolverState* S) {
    drop_graph(S);
    for (GridOp& g : S->coarse) grid_free(&g);
    S->coarse.clear();
    S->levels = 0;
}

// Workspace buffers are carved from one device allocation (one hipMalloc
// and one hipFree per workspace instead of one per buffer): the layout runs
// once to size the arena (plan) and once to hand out 256-byte aligned
// sub-ranges.
static int alloc(SolverState* S, void** p, size_t bytes) {
    bytes = ((bytes ? bytes : 16) + 255) & ~static_cast<size_t>(255);
    if (S->arena_plan) {
        *p = nullptr;
        S->arena_size += bytes;
        return HELM27_OK;
    }
    if (S->arena_used + bytes > S->arena_size) {
        *p = nullptr;
        return HELM27_ENOMEM;
    }
    *p = static_cast<char*>(S->arena) + S->arena_used;
    S->arena_used += bytes;
    return HELM27_OK;
}

// Automatic depth: halve the grid while the coarser grid keeps at least
// 8192 points and 3 nodes per axis (at least two levels when possible, at
// most eight).  Coarse grids below that size cost a launch per sweep while
// doing almost no work.
static int auto_levels(const GridOp& g) {
    int nx = g.nx, ny = g.ny, nz = g.nz, levels = 1;
    while (levels < 8) {
        const int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
        if (cx < 3 || cy < 3 || cz < 3) break;
        if (levels >= 2 && static_cast<int64_t>(cx) * cy * cz < 8192) break;
        nx = cx;
        ny = cy;
        nz = cz;
        ++levels;
    }
    return levels;
}

// Coarse grids: node i of level l+1 sits on node 2i of level l.
// Each coarse level rediscretises the operator at its own h_l = 2^l h, so its
// rows have G = c/(f h_l).  They take the operator's table (clamped); with
// `widen` (mg_coarse_table = 1) a level whose G range that table does not
// reach gets a table widened for it (same axis grid and fit settings).  The
// rows that still fall outside are counted.
static int build_hierarchy(helm27_op* op, SolverState* S, int levels, bool widen_coarse, hipStream_t s) {
    free_hierarchy(S);
    S->coarse_clamped = 0;
    S->coarse_tables = 0;
    const GridOp* prev = &op->g;
    // select-index counters, 4 per level (clamped rows, invalid, min, max bits)
    const int n_lv = levels > 1 ? levels - 1 : 1;
    unsigned long long* d_cnt = nullptr;
    if (hipMalloc(&d_cnt, 4 * sizeof(unsigned long long) * n_lv) != hipSuccess) return HELM27_ENOMEM;
    if (hipMemsetAsync(d_cnt, 0, 4 * sizeof(unsigned long long) * n_lv, s) != hipSuccess) {
        hipFree(d_cnt);
        return HELM27_EDEVICE;
    }
    int st = HELM27_OK;
    const helm27_table& base = op->table;
    const bool widen = widen_coarse && base.lambda >= 0;
    S->coarse.reserve(levels > 1 ? levels - 1 : 0);
    for (int l = 1; l < levels; ++l) {
        const int cx = (prev->nx + 1) / 2, cy = (prev->ny + 1) / 2, cz = (prev->nz + 1) / 2;
        if (cx < 3 || cy < 3 || cz < 3) break;
        S->coarse.emplace_back();
        GridOp& c = S->coarse.back();
        c.nx = cx;
        c.ny = cy;
        c.nz = cz;
        c.N = static_cast<int64_t>(cx) * cy * cz;
        c.h = prev->h * 2.0;
        c.omega = prev->omega;
        c.R = prev->R;
        c.c_ref = prev->c_ref;
        c.mass_a = prev->mass_a;
        c.att_re = prev->att_re;
        c.att_im = prev->att_im;
        for (int a = 0; a < 3; ++a) {
            c.npml[a] = 0;
            c.pml_lo[a] = prev->pml_lo[a];
            c.pml_hi[a] = prev->pml_hi[a];
            c.pml_L[a] = prev->pml_L[a];
        }
        if (hipMalloc(&c.d_c, c.N * sizeof(float)) != hipSuccess ||
            hipMalloc(&c.d_idx, c.N * sizeof(uint16_t)) != hipSuccess) {
            st = HELM27_ENOMEM;
            break;
        }
        c.bytes += c.N * (sizeof(float) + sizeof(uint16_t));
        if ((st = inject_velocity(prev->d_c, prev->nx, prev->ny, c.d_c, cx, cy, cz, s))) break;
        const double fh = op->freq * c.h;
        const helm27_table* T = &base;
        helm27_table* own = nullptr;
        if (widen) {
            const bool inv = base.spacing == HELM27_SPACING_INVG;
            const double need_lo = inv ? fh / static_cast<double>(op->cmax) : static_cast<double>(op->cmin) / fh;
            const double need_hi = inv ? fh / static_cast<double>(op->cmin) : static_cast<double>(op->cmax) / fh;
            double v_min = 0;
            int n_w = 0;
            if ((st = widen_range(&base, need_lo, need_hi, &v_min, &n_w))) break;
            if (n_w != base.n_g) {
                if ((st = build_table_like(&base, v_min, n_w, &own))) break;
                T = own;
                ++S->coarse_tables;
            }
        }
        const int n_g = T->n_g;
        st = launch_select_index(c.d_c, c.d_idx, c.N, fh, T->g_min, T->dg, n_g, T->spacing, d_cnt + 4 * (l - 1), s);
        if (!st) st = grid_setup(&c, T->w7.data(), n_g, op->g.fixed);
        if (!st) {
            const int ia = host_index(op->cmin, fh, T->g_min, T->dg, n_g, T->spacing);
            const int ib = host_index(op->cmax, fh, T->g_min, T->dg, n_g, T->spacing);
            c.idx_lo = std::min(ia, ib);
            c.idx_hi = std::max(ia, ib);
        }
        delete own;
        if (st) break;
        prev = &c;
    }
    std::vector<unsigned long long> cnt(4 * static_cast<size_t>(n_lv), 0);
    if ((hipMemcpyAsync(cnt.data(), d_cnt, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s) !=
             hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess) &&
        st == HELM27_OK)
        st = HELM27_EDEVICE;
    hipFree(d_cnt);
    for (size_t l = 0; l < S->coarse.size(); ++l) S->coarse_clamped += static_cast<int64_t>(cnt[4 * l]);
    S->levels = 1 + static_cast<int>(S->coarse.size());
    return st;
}

static const GridOp& level_grid(const helm27_op* op, const SolverState* S, int l) {
    return l == 0 ? op->g : S->coarse[l - 1];
}

static int workspace_layout(helm27_op* op, SolverState* S, int nrhs, int m, int prec);

static int ensure_workspace(helm27_op* op, SolverState* S, int nrhs, int m, int prec) {
    if (S->nrhs == nrhs && S->m == m && S->prec == prec && S->N == op->g.N &&
        static_cast<int>(S->X.size()) == S->levels)
        return HELM27_OK;
    free_workspace(S);
    S->arena_plan = true;
    S->arena_size = 0;
    int st = workspace_layout(op, S, nrhs, m, prec);
    S->arena_plan = false;
    if (st) return st;
    if (hipMalloc(&S->arena, S->arena_size) != hipSuccess) {
        S->arena = nullptr;
        S->arena_size = 0;
        return HELM27_ENOMEM;
    }
    S->bufs.push_back(S->arena);
    S->arena_used = 0;
    if ((st = workspace_layout(op, S, nrhs, m, prec))) return st;
    if (hipHostMalloc(reinterpret_cast<void**>(&S->h_est), 3 * static_cast<size_t>(nrhs) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        S->h_est = nullptr;
        return HELM27_ENOMEM;
    }
    for (int k = 0; k < 2; ++k)
        if (!S->est_ev[k]) H27_CHECK_HIP(hipEventCreateWithFlags(&S->est_ev[k], hipEventDisableTiming));
    if (!S->beta_ev) H27_CHECK_HIP(hipEventCreateWithFlags(&S->beta_ev, hipEventDisableTiming));
    S->nrhs = nrhs;
    S->m = m;
    S->prec = prec;
    S->N = op->g.N;
    return HELM27_OK;
}

// The workspace layout: every device buffer of the solver for nrhs
// right-hand sides, restart m and inner precision prec (bytes per real).
static int workspace_layout(helm27_op* op, SolverState* S, int nrhs, int m, int prec) {
    const int64_t N = op->g.N;
    const size_t vb = static_cast<size_t>(2 * prec);   // complex element bytes
    const size_t vec = static_cast<size_t>(N) * nrhs * vb;
    int st;
    if ((st = alloc(S, &S->V, vec * (m + 1)))) return st;
    if ((st = alloc(S, &S->w, vec))) return st;
    if ((st = alloc(S, &S->e, vec))) return st;
    if ((st = alloc(S, &S->rin, vec))) return st;
    if ((st = alloc(S, &S->tmp, vec))) return st;
    if ((st = alloc(S, &S->vin, vec))) return st;
    if ((st = alloc(S, &S->vy, vec))) return st;
    S->Dv.assign(S->levels, nullptr);
    S->X.resize(S->levels);
    S->T.resize(S->levels);
    S->B.resize(S->levels);
    S->Rr.resize(S->levels);
    for (int l = 0; l < S->levels; ++l) {
        const size_t lv = static_cast<size_t>(level_grid(op, S, l).N) * nrhs * vb;
        if ((st = alloc(S, &S->X[l], lv))) return st;
        if ((st = alloc(S, &S->T[l], lv))) return st;
        if ((st = alloc(S, &S->Rr[l], lv))) return st;
        if (l > 0) {
            if ((st = alloc(S, &S->B[l], lv))) return st;
        } else {
            S->B[l] = nullptr;
        }
        const GridOp& Gl = level_grid(op, S, l);
        if (stencil_wave_path(Gl, prec == 8))
            if ((st = alloc(S, &S->Dv[l], static_cast<size_t>(Gl.N) * vb))) return st;
    }
    void* p;
    if ((st = alloc(S, &p, static_cast<size_t>(N) * nrhs * sizeof(double2)))) return st;
    S->r64 = static_cast<double2*>(p);
    S->max_blocks = 1024;
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * (m + 2 > 8 ? m + 2 : 8) * S->max_blocks * 2 * sizeof(double))))
        return st;
    S->d_partial = static_cast<double*>(p);
    const int ldh = m + 1;
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * ldh * sizeof(double2)))) return st;
    S->d_hcol = static_cast<double2*>(p);
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * ldh * sizeof(double2)))) return st;
    S->d_htmp = static_cast<double2*>(p);
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * ldh * sizeof(double2)))) return st;
    S->d_y = static_cast<double2*>(p);
    double* dd[7];
    for (int k = 0; k < 7; ++k) {
        if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * sizeof(double)))) return st;
        dd[k] = static_cast<double*>(p);
    }
    S->d_nrm = dd[0];
    S->d_beta = dd[1];
    S->d_est = dd[2];
    S->d_rn = dd[3];
    S->d_bn = dd[4];
    S->d_n0 = dd[5];
    S->d_n1 = dd[6];
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * (m + 1) * m * sizeof(double2)))) return st;
    S->d_H = static_cast<double2*>(p);
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * m * sizeof(double)))) return st;
    S->d_cs = static_cast<double*>(p);
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * m * sizeof(double2)))) return st;
    S->d_sn = static_cast<double2*>(p);
    if ((st = alloc(S, &p, static_cast<size_t>(nrhs) * (m + 1) * sizeof(double2)))) return st;
    S->d_g = static_cast<double2*>(p);
    return HELM27_OK;
}

struct Ctx {
    helm27_op* op;
    SolverState* S;
    const helm27_solve_opts* o;
    hipStream_t s;
    int nrhs;
};

// the physical operator of the solve (MODE_APPLY: y = A x, MODE_RESID:
// y = b - A x): the recompute kernels, or for the transposed problem the
// stored coefficients read transposed
template <typename R>
static int phys_apply(const Ctx& c, int mode, const void* x, void* y, const void* b) {
    if (c.o->transpose) {
        const void* coef = sizeof(R) == 4 ? c.op->d_coef_f : c.op->d_coef_d;
        if (!coef) return HELM27_EINVAL;
        return launch_apply_stored_t<R>(c.op->g, coef, x, y, mode == MODE_RESID ? b : nullptr, c.nrhs, c.s);
    }
    return launch_stencil<R>(c.op->g, mode, 1.0, 0.0, x, y, b, 0.0, c.nrhs, c.s);
}

// omega D^-1 of the shifted operator on every level that has a Dv buffer:
// the first-sweep kernel applied to b = 1 (recomputed when the shift, omega
// or the precision change).  Runs outside any graph recording.
template <typename R>
static int ensure_dinv(const Ctx& c) {
    SolverState* S = c.S;
    const double key[3] = {c.o->mg_shift_re, c.o->mg_shift, c.o->mg_omega};
    if (S->dv_ok && key[0] == S->dv_key[0] && key[1] == S->dv_key[1] && key[2] == S->dv_key[2]) return HELM27_OK;
    int st;
    for (int l = 0; l < S->levels && l < static_cast<int>(S->Dv.size()); ++l) {
        if (!S->Dv[l]) continue;
        const GridOp& G = level_grid(c.op, S, l);
        if ((st = fill_one<R>(S->Rr[l], G.N, c.s))) return st;
        if ((st = launch_stencil<R>(G, MODE_JACOBI0, key[0], key[1], nullptr, S->Dv[l], S->Rr[l], key[2], 1, c.s)))
            return st;
    }
    for (int k = 0; k < 3; ++k) S->dv_key[k] = key[k];
    S->dv_ok = true;
    return HELM27_OK;
}

static int level_pre(const Ctx& c, int l) {
    return l == c.S->levels - 1 ? c.o->mg_coarse_sweeps : c.o->mg_pre;
}

// One V-cycle on level l for right-hand side b (inner precision R); returns
// the buffer that holds the result.  y0 (optional) holds the first sweep
// dinv * b, formed by the kernel that produced b.
template <typename R>
static int vcycle(const Ctx& c, int l, const void* b, void** out, void* y0 = nullptr) {
    SolverState* S = c.S;
    const GridOp& G = level_grid(c.op, S, l);
    const int64_t bytes = G.N * c.nrhs * static_cast<int64_t>(2 * sizeof(R));
    void* x = S->X[l];
    void* t = S->T[l];
    int st;
    const bool coarsest = l == S->levels - 1;
    const double a = c.o->mg_shift_re, bshift = c.o->mg_shift;
    const int pre = level_pre(c, l);
    // the iterate starts at zero: the first sweep is omega D^-1 b = dinv * b
    const bool zero_sweep = pre > 0 && S->Dv[l];
    if (zero_sweep) {
        if (y0) {
            x = y0;
        } else if ((st = dinv_scale<R>(S->Dv[l], b, x, G.N, c.nrhs, c.s))) {
            return st;
        }
    } else if ((st = fill_zero(x, bytes, c.s))) {
        return st;
    }
    for (int k = zero_sweep ? 1 : 0; k < pre; ++k) {
        if ((st = launch_stencil<R>(G, MODE_JACOBI, a, bshift, x, t, b, c.o->mg_omega, c.nrhs, c.s))) return st;
        std::swap(x, t);
    }
    if (!coarsest) {
        const GridOp& Gc = level_grid(c.op, S, l + 1);
        if ((st = launch_stencil<R>(G, MODE_RESID, a, bshift, x, S->Rr[l], b, 0.0, c.nrhs, c.s))) return st;
        // the restriction also forms the coarse level's first sweep
        void* yc = level_pre(c, l + 1) > 0 && S->Dv[l + 1] ? S->X[l + 1] : nullptr;
        if ((st = mg_restrict<R>(S->Rr[l], G.nx, G.ny, G.nz, S->B[l + 1], Gc.nx, Gc.ny, Gc.nz, c.nrhs, c.s,
                                 yc ? S->Dv[l + 1] : nullptr, yc)))
            return st;
        void* xc = nullptr;
        if ((st = vcycle<R>(c, l + 1, S->B[l + 1], &xc, yc))) return st;
        if ((st = mg_prolong_add<R>(xc, Gc.nx, Gc.ny, Gc.nz, x, G.nx, G.ny, G.nz, c.nrhs, c.s))) return st;
        for (int k = 0; k < c.o->mg_post; ++k) {
            if ((st = launch_stencil<R>(G, MODE_JACOBI, a, bshift, x, t, b, c.o->mg_omega, c.nrhs, c.s))) return st;
            std::swap(x, t);
        }
    }
    *out = x;
    return HELM27_OK;
}

// z = M^-1 v (or z = v without preconditioner); returns the result buffer.
template <typename R>
static int precond(const Ctx& c, const void* v, void** z) {
    if (c.S->levels <= 0 || c.o->mg_levels == 0) {
        *z = const_cast<void*>(v);
        return HELM27_OK;
    }
    return vcycle<R>(c, 0, v, z);
}

// dinv * vin is formed by the kernels that write vin when the finest level
// has a Dv buffer and a pre-sweep
static void* vin_y0(const Ctx& c) {
    return level_pre(c, 0) > 0 && !c.S->Dv.empty() && c.S->Dv[0] ? c.S->vy : nullptr;
}

static bool use_vgraph(const Ctx& c) {
    return c.o->use_graph && c.S->levels > 0 && c.o->mg_levels != 0 && !c.S->graph_failed;
}

// The V-cycle on S->vin replayed from one hipGraph: the launch sequence
// depends only on the hierarchy, the right-hand-side count, the precision, the
// smoother options and the tile tuning, which key the graph.  The graph is
// built node by node from the same launchers (kernel nodes only: the zero
// fills are kernels), so a replay runs exactly the eager kernels.  Falls back
// to eager launches if building the graph fails.
template <typename R>
static int precond_vin(const Ctx& c, void** z) {
    SolverState* S = c.S;
    const GridOp& G = c.op->g;
    const double kd[3] = {c.o->mg_shift_re, c.o->mg_shift, c.o->mg_omega};
    const int ki[10] = {c.nrhs, static_cast<int>(sizeof(R)), c.o->mg_pre, c.o->mg_post, c.o->mg_coarse_sweeps,
                        G.plain_ry[0], G.plain_ry[1], G.kernel_variant, G.wave_zchunk, G.auto_tile ? 1 : 0};
    bool same = S->vgraph != nullptr;
    for (int k = 0; k < 3 && same; ++k) same = S->gkey_d[k] == kd[k];
    for (int k = 0; k < 10 && same; ++k) same = S->gkey_i[k] == ki[k];
    if (!same) {
        drop_graph(S);
        GraphRec rec;
        if (hipGraphCreate(&rec.graph, 0) != hipSuccess) {
            S->graph_failed = true;
            return precond<R>(c, S->vin, z);
        }
        void* out = nullptr;
        graph_rec() = &rec;
        const int st = vcycle<R>(c, 0, S->vin, &out, vin_y0(c));
        graph_rec() = nullptr;
        hipGraphExec_t ex = nullptr;
        if (st || rec.err != hipSuccess || hipGraphInstantiate(&ex, rec.graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(rec.graph);
            (void)hipGetLastError();
            S->graph_failed = true;
            if (st) return st;
            return precond<R>(c, S->vin, z);
        }
        hipGraphDestroy(rec.graph);
        S->vgraph = ex;
        S->vgraph_out = out;
        for (int k = 0; k < 3; ++k) S->gkey_d[k] = kd[k];
        for (int k = 0; k < 10; ++k) S->gkey_i[k] = ki[k];
    }
    H27_CHECK_HIP(hipGraphLaunch(S->vgraph, c.s));
    *z = S->vgraph_out;
    return HELM27_OK;
}

static int read_host(std::vector<double>* h, const double* d, int n, hipStream_t s) {
    h->resize(n);
    H27_CHECK_HIP(hipMemcpyAsync(h->data(), d, n * sizeof(double), hipMemcpyDeviceToHost, s));
    H27_CHECK_HIP(hipStreamSynchronize(s));
    return HELM27_OK;
}

// Waits for the pinned copy of Arnoldi step j's residual estimates; done when
// every right-hand side is at or below its threshold.
static int check_est(const Ctx& c, int j, const std::vector<double>& thr, const std::vector<double>& bn, int it,
                     bool* done) {
    H27_CHECK_HIP(hipEventSynchronize(c.S->est_ev[j & 1]));
    const double* est = c.S->h_est + (j & 1) * c.nrhs;
    *done = true;
    for (int q = 0; q < c.nrhs; ++q) {
        if (!std::isfinite(est[q])) return HELM27_ENUMERIC;
        if (est[q] > thr[q] * bn[q]) *done = false;
    }
    if (c.o->verbose)
        std::fprintf(stderr, "helm27: gmres it %d est[0] %.3e (target %.3e)\n", it, est[0], thr[0] * bn[0]);
    return HELM27_OK;
}

// GMRES(m) on A x = rhs (inner precision R), x starting at zero.  Stops when
// every right-hand side's residual estimate is <= thr[rhs] * ||rhs||.
template <typename R>
static int gmres_inner(const Ctx& c, const void* rhs, void* x, const std::vector<double>& thr, int max_it,
                       int* iters, bool* conv) {
    SolverState* S = c.S;
    const GridOp& G = c.op->g;
    const int nrhs = c.nrhs, m = S->m, ldh = m + 1;
    const int64_t N = G.N;
    const int64_t vstride = N * nrhs;
    const int64_t vbytes = vstride * static_cast<int64_t>(2 * sizeof(R));
    const size_t eb = 2 * sizeof(R);
    int st;
    if ((st = fill_zero(x, vbytes, c.s))) return st;
    if ((st = ensure_dinv<R>(c))) return st;
    std::vector<double> bn;
    if ((st = norms<R>(rhs, N, nrhs, S->d_partial, S->max_blocks, S->d_nrm, c.s))) return st;
    if ((st = read_host(&bn, S->d_nrm, nrhs, c.s))) return st;
    for (double v : bn)
        if (!std::isfinite(v)) return HELM27_ENUMERIC;
    int it = 0;
    *conv = false;
    bool first = true;
    int last_k = -1;   // steps of the last cycle that updated x
    while (it < max_it) {
        const void* r;
        if (first) {
            r = rhs;
        } else {
            if ((st = phys_apply<R>(c, MODE_RESID, x, S->w, rhs))) return st;
            r = S->w;
        }
        if ((st = norms<R>(r, N, nrhs, S->d_partial, S->max_blocks, S->d_beta, c.s))) return st;
        // the restart norms go to pinned memory; the host checks them once the
        // cycle's first Arnoldi step is queued (no device idle for the round
        // trip).  If they already meet the thresholds, that step is dropped
        // and x stays as it is.
        double* h_beta = S->h_est + 2 * nrhs;
        H27_CHECK_HIP(hipMemcpyAsync(h_beta, S->d_beta, nrhs * sizeof(double), hipMemcpyDeviceToHost, c.s));
        H27_CHECK_HIP(hipEventRecord(S->beta_ev, c.s));
        bool beta_checked = false, beta_conv = false;
        first = false;
        const bool g = use_vgraph(c);
        void* y0 = g ? vin_y0(c) : nullptr;
        const void* dv0 = y0 ? S->Dv[0] : nullptr;
        if ((st = scale_by_norm<R, R>(r, S->V, N, nrhs, S->d_beta, 0, c.s, g ? S->vin : nullptr, dv0, y0))) return st;
        if ((st = givens_init(S->d_g, m, nrhs, S->d_beta, c.s))) return st;
        int k = 0;
        bool cyc_conv = false;
        for (int j = 0; j < m && it < max_it; ++j) {
            void* vj = static_cast<char*>(S->V) + static_cast<size_t>(j) * vstride * eb;
            void* z = nullptr;
            if ((st = g ? precond_vin<R>(c, &z) : precond<R>(c, vj, &z))) return st;
            if ((st = phys_apply<R>(c, MODE_APPLY, z, S->w, nullptr))) return st;
            // classical Gram-Schmidt: h = V^H w (and ||w||); w -= V h (and ||w||);
            // then, per right-hand side only where the first pass cancelled
            // more than 1 - 1/sqrt(2) of the norm: h2 = V^H w (h += h2 in the
            // reduction) and w -= V h2; ||w|| of the result in the last pass
            if ((st = mdot<R>(S->V, vstride, j + 1, S->w, N, nrhs, S->d_partial, S->max_blocks, S->d_hcol, nullptr, ldh,
                              c.s, S->d_n0)))
                return st;
            if ((st = cgs_update<R>(S->V, vstride, j + 1, S->d_hcol, ldh, S->w, N, nrhs, S->d_partial, S->max_blocks,
                                    S->d_n1, c.s)))
                return st;
            const double* g0 = c.o->reorth_always ? nullptr : S->d_n0;
            if ((st = mdot<R>(S->V, vstride, j + 1, S->w, N, nrhs, S->d_partial, S->max_blocks, S->d_htmp, S->d_hcol,
                              ldh, c.s, nullptr, g0, S->d_n1)))
                return st;
            if ((st = cgs_update<R>(S->V, vstride, j + 1, S->d_htmp, ldh, S->w, N, nrhs, S->d_partial, S->max_blocks,
                                    S->d_nrm, c.s, g0, S->d_n1)))
                return st;
            void* vj1 = static_cast<char*>(S->V) + static_cast<size_t>(j + 1) * vstride * eb;
            const bool feed = g && j + 1 < m;   // v_{j+1} is the next V-cycle's input
            if ((st = scale_by_norm<R, R>(S->w, vj1, N, nrhs, S->d_nrm, 0, c.s, feed ? S->vin : nullptr,
                                          feed ? dv0 : nullptr, feed ? y0 : nullptr)))
                return st;
            if ((st = givens_step(j, m, nrhs, S->d_hcol, ldh, S->d_nrm, S->d_H, S->d_cs, S->d_sn, S->d_g, S->d_est, c.s)))
                return st;
            ++it;
            k = j + 1;
            // the estimate of step j goes to pinned memory; the host then
            // checks step j - 1, whose copy is normally complete while step j
            // runs, so the device never waits for the host between steps.  If
            // step j - 1 converged, step j is dropped (k = j): its kernels
            // touched only column j, g[j..j+1] and v_{j+1}, none of which the
            // solution update with k = j reads.
            H27_CHECK_HIP(hipMemcpyAsync(S->h_est + (j & 1) * nrhs, S->d_est, nrhs * sizeof(double),
                                         hipMemcpyDeviceToHost, c.s));
            H27_CHECK_HIP(hipEventRecord(S->est_ev[j & 1], c.s));
            if (!beta_checked) {
                beta_checked = true;
                H27_CHECK_HIP(hipEventSynchronize(S->beta_ev));
                beta_conv = true;
                for (int q = 0; q < nrhs; ++q) {
                    if (!std::isfinite(h_beta[q])) return HELM27_ENUMERIC;
                    if (h_beta[q] > thr[q] * bn[q]) beta_conv = false;
                }
                if (beta_conv) {
                    --it;
                    break;
                }
            }
            if (j > 0) {
                bool done = false;
                if ((st = check_est(c, j - 1, thr, bn, it - 1, &done))) return st;
                if (done) {
                    --it;
                    k = j;
                    cyc_conv = true;
                    break;
                }
            }
        }
        if (beta_conv) {   // converged before this cycle: x is final
            S->last_est = 0;
            for (int q = 0; q < nrhs; ++q) S->last_est = std::max(S->last_est, h_beta[q] / bn[q]);
            last_k = -1;
            *conv = true;
            break;
        }
        if (!beta_checked) {   // no step ran (max_it reached): check the restart norms
            H27_CHECK_HIP(hipEventSynchronize(S->beta_ev));
            bool all = true;
            for (int q = 0; q < nrhs; ++q) {
                if (!std::isfinite(h_beta[q])) return HELM27_ENUMERIC;
                if (h_beta[q] > thr[q] * bn[q]) all = false;
            }
            if (all) *conv = true;
            last_k = 0;   // g was re-initialised: g_0 = beta, the residual x leaves
            break;
        }
        if (!cyc_conv && k > 0) {
            bool done = false;
            if ((st = check_est(c, k - 1, thr, bn, it, &done))) return st;
            cyc_conv = done;
        }
        if ((st = upper_solve(k, m, nrhs, S->d_H, S->d_g, S->d_y, ldh, c.s))) return st;
        last_k = k;
        void* z = nullptr;
        if (g) {
            if ((st = combine<R>(S->V, vstride, k, S->d_y, ldh, S->vin, N, nrhs, 0, c.s, dv0, y0))) return st;
            if ((st = precond_vin<R>(c, &z))) return st;
        } else {
            if ((st = combine<R>(S->V, vstride, k, S->d_y, ldh, S->tmp, N, nrhs, 0, c.s))) return st;
            if ((st = precond<R>(c, S->tmp, &z))) return st;
        }
        if ((st = add_inplace<R>(x, z, vstride, c.s))) return st;
        if (cyc_conv) {
            *conv = true;
            break;
        }
    }
    if (last_k >= 0 && S->last_est >= 0) {
        // the last cycle's Givens estimate |g_k| of the residual it leaves
        // (absolute: g_0 = beta is the cycle's starting residual); g is
        // re-initialised only when a cycle starts, so it is still that cycle's
        std::vector<double2> gk(static_cast<size_t>(nrhs) * ldh);
        H27_CHECK_HIP(hipMemcpyAsync(gk.data(), S->d_g, gk.size() * sizeof(double2), hipMemcpyDeviceToHost, c.s));
        H27_CHECK_HIP(hipStreamSynchronize(c.s));
        S->last_est = 0;
        for (int q = 0; q < nrhs; ++q) {
            const double2 v = gk[static_cast<size_t>(q) * ldh + last_k];
            S->last_est = std::max(S->last_est, std::hypot(v.x, v.y) / bn[q]);
        }
    }
    *iters = it;
    return HELM27_OK;
}

static int solve_core(helm27_op* op, const double2* b, double2* u, int nrhs, const helm27_solve_opts* o,
                      helm27_solve_stats* stats, hipStream_t s) {
    SolverState* S = static_cast<SolverState*>(op->solver);
    const int want_levels = o->mg_levels > 0 ? o->mg_levels : (o->mg_levels < 0 ? auto_levels(op->g) : 0);
    if (want_levels != S->req_levels || o->mg_coarse_table != S->req_coarse_table) {
        free_workspace(S);
        free_hierarchy(S);
        if (want_levels > 0) {
            const int st = build_hierarchy(op, S, want_levels, o->mg_coarse_table == 1, s);
            if (st) return st;
        }
        S->req_levels = want_levels;
        S->req_coarse_table = o->mg_coarse_table;
    }
    const int prec = o->precision == HELM27_C128 ? 8 : 4;
    int st = ensure_workspace(op, S, nrhs, o->restart, prec);
    if (st) return st;
    Ctx c{op, S, o, s, nrhs};
    const GridOp& G = op->g;
    const int64_t N = G.N;
    if ((st = fill_zero(u, N * nrhs * static_cast<int64_t>(sizeof(double2)), s))) return st;
    std::vector<double> bn, rn;
    if ((st = norms<double>(b, N, nrhs, S->d_partial, S->max_blocks, S->d_bn, s))) return st;
    if ((st = read_host(&bn, S->d_bn, nrhs, s))) return st;
    for (double v : bn)
        if (!std::isfinite(v)) return HELM27_ENUMERIC;
    int outer = 0, inner_total = 0;
    bool converged = false;
    double maxrel = 0;
    for (;;) {
        if ((st = phys_apply<double>(c, MODE_RESID, u, S->r64, b))) return st;
        if ((st = norms<double>(S->r64, N, nrhs, S->d_partial, S->max_blocks, S->d_rn, s))) return st;
        if ((st = read_host(&rn, S->d_rn, nrhs, s))) return st;
        maxrel = 0;
        for (int k = 0; k < nrhs; ++k) {
            if (!std::isfinite(rn[k])) return HELM27_ENUMERIC;
            const double rel = bn[k] > 0 ? rn[k] / bn[k] : 0.0;
            maxrel = std::max(maxrel, rel);
        }
        if (o->verbose) std::fprintf(stderr, "helm27: outer %d max relres %.3e\n", outer, maxrel);
        if (maxrel <= o->tol) {
            converged = true;
            break;
        }
        if (outer >= o->max_outer) break;
        // inner thresholds relative to the normalised residual
        std::vector<double> thr(nrhs);
        for (int k = 0; k < nrhs; ++k) {
            const double need = (bn[k] > 0 && rn[k] > 0) ? 0.5 * o->tol * bn[k] / rn[k] : 1.0;
            thr[k] = std::min(1.0, std::max(need, o->inner_tol));
            if (prec == 8) thr[k] = std::min(1.0, need);
        }
        int its = 0;
        bool ic = false;
        if (prec == 4) {
            if ((st = scale_by_norm<double, float>(S->r64, S->rin, N, nrhs, S->d_rn, 0, s))) return st;
            if ((st = gmres_inner<float>(c, S->rin, S->e, thr, o->max_inner, &its, &ic))) return st;
            if ((st = refine_update<float>(u, S->e, N, nrhs, S->d_rn, s))) return st;
        } else {
            if ((st = scale_by_norm<double, double>(S->r64, S->rin, N, nrhs, S->d_rn, 0, s))) return st;
            if ((st = gmres_inner<double>(c, S->rin, S->e, thr, o->max_inner, &its, &ic))) return st;
            if ((st = refine_update<double>(u, S->e, N, nrhs, S->d_rn, s))) return st;
        }
        inner_total += its;
        ++outer;
        if (its == 0) break;   // no progress possible
    }
    if (stats) {
        stats->outer_iters = outer;
        stats->inner_iters = inner_total;
        stats->converged = converged ? 1 : 0;
        stats->max_relres = maxrel;
        stats->mg_levels = o->mg_levels == 0 ? 1 : S->levels;
        stats->coarse_clamped = o->mg_levels == 0 ? 0 : S->coarse_clamped;
        stats->coarse_tables = o->mg_levels == 0 ? 0 : S->coarse_tables;
        stats->inner_est = S->last_est;
    }
    return converged ? HELM27_OK : HELM27_ENOCONV;
}

}  // namespace h27

using namespace h27;

void solver_free(helm27_op* op) {
    if (!op || !op->solver) return;
    SolverState* S = static_cast<SolverState*>(op->solver);
    free_workspace(S);
    free_hierarchy(S);
    for (hipEvent_t e : S->est_ev)
        if (e) hipEventDestroy(e);
    if (S->beta_ev) hipEventDestroy(S->beta_ev);
    hipFree(S->d_lin);
    hipFree(S->d_amp);
    hipFree(S->d_b);
    delete S;
    op->solver = nullptr;
}

extern "C" void helm27_solve_opts_default(helm27_solve_opts* o) {
    if (!o) return;
    o->tol = 1e-6;
    o->restart = 28;
    o->max_inner = 600;
    o->max_outer = 10;
    o->inner_tol = 1e-3;
    o->precision = HELM27_C64;
    o->mg_levels = -1;
    o->mg_shift = 1.0;
    o->mg_shift_re = 0.0;
    o->mg_pre = 2;
    o->mg_post = 1;
    o->mg_omega = 0.6;
    o->mg_coarse_sweeps = 3;
    o->use_graph = 1;
    o->reorth_always = 0;
    o->mg_coarse_table = 0;
    o->transpose = 0;
    o->verbose = 0;
}

static int check_opts(const helm27_solve_opts* o) {
    if (!(o->tol > 0) || o->restart < 1 || o->restart > 63 || o->max_inner < 1 || o->max_outer < 0 ||
        !(o->inner_tol > 0) || o->inner_tol >= 1 || (o->precision != HELM27_C64 && o->precision != HELM27_C128) ||
        o->mg_levels < -1 || o->mg_levels > 8 || o->mg_pre < 0 || o->mg_post < 0 || o->mg_coarse_sweeps < 0 ||
        !(o->mg_omega > 0) || !std::isfinite(o->mg_shift) || !std::isfinite(o->mg_shift_re) ||
        (o->mg_coarse_table != 0 && o->mg_coarse_table != 1) || (o->transpose != 0 && o->transpose != 1))
        return HELM27_EINVAL;
    return HELM27_OK;
}

extern "C" int helm27_solve_rhs(helm27_op* op, const void* b, void* u, int nrhs, const helm27_solve_opts* opts,
                                helm27_solve_stats* stats, void* stream) {
    if (!op || !b || !u || nrhs <= 0) return HELM27_EINVAL;
    helm27_solve_opts o;
    if (opts) o = *opts;
    else helm27_solve_opts_default(&o);
    int st = check_opts(&o);
    if (st) return st;
    if (!op->solver) {
        op->solver = new (std::nothrow) SolverState;
        if (!op->solver) return HELM27_ENOMEM;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = solve_core(op, static_cast<const double2*>(b), static_cast<double2*>(u), nrhs, &o, stats, s);
    if (hipStreamSynchronize(s) != hipSuccess && st == HELM27_OK) st = HELM27_EDEVICE;
    if (stats) stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

extern "C" int helm27_solve(helm27_op* op, const double* src, void* u, int nrhs, const helm27_solve_opts* opts,
                            helm27_solve_stats* stats, void* stream) {
    if (!op || !src || !u || nrhs <= 0) return HELM27_EINVAL;
    const GridOp& G = op->g;
    std::vector<int64_t> lin(nrhs);
    std::vector<double2> amp(nrhs);
    const int dims[3] = {G.nx, G.ny, G.nz};
    for (int k = 0; k < nrhs; ++k) {
        int p[3];
        for (int a = 0; a < 3; ++a) {
            const double v = src[5 * k + a];
            if (!(v == std::floor(v))) return HELM27_EINVAL;
            p[a] = static_cast<int>(v);
            if (p[a] < G.npml[a] || p[a] > dims[a] - 1 - G.npml[a]) return HELM27_ERANGE;
        }
        if (!std::isfinite(src[5 * k + 3]) || !std::isfinite(src[5 * k + 4])) return HELM27_ENUMERIC;
        lin[k] = p[0] + static_cast<int64_t>(G.nx) * (p[1] + static_cast<int64_t>(G.ny) * p[2]);
        amp[k].x = src[5 * k + 3];
        amp[k].y = src[5 * k + 4];
    }
    if (!op->solver) {
        op->solver = new (std::nothrow) SolverState;
        if (!op->solver) return HELM27_ENOMEM;
    }
    SolverState* S = static_cast<SolverState*>(op->solver);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (S->src_cap < nrhs) {
        hipFree(S->d_lin);
        hipFree(S->d_amp);
        hipFree(S->d_b);
        S->d_lin = nullptr;
        S->d_amp = nullptr;
        S->d_b = nullptr;
        S->src_cap = 0;
        if (hipMalloc(&S->d_lin, nrhs * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&S->d_amp, nrhs * sizeof(double2)) != hipSuccess ||
            hipMalloc(&S->d_b, static_cast<size_t>(G.N) * nrhs * sizeof(double2)) != hipSuccess)
            return HELM27_ENOMEM;
        S->src_cap = nrhs;
    }
    double2* b = S->d_b;
    int st = HELM27_OK;
    if (hipMemcpyAsync(S->d_lin, lin.data(), nrhs * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(S->d_amp, amp.data(), nrhs * sizeof(double2), hipMemcpyHostToDevice, s) != hipSuccess)
        st = HELM27_EDEVICE;
    if (!st) st = fill_zero(b, G.N * nrhs * static_cast<int64_t>(sizeof(double2)), s);
    if (!st) st = inject_sources(b, G.N, S->d_lin, S->d_amp, nrhs, G.h, s);
    if (!st) st = helm27_solve_rhs(op, b, u, nrhs, opts, stats, stream);
    else hipStreamSynchronize(s);
    return st;
}

void h27::solver_trim(helm27_op* op) {
    if (!op || !op->solver) return;
    SolverState* S = static_cast<SolverState*>(op->solver);
    free_workspace(S);
    hipFree(S->d_lin);
    hipFree(S->d_amp);
    hipFree(S->d_b);
    S->d_lin = nullptr;
    S->d_amp = nullptr;
    S->d_b = nullptr;
    S->src_cap = 0;
}

size_t h27::solve_footprint(int64_t N, int nrhs, int restart, int precision, int levels) {
    const double e = precision == HELM27_C128 ? 16.0 : 8.0;   // complex element bytes, inner precision
    const double n = static_cast<double>(N) * nrhs;
    double bytes = n * e * (restart + 1 + 6);                   // Krylov basis, w, e, rin, tmp, vin, vy
    double lv = 0, f = 1, pl = 0;
    if (levels < 0) levels = 8;                                 // automatic depth: bound
    for (int l = 0; l < levels; ++l, f /= 8) {
        lv += f * (l == 0 ? 3 : 4);
        pl += f;
    }
    bytes += n * e * lv;                                        // multigrid vectors
    bytes += static_cast<double>(N) * e * pl;                   // omega D^-1 per level
    bytes += n * 16.0 * 2;                                      // FP64 residual and right-hand side
    bytes += static_cast<double>(N) * 7.0;                      // coarse grids (velocity + index + ...)
    bytes += static_cast<double>(nrhs) * (restart + 2) * 1024 * 16;   // reduction partials
    return static_cast<size_t>(bytes * 1.05) + (16u << 20);
}

// Several operators at once (one model at several frequencies, Sec. 1):
// every solve runs from its own host thread on its own stream, so their
// kernels overlap on the device; each operator's solve is the same sequence
// of launches as alone, so its result is bit-identical to a lone solve.
extern "C" int helm27_solve_many(helm27_op* const* ops, int nops, const double* const* src, const int* nrhs,
                                 void* const* u, const helm27_solve_opts* opts, helm27_solve_stats* stats) {
    if (!ops || !src || !nrhs || !u || nops <= 0) return HELM27_EINVAL;
    for (int k = 0; k < nops; ++k) {
        if (!ops[k] || !src[k] || !u[k] || nrhs[k] <= 0) return HELM27_EINVAL;
        for (int j = 0; j < k; ++j)
            if (ops[j] == ops[k]) return HELM27_EINVAL;   // one solve per operator at a time
    }
    int dev = 0;
    H27_CHECK_HIP(hipGetDevice(&dev));
    std::vector<int> status(nops, HELM27_OK);
    std::vector<hipStream_t> streams(nops, nullptr);
    for (int k = 0; k < nops; ++k) {
        if (hipSetDevice(ops[k]->ctx->device) != hipSuccess || hipStreamCreate(&streams[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) hipStreamDestroy(streams[j]);
            (void)hipSetDevice(dev);
            return HELM27_EDEVICE;
        }
    }
    auto work = [&](int k) {
        if (hipSetDevice(ops[k]->ctx->device) != hipSuccess) {
            status[k] = HELM27_EDEVICE;
            return;
        }
        status[k] = helm27_solve(ops[k], src[k], u[k], nrhs[k], opts, stats ? &stats[k] : nullptr, streams[k]);
    };
    std::vector<std::thread> pool;
    try {
        for (int k = 1; k < nops; ++k) pool.emplace_back(work, k);
    } catch (...) {
        for (std::thread& t : pool) t.join();
        for (hipStream_t st : streams) hipStreamDestroy(st);
        (void)hipSetDevice(dev);
        return HELM27_ENOMEM;
    }
    work(0);
    for (std::thread& t : pool) t.join();
    for (hipStream_t st : streams) hipStreamDestroy(st);
    (void)hipSetDevice(dev);
    for (int k = 0; k < nops; ++k)
        if (status[k] != HELM27_OK && status[k] != HELM27_ENOCONV) return status[k];
    for (int k = 0; k < nops; ++k)
        if (status[k] == HELM27_ENOCONV) return HELM27_ENOCONV;
    return HELM27_OK;
}
