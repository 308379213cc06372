// Operator construction (weights per row, PML profiles, tiling) and the apply /
// export entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "stencil.h"

namespace h27 {

// PML stretching along one axis (paper Sec. 2.1: d/dx -> (1/xi) d/dx with
// xi = 1 + i gamma/omega).  Profile: a layer of width L beyond [x_lo, x_hi]
// with gamma(d) = gamma_max (1 - cos(pi d / (2 L))) at depth d into the layer
// and gamma_max = c_ref ln(1/R) / (2 L (1 - 2/pi)), which makes
// exp(-(2/c_ref) int_0^L gamma) = R; the same formula holds beyond the last
// node.  Evaluated at nodes x = i h and half nodes (i +- 1/2) h, so every
// multigrid level samples the same physical stretching.
static double pml_gamma(double x, double x_lo, double x_hi, double L, double c_ref, double R) {
    double d = 0.0;
    if (x < x_lo) d = x_lo - x;
    if (x > x_hi) d = x - x_hi;
    if (d <= 0.0 || L <= 0.0) return 0.0;
    const double pi = 3.14159265358979323846;
    const double gmax = c_ref * std::log(1.0 / R) / (2.0 * L * (1.0 - 2.0 / pi));
    return gmax * (1.0 - std::cos(pi * d / (2.0 * L)));
}

void axis_nodes(int n, double h, double x_lo, double x_hi, double L, double omega, double c_ref, double R,
                std::vector<AxisNode<double>>* out) {
    out->assign(n, AxisNode<double>{});
    for (int i = 0; i < n; ++i) {
        const double gn = pml_gamma(i * h, x_lo, x_hi, L, c_ref, R);
        const double gm = pml_gamma((i - 0.5) * h, x_lo, x_hi, L, c_ref, R);
        const double gp = pml_gamma((i + 0.5) * h, x_lo, x_hi, L, c_ref, R);
        AxisNode<double>& a = (*out)[i];
        a.xi_re = 1.0;
        a.xi_im = gn / omega;
        // 1 / (1 + i s) = (1 - i s) / (1 + s^2)
        const double sm = gm / omega, sp = gp / omega;
        a.tm_re = 1.0 / (1.0 + sm * sm);
        a.tm_im = -sm / (1.0 + sm * sm);
        a.tp_re = 1.0 / (1.0 + sp * sp);
        a.tp_im = -sp / (1.0 + sp * sp);
        a.um_re = 0.5;
        a.um_im = 0.5 * sm;
        a.up_re = 0.5;
        a.up_im = 0.5 * sp;
        a.plain = (gn == 0.0 && gm == 0.0 && gp == 0.0) ? 1 : 0;
        a.pad = 0;
    }
}

static void plain_range(const std::vector<AxisNode<double>>& a, int* lo, int* hi) {
    const int n = static_cast<int>(a.size());
    int l = 0;
    while (l < n && !a[l].plain) ++l;
    int h = l;
    while (h < n && a[h].plain) ++h;
    *lo = l;
    *hi = h;
}

void make_tiling(int nx, int ny, const int plo[2], const int phi[2], Tiling* t, int zchunk, int nz) {
    // plain tile height in rows: kPlainTY (4) threads x 2 rows
    const int TW = kPlainTX, TH = kPlainTY * kRows, F = kFrameT;
    Tiling T;
    int px0 = plo[0], px1 = phi[0], py0 = plo[1], py1 = phi[1];
    if (px1 <= px0 || py1 <= py0) {
        px0 = px1 = py0 = py1 = 0;
    }
    T.plain_x0 = px0;
    T.plain_y0 = py0;
    T.plain_w = px1 - px0;
    T.plain_h = py1 - py0;
    T.n_plain_tiles_x = T.plain_w > 0 ? (T.plain_w + TW - 1) / TW : 0;
    T.n_plain_tiles_y = T.plain_h > 0 ? (T.plain_h + TH - 1) / TH : 0;
    T.n_plain_blocks = T.n_plain_tiles_x * T.n_plain_tiles_y;
    Rect r[4];
    if (T.plain_w == 0) {
        r[0] = {0, 0, nx, ny};
        r[1] = r[2] = r[3] = {0, 0, 0, 0};
    } else {
        r[0] = {0, 0, nx, py0};                 // bottom strip (y < py0)
        r[1] = {0, py1, nx, ny - py1};          // top strip
        r[2] = {0, py0, px0, py1 - py0};        // left strip
        r[3] = {px1, py0, nx - px1, py1 - py0}; // right strip
    }
    T.n_frame_blocks = 0;
    for (int k = 0; k < 4; ++k) {
        T.frame[k] = r[k];
        const bool empty = r[k].w <= 0 || r[k].h <= 0;
        T.frame_tiles_x[k] = empty ? 0 : (r[k].w + F - 1) / F;
        T.frame_tiles_y[k] = empty ? 0 : (r[k].h + F - 1) / F;
        T.n_frame_blocks += T.frame_tiles_x[k] * T.frame_tiles_y[k];
    }
    if (zchunk <= 0) {
        // enough blocks to fill 256 CUs a few times over, but long z marches
        const int64_t cols = T.n_plain_blocks + T.n_frame_blocks;
        int zc = static_cast<int>((cols * nz) / 2048);
        zc = std::max(2, std::min(16, zc));
        zchunk = zc;
    }
    T.zchunk = std::min(zchunk, nz);
    T.n_zchunks = (nz + T.zchunk - 1) / T.zchunk;
    *t = T;
}

void grid_free(GridOp* g) {
    hipFree(g->d_c);
    hipFree(g->d_idx);
    hipFree(g->d_setup);   // entry and axis arrays
    hipFree(g->d_row_f);
    hipFree(g->d_row_d);
    *g = GridOp{};
}

template <typename R>
static EntryCoef<R> entry_from_w7(const double* w) {
    // stiffness in tensor form: 1 * sum T + beta2 sum TT + beta3 TTT, with
    // beta2 = w_s2/6 + w_s3/2 and beta3 = 3 w_s3 / 8 (the rotated families'
    // symbols); the interior class values follow from them.
    const double b2 = w[1] / 6.0 + w[2] / 2.0;
    const double b3 = 3.0 * w[2] / 8.0;
    EntryCoef<R> e;
    e.s0 = static_cast<R>(-6.0 + 12.0 * b2 - 8.0 * b3);
    e.s1 = static_cast<R>(1.0 - 4.0 * b2 + 4.0 * b3);
    e.s2 = static_cast<R>(b2 - 2.0 * b3);
    e.s3 = static_cast<R>(b3);
    e.beta2 = static_cast<R>(b2);
    e.beta3 = static_cast<R>(b3);
    e.m0 = static_cast<R>(w[3]);
    e.m1 = static_cast<R>(w[4]);
    e.m2 = static_cast<R>(w[5]);
    e.m3 = static_cast<R>(w[6]);
    e.pad0 = e.pad1 = R(0);
    return e;
}

// The same binary64 formula as the device index selection.
int host_index(float c, double fh, double gmin, double dg, int n_g, int invg) {
    const double G = invg ? fh / static_cast<double>(c) : static_cast<double>(c) / fh;
    const double t = (G - gmin) / dg;
    const double raw = std::floor(t + 0.5);
    if (!(raw >= 0.0)) return 0;
    if (raw > static_cast<double>(n_g - 1)) return n_g - 1;
    return static_cast<int>(raw);
}

int widen_range(const helm27_table* t, double need_lo, double need_hi, double* v_min, int* n_g) {
    const double v0 = t->g_min, dv = t->dg;
    const double v1 = v0 + (t->n_g - 1) * dv;
    double k_lo = need_lo < v0 ? std::ceil((v0 - need_lo) / dv) : 0.0;
    // keep the first abscissa in the axis' domain: G > 0, s = 1/G >= 0
    const double k_max = t->spacing == HELM27_SPACING_INVG ? std::floor(v0 / dv + 1e-9) : std::ceil(v0 / dv) - 1.0;
    if (k_lo > k_max) k_lo = std::max(0.0, k_max);
    const double k_hi = need_hi > v1 ? std::ceil((need_hi - v1) / dv) : 0.0;
    const double n = t->n_g + k_lo + k_hi;
    if (n > 65535.0) return HELM27_ERANGE;
    *v_min = k_lo > 0 ? v0 - k_lo * dv : v0;
    *n_g = static_cast<int>(n);
    return HELM27_OK;
}

// Fill the weight tables, PML axes and tiling of a grid whose velocity is
// already on the device (d_c) and whose index has been selected.
int grid_setup(GridOp* g, const double* w7, int n_g, int fixed) {
    g->n_g = n_g;
    g->fixed = fixed;
    // the table entries (FP32, FP64) and the three axes' PML nodes (FP64,
    // FP32) go to the device in one allocation and one copy, each array at a
    // 256-byte aligned offset
    std::vector<unsigned char> host;
    auto put = [&host](const void* src, size_t bytes) {
        const size_t off = (host.size() + 255) & ~static_cast<size_t>(255);
        host.resize(off + bytes);
        std::memcpy(host.data() + off, src, bytes);
        return off;
    };
    std::vector<EntryCoef<float>> ef(n_g);
    std::vector<EntryCoef<double>> ed(n_g);
    for (int i = 0; i < n_g; ++i) {
        ef[i] = entry_from_w7<float>(w7 + 7 * i);
        ed[i] = entry_from_w7<double>(w7 + 7 * i);
    }
    const size_t o_ef = put(ef.data(), ef.size() * sizeof(ef[0]));
    const size_t o_ed = put(ed.data(), ed.size() * sizeof(ed[0]));
    size_t o_axd[3], o_axf[3];
    const int dims[3] = {g->nx, g->ny, g->nz};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        std::vector<AxisNode<double>> nd;
        axis_nodes(dims[a], g->h, g->pml_lo[a], g->pml_hi[a], g->pml_L[a], g->omega, g->c_ref, g->R, &nd);
        std::vector<AxisNode<float>> nf(nd.size());
        for (size_t i = 0; i < nd.size(); ++i) {
            const AxisNode<double>& s = nd[i];
            nf[i] = AxisNode<float>{static_cast<float>(s.xi_re), static_cast<float>(s.xi_im),
                                    static_cast<float>(s.tm_re), static_cast<float>(s.tm_im),
                                    static_cast<float>(s.tp_re), static_cast<float>(s.tp_im),
                                    static_cast<float>(s.um_re), static_cast<float>(s.um_im),
                                    static_cast<float>(s.up_re), static_cast<float>(s.up_im), s.plain, 0};
        }
        o_axd[a] = put(nd.data(), nd.size() * sizeof(nd[0]));
        o_axf[a] = put(nf.data(), nf.size() * sizeof(nf[0]));
        plain_range(nd, &lo[a], &hi[a]);
    }
    if (hipMalloc(&g->d_setup, host.size()) != hipSuccess) {
        g->d_setup = nullptr;
        return HELM27_ENOMEM;
    }
    g->bytes += host.size();
    H27_CHECK_HIP(hipMemcpy(g->d_setup, host.data(), host.size(), hipMemcpyHostToDevice));
    unsigned char* base = static_cast<unsigned char*>(g->d_setup);
    g->d_entry_f = reinterpret_cast<EntryCoef<float>*>(base + o_ef);
    g->d_entry_d = reinterpret_cast<EntryCoef<double>*>(base + o_ed);
    for (int a = 0; a < 3; ++a) {
        g->d_ax_d[a] = reinterpret_cast<AxisNode<double>*>(base + o_axd[a]);
        g->d_ax_f[a] = reinterpret_cast<AxisNode<float>*>(base + o_axf[a]);
    }
    g->zp_lo = lo[2];
    g->zp_hi = hi[2];
    make_tiling(g->nx, g->ny, lo, hi, &g->tiling, 0, g->nz);
    return HELM27_OK;
}

}  // namespace h27

using namespace h27;

extern "C" int helm27_create(helm27_ctx** out, int device, size_t hbm_budget_bytes) {
    if (!out) return HELM27_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HELM27_EINVAL;
    H27_CHECK_HIP(hipSetDevice(device));
    helm27_ctx* c = new (std::nothrow) helm27_ctx;
    if (!c) return HELM27_ENOMEM;
    c->device = device;
    if (hbm_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) hbm_budget_bytes = static_cast<size_t>(0.9 * fr);
    }
    c->hbm_budget = hbm_budget_bytes;
    // the no-allocation entry point's scratch array: its address on this device
    const int st = h27::noalloc_init(device);
    if (st) {
        delete c;
        return st;
    }
    *out = c;
    return HELM27_OK;
}

void helm27_serve_shutdown(helm27_ctx* ctx);  // serve.cpp

extern "C" void helm27_destroy(helm27_ctx* ctx) {
    if (!ctx) return;
    helm27_serve_shutdown(ctx);
    delete ctx;
}

extern "C" const char* helm27_strerror(int st) {
    switch (st) {
        case HELM27_OK: return "ok";
        case HELM27_EINVAL: return "invalid argument";
        case HELM27_ENOMEM: return "out of memory";
        case HELM27_EADMIT: return "request exceeds the HBM budget";
        case HELM27_ENOCONV: return "no convergence within the iteration limit";
        case HELM27_ENUMERIC: return "NaN/Inf or breakdown";
        case HELM27_EDEVICE: return "HIP device error";
        case HELM27_ERANGE: return "source outside the grid or inside the PML";
        case HELM27_ENOTFOUND: return "unknown ticket";
        case HELM27_EAGAIN: return "not ready";
        default: return "unknown status";
    }
}

namespace h27 {
// Assembly on a given stream (the serving workers use their own streams).
int op_create(helm27_ctx* ctx, const helm27_table* t, const float* vel, int nx, int ny, int nz, double h,
              double freq, const helm27_pml* pml, int flags, hipStream_t stream, helm27_op** out) {
    if (!ctx || !t || !vel || !out) return HELM27_EINVAL;
    if (nx < 3 || ny < 3 || nz < 3 || !(h > 0) || !(freq > 0)) return HELM27_EINVAL;
    const int wmode = flags & 0x3;
    if (wmode == 3) return HELM27_EINVAL;
    if (flags & ~(0x3 | HELM27_STORE_C64 | HELM27_STORE_C128 | HELM27_EXTEND_TABLE | HELM27_MASS_A))
        return HELM27_EINVAL;
    if ((flags & HELM27_EXTEND_TABLE) && t->lambda < 0) return HELM27_EINVAL;   // fit settings unknown
    helm27_pml P{{8, 8, 8}, 1e-3, 0.0};
    if (pml) P = *pml;
    const int dims[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a)
        if (P.npml[a] < 0 || 2 * P.npml[a] + 1 > dims[a]) return HELM27_EINVAL;
    if (!(P.R > 0) || P.R >= 1) P.R = 1e-3;
    H27_CHECK_HIP(hipSetDevice(ctx->device));

    const int64_t N = static_cast<int64_t>(nx) * ny * nz;
    helm27_op* op = new (std::nothrow) helm27_op;
    if (!op) return HELM27_ENOMEM;
    op->ctx = ctx;
    GridOp& g = op->g;
    g.nx = nx; g.ny = ny; g.nz = nz; g.N = N;
    g.h = h;
    g.omega = 2.0 * 3.14159265358979323846 * freq;
    for (int a = 0; a < 3; ++a) {
        g.npml[a] = P.npml[a];
        g.pml_L[a] = P.npml[a] * h;
        g.pml_lo[a] = P.npml[a] * h;
        g.pml_hi[a] = (dims[a] - 1 - P.npml[a]) * h;
    }
    g.R = P.R;
    op->freq = freq;
    op->flags = flags;
    op->table = *t;
    g.mass_a = (flags & HELM27_MASS_A) ? 1 : 0;
    const double fh = freq * h;

    int st = HELM27_OK;
    unsigned long long* d_cnt = nullptr;
    auto fail = [&](int s) {
        hipFree(d_cnt);
        helm27_op_destroy(op);
        return s;
    };
    // the velocity goes to the device as given (host or device pointer); the
    // index kernel validates it and finds its range on the device
    if (hipMalloc(&g.d_c, N * sizeof(float)) != hipSuccess) return fail(HELM27_ENOMEM);
    if (hipMalloc(&g.d_idx, N * sizeof(uint16_t)) != hipSuccess) return fail(HELM27_ENOMEM);
    g.bytes += N * (sizeof(float) + sizeof(uint16_t));
    if (hipMemcpyAsync(g.d_c, vel, N * sizeof(float), hipMemcpyDefault, stream) != hipSuccess)
        return fail(HELM27_EDEVICE);
    unsigned long long cnt[4] = {0, 0, 0x7F800000ull, 0};   // clamped, invalid, min bits (+inf), max bits
    if (hipMalloc(&d_cnt, sizeof(cnt)) != hipSuccess) return fail(HELM27_ENOMEM);
    // index pass with the operator's table: counts, validation, range
    auto index_pass = [&]() {
        unsigned long long c0[4] = {0, 0, 0x7F800000ull, 0};
        const helm27_table& T = op->table;
        if (hipMemcpyAsync(d_cnt, c0, sizeof(c0), hipMemcpyHostToDevice, stream) != hipSuccess) return HELM27_EDEVICE;
        int s2 = launch_select_index(g.d_c, g.d_idx, N, fh, T.g_min, T.dg, T.n_g, T.spacing, d_cnt, stream);
        if (s2) return s2;
        if (hipMemcpyAsync(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return HELM27_EDEVICE;
        return HELM27_OK;
    };
    if ((st = index_pass())) return fail(st);
    if (cnt[1] != 0) return fail(HELM27_EINVAL);
    if ((flags & HELM27_EXTEND_TABLE) && cnt[0] != 0) {
        // widen the table over the model's range on the same axis grid and index again
        float c_lo, c_hi;
        const unsigned lo = static_cast<unsigned>(cnt[2]), hi = static_cast<unsigned>(cnt[3]);
        std::memcpy(&c_lo, &lo, sizeof(float));
        std::memcpy(&c_hi, &hi, sizeof(float));
        const bool inv = t->spacing == HELM27_SPACING_INVG;
        const double need_lo = inv ? fh / static_cast<double>(c_hi) : static_cast<double>(c_lo) / fh;
        const double need_hi = inv ? fh / static_cast<double>(c_lo) : static_cast<double>(c_hi) / fh;
        double v_min = 0;
        int n_w = 0;
        if ((st = widen_range(t, need_lo, need_hi, &v_min, &n_w))) return fail(st);
        helm27_table* wide = nullptr;
        if ((st = build_table_like(t, v_min, n_w, &wide))) return fail(st);
        op->table = *wide;
        delete wide;
        if ((st = index_pass())) return fail(st);
    }
    hipFree(d_cnt);
    d_cnt = nullptr;
    op->n_clamped = static_cast<int64_t>(cnt[0]);
    float cmin, cmax;
    {
        const unsigned lo = static_cast<unsigned>(cnt[2]), hi = static_cast<unsigned>(cnt[3]);
        std::memcpy(&cmin, &lo, sizeof(float));
        std::memcpy(&cmax, &hi, sizeof(float));
    }
    op->cmin = cmin;
    op->cmax = cmax;
    op->g_min_model = static_cast<double>(cmin) / fh;
    op->g_max_model = static_cast<double>(cmax) / fh;
    g.c_ref = P.c_ref > 0 ? P.c_ref : static_cast<double>(cmax);

    const helm27_table& T = op->table;
    if ((st = grid_setup(&g, T.w7.data(), T.n_g, wmode == HELM27_WEIGHTS_FIXED ? 1 : 0))) return fail(st);
    // the explicit tile shape a large grid starts from when one of its
    // settings is changed (launches choose per call while auto_tile is set)
    if (g.N >= (int64_t(1) << 23)) {
        g.kernel_variant = 2;
        g.plain_ry[0] = 1;
        g.wave_zchunk = 16;
    }
    // idx is monotone in c, so the smallest / largest velocities give its range
    {
        const int ia = host_index(cmin, fh, T.g_min, T.dg, T.n_g, T.spacing);
        const int ib = host_index(cmax, fh, T.g_min, T.dg, T.n_g, T.spacing);
        g.idx_lo = std::min(ia, ib);
        g.idx_hi = std::max(ia, ib);
    }
    if (wmode == HELM27_WEIGHTS_GAM) {
        if (hipMalloc(&g.d_row_f, N * sizeof(EntryCoef<float>)) != hipSuccess) return fail(HELM27_ENOMEM);
        if (hipMalloc(&g.d_row_d, N * sizeof(EntryCoef<double>)) != hipSuccess) return fail(HELM27_ENOMEM);
        g.bytes += N * (sizeof(EntryCoef<float>) + sizeof(EntryCoef<double>));
        if ((st = launch_gam_average<float>(g, g.d_row_f, stream))) return fail(st);
        if ((st = launch_gam_average<double>(g, g.d_row_d, stream))) return fail(st);
    }
    if (flags & HELM27_STORE_C64) {
        if (hipMalloc(&op->d_coef_f, coef_elems(N) * sizeof(float2)) != hipSuccess) return fail(HELM27_ENOMEM);
        g.bytes += coef_elems(N) * sizeof(float2);
        if ((st = launch_fill_stored<float>(g, op->d_coef_f, 1.0, 0.0, stream))) return fail(st);
    }
    if (flags & HELM27_STORE_C128) {
        if (hipMalloc(&op->d_coef_d, coef_elems(N) * sizeof(double2)) != hipSuccess) return fail(HELM27_ENOMEM);
        g.bytes += coef_elems(N) * sizeof(double2);
        if ((st = launch_fill_stored<double>(g, op->d_coef_d, 1.0, 0.0, stream))) return fail(st);
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return fail(HELM27_EDEVICE);
    *out = op;
    return HELM27_OK;
}
}  // namespace h27

extern "C" int helm27_assemble(helm27_ctx* ctx, const helm27_table* t, const float* vel, int nx, int ny, int nz,
                               double h, double freq, const helm27_pml* pml, int flags, helm27_op** out) {
    return h27::op_create(ctx, t, vel, nx, ny, nz, h, freq, pml, flags, nullptr, out);
}

void solver_free(helm27_op* op);  // solver.cpp

extern "C" void helm27_op_destroy(helm27_op* op) {
    if (!op) return;
    solver_free(op);
    grid_free(&op->g);
    hipFree(op->d_coef_f);
    hipFree(op->d_coef_d);
    delete op;
}

extern "C" int helm27_op_info(const helm27_op* op, helm27_op_desc* o) {
    if (!op || !o) return HELM27_EINVAL;
    o->nx = op->g.nx;
    o->ny = op->g.ny;
    o->nz = op->g.nz;
    o->h = op->g.h;
    o->freq = op->freq;
    o->omega = op->g.omega;
    o->n_g = op->g.n_g;
    o->n_clamped = op->n_clamped;
    o->g_min_model = op->g_min_model;
    o->g_max_model = op->g_max_model;
    o->device_bytes = op->g.bytes;
    o->auto_tile = op->g.auto_tile ? 1 : 0;
    o->kernel_variant = op->g.kernel_variant;
    o->rows_fp32 = op->g.plain_ry[0];
    o->rows_fp64 = op->g.plain_ry[1];
    o->zchunk = op->g.wave_zchunk;
    o->rhs_block = op->g.rhs_block;
    o->rhs_order = op->g.rhs_order;
    o->table_spacing = op->table.spacing;
    o->table_min = op->table.g_min;
    o->table_step = op->table.dg;
    return HELM27_OK;
}

extern "C" int helm27_op_table_weights(const helm27_op* op, double* w7) {
    if (!op || !w7) return HELM27_EINVAL;
    std::memcpy(w7, op->table.w7.data(), op->table.w7.size() * sizeof(double));
    return HELM27_OK;
}

extern "C" int helm27_export_index(const helm27_op* op, uint16_t* idx) {
    if (!op || !idx) return HELM27_EINVAL;
    H27_CHECK_HIP(hipMemcpy(idx, op->g.d_idx, op->g.N * sizeof(uint16_t), hipMemcpyDeviceToHost));
    return HELM27_OK;
}

extern "C" int helm27_export_csr(const helm27_op* op, int64_t* nnz_out, int64_t* indptr, int64_t* indices,
                                 double* vals) {
    if (!op) return HELM27_EINVAL;
    const GridOp& g = op->g;
    const int64_t nnz = static_cast<int64_t>(3 * g.nx - 2) * (3 * g.ny - 2) * (3 * g.nz - 2);
    if (nnz_out) *nnz_out = nnz;
    if (!indptr) return HELM27_OK;
    if (!indices || !vals) return HELM27_EINVAL;
    void* d_coef = nullptr;
    if (hipMalloc(&d_coef, coef_elems(g.N) * sizeof(double2)) != hipSuccess) return HELM27_ENOMEM;
    int st = launch_fill_stored<double>(g, d_coef, 1.0, 0.0, nullptr);
    std::vector<double> hco;
    if (st == HELM27_OK) {
        hco.resize(static_cast<size_t>(coef_elems(g.N)) * 2);
        if (hipMemcpy(hco.data(), d_coef, hco.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            st = HELM27_EDEVICE;
    }
    hipFree(d_coef);
    if (st) return st;
    int64_t k = 0;
    indptr[0] = 0;
    const int64_t plane = static_cast<int64_t>(g.nx) * g.ny;
    for (int64_t i = 0; i < g.N; ++i) {
        const int x = static_cast<int>(i % g.nx), y = static_cast<int>((i / g.nx) % g.ny),
                  z = static_cast<int>(i / plane);
        for (int s = 0; s < 27; ++s) {
            const int dz = s / 9 - 1, dy = (s / 3) % 3 - 1, dx = s % 3 - 1;
            if (x + dx < 0 || x + dx >= g.nx || y + dy < 0 || y + dy >= g.ny || z + dz < 0 || z + dz >= g.nz)
                continue;
            indices[k] = i + dx + static_cast<int64_t>(g.nx) * dy + plane * dz;
            vals[2 * k] = hco[2 * static_cast<size_t>(coef_at(i, s))];
            vals[2 * k + 1] = hco[2 * static_cast<size_t>(coef_at(i, s)) + 1];
            ++k;
        }
        indptr[i + 1] = k;
    }
    return k == nnz ? HELM27_OK : HELM27_EDEVICE;
}

extern "C" int helm27_apply(helm27_op* op, const void* u, void* y, int nrhs, int dtype, int variant, void* stream) {
    if (!op || !u || !y || nrhs <= 0) return HELM27_EINVAL;
    if (u == y) return HELM27_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (variant == HELM27_RECOMPUTE) {
        if (dtype == HELM27_C64) return launch_stencil<float>(op->g, 0, 1.0, 0.0, u, y, nullptr, 0.0, nrhs, s);
        if (dtype == HELM27_C128) return launch_stencil<double>(op->g, 0, 1.0, 0.0, u, y, nullptr, 0.0, nrhs, s);
        return HELM27_EINVAL;
    }
    if (variant == HELM27_STORED) {
        if (dtype == HELM27_C64) {
            if (!op->d_coef_f) return HELM27_EINVAL;
            return launch_apply_stored<float>(op->g, op->d_coef_f, u, y, nrhs, s);
        }
        if (dtype == HELM27_C128) {
            if (!op->d_coef_d) return HELM27_EINVAL;
            return launch_apply_stored<double>(op->g, op->d_coef_d, u, y, nrhs, s);
        }
    }
    if (variant == HELM27_STORED_T) {
        if (dtype == HELM27_C64) {
            if (!op->d_coef_f) return HELM27_EINVAL;
            return launch_apply_stored_t<float>(op->g, op->d_coef_f, u, y, nullptr, nrhs, s);
        }
        if (dtype == HELM27_C128) {
            if (!op->d_coef_d) return HELM27_EINVAL;
            return launch_apply_stored_t<double>(op->g, op->d_coef_d, u, y, nullptr, nrhs, s);
        }
    }
    return HELM27_EINVAL;
}

extern "C" int helm27_apply_many(helm27_op* const* ops, int n_ops, const void* const* u, void* const* y,
                                 const int* nrhs, int dtype, void* stream) {
    if (n_ops < 0 || (n_ops > 0 && (!ops || !u || !y || !nrhs))) return HELM27_EINVAL;
    if (dtype != HELM27_C64 && dtype != HELM27_C128) return HELM27_EINVAL;
    std::vector<const GridOp*> g(static_cast<size_t>(n_ops));
    for (int i = 0; i < n_ops; ++i) {
        if (!ops[i] || nrhs[i] < 0) return HELM27_EINVAL;
        if (nrhs[i] > 0 && (!u[i] || !y[i] || u[i] == y[i])) return HELM27_EINVAL;
        if (i > 0 && ops[i]->ctx != ops[0]->ctx) return HELM27_EINVAL;
        g[i] = &ops[i]->g;
    }
    if (n_ops == 0) return HELM27_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return dtype == HELM27_C64 ? launch_stencil_batch<float>(g.data(), n_ops, u, y, nrhs, s)
                               : launch_stencil_batch<double>(g.data(), n_ops, u, y, nrhs, s);
}

extern "C" int helm27_set_tuning(helm27_op* op, int dtype, int rows_per_wave) {
    if (!op || rows_per_wave < 1 || rows_per_wave > 4) return HELM27_EINVAL;
    if (dtype == HELM27_C64) op->g.plain_ry[0] = rows_per_wave;
    else if (dtype == HELM27_C128) op->g.plain_ry[1] = rows_per_wave;
    else return HELM27_EINVAL;
    op->g.auto_tile = false;
    return HELM27_OK;
}

extern "C" int helm27_tune(helm27_op* op, int nrhs, int dtype, void* stream, int* best_rows) {
    if (!op || nrhs <= 0 || (dtype != HELM27_C64 && dtype != HELM27_C128)) return HELM27_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t vb = dtype == HELM27_C64 ? 8 : 16;
    const size_t bytes = static_cast<size_t>(op->g.N) * nrhs * vb;
    void *u = nullptr, *y = nullptr;
    if (hipMalloc(&u, bytes) != hipSuccess) return HELM27_ENOMEM;
    if (hipMalloc(&y, bytes) != hipSuccess) {
        hipFree(u);
        return HELM27_ENOMEM;
    }
    int st = HELM27_OK;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (hipMemsetAsync(u, 0, bytes, s) != hipSuccess) st = HELM27_EDEVICE;
    const int slot = dtype == HELM27_C64 ? 0 : 1;
    float best = 1e30f;
    int best_ry = op->g.plain_ry[slot], best_zc = op->g.wave_zchunk, best_var = op->g.kernel_variant;
    int best_nb = op->g.rhs_block, best_order = op->g.rhs_order;
    op->g.auto_tile = false;   // the tuner measures explicit shapes and keeps the fastest
    const int zchunks[5] = {0, 8, 16, 32, 64};   // 0 = automatic
    const int variants[2] = {0, 2};
    // right-hand sides per box wavefront: 1, and for several FP32 right-hand
    // sides 2 and 4 (block tiles, one row per wavefront)
    const int nbs[3] = {1, 2, 4};
    const int n_nb = (dtype == HELM27_C64 && nrhs >= 2) ? (nrhs >= 4 ? 3 : 2) : 1;
    const int n_order = nrhs >= 2 ? 2 : 1;   // right-hand side slowest, then fastest
    for (int oi = 0; oi < n_order && st == HELM27_OK; ++oi)
    for (int ni = 0; ni < n_nb && st == HELM27_OK; ++ni)
    for (int vi = 0; vi < 2 && st == HELM27_OK; ++vi)
    for (int ry = 1; ry <= 4 && st == HELM27_OK; ++ry) {
        if (ni > 0 && (vi == 0 || ry > 1)) continue;   // grouped right-hand sides: variant 2, one row
        for (int zi = 0; zi < 5 && st == HELM27_OK; ++zi) {
            if (zchunks[zi] > op->g.nz) continue;
            op->g.rhs_block = nbs[ni];
            op->g.rhs_order = oi == 0 ? 2 : 1;
            op->g.kernel_variant = variants[vi];
            op->g.plain_ry[slot] = ry;
            op->g.wave_zchunk = zchunks[zi];
            if (!stencil_wave_path(op->g, dtype == HELM27_C128)) continue;
            for (int w = 0; w < 2 && st == HELM27_OK; ++w)
                st = helm27_apply(op, u, y, nrhs, dtype, HELM27_RECOMPUTE, s);
            (void)hipEventRecord(e0, s);
            const int reps = 10;
            for (int r = 0; r < reps && st == HELM27_OK; ++r)
                st = helm27_apply(op, u, y, nrhs, dtype, HELM27_RECOMPUTE, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) st = HELM27_EDEVICE;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (st == HELM27_OK && ms < best) {
                best = ms;
                best_ry = ry;
                best_zc = zchunks[zi];
                best_var = variants[vi];
                best_nb = nbs[ni];
                best_order = oi == 0 ? 2 : 1;
            }
        }
    }
    op->g.plain_ry[slot] = best_ry;
    op->g.wave_zchunk = best_zc;
    op->g.kernel_variant = best_var;
    op->g.rhs_block = n_nb > 1 ? best_nb : op->g.rhs_block;
    op->g.rhs_order = n_order > 1 ? best_order : op->g.rhs_order;
    if (best_rows) *best_rows = best_ry;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hipFree(u);
    hipFree(y);
    return st;
}

extern "C" int helm27_set_kernel_variant(helm27_op* op, int variant) {
    if (!op || variant < 0 || variant > 2) return HELM27_EINVAL;
    op->g.kernel_variant = variant;
    op->g.auto_tile = false;
    return HELM27_OK;
}

extern "C" int helm27_set_attenuation(helm27_op* op, double Q) {
    if (!op || std::isnan(Q) || Q < 0) return HELM27_EINVAL;
    // k^2 = omega^2 / c~^2 with c~ = c (1 - i/(2Q)): factor 1 / (1 - i/(2Q))^2
    double re = 1.0, im = 0.0;
    if (Q > 0 && std::isfinite(Q)) {
        const double a = 1.0, b = -0.5 / Q;             // 1 - i/(2Q)
        const double sr = a * a - b * b, si = 2.0 * a * b;   // (1 - i/(2Q))^2
        const double d = sr * sr + si * si;
        re = sr / d;
        im = -si / d;
    }
    op->g.att_re = re;
    op->g.att_im = im;
    solver_free(op);   // coarse levels are rebuilt with the new factor
    hipStream_t s = nullptr;
    int st = HELM27_OK;
    if (op->d_coef_f && (st = h27::launch_fill_stored<float>(op->g, op->d_coef_f, 1.0, 0.0, s))) return st;
    if (op->d_coef_d && (st = h27::launch_fill_stored<double>(op->g, op->d_coef_d, 1.0, 0.0, s))) return st;
    H27_CHECK_HIP(hipStreamSynchronize(s));
    return HELM27_OK;
}

extern "C" int helm27_set_rhs_block(helm27_op* op, int nb) {
    if (!op || !(nb == 0 || nb == 1 || nb == 2 || nb == 4)) return HELM27_EINVAL;
    op->g.rhs_block = nb;
    return HELM27_OK;
}

extern "C" int helm27_set_rhs_order(helm27_op* op, int order) {
    if (!op || order < 0 || order > 2) return HELM27_EINVAL;
    op->g.rhs_order = order;
    return HELM27_OK;
}

extern "C" int helm27_set_zchunk(helm27_op* op, int zchunk) {
    if (!op || zchunk < 0 || zchunk == 1 || zchunk > 4096) return HELM27_EINVAL;
    op->g.wave_zchunk = zchunk;
    op->g.auto_tile = false;
    return HELM27_OK;
}
