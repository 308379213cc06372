// Matrix-free 27-point stencil kernels (apply, residual, damped Jacobi).
//
// Operator (paper Sec. 2.1, [M + S] p with per-row weights, Sec. 3.1): for an
// output row at node (i, j, k) with table entry E and k^2 = omega^2 / c^2,
//
//   A u = sigma * [ sum_a T_a + beta2 sum_{a<b} T_a T_b + beta3 T_x T_y T_z ] u
//       + kappa * [ m0 XXX + 2 m1 sum UXX + 4 m2 sum UUX + 8 m3 UUU ] u
//
// with sigma = 1/h^2, kappa = k^2 (physical operator) or k^2 (a + i b) (the
// complex-shifted operator of the preconditioner), 1D factors T (stretched second
// difference), U (stretched neighbour half-sum), X (stretch at the node); an
// axis absent from a product contributes X.  In the unstretched interior this
// is exactly the weighted sum of the Cartesian, 45-degree-rotated and
// cube-diagonal stencils plus the consistent mass of Sec. 2.1.
//
// Evaluation: each block owns a tile of (x, y) columns and marches along z.
// A plane of u with a one-node halo is staged in LDS (double buffered, the
// next plane's global loads in flight while the current one is used).  Each
// input plane is reduced per column to a few in-plane contractions that are
// kept in registers for three consecutive planes, and the output row of the
// middle plane is formed from them:
//   * plain tiles (x and y unstretched, 64-wide rows -> coalesced along x):
//     centre c, 4-face sum f, 4-diagonal sum e per plane; the output is a
//     9-term combination whose coefficients are real in the interior and
//     complex in z-PML planes (uniform per plane, so no divergence);
//   * frame tiles (x- or y-PML columns, 16 x 16): the separable contractions
//     a = XX u, b = (TX + XT) u, c = TT u, d = (UX + XU) u, e = UU u with the
//     column's complex 1D factors, then the same z combination.
#include <algorithm>

#include "stencil.h"

namespace h27 {

template <typename R>
__device__ __forceinline__ EntryCoef<R> row_entry(const GridData<R>& g, int64_t i) {
    if (g.rowcoef) return g.rowcoef[i];
    const int e = g.fixed ? 0 : static_cast<int>(g.idx[i]);
    return g.entry[e];
}

template <typename R>
__device__ __forceinline__ Cx<R> nd(R re, R im) { return Cx<R>{re, im}; }

template <typename R, int MODE>
__device__ __forceinline__ void epilogue(const StencilArgs<R>& a, int rhs, int64_t i, Cx<R> acc,
                                         Cx<R> diag, Cx<R> xcen) {
    using V = typename V2<R>::T;
    V* y = a.y + static_cast<int64_t>(rhs) * a.g.N;
    if (MODE == MODE_APPLY) {
        st<R>(y + i, acc);
    } else {
        const Cx<R> bb = ld<R>(a.b + static_cast<int64_t>(rhs) * a.g.N + i);
        const Cx<R> r = bb - acc;
        if (MODE == MODE_RESID) {
            st<R>(y + i, r);
        } else {
            const Cx<R> q = r * cinv(diag);
            st<R>(y + i, xcen + a.omega_j * q);
        }
    }
}

// ---------------------------------------------------------------------------
// plain tiles
template <typename R, int MODE, bool SHIFTED, int ROWS>
__device__ __forceinline__ void plain_tile(const StencilArgs<R>& a, int tile, int z0, int z1, int rhs,
                                           typename V2<R>::T* lds) {
    using V = typename V2<R>::T;
    constexpr int TH = kPlainTY * ROWS;
    constexpr int LW = kPlainTX + 2, LH = TH + 2, LN = LW * LH;
    constexpr int NL = (LN + kBlock - 1) / kBlock;
    const GridData<R>& g = a.g;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int bx = tile % a.ptx, by = tile / a.ptx;
    const int x0 = a.px0 + bx * kPlainTX, y0 = a.py0 + by * TH;
    const int xe = a.px0 + a.pw, ye = a.py0 + a.ph;
    const int gx = x0 + tx;
    const bool colx = gx < xe;
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;

    V pre[NL];
    auto load_plane = [&](int q) {
#pragma unroll
        for (int s = 0; s < NL; ++s) {
            const int e = threadIdx.x + s * kBlock;
            V v;
            v.x = R(0);
            v.y = R(0);
            if (e < LN && q >= 0 && q < g.nz) {
                const int ly = e / LW, lx = e - ly * LW;
                const int xx = x0 - 1 + lx, yy = y0 - 1 + ly;
                if (xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny)
                    v = u[static_cast<int64_t>(q) * g.plane + static_cast<int64_t>(yy) * g.nx + xx];
            }
            pre[s] = v;
        }
    };

    Cx<R> cA[ROWS], fA[ROWS], eA[ROWS], cB[ROWS], fB[ROWS], eB[ROWS], cC[ROWS], fC[ROWS], eC[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        cA[r] = fA[r] = eA[r] = cB[r] = fB[r] = eB[r] = cC[r] = fC[r] = eC[r] = zero<R>();
    }
    int buf = 0;
    load_plane(z0 - 1);
    for (int q = z0 - 1; q <= z1; ++q) {
        V* L = lds + buf * LN;
#pragma unroll
        for (int s = 0; s < NL; ++s) {
            const int e = threadIdx.x + s * kBlock;
            if (e < LN) L[e] = pre[s];
        }
        if (q + 1 <= z1) load_plane(q + 1);
        __syncthreads();
        Cx<R> m[ROWS + 2], sx[ROWS + 2];
#pragma unroll
        for (int k = 0; k < ROWS + 2; ++k) {
            const V* row = L + (ty * ROWS + k) * LW + tx;
            const Cx<R> l = ld<R>(row), c = ld<R>(row + 1), rr = ld<R>(row + 2);
            m[k] = c;
            sx[k] = l + rr;
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            cA[r] = cB[r]; fA[r] = fB[r]; eA[r] = eB[r];
            cB[r] = cC[r]; fB[r] = fC[r]; eB[r] = eC[r];
            cC[r] = m[r + 1];
            fC[r] = sx[r + 1] + m[r] + m[r + 2];
            eC[r] = sx[r] + sx[r + 2];
        }
        buf ^= 1;
        const int zo = q - 1;
        if (zo < z0) continue;
        const AxisNode<R> Z = g.az[zo];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = y0 + ty * ROWS + r;
            if (!colx || gy >= ye) continue;
            const int64_t i = static_cast<int64_t>(zo) * g.plane + static_cast<int64_t>(gy) * g.nx + gx;
            const EntryCoef<R> E = row_entry(g, i);
            const R cv = static_cast<R>(g.c[i]);
            const R kap = g.omega2 / (cv * cv);
            const R sig = g.inv_h2;
            Cx<R> acc = zero<R>(), diag = zero<R>();
            if (Z.plain) {
                const Cx<R> Fc = fB[r] + cA[r] + cC[r];
                const Cx<R> Ec = eB[r] + fA[r] + fC[r];
                const Cx<R> Co = eA[r] + eC[r];
                const R A0 = sig * E.s0 + kap * E.m0, A1 = sig * E.s1 + kap * E.m1;
                const R A2 = sig * E.s2 + kap * E.m2, A3 = sig * E.s3 + kap * E.m3;
                if (SHIFTED) {
                    const R kr = kap * (g.shift_re - R(1)), ks = kap * g.shift_im;
                    const Cx<R> K0 = nd(A0 + kr * E.m0, ks * E.m0), K1 = nd(A1 + kr * E.m1, ks * E.m1);
                    const Cx<R> K2 = nd(A2 + kr * E.m2, ks * E.m2), K3 = nd(A3 + kr * E.m3, ks * E.m3);
                    cmac(acc, K0, cB[r]);
                    cmac(acc, K1, Fc);
                    cmac(acc, K2, Ec);
                    cmac(acc, K3, Co);
                    diag = K0;
                } else {
                    rmac(acc, A0, cB[r]);
                    rmac(acc, A1, Fc);
                    rmac(acc, A2, Ec);
                    rmac(acc, A3, Co);
                    diag = nd(A0, R(0));
                }
            } else {
                const Cx<R> tm = nd(Z.tm_re, Z.tm_im), tp = nd(Z.tp_re, Z.tp_im);
                const Cx<R> t0 = -(tm + tp);
                const Cx<R> xz = nd(Z.xi_re, Z.xi_im);
                const Cx<R> um = nd(Z.um_re, Z.um_im), up = nd(Z.up_re, Z.up_im);
                const Cx<R> kc = SHIFTED ? nd(kap * g.shift_re, kap * g.shift_im) : nd(kap, R(0));
                const Cx<R> kum = kc * um, kup = kc * up, kxz = kc * xz;
                // planes zo -/+ 1: T_z (s1 c + s2 f + s3 e) sigma + U_z 2 (m1 c + m2 f + m3 e) kappa
                const Cx<R> Kcm = (sig * E.s1) * tm + (R(2) * E.m1) * kum;
                const Cx<R> Kfm = (sig * E.s2) * tm + (R(2) * E.m2) * kum;
                const Cx<R> Kem = (sig * E.s3) * tm + (R(2) * E.m3) * kum;
                const Cx<R> Kcp = (sig * E.s1) * tp + (R(2) * E.m1) * kup;
                const Cx<R> Kfp = (sig * E.s2) * tp + (R(2) * E.m2) * kup;
                const Cx<R> Kep = (sig * E.s3) * tp + (R(2) * E.m3) * kup;
                // plane zo: T_z(0) (s1 c + s2 f + s3 e) sigma
                //          + X_z [(-4 + 4 b2) c + (1 - 2 b2) f + b2 e] sigma + X_z (m0 c + m1 f + m2 e) kappa
                const Cx<R> Kc0 = (sig * E.s1) * t0 + (sig * (R(4) * E.beta2 - R(4))) * xz + E.m0 * kxz;
                const Cx<R> Kf0 = (sig * E.s2) * t0 + (sig * (R(1) - R(2) * E.beta2)) * xz + E.m1 * kxz;
                const Cx<R> Ke0 = (sig * E.s3) * t0 + (sig * E.beta2) * xz + E.m2 * kxz;
                cmac(acc, Kcm, cA[r]);
                cmac(acc, Kfm, fA[r]);
                cmac(acc, Kem, eA[r]);
                cmac(acc, Kc0, cB[r]);
                cmac(acc, Kf0, fB[r]);
                cmac(acc, Ke0, eB[r]);
                cmac(acc, Kcp, cC[r]);
                cmac(acc, Kfp, fC[r]);
                cmac(acc, Kep, eC[r]);
                diag = Kc0;
            }
            epilogue<R, MODE>(a, rhs, i, acc, diag, cB[r]);
        }
    }
}

// ---------------------------------------------------------------------------
// frame tiles
template <typename R, int MODE, bool SHIFTED>
__device__ __forceinline__ void frame_tile(const StencilArgs<R>& a, int fb, int z0, int z1, int rhs,
                                           typename V2<R>::T* lds) {
    using V = typename V2<R>::T;
    constexpr int LW = kFrameT + 2, LN = LW * LW;
    constexpr int NL = (LN + kBlock - 1) / kBlock;
    const GridData<R>& g = a.g;
    int k = 0;
    while (k < 3 && fb >= a.fstart[k + 1]) ++k;
    const int t = fb - a.fstart[k];
    const int bx = t % a.ftx[k], by = t / a.ftx[k];
    const int x0 = a.fx0[k] + bx * kFrameT, y0 = a.fy0[k] + by * kFrameT;
    const int tx = threadIdx.x & (kFrameT - 1), ty = threadIdx.x / kFrameT;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool valid = gx < a.fx0[k] + a.fw[k] && gy < a.fy0[k] + a.fh[k];
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;

    // column factors
    Cx<R> txm = zero<R>(), txp = zero<R>(), xix = zero<R>(), uxm = zero<R>(), uxp = zero<R>();
    Cx<R> tym = zero<R>(), typ = zero<R>(), xiy = zero<R>(), uym = zero<R>(), uyp = zero<R>();
    if (valid) {
        const AxisNode<R> X = g.ax[gx];
        const AxisNode<R> Y = g.ay[gy];
        txm = nd(X.tm_re, X.tm_im); txp = nd(X.tp_re, X.tp_im); xix = nd(X.xi_re, X.xi_im);
        uxm = nd(X.um_re, X.um_im); uxp = nd(X.up_re, X.up_im);
        tym = nd(Y.tm_re, Y.tm_im); typ = nd(Y.tp_re, Y.tp_im); xiy = nd(Y.xi_re, Y.xi_im);
        uym = nd(Y.um_re, Y.um_im); uyp = nd(Y.up_re, Y.up_im);
    }
    const Cx<R> tx0 = -(txm + txp), ty0 = -(tym + typ);
    const Cx<R> xixy = xix * xiy;
    // in-plane contraction weights of the centre node (for the Jacobi diagonal)
    const Cx<R> a_c = xixy, b_c = tx0 * xiy + xix * ty0, c_c = tx0 * ty0;

    V pre[NL];
    auto load_plane = [&](int q) {
#pragma unroll
        for (int s = 0; s < NL; ++s) {
            const int e = threadIdx.x + s * kBlock;
            V v;
            v.x = R(0);
            v.y = R(0);
            if (e < LN && q >= 0 && q < g.nz) {
                const int ly = e / LW, lx = e - ly * LW;
                const int xx = x0 - 1 + lx, yy = y0 - 1 + ly;
                if (xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny)
                    v = u[static_cast<int64_t>(q) * g.plane + static_cast<int64_t>(yy) * g.nx + xx];
            }
            pre[s] = v;
        }
    };

    Cx<R> aP[3], bP[3], cP[3], dP[3], eP[3];
    Cx<R> cenB = zero<R>(), cenC = zero<R>();
#pragma unroll
    for (int p = 0; p < 3; ++p) aP[p] = bP[p] = cP[p] = dP[p] = eP[p] = zero<R>();
    int buf = 0;
    load_plane(z0 - 1);
    for (int q = z0 - 1; q <= z1; ++q) {
        V* L = lds + buf * LN;
#pragma unroll
        for (int s = 0; s < NL; ++s) {
            const int e = threadIdx.x + s * kBlock;
            if (e < LN) L[e] = pre[s];
        }
        if (q + 1 <= z1) load_plane(q + 1);
        __syncthreads();
        Cx<R> v[3][3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) v[dy][dx] = ld<R>(L + (ty + dy) * LW + tx + dx);
        Cx<R> RT[3], RU[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            RT[dy] = txm * v[dy][0] + tx0 * v[dy][1] + txp * v[dy][2];
            RU[dy] = uxm * v[dy][0] + uxp * v[dy][2];
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            aP[p] = aP[p + 1]; bP[p] = bP[p + 1]; cP[p] = cP[p + 1]; dP[p] = dP[p + 1]; eP[p] = eP[p + 1];
        }
        cenB = cenC;
        cenC = v[1][1];
        aP[2] = xixy * v[1][1];
        bP[2] = xiy * RT[1] + xix * (tym * v[0][1] + ty0 * v[1][1] + typ * v[2][1]);
        cP[2] = tym * RT[0] + ty0 * RT[1] + typ * RT[2];
        dP[2] = xiy * RU[1] + xix * (uym * v[0][1] + uyp * v[2][1]);
        eP[2] = uym * RU[0] + uyp * RU[2];
        buf ^= 1;
        const int zo = q - 1;
        if (zo < z0 || !valid) continue;
        const AxisNode<R> Z = g.az[zo];
        const int64_t i = static_cast<int64_t>(zo) * g.plane + static_cast<int64_t>(gy) * g.nx + gx;
        const EntryCoef<R> E = row_entry(g, i);
        const R cv = static_cast<R>(g.c[i]);
        const R kap = g.omega2 / (cv * cv);
        const R sig = g.inv_h2;
        const Cx<R> kc = SHIFTED ? nd(kap * g.shift_re, kap * g.shift_im) : nd(kap, R(0));
        const Cx<R> tzm = nd(Z.tm_re, Z.tm_im), tzp = nd(Z.tp_re, Z.tp_im);
        const Cx<R> tz0 = -(tzm + tzp);
        const Cx<R> xz = nd(Z.xi_re, Z.xi_im);
        const Cx<R> uzm = nd(Z.um_re, Z.um_im), uzp = nd(Z.up_re, Z.up_im);
        const R b2 = E.beta2, b3 = E.beta3;
        Cx<R> PT[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            PT[p] = aP[p];
            rmac(PT[p], b2, bP[p]);
            rmac(PT[p], b3, cP[p]);
        }
        Cx<R> PUm = zero<R>(), PUp = zero<R>();
        rmac(PUm, R(2) * E.m1, aP[0]); rmac(PUm, R(4) * E.m2, dP[0]); rmac(PUm, R(8) * E.m3, eP[0]);
        rmac(PUp, R(2) * E.m1, aP[2]); rmac(PUp, R(4) * E.m2, dP[2]); rmac(PUp, R(8) * E.m3, eP[2]);
        Cx<R> PXs = bP[1];
        rmac(PXs, b2, cP[1]);
        Cx<R> PXm = zero<R>();
        rmac(PXm, E.m0, aP[1]); rmac(PXm, R(2) * E.m1, dP[1]); rmac(PXm, R(4) * E.m2, eP[1]);
        Cx<R> stiff = tzm * PT[0];
        cmac(stiff, tz0, PT[1]);
        cmac(stiff, tzp, PT[2]);
        cmac(stiff, xz, PXs);
        Cx<R> mass = uzm * PUm;
        cmac(mass, uzp, PUp);
        cmac(mass, xz, PXm);
        Cx<R> acc = sig * stiff;
        cmac(acc, kc, mass);
        Cx<R> diag = zero<R>();
        if (MODE == MODE_JACOBI) {
            Cx<R> pc = a_c;
            rmac(pc, b2, b_c);
            rmac(pc, b3, c_c);
            Cx<R> pxs = b_c;
            rmac(pxs, b2, c_c);
            diag = sig * (tz0 * pc + xz * pxs) + (E.m0 * kc) * (xz * a_c);
        }
        epilogue<R, MODE>(a, rhs, i, acc, diag, cenB);
    }
}

template <typename R, int MODE, bool SHIFTED, int ROWS>
__global__ __launch_bounds__(kBlock) void stencil27_kernel(StencilArgs<R> a) {
    constexpr int TH = kPlainTY * ROWS;
    constexpr int LNP = (kPlainTX + 2) * (TH + 2);
    constexpr int LNF = (kFrameT + 2) * (kFrameT + 2);
    constexpr int LNMAX = LNP > LNF ? LNP : LNF;
    __shared__ typename V2<R>::T lds[2 * LNMAX];
    const int bid = blockIdx.x;
    const int z0 = blockIdx.y * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.g.nz);
    for (int rhs = blockIdx.z; rhs < a.nrhs; rhs += gridDim.z) {
        if (bid < a.n_plain_blocks)
            plain_tile<R, MODE, SHIFTED, ROWS>(a, bid, z0, z1, rhs, lds);
        else
            frame_tile<R, MODE, SHIFTED>(a, bid - a.n_plain_blocks, z0, z1, rhs, lds);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
template <typename R>
static GridData<R> grid_data(const GridOp& g, double shift_re, double shift_im);

template <>
GridData<float> grid_data<float>(const GridOp& g, double shift_re, double shift_im) {
    GridData<float> d{};
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.plane = static_cast<int64_t>(g.nx) * g.ny;
    d.N = g.N;
    d.c = g.d_c; d.idx = g.d_idx; d.entry = g.d_entry_f; d.rowcoef = g.d_row_f; d.fixed = g.fixed;
    d.ax = g.d_ax_f[0]; d.ay = g.d_ax_f[1]; d.az = g.d_ax_f[2];
    d.omega2 = static_cast<float>(g.omega * g.omega);
    d.inv_h2 = static_cast<float>(1.0 / (g.h * g.h));
    // mass factor = requested shift x the medium's attenuation factor
    d.shift_re = static_cast<float>(shift_re * g.att_re - shift_im * g.att_im);
    d.shift_im = static_cast<float>(shift_re * g.att_im + shift_im * g.att_re);
    d.mass_a = g.mass_a;
    d.zlo = g.zp_lo;
    d.zhi = g.zp_hi;
    return d;
}

template <>
GridData<double> grid_data<double>(const GridOp& g, double shift_re, double shift_im) {
    GridData<double> d{};
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.plane = static_cast<int64_t>(g.nx) * g.ny;
    d.N = g.N;
    d.c = g.d_c; d.idx = g.d_idx; d.entry = g.d_entry_d; d.rowcoef = g.d_row_d; d.fixed = g.fixed;
    d.ax = g.d_ax_d[0]; d.ay = g.d_ax_d[1]; d.az = g.d_ax_d[2];
    d.omega2 = g.omega * g.omega;
    d.inv_h2 = 1.0 / (g.h * g.h);
    d.shift_re = shift_re * g.att_re - shift_im * g.att_im;
    d.shift_im = shift_re * g.att_im + shift_im * g.att_re;
    d.mass_a = g.mass_a;
    d.zlo = g.zp_lo;
    d.zhi = g.zp_hi;
    return d;
}

template <typename R, int MODE, bool SHIFTED>
static int launch_mode(const StencilArgs<R>& args, dim3 grid, hipStream_t s) {
    H27_CHECK_HIP(launch(stencil27_kernel<R, MODE, SHIFTED, kRows>, grid, dim3(kBlock), 0, s, args));
    return HELM27_OK;
}

// LDS bytes one block may use on the current device (queried once per device)
static size_t lds_limit() {
    static std::mutex mu;
    static std::vector<size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 64 * 1024;
    std::lock_guard<std::mutex> lk(mu);
    if (static_cast<size_t>(dev) >= cache.size()) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int v = 0;
        cache[dev] = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0
                         ? static_cast<size_t>(v)
                         : 64 * 1024;
    }
    return cache[dev];
}

// whether the wavefront kernel serves this grid (else the LDS-tiled kernel)
bool stencil_wave_path(const GridOp& g, bool fp64) {
    const int n_tab = g.idx_hi - g.idx_lo + 1;   // the table slice the grid's indices span
    // the wavefront kernel addresses one right-hand side with 32-bit buffer
    // offsets: its byte size must stay below 2^31
    const int ry = g.mass_a ? 1 : g.plain_ry[fp64 ? 1 : 0];
    const size_t ring = g.kernel_variant == 2 ? wave_ring_bytes(ry, 1, fp64, g.mass_a != 0) : 0;
    // the first mass form runs on the wavefront kernels only
    return (g.kernel_variant == 0 || g.kernel_variant == 2 || g.mass_a) && n_tab > 0 &&
           static_cast<int64_t>(g.N) * (fp64 ? 16 : 8) < (int64_t(1) << 31) &&
           wave_ring_offset(g.d_row_f ? 0 : n_tab, z_lds_nodes(g.nz, g.zp_lo, g.zp_hi), fp64) + ring <= lds_limit();
}

template <typename R>
static int build_wave_args(const GridOp& g, const GridData<R>& gd, const void* u, void* y, const void* b,
                           double omega_j, int nrhs, bool batch, WaveArgs<R>& w, int& RY) {
    const Tiling& t = g.tiling;
    const int n_tab = g.idx_hi - g.idx_lo + 1;
    w.g = gd;
    constexpr bool fp64 = sizeof(R) == 8;
    RY = g.plain_ry[fp64 ? 1 : 0];
    int variant = g.kernel_variant, zc_set = g.wave_zchunk;
    if (batch) {
        // batched small grids: per-wavefront tiles (two rows in FP32, one
        // in FP64 or with the first mass form), automatic z chunks
        RY = fp64 ? 1 : 2;
        variant = 0;
        zc_set = 0;
    } else if (g.auto_tile) {
        // HBM-bound launches (2^23 or more point-RHS pairs): box rows shared
        // across the block (variant 2), one row per wavefront in 32-plane
        // chunks for one RHS, two rows in 16-plane chunks for several
        // (400x400x200: 181 us against 185 us with 16-plane chunks and
        // 203-213 us for variant 0; 201x201x101 x 16 RHS: 390 us against
        // 431 us); smaller launches keep the latency-friendlier
        // per-wavefront tiles with automatic chunks
        const bool big = static_cast<int64_t>(g.N) * nrhs >= (int64_t(1) << 23);
        RY = fp64 ? g.plain_ry[1] : (big && nrhs >= 2 ? 2 : (big ? 1 : 2));
        variant = 0;
        zc_set = 0;
        const size_t ring = wave_ring_bytes(g.mass_a ? 1 : RY, 1, fp64, g.mass_a != 0);
        if (big && wave_ring_offset(g.d_row_f ? 0 : n_tab, z_lds_nodes(g.nz, g.zp_lo, g.zp_hi), fp64) + ring <= lds_limit()) {
            variant = 2;
            zc_set = nrhs == 1 ? 32 : 16;
        }
    }
    const int RQ = frame_rows<R>();
    w.n_items = 0;
    // several right-hand sides per box wavefront (FP32 block tiles, one
    // row per wavefront) when asked for (helm27_set_rhs_block or the
    // tuner), the group's vectors are addressable with 32-bit buffer
    // offsets and its row ring fits in LDS.  Automatic: one (measured on
    // 400x400x200 x 16 and 201x201x101 x 64: groups of 2 or 4 change the
    // time by -4 % to +4 %; the per-RHS cost is the row traffic of u
    // and y, not the per-point data the groups share)
    if (g.mass_a) {   // first mass form: one row per wavefront (two spill registers)
        RY = 1;
        if (variant == 1) variant = 0;
    }
    int NB = 1;
    if (!fp64 && nrhs >= 2 && g.rhs_block > 1 && !g.mass_a && !batch) {
        NB = g.rhs_block;
        const bool fits = static_cast<int64_t>(g.N) * 8 * NB < (int64_t(1) << 31) &&
                          wave_ring_offset(g.d_row_f ? 0 : n_tab, z_lds_nodes(g.nz, g.zp_lo, g.zp_hi), fp64) + wave_ring_bytes(1, NB, fp64) <=
                              lds_limit();
        if (!fits) NB = 1;
    }
    if (NB > 1) {
        variant = 2;
        RY = 1;
        if (g.auto_tile) zc_set = static_cast<int64_t>(g.N) * nrhs >= (int64_t(1) << 23) ? 32 : 0;
    }
    w.nb = NB;
    w.ngrp = (nrhs + NB - 1) / NB;
    // multi-RHS item order: right-hand side slowest by default (each
    // right-hand side's pass keeps its tiles' shared halo rows and planes
    // close in time, as a single-RHS launch does; 201x201x101 x 64:
    // 1.81 -> 1.52 ms), or fastest (the per-point data of a tile are
    // shared by its right-hand sides in L2)
    w.rhs_outer = g.rhs_order == 1 ? 0 : 1;
    const int TC = kWaveCols;
    w.px0 = t.plain_x0; w.py0 = t.plain_y0; w.pw = t.plain_w; w.ph = t.plain_h;
    Rect fr[4] = {t.frame[0], t.frame[1], t.frame[2], t.frame[3]};
    // The box is cut into 62-column tiles; a last partial tile costs as
    // much as a full one.  When the left / right strips (14-column lane
    // groups) have room for those leftover columns in the groups they
    // already use, they take them (the general formula holds for
    // unstretched columns too) and the box becomes whole tiles
    // (400 wide with an 8-node PML: 6 tiles instead of 6 + 12 columns).
    if (w.pw > TC && fr[2].w > 0 && fr[3].w > 0) {
        const int left = w.pw % TC;
        const int capl = 14 * ((fr[2].w + 13) / 14) - fr[2].w, capr = 14 * ((fr[3].w + 13) / 14) - fr[3].w;
        if (left > 0 && left <= capl + capr) {
            const int a = std::min(left, capl);
            w.px0 += a;
            w.pw -= left;
            fr[2].w += a;
            fr[3].x0 = w.px0 + w.pw;
            fr[3].w = g.nx - fr[3].x0;
        }
    }
    // variant 2: box tiles grouped blk_waves along y per block item (rows shared in LDS)
    w.blk = variant == 2 ? 1 : 0;
    const int BW = blk_waves(fp64);
    const int rows_per_tile = w.blk ? BW * RY : RY;
    w.ntx = w.pw > 0 ? (w.pw + TC - 1) / TC : 0;
    w.nty = w.ph > 0 ? (w.ph + rows_per_tile - 1) / rows_per_tile : 0;
    w.n_plain = w.ntx * w.nty;
    int accf = 0;
    for (int k = 0; k < 4; ++k) {
        const Rect& r = fr[k];
        w.fx0[k] = r.x0; w.fy0[k] = r.y0; w.fw[k] = r.w; w.fh[k] = r.h;
        // lanes always run along x: whole-wave groups (62 columns) for strips
        // spanning x (bottom / top, or the whole grid), 16-lane groups (14
        // columns, 4 groups stacked along y) for the narrow left / right strips
        const bool wide = !(k >= 2 && t.plain_w > 0);
        w.flx[k] = wide ? 1 : 0;
        const int cols = wide ? kWaveCols : 14, rows = wide ? RQ : 4 * RQ;
        const bool empty = r.w <= 0 || r.h <= 0;
        w.fnl[k] = empty ? 1 : (r.w + cols - 1) / cols;
        w.fnq[k] = empty ? 0 : (r.h + rows - 1) / rows;
        w.fstart[k] = accf;
        accf += empty ? 0 : w.fnl[k] * w.fnq[k];
    }
    w.fstart[4] = accf;
    w.n_frame = accf;
    // work items: wavefront items (variant 0) or block items of BW wavefronts (variant 2)
    const int64_t tiles = static_cast<int64_t>(w.blk ? (w.n_frame + BW - 1) / BW + w.n_plain : w.n_plain + w.n_frame) *
                          w.ngrp;
    if (tiles <= 0) return HELM27_OK;   // nothing to do (n_items stays 0)
    const int64_t target = w.blk ? 1024 : 4096;
    int64_t nzc = (target + tiles - 1) / tiles;
    int zc = static_cast<int>((g.nz + nzc - 1) / nzc);
    zc = std::max(2, std::min(16, zc));
    if (zc_set > 0) zc = zc_set;
    w.zchunk = std::min(zc, g.nz);
    w.nzc = (g.nz + w.zchunk - 1) / w.zchunk;
    w.nrhs = nrhs;
    const int64_t items = tiles * w.nzc;
    if (items > (int64_t(1) << 30)) return HELM27_EINVAL;
    w.n_items = static_cast<int>(items);
    w.tab_lo = g.idx_lo;
    w.n_tab = n_tab;
    // launches whose input and output vectors together exceed the 256 MiB
    // last-level cache store an apply's output non-temporally and read their
    // per-point data non-temporally when every point is visited by one
    // right-hand-side group only (several groups re-read them; smaller
    // launches keep everything cached for the solver's next kernel).  Only
    // unshifted block-tile applies have the non-temporal instances.
    const bool big = 2.0 * static_cast<double>(g.N) * nrhs * sizeof(typename V2<R>::T) >= 256.0 * (1 << 20);
    w.nt_store = big && !batch ? 1 : 0;
    w.nt_meta = big && w.ngrp == 1 ? 1 : 0;
    w.u = static_cast<const typename V2<R>::T*>(u);
    w.y = static_cast<typename V2<R>::T*>(y);
    w.b = static_cast<const typename V2<R>::T*>(b);
    w.omega_j = static_cast<R>(omega_j);
    return HELM27_OK;
}

template <typename R>
int launch_stencil(const GridOp& g, int mode, double shift_re, double shift_im, const void* u, void* y, const void* b,
                   double omega_j, int nrhs, hipStream_t s) {
    if (nrhs <= 0) return HELM27_OK;
    const Tiling& t = g.tiling;
    StencilArgs<R> a{};
    a.g = grid_data<R>(g, shift_re, shift_im);
    const bool shifted = !(shift_re * g.att_re - shift_im * g.att_im == 1.0 &&
                           shift_re * g.att_im + shift_im * g.att_re == 0.0);
    if (!a.g.entry || !a.g.ax || !a.g.ay || !a.g.az) return HELM27_EINVAL;
    a.px0 = t.plain_x0; a.py0 = t.plain_y0; a.pw = t.plain_w; a.ph = t.plain_h;
    a.ptx = t.n_plain_tiles_x > 0 ? t.n_plain_tiles_x : 1;
    a.rows = kRows;
    int acc = 0;
    for (int k = 0; k < 4; ++k) {
        a.fx0[k] = t.frame[k].x0; a.fy0[k] = t.frame[k].y0; a.fw[k] = t.frame[k].w; a.fh[k] = t.frame[k].h;
        a.ftx[k] = t.frame_tiles_x[k] > 0 ? t.frame_tiles_x[k] : 1;
        a.fstart[k] = acc;
        acc += t.frame_tiles_x[k] * t.frame_tiles_y[k];
    }
    a.fstart[4] = acc;
    a.n_plain_blocks = t.n_plain_blocks;
    a.zchunk = t.zchunk;
    a.nrhs = nrhs;
    a.u = static_cast<const typename V2<R>::T*>(u);
    a.y = static_cast<typename V2<R>::T*>(y);
    a.b = static_cast<const typename V2<R>::T*>(b);
    a.omega_j = static_cast<R>(omega_j);
    // Default: the wavefront-per-tile kernel for the whole grid (box + frame
    // work items in one launch).  Variant 1 keeps the LDS-tiled kernel below.
    const int n_tab = g.idx_hi - g.idx_lo + 1;
    const bool use_wave = stencil_wave_path(g, sizeof(R) == 8);
    if ((mode == MODE_JACOBI0 || g.mass_a) && !use_wave) return HELM27_EINVAL;   // wavefront kernel only
    if (use_wave) {
        WaveArgs<R> w{};
        int RY = 1;
        const int st = build_wave_args<R>(g, a.g, u, y, b, omega_j, nrhs, false, w, RY);
        if (st != HELM27_OK || w.n_items == 0) return st;
        return launch_wave<R>(w, mode, shifted, RY, frame_rows<R>(), s);
    }
    const int nblk = a.n_plain_blocks + t.n_frame_blocks;
    if (nblk == 0) return HELM27_OK;
    const int per_rhs = nblk * t.n_zchunks;
    int groups = (4096 + per_rhs - 1) / per_rhs;
    if (groups > nrhs) groups = nrhs;
    if (groups < 1) groups = 1;
    if (groups > 65535) groups = 65535;
    dim3 grid(nblk, t.n_zchunks, groups);
    const bool sh = shifted;
    switch (mode) {
        case MODE_APPLY:
            return sh ? launch_mode<R, MODE_APPLY, true>(a, grid, s) : launch_mode<R, MODE_APPLY, false>(a, grid, s);
        case MODE_RESID:
            return sh ? launch_mode<R, MODE_RESID, true>(a, grid, s) : launch_mode<R, MODE_RESID, false>(a, grid, s);
        case MODE_JACOBI:
            return sh ? launch_mode<R, MODE_JACOBI, true>(a, grid, s) : launch_mode<R, MODE_JACOBI, false>(a, grid, s);
        default:
            return HELM27_EINVAL;
    }
}

// y_i = A_i u_i for several grids: fused launches of the wavefront kernel,
// grouped by kernel instance (attenuation, per-row coefficients, mass form)
template <typename R>
int launch_stencil_batch(const GridOp* const* g, int n, const void* const* u, void* const* y, const int* nrhs,
                         hipStream_t s) {
    constexpr bool fp64 = sizeof(R) == 8;
    std::vector<WaveArgs<R>> w(static_cast<size_t>(n));
    std::vector<int> key(static_cast<size_t>(n), -1);
    for (int i = 0; i < n; ++i) {
        const GridOp& G = *g[i];
        if (nrhs[i] == 0) continue;
        const int n_tab = G.idx_hi - G.idx_lo + 1;
        if (n_tab <= 0 || static_cast<int64_t>(G.N) * (fp64 ? 16 : 8) >= (int64_t(1) << 31) ||
            wave_ring_offset(G.d_row_f ? 0 : n_tab, z_lds_nodes(G.nz, G.zp_lo, G.zp_hi), fp64) > lds_limit())
            return HELM27_EINVAL;
        const GridData<R> gd = grid_data<R>(G, 1.0, 0.0);
        if (!gd.entry || !gd.ax || !gd.ay || !gd.az) return HELM27_EINVAL;
        const bool shifted = !(G.att_re == 1.0 && G.att_im == 0.0);
        int RY = 1;
        const int st = build_wave_args<R>(G, gd, u[i], y[i], nullptr, 0.0, nrhs[i], true, w[i], RY);
        if (st != HELM27_OK) return st;
        if (w[i].n_items == 0) continue;
        key[i] = (shifted ? 1 : 0) | (gd.rowcoef ? 2 : 0) | (G.mass_a ? 4 : 0);
    }
    std::vector<const WaveArgs<R>*> grp;
    for (int k = 0; k < 8; ++k) {
        grp.clear();
        for (int i = 0; i < n; ++i)
            if (key[i] == k) grp.push_back(&w[i]);
        if (grp.empty()) continue;
        const int st = launch_wave_batch<R>(grp.data(), static_cast<int>(grp.size()), (k & 1) != 0, (k & 2) != 0,
                                            (k & 4) != 0, s);
        if (st != HELM27_OK) return st;
    }
    return HELM27_OK;
}

template int launch_stencil_batch<float>(const GridOp* const*, int, const void* const*, void* const*, const int*,
                                         hipStream_t);
template int launch_stencil_batch<double>(const GridOp* const*, int, const void* const*, void* const*, const int*,
                                          hipStream_t);

template int launch_stencil<float>(const GridOp&, int, double, double, const void*, void*, const void*, double, int, hipStream_t);
template int launch_stencil<double>(const GridOp&, int, double, double, const void*, void*, const void*, double, int, hipStream_t);

}  // namespace h27
