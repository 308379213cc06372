// Wavefront-per-tile 27-point stencil (apply, residual, damped Jacobi).
//
// Operator (paper Sec. 2.1 with per-row weights, Sec. 3.1): for an output row
// with table entry E and kappa = k^2 (a + i b) ((a, b) = (1, 0) for the
// physical operator),
//   A u = (1/h^2) [ sum_a T_a + beta2 sum_{a<b} T_a T_b + beta3 T_x T_y T_z ] u
//       + kappa   [ m0 XXX + 2 m1 sum UXX + 4 m2 sum UUX + 8 m3 UUU ] u
// with T, U, X the (stretched) 1D second difference, neighbour half-sum and
// node stretch; an axis absent from a product contributes X.
//
// One wavefront per work item: 62 output columns along its lane axis (lanes
// 0 and 63 are halo), R rows along the other in-plane axis, a chunk of z
// planes marched in registers, one right-hand side.
//   * All control flow is wave-uniform (scalar registers): the work item, the
//     z loop, the plane kind, the row count and the grid-edge case.
//   * In-plane neighbours along the lane axis come from cross-lane DPP shifts
//     of the values the wave loaded, along the row axis from the R + 2 rows it
//     loads per plane, along z from the previous planes kept in registers.
//   * Software pipeline: the loads of plane q + 2 and the per-point data of
//     output plane q are issued before plane q is combined; loads go to
//     clamped (always valid) addresses and the zero outside the grid is
//     applied when the plane is used.  The z loop is unrolled three times so
//     the three load buffers, plane slots and per-point slots rotate by
//     renaming, not copying.
//   * The slice of the weight table the grid uses is staged in LDS per block
//     (stiffness weights pre-scaled by 1/h^2).
//   * Blocks are renumbered so that each XCD (blocks dispatched round-robin
//     over the 8 XCDs) runs a contiguous range of work items, and rows shared
//     by neighbouring tiles are re-read from its own L2.
// Two kinds of work items share a launch:
//   * box tiles (x and y unstretched, lanes along x): per plane the centre c,
//     4-face sum f and 4-diagonal sum e; the output is a 9-term combination
//     with real coefficients, complex in z-PML planes (uniform per plane);
//   * PML-frame tiles (lanes along x in groups of 64 or 16): the separable
//     contractions a = XX u, b = (TX + XT) u, c = TT u, d = (UX + XU) u,
//     e = UU u with the complex 1D factors of the lane node and of the row
//     node, then the same z combination.
#include "stencil.h"

namespace h27 {

// LDS copy of one table entry: s = stiffness class weights times 1/h^2,
// m = mass class weights, b2 / b3 = unscaled beta2 / beta3 (frame formula).
template <typename R>
struct TabEntry {
    R s[4];
    R m[4];
    R b2, b3, pad0, pad1;
};

// lane i <- lane i + 1 (wshl) and lane i <- lane i - 1 (wshr), whole wavefront
__device__ __forceinline__ float wshl(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float wshr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double wshl(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double wshr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// the same within each row of 16 lanes
__device__ __forceinline__ float rshl(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
}
__device__ __forceinline__ float rshr(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));
}
__device__ __forceinline__ double rshl(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x101, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x101, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double rshr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b & 0xffffffffLL), 0x111, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), 0x111, 0xF, 0xF, true);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// neighbours along the lane axis for a lane-group width of 64 (whole wave) or 16 (DPP rows)
template <int LW, typename R>
__device__ __forceinline__ Cx<R> nxt_g(Cx<R> v) {
    if (LW == 64) return Cx<R>{wshl(v.re), wshl(v.im)};
    return Cx<R>{rshl(v.re), rshl(v.im)};
}
template <int LW, typename R>
__device__ __forceinline__ Cx<R> prv_g(Cx<R> v) {
    if (LW == 64) return Cx<R>{wshr(v.re), wshr(v.im)};
    return Cx<R>{rshr(v.re), rshr(v.im)};
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// reciprocal: v_rcp_f32 (1 ulp) in the FP32 kernels, a correctly rounded
// division in the FP64 kernels
__device__ __forceinline__ float rcp_of(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_of(double x) { return 1.0 / x; }

template <typename R>
__device__ __forceinline__ Cx<R> inv_of(Cx<R> a) {
    const R d = rcp_of(a.re * a.re + a.im * a.im);
    return Cx<R>{a.re * d, -a.im * d};
}

// the value a mode stores for the operator row acc = (A u)_i
template <typename R, int MODE>
__device__ __forceinline__ Cx<R> finish(R omega_j, Cx<R> acc, Cx<R> diag, Cx<R> xcen,
                                        typename V2<R>::T bb) {
    if (MODE == MODE_APPLY) return acc;
    const Cx<R> rr{bb.x - acc.re, bb.y - acc.im};
    if (MODE == MODE_RESID) return rr;
    return xcen + omega_j * (rr * inv_of(diag));
}

// per-point data of one output plane: table index, velocity and (residual /
// Jacobi modes) the right-hand side
template <typename R, int NR>
struct Meta {
    int idx[NR];
    float c[NR];
    typename V2<R>::T b[NR];
};

template <typename R, int NR>
struct BoxPlane {
    Cx<R> c[NR], f[NR], e[NR];
};

// ---------------------------------------------------------------------------
// unstretched-box tile
template <typename R, int MODE, bool SHIFTED, int RY, bool ROWC>
__device__ __forceinline__ void box_item(const WaveArgs<R>& a, const TabEntry<R>* tab, const AxisNode<R>* zn,
                                         int tile, int zc, int rhs, int lane) {
    using V = typename V2<R>::T;
    const GridData<R>& g = a.g;
    const int tx = tile % a.ntx, ty = tile / a.ntx;
    const int xb = a.px0 + tx * kWaveCols - 1;              // x of lane 0
    const int gx = xb + lane;
    const bool outx = lane >= 1 && lane <= kWaveCols && gx < a.px0 + a.pw;
    const bool inx = gx >= 0 && gx < g.nx;
    const int gxc = min(max(gx, 0), g.nx - 1);
    const int y0 = a.py0 + ty * RY;
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const int nrow = min(RY, a.py0 + a.ph - y0);            // output rows of this tile
    const bool edge = xb < 0 || xb + 63 >= g.nx || y0 - 1 < 0 || y0 + RY >= g.ny;
    unsigned off[RY + 2];
    bool okk[RY + 2];
#pragma unroll
    for (int k = 0; k < RY + 2; ++k) {
        const int yy = y0 - 1 + k;
        okk[k] = inx && yy >= 0 && yy < g.ny;
        off[k] = static_cast<unsigned>(min(max(yy, 0), g.ny - 1) * g.nx + gxc);
    }
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;
    V* const yrhs = a.y + static_cast<int64_t>(rhs) * g.N;
    const V* brhs = (MODE == MODE_APPLY) ? nullptr : a.b + static_cast<int64_t>(rhs) * g.N;
    const R sig = g.inv_h2;

    auto load = [&](int q, V (&L)[RY + 2]) __attribute__((always_inline)) {
        const int qc = min(max(q, 0), g.nz - 1);
        const V* p = u + static_cast<int64_t>(qc) * g.plane;
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) L[k] = p[off[k]];
    };
    auto load_meta = [&](int q, Meta<R, RY>& M) __attribute__((always_inline)) {
        const int64_t pb = static_cast<int64_t>(q) * g.plane;
        const uint16_t* ip = g.idx + pb;
        const float* cp = g.c + pb;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!ROWC) M.idx[r] = static_cast<int>(ip[off[r + 1]]);
            M.c[r] = cp[off[r + 1]];
            if (MODE != MODE_APPLY) M.b[r] = brhs[pb + off[r + 1]];
        }
    };
    // plane q from its raw loads: zero outside the grid
    auto unpack = [&](int q, const V (&L)[RY + 2], Cx<R> (&U)[RY + 2]) __attribute__((always_inline)) {
        if (q < 0 || q >= g.nz) {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) U[k] = zero<R>();
        } else if (edge) {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) U[k] = Cx<R>{okk[k] ? L[k].x : R(0), okk[k] ? L[k].y : R(0)};
        } else {
#pragma unroll
            for (int k = 0; k < RY + 2; ++k) U[k] = Cx<R>{L[k].x, L[k].y};
        }
    };
    auto output = [&](int zo, const Meta<R, RY>& M, const BoxPlane<R, RY>& A, const BoxPlane<R, RY>& B,
                      const BoxPlane<R, RY>& C) __attribute__((always_inline)) {
        const AxisNode<R> Z = zn[zo];
        const int64_t pb = static_cast<int64_t>(zo) * g.plane;
        V* yp = yrhs + pb;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            R s0, s1, s2, s3, m0, m1, m2, m3;
            if (ROWC) {
                const EntryCoef<R> F = g.rowcoef[pb + off[r + 1]];
                s0 = sig * F.s0; s1 = sig * F.s1; s2 = sig * F.s2; s3 = sig * F.s3;
                m0 = F.m0; m1 = F.m1; m2 = F.m2; m3 = F.m3;
            } else {
                const TabEntry<R>& E = tab[M.idx[r] - a.tab_lo];
                s0 = E.s[0]; s1 = E.s[1]; s2 = E.s[2]; s3 = E.s[3];
                m0 = E.m[0]; m1 = E.m[1]; m2 = E.m[2]; m3 = E.m[3];
            }
            const R cvr = static_cast<R>(M.c[r]);
            const R kap = g.omega2 * rcp_of(cvr * cvr);
            Cx<R> acc, diag;
            if (Z.plain) {
                const Cx<R> Fc = B.f[r] + A.c[r] + C.c[r];
                const Cx<R> Ec = B.e[r] + A.f[r] + C.f[r];
                const Cx<R> Co = A.e[r] + C.e[r];
                if (SHIFTED) {
                    const R kr = kap * g.shift_re, ks = kap * g.shift_im;
                    const Cx<R> K0{s0 + kr * m0, ks * m0}, K1{s1 + kr * m1, ks * m1};
                    const Cx<R> K2{s2 + kr * m2, ks * m2}, K3{s3 + kr * m3, ks * m3};
                    acc = K0 * B.c[r];
                    cmac(acc, K1, Fc);
                    cmac(acc, K2, Ec);
                    cmac(acc, K3, Co);
                    diag = K0;
                } else {
                    const R A0 = s0 + kap * m0, A1 = s1 + kap * m1, A2 = s2 + kap * m2, A3 = s3 + kap * m3;
                    acc = A0 * B.c[r];
                    rmac(acc, A1, Fc);
                    rmac(acc, A2, Ec);
                    rmac(acc, A3, Co);
                    diag = Cx<R>{A0, R(0)};
                }
            } else {
                // z-stretched plane: stiffness sig (s1 T_z + ...), mass kappa (2 m1 U_z + ...)
                const R b2 = s2 + R(2) * s3;   // sig * beta2
                const Cx<R> tm{Z.tm_re, Z.tm_im}, tp{Z.tp_re, Z.tp_im};
                const Cx<R> t0 = -(tm + tp);
                const Cx<R> xz{Z.xi_re, Z.xi_im};
                const Cx<R> um{Z.um_re, Z.um_im}, up{Z.up_re, Z.up_im};
                const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
                const Cx<R> kum = kc * um, kup = kc * up, kxz = kc * xz;
                const Cx<R> Kcm = s1 * tm + (R(2) * m1) * kum;
                const Cx<R> Kfm = s2 * tm + (R(2) * m2) * kum;
                const Cx<R> Kem = s3 * tm + (R(2) * m3) * kum;
                const Cx<R> Kcp = s1 * tp + (R(2) * m1) * kup;
                const Cx<R> Kfp = s2 * tp + (R(2) * m2) * kup;
                const Cx<R> Kep = s3 * tp + (R(2) * m3) * kup;
                const Cx<R> Kc0 = s1 * t0 + (R(4) * b2 - R(4) * sig) * xz + m0 * kxz;
                const Cx<R> Kf0 = s2 * t0 + (sig - R(2) * b2) * xz + m1 * kxz;
                const Cx<R> Ke0 = s3 * t0 + b2 * xz + m2 * kxz;
                acc = Kcm * A.c[r];
                cmac(acc, Kfm, A.f[r]);
                cmac(acc, Kem, A.e[r]);
                cmac(acc, Kc0, B.c[r]);
                cmac(acc, Kf0, B.f[r]);
                cmac(acc, Ke0, B.e[r]);
                cmac(acc, Kcp, C.c[r]);
                cmac(acc, Kfp, C.f[r]);
                cmac(acc, Kep, C.e[r]);
                diag = Kc0;
            }
            V bb{};
            if (MODE != MODE_APPLY) bb = M.b[r];
            const Cx<R> o = finish<R, MODE>(a.omega_j, acc, diag, B.c[r], bb);
            if (outx && r < nrow) {
                V ov;
                ov.x = o.re;
                ov.y = o.im;
                yp[off[r + 1]] = ov;
            }
        }
    };
    // one z step: plane q enters, output plane q - 1 leaves
    // plane q + 2 and the per-point data of plane q + 1 are loaded two steps
    // ahead of their use; past the chunk the last plane is loaded again, so
    // every step issues the same loads and the waits stay exact
    auto step = [&](int q, bool out, const V (&Lc)[RY + 2], V (&Ln)[RY + 2], const BoxPlane<R, RY>& A,
                    const BoxPlane<R, RY>& B, BoxPlane<R, RY>& C, const Meta<R, RY>& Mc, Meta<R, RY>& Mn)
                    __attribute__((always_inline)) {
        load(min(q + 2, z1), Ln);
        load_meta(min(q + 1, z1 - 1), Mn);
        Cx<R> U[RY + 2];
        unpack(q, Lc, U);
        Cx<R> sx[RY + 2];
#pragma unroll
        for (int k = 0; k < RY + 2; ++k) sx[k] = nxt_g<64>(U[k]) + prv_g<64>(U[k]);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            C.c[r] = U[r + 1];
            C.f[r] = sx[r + 1] + U[r] + U[r + 2];
            C.e[r] = sx[r] + sx[r + 2];
        }
        if (out) output(q - 1, Mc, A, B, C);
    };

    // slot k % 3 (k = q - z0 + 1) holds the loads, the plane sums and the
    // per-point data of plane q
    V L0[RY + 2], L1[RY + 2], L2[RY + 2];
    BoxPlane<R, RY> P0, P1, P2;
    Meta<R, RY> M0, M1, M2;
    load(z0 - 1, L0);
    load(z0, L1);
    // planes z0 - 1 and z0 enter without an output; then one output per step
    step(z0 - 1, false, L0, L2, P1, P2, P0, M2, M1);
    step(z0, false, L1, L0, P2, P0, P1, M0, M2);
    int q = z0 + 1;
    for (;;) {
        step(q, true, L2, L1, P0, P1, P2, M1, M0);
        if (++q > z1) break;
        step(q, true, L0, L2, P1, P2, P0, M2, M1);
        if (++q > z1) break;
        step(q, true, L1, L0, P2, P0, P1, M0, M2);
        if (++q > z1) break;
    }
}

// ---------------------------------------------------------------------------
// PML-frame tile: lanes along x in groups of LW (LW - 2 output columns each,
// halo at both ends), 64 / LW groups stacked along y, RQ rows per lane
template <typename R>
struct Factors {
    Cx<R> tm, tp, t0, xi, um, up;
};
template <typename R>
__device__ __forceinline__ Factors<R> factors(const AxisNode<R>& n) {
    Factors<R> f;
    f.tm = Cx<R>{n.tm_re, n.tm_im};
    f.tp = Cx<R>{n.tp_re, n.tp_im};
    f.t0 = -(f.tm + f.tp);
    f.xi = Cx<R>{n.xi_re, n.xi_im};
    f.um = Cx<R>{n.um_re, n.um_im};
    f.up = Cx<R>{n.up_re, n.up_im};
    return f;
}

template <typename R, int NR>
struct FramePlane {
    Cx<R> a[NR], b[NR], c[NR], d[NR], e[NR], u[NR];
};

template <typename R, int MODE, bool SHIFTED, int RQ, int LW, bool ROWC>
__device__ __forceinline__ void frame_item(const WaveArgs<R>& a, const TabEntry<R>* tab, const AxisNode<R>* zn,
                                           int fr, int ft, int zc, int rhs, int lane) {
    using V = typename V2<R>::T;
    const GridData<R>& g = a.g;
    constexpr int NG = 64 / LW;
    const int lx = lane % LW, ly = lane / LW;
    const int tl = ft % a.fnl[fr], tq = ft / a.fnl[fr];
    const int x_org = a.fx0[fr], x_ext = a.fw[fr];
    const int y_org = a.fy0[fr], y_ext = a.fh[fr];
    const int lc = x_org + tl * (LW - 2) - 1 + lx;
    const bool outl = lx >= 1 && lx <= LW - 2 && lc < x_org + x_ext;
    const bool inl = lc >= 0 && lc < g.nx;
    const int lcc = min(max(lc, 0), g.nx - 1);
    const int q0 = y_org + (tq * NG + ly) * RQ;
    const int z0 = zc * a.zchunk;
    const int z1 = min(z0 + a.zchunk, g.nz);
    const Factors<R> FL = factors<R>(g.ax[lcc]);
    Factors<R> FQ[RQ];
    Cx<R> xLQ[RQ];
    unsigned off[RQ + 2];
    bool okk[RQ + 2];
#pragma unroll
    for (int k = 0; k < RQ + 2; ++k) {
        const int qq = q0 - 1 + k;
        okk[k] = inl && qq >= 0 && qq < g.ny;
        off[k] = static_cast<unsigned>(min(max(qq, 0), g.ny - 1) * g.nx + lcc);
    }
    bool outr[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        FQ[r] = factors<R>(g.ay[min(q0 + r, g.ny - 1)]);
        xLQ[r] = FL.xi * FQ[r].xi;
        outr[r] = outl && (q0 + r < y_org + y_ext);
    }
    const V* u = a.u + static_cast<int64_t>(rhs) * g.N;
    V* const yrhs = a.y + static_cast<int64_t>(rhs) * g.N;
    const V* brhs = (MODE == MODE_APPLY) ? nullptr : a.b + static_cast<int64_t>(rhs) * g.N;
    const R sig = g.inv_h2;

    auto load = [&](int q, V (&L)[RQ + 2]) __attribute__((always_inline)) {
        const int qc = min(max(q, 0), g.nz - 1);
        const V* p = u + static_cast<int64_t>(qc) * g.plane;
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) L[k] = p[off[k]];
    };
    auto load_meta = [&](int q, Meta<R, RQ>& M) __attribute__((always_inline)) {
        const int64_t pb = static_cast<int64_t>(q) * g.plane;
        const uint16_t* ip = g.idx + pb;
        const float* cp = g.c + pb;
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            if (!ROWC) M.idx[r] = static_cast<int>(ip[off[r + 1]]);
            M.c[r] = cp[off[r + 1]];
            if (MODE != MODE_APPLY) M.b[r] = brhs[pb + off[r + 1]];
        }
    };
    auto unpack = [&](int q, const V (&L)[RQ + 2], Cx<R> (&U)[RQ + 2]) __attribute__((always_inline)) {
        if (q < 0 || q >= g.nz) {
#pragma unroll
            for (int k = 0; k < RQ + 2; ++k) U[k] = zero<R>();
        } else {
#pragma unroll
            for (int k = 0; k < RQ + 2; ++k) U[k] = Cx<R>{okk[k] ? L[k].x : R(0), okk[k] ? L[k].y : R(0)};
        }
    };
    auto output = [&](int zo, const Meta<R, RQ>& M, const FramePlane<R, RQ>& A, const FramePlane<R, RQ>& B,
                      const FramePlane<R, RQ>& C) __attribute__((always_inline)) {
        const AxisNode<R> Z = zn[zo];
        const bool plainz = Z.plain != 0;
        const Factors<R> FZ = factors<R>(Z);
        const int64_t pb = static_cast<int64_t>(zo) * g.plane;
        V* yp = yrhs + pb;
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            R b2, b3, m0, m1, m2, m3;
            if (ROWC) {
                const EntryCoef<R> E = g.rowcoef[pb + off[r + 1]];
                b2 = E.beta2; b3 = E.beta3; m0 = E.m0; m1 = E.m1; m2 = E.m2; m3 = E.m3;
            } else {
                const TabEntry<R>& E = tab[M.idx[r] - a.tab_lo];
                b2 = E.b2; b3 = E.b3;
                m0 = E.m[0]; m1 = E.m[1]; m2 = E.m[2]; m3 = E.m[3];
            }
            const R cvr = static_cast<R>(M.c[r]);
            const R kap = g.omega2 * rcp_of(cvr * cvr);
            const Cx<R> kc = SHIFTED ? Cx<R>{kap * g.shift_re, kap * g.shift_im} : Cx<R>{kap, R(0)};
            Cx<R> PTA = A.a[r], PTB = B.a[r], PTC = C.a[r];
            rmac(PTA, b2, A.b[r]); rmac(PTA, b3, A.c[r]);
            rmac(PTB, b2, B.b[r]); rmac(PTB, b3, B.c[r]);
            rmac(PTC, b2, C.b[r]); rmac(PTC, b3, C.c[r]);
            const R w1 = R(2) * m1, w2 = R(4) * m2, w3 = R(8) * m3;
            Cx<R> PUA = w1 * A.a[r], PUC = w1 * C.a[r];
            rmac(PUA, w2, A.d[r]); rmac(PUA, w3, A.e[r]);
            rmac(PUC, w2, C.d[r]); rmac(PUC, w3, C.e[r]);
            Cx<R> PXs = B.b[r];
            rmac(PXs, b2, B.c[r]);
            Cx<R> PXm = m0 * B.a[r];
            rmac(PXm, w1, B.d[r]); rmac(PXm, w2, B.e[r]);
            Cx<R> stiff, mass;
            if (plainz) {   // T_z = (1, -2, 1), X_z = 1, U_z = (1/2, 0, 1/2)
                stiff = PTA + PTC + PXs - R(2) * PTB;
                mass = PXm + R(0.5) * (PUA + PUC);
            } else {
                stiff = FZ.tm * PTA;
                cmac(stiff, FZ.t0, PTB);
                cmac(stiff, FZ.tp, PTC);
                cmac(stiff, FZ.xi, PXs);
                mass = FZ.um * PUA;
                cmac(mass, FZ.up, PUC);
                cmac(mass, FZ.xi, PXm);
            }
            Cx<R> acc = sig * stiff;
            cmac(acc, kc, mass);
            Cx<R> diag = zero<R>();
            if (MODE == MODE_JACOBI) {
                const Factors<R>& Q = FQ[r];
                const Cx<R> ac = xLQ[r];
                const Cx<R> bc = FL.t0 * Q.xi + FL.xi * Q.t0;
                const Cx<R> cc = FL.t0 * Q.t0;
                Cx<R> pc = ac;
                rmac(pc, b2, bc);
                rmac(pc, b3, cc);
                Cx<R> pxs = bc;
                rmac(pxs, b2, cc);
                diag = sig * (FZ.t0 * pc + FZ.xi * pxs) + (m0 * kc) * (FZ.xi * ac);
            }
            V bb{};
            if (MODE != MODE_APPLY) bb = M.b[r];
            const Cx<R> o = finish<R, MODE>(a.omega_j, acc, diag, B.u[r], bb);
            if (outr[r]) {
                V ov;
                ov.x = o.re;
                ov.y = o.im;
                yp[off[r + 1]] = ov;
            }
        }
    };
    // plane q + 2 and the per-point data of plane q + 1 are loaded two steps
    // ahead of their use; past the chunk the last plane is loaded again, so
    // every step issues the same loads and the waits stay exact
    auto step = [&](int q, bool out, const V (&Lc)[RQ + 2], V (&Ln)[RQ + 2], const FramePlane<R, RQ>& A,
                    const FramePlane<R, RQ>& B, FramePlane<R, RQ>& C, const Meta<R, RQ>& Mc, Meta<R, RQ>& Mn)
                    __attribute__((always_inline)) {
        load(min(q + 2, z1), Ln);
        load_meta(min(q + 1, z1 - 1), Mn);
        Cx<R> U[RQ + 2];
        unpack(q, Lc, U);
        Cx<R> RT[RQ + 2], RU[RQ + 2];
#pragma unroll
        for (int k = 0; k < RQ + 2; ++k) {
            const Cx<R> vm = prv_g<LW>(U[k]), vp = nxt_g<LW>(U[k]);
            RT[k] = FL.tm * vm + FL.t0 * U[k] + FL.tp * vp;
            RU[k] = FL.um * vm + FL.up * vp;
        }
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            const Factors<R>& Q = FQ[r];
            C.u[r] = U[r + 1];
            C.a[r] = xLQ[r] * U[r + 1];
            C.b[r] = Q.xi * RT[r + 1] + FL.xi * (Q.tm * U[r] + Q.t0 * U[r + 1] + Q.tp * U[r + 2]);
            C.c[r] = Q.tm * RT[r] + Q.t0 * RT[r + 1] + Q.tp * RT[r + 2];
            C.d[r] = Q.xi * RU[r + 1] + FL.xi * (Q.um * U[r] + Q.up * U[r + 2]);
            C.e[r] = Q.um * RU[r] + Q.up * RU[r + 2];
        }
        if (out) output(q - 1, Mc, A, B, C);
    };

    // slot k % 3 (k = q - z0 + 1) holds the loads, the plane sums and the
    // per-point data of plane q
    V L0[RQ + 2], L1[RQ + 2], L2[RQ + 2];
    FramePlane<R, RQ> P0, P1, P2;
    Meta<R, RQ> M0, M1, M2;
    load(z0 - 1, L0);
    load(z0, L1);
    // planes z0 - 1 and z0 enter without an output; then one output per step
    step(z0 - 1, false, L0, L2, P1, P2, P0, M2, M1);
    step(z0, false, L1, L0, P2, P0, P1, M0, M2);
    int q = z0 + 1;
    for (;;) {
        step(q, true, L2, L1, P0, P1, P2, M1, M0);
        if (++q > z1) break;
        step(q, true, L0, L2, P1, P2, P0, M2, M1);
        if (++q > z1) break;
        step(q, true, L1, L0, P2, P0, P1, M0, M2);
        if (++q > z1) break;
    }
}

// register budget: 4 waves per SIMD (128 VGPRs) for FP32, 2 for FP64
template <typename R, int MODE, bool SHIFTED, int RY, int RQ, bool ROWC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2)))
void wave27_kernel(WaveArgs<R> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const GridData<R>& g = a.g;
    const int n_tab = ROWC ? 0 : a.n_tab;
    TabEntry<R>* tab = reinterpret_cast<TabEntry<R>*>(smem_raw);
    AxisNode<R>* zn = reinterpret_cast<AxisNode<R>*>(smem_raw + static_cast<size_t>(n_tab) * sizeof(TabEntry<R>));
    const R sig = g.inv_h2;
    for (int t = threadIdx.x; t < n_tab; t += kBlock) {
        const EntryCoef<R> E = g.entry[g.fixed ? 0 : a.tab_lo + t];   // fixed weights: one entry everywhere
        TabEntry<R> e;
        e.s[0] = sig * E.s0; e.s[1] = sig * E.s1; e.s[2] = sig * E.s2; e.s[3] = sig * E.s3;
        e.m[0] = E.m0; e.m[1] = E.m1; e.m[2] = E.m2; e.m[3] = E.m3;
        e.b2 = E.s2 + R(2) * E.s3;
        e.b3 = E.s3;
        e.pad0 = e.pad1 = R(0);
        tab[t] = e;
    }
    for (int t = threadIdx.x; t < g.nz; t += kBlock) zn[t] = g.az[t];
    __syncthreads();
    // XCD-contiguous block order: block b runs on XCD b % 8; the grid is at
    // most one resident wave per slot and each wave strides over the items
    const int nb = static_cast<int>(gridDim.x);
    const int bx = static_cast<int>(blockIdx.x);
    const int xcd = bx & 7, q8 = nb >> 3, r8 = nb & 7;
    const int lb = xcd * q8 + min(xcd, r8) + (bx >> 3);
    const int wave = uni(static_cast<int>(threadIdx.x) >> 6);
    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int ntile = a.n_frame + a.n_plain;
    for (int item = lb * (kBlock / 64) + wave; item < a.n_items; item += nb * (kBlock / 64)) {
        // item order: right-hand side fastest, then tile, then z chunk
        const int rhs = item % a.nrhs;
        const int t = item / a.nrhs;
        const int tile = t % ntile;
        const int zc = t / ntile;
        if (tile < a.n_frame) {
            int k = 0;
            while (k < 3 && tile >= a.fstart[k + 1]) ++k;
            if (a.flx[k])
                frame_item<R, MODE, SHIFTED, RQ, 64, ROWC>(a, tab, zn, k, tile - a.fstart[k], zc, rhs, lane);
            else
                frame_item<R, MODE, SHIFTED, RQ, 16, ROWC>(a, tab, zn, k, tile - a.fstart[k], zc, rhs, lane);
        } else {
            box_item<R, MODE, SHIFTED, RY, ROWC>(a, tab, zn, tile - a.n_frame, zc, rhs, lane);
        }
    }
}

template <typename R> struct FrameRows;
template <> struct FrameRows<float> { static constexpr int value = 1; };
template <> struct FrameRows<double> { static constexpr int value = 1; };

// blocks of one kernel that fit on the device at once (cached per kernel and
// LDS size; queried on the current device)
static int resident_blocks(const void* fn, size_t lds) {
    struct Entry { const void* fn; size_t lds; int dev; int blocks; };
    static thread_local Entry cache[64] = {};
    static thread_local int next = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    for (const Entry& e : cache)
        if (e.fn == fn && e.lds == lds && e.dev == dev) return e.blocks;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const int blocks = per_cu * cus;
    cache[next] = Entry{fn, lds, dev, blocks};
    next = (next + 1) % 64;
    return blocks;
}

template <typename R, int MODE, bool SHIFTED, int RY, bool ROWC>
static int launch_wave_k(const WaveArgs<R>& a, hipStream_t s) {
    constexpr int RQ = FrameRows<R>::value;
    const void* fn = reinterpret_cast<const void*>(&wave27_kernel<R, MODE, SHIFTED, RY, RQ, ROWC>);
    const size_t lds = wave_lds_bytes(ROWC ? 0 : a.n_tab, a.g.nz, sizeof(R) == 8);
    int blocks = (a.n_items + (kBlock / 64) - 1) / (kBlock / 64);
    const int cap = resident_blocks(fn, lds);
    if (cap <= 0) return HELM27_EDEVICE;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL((wave27_kernel<R, MODE, SHIFTED, RY, RQ, ROWC>), dim3(blocks), dim3(kBlock), lds, s, a);
    H27_CHECK_HIP(hipGetLastError());
    return HELM27_OK;
}

template <typename R, int MODE, bool SHIFTED, int RY>
static int launch_wave_ry(const WaveArgs<R>& a, hipStream_t s) {
    return a.g.rowcoef ? launch_wave_k<R, MODE, SHIFTED, RY, true>(a, s)
                       : launch_wave_k<R, MODE, SHIFTED, RY, false>(a, s);
}

template <typename R, int MODE, bool SHIFTED>
static int launch_wave_mode(const WaveArgs<R>& a, int ry, hipStream_t s) {
    switch (ry) {
        case 1: return launch_wave_ry<R, MODE, SHIFTED, 1>(a, s);
        case 2: return launch_wave_ry<R, MODE, SHIFTED, 2>(a, s);
        case 3: return launch_wave_ry<R, MODE, SHIFTED, 3>(a, s);
        case 4: return launch_wave_ry<R, MODE, SHIFTED, 4>(a, s);
        default: return HELM27_EINVAL;
    }
}

template <typename R>
int launch_wave(const WaveArgs<R>& a, int mode, bool shifted, int ry, int rq, hipStream_t s) {
    (void)rq;
    if (a.n_items <= 0) return HELM27_OK;
    switch (mode) {
        case MODE_APPLY:
            return shifted ? launch_wave_mode<R, MODE_APPLY, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_APPLY, false>(a, ry, s);
        case MODE_RESID:
            return shifted ? launch_wave_mode<R, MODE_RESID, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_RESID, false>(a, ry, s);
        case MODE_JACOBI:
            return shifted ? launch_wave_mode<R, MODE_JACOBI, true>(a, ry, s)
                           : launch_wave_mode<R, MODE_JACOBI, false>(a, ry, s);
        default:
            return HELM27_EINVAL;
    }
}
template int launch_wave<float>(const WaveArgs<float>&, int, bool, int, int, hipStream_t);
template int launch_wave<double>(const WaveArgs<double>&, int, bool, int, int, hipStream_t);

template <typename R>
int frame_rows() { return FrameRows<R>::value; }
template int frame_rows<float>();
template int frame_rows<double>();

size_t wave_lds_bytes(int n_tab, int nz, bool fp64) {
    return fp64 ? static_cast<size_t>(n_tab) * sizeof(TabEntry<double>) + static_cast<size_t>(nz) * sizeof(AxisNode<double>)
                : static_cast<size_t>(n_tab) * sizeof(TabEntry<float>) + static_cast<size_t>(nz) * sizeof(AxisNode<float>);
}

}  // namespace h27
